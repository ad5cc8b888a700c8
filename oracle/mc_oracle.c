/*
 * mc_oracle.c -- plain, slow, double-precision CPU oracle for the Monte Carlo
 * path engine ("Tensor Processing Units for Financial Monte Carlo",
 * Belletti et al., arXiv:1906.02818).
 *
 * TEST INFRASTRUCTURE ONLY. It exists to check the HIP library. Only the tests,
 * the smoke check and the CPU-baseline leg of the benchmark may load it. It
 * shares no code, header, table or helper with the HIP library; the only thing
 * the two sides agree on is the published definition of Philox4x32-10 and the
 * counter layout written down below, which each side implements on its own.
 *
 * Style: one path at a time, one time step at a time, every quantity in
 * double precision, in the order the method states it. No blocking, fusion
 * or reordering. OpenMP only splits the independent paths across threads;
 * every path writes its own output row, so the result does not depend on the
 * thread count.
 *
 * Per-path outputs are written row-major: out[p * n_channels + c].
 *
 * The arithmetic-Asian call price (GBM channel "asian", Heston channel
 * "asian") has no closed form for many fixings. It is pinned by its K = 0
 * mean (exact), its zero-volatility value at any K (exact), its ordering
 * against the geometric Asian, its pathwise tangents, its one-fixing case
 * (the European call) and, at K > 0 with volatility, the two-fixing price
 * (a one-dimensional quadrature of a Black-Scholes inner expectation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------ */
/* 1. Philox4x32-10: the keyed counter-based generator of Salmon, Moraes,    */
/*    Dror and Shaw (SC'11), which the paper uses on GPUs (Sec. IV-A, Sec.   */
/*    VI). Ten rounds; each round multiplies counter words 0 and 2 by the    */
/*    two Philox multipliers as full 32x32->64-bit products and mixes the    */
/*    halves with words 1, 3 and the key; the key is bumped by the two Weyl  */
/*    constants between rounds.                                              */
/* ------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                       uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {            /* key schedule between rounds */
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* 2. Counter layout (the paper leaves it open; this is the reading the     */
/*    library must follow). Normal number k of path p in stream `tag` comes  */
/*    from Philox block j = floor(k/4), counter (j, p mod 2^32, p >> 32,    */
/*    tag), key (seed mod 2^32, seed >> 32), and uses slot k mod 4 of that   */
/*    block. Per time step i a model with d normals per step uses            */
/*    k = i*d + a, a = 0..d-1.                                               */
/* ------------------------------------------------------------------------ */
void orc_block_words(uint64_t seed, uint32_t tag, uint64_t path, uint64_t j,
                     uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)j, (uint32_t)(path & 0xffffffffu),
                       (uint32_t)(path >> 32), tag};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    (void)(j >> 32);            /* blocks beyond 2^32 per path are not used */
    orc_philox4x32_10(ctr, key, out);
}

/* 3. Uniform in the open interval (0,1): u = (2*(w >> 9) + 1) / 2^24.
 *    Odd multiples of 2^-24, so 0 and 1 never occur and u -> 1-u maps the
 *    set onto itself. */
double orc_uniform(uint32_t w)
{
    return (double)(2u * (w >> 9) + 1u) * 0x1p-24;
}

/* 4. Box-Muller on one Philox block: slots 0,1 use words (w0 radius, w1
 *    angle) as r cos, r sin; slots 2,3 use (w2 radius, w3 angle). */
static void box_muller_block(const uint32_t w[4], double z[4])
{
    for (int h = 0; h < 2; ++h) {
        double u_r = orc_uniform(w[2 * h]);
        double u_a = orc_uniform(w[2 * h + 1]);
        double rad = sqrt(-2.0 * log(u_r));
        double ang = 2.0 * M_PI * u_a;
        z[2 * h] = rad * cos(ang);
        z[2 * h + 1] = rad * sin(ang);
    }
}

/* Normal number k of path `path`. */
double orc_normal(uint64_t seed, uint32_t tag, uint64_t path, uint64_t k)
{
    uint32_t w[4];
    double z[4];
    orc_block_words(seed, tag, path, k / 4, w);
    box_muller_block(w, z);
    return z[k % 4];
}

/* Normals k0 .. k0+count-1 of one path (convenience for the tests). */
void orc_normals(uint64_t seed, uint32_t tag, uint64_t path, uint64_t k0,
                 uint64_t count, double *z)
{
    for (uint64_t i = 0; i < count; ++i)
        z[i] = orc_normal(seed, tag, path, k0 + i);
}

/* Raw words of sampled (path, block) pairs, for the bit-exact tests. */
void orc_words_many(uint64_t seed, uint32_t tag, uint64_t n,
                    const uint64_t *paths, const uint64_t *blocks,
                    uint32_t *out /* n x 4 */)
{
    for (uint64_t i = 0; i < n; ++i)
        orc_block_words(seed, tag, paths[i], blocks[i], out + 4 * i);
}

/* The normals of one path are drawn block by block in index order. This
 * small cursor keeps the current block so that a path costs one Philox call
 * per four normals, exactly like reading orc_normal(k) for k = 0,1,2,... */
typedef struct {
    uint64_t seed, path;
    uint32_t tag;
    uint64_t next_k;
    uint64_t block;
    double z[4];
    /* Sobol' source (section 11): when V is set, block j's words are the
     * shifted Sobol' coordinates 4j .. 4j+3 of point `path`. */
    const uint32_t *V, *shift;
} normal_stream;

uint32_t orc_sobol_word(const uint32_t *V, int dim, uint64_t point);

static void ns_init(normal_stream *s, uint64_t seed, uint32_t tag, uint64_t path)
{
    s->seed = seed; s->tag = tag; s->path = path; s->next_k = 0;
    s->block = UINT64_MAX;
    s->V = NULL;
    s->shift = NULL;
}

static double ns_next(normal_stream *s)
{
    uint64_t k = s->next_k++;
    uint64_t j = k / 4;
    if (j != s->block) {
        uint32_t w[4];
        if (s->V) {
            for (int t = 0; t < 4; ++t)
                w[t] = orc_sobol_word(s->V, (int)(4 * j) + t, s->path) ^ s->shift[4 * j + t];
        } else {
            orc_block_words(s->seed, s->tag, s->path, j, w);
        }
        box_muller_block(w, s->z);
        s->block = j;
    }
    return s->z[k % 4];
}

static double pos(double x) { return x > 0.0 ? x : 0.0; }

/* ------------------------------------------------------------------------ */
/* 5. One-dimensional GBM under the risk-neutral measure, dS = r S dt +      */
/*    sigma S dW, discretised by Euler-Maruyama (Eq. 1 with mu = r S,        */
/*    sigma(S) = sigma S; scheme of Sec. II-A.1). Two schemes:               */
/*      scheme 0 (log-Euler): x = ln S, x += (r - sigma^2/2) dt              */
/*                                          + sigma sqrt(dt) Z               */
/*      scheme 1 (Euler on S): S *= 1 + r dt + sigma sqrt(dt) Z              */
/*    `coarsen` c >= 1 couples a coarse path to a fine one as in multilevel  */
/*    Monte Carlo (Sec. V-B): coarse step k uses Z = (sum of the c fine      */
/*    normals k*c .. k*c+c-1) / sqrt(c); the step count n is the coarse one. */
/*                                                                           */
/*    Per-path channels (discount factor e^{-rT} included):                  */
/*      0 European call (S_n - K)+                                           */
/*      1 arithmetic-average Asian call (A - K)+, A = mean of S_1..S_n       */
/*      2 geometric-average Asian call (G - K)+, G = exp(mean of ln S_i)     */
/*      3 discretely monitored up-and-out call (S_n - K)+ 1{S_i < B all i}   */
/*      4 pathwise delta of 0     5 pathwise vega (d/dsigma) of 0            */
/*      6 pathwise delta of 1     7 pathwise vega of 1                       */
/*      8 e^{-rT} S_n             9 (Brownian-bridge) up-and-out call with   */
/*                                  continuous monitoring, see below         */
/*     10 knock-out margin max_i ln(S_i/B) of channel 3                      */
/*     11 knock-out margin max_i (m_i - ln B) of channel 9                   */
/*    The pathwise derivatives are forward tangents (Sec. I-A.3 greeks).     */
/*    Channel 9: between grid values x, y of ln S the maximum of the         */
/*    Brownian bridge is drawn as m = (x + y + sqrt((x-y)^2                  */
/*    - 2 dt sigma^2 ln U))/2 with U uniform (Sec. VI-A.1, exotic put);      */
/*    U is word (i mod 4) of block floor(i/4) of stream tag+5, scheme 0 only.*/
/* ------------------------------------------------------------------------ */
#define GBM_CH 12

/* extras = 0 computes the payoff channels 0-3 and 8 only (the others are
   NaN): no tangents, no Brownian-bridge stream, no margins. */
static void gbm_one_path(const double *prm, int n, int scheme, int coarsen,
                         uint64_t seed, uint32_t tag, uint64_t path, int extras,
                         double *o)
{
    const double S0 = prm[0], r = prm[1], sig = prm[2], T = prm[3];
    const double K = prm[4], B = prm[5];
    const double dt = T / n;
    const double sdt = sqrt(dt);
    const double disc = exp(-r * T);
    normal_stream ns;
    ns_init(&ns, seed, tag, path);

    double S = S0, x = log(S0);
    double dS_dS0 = 1.0, dS_dsig = 0.0;     /* tangents of S_i */
    double dx_dsig = 0.0;                   /* tangent of x_i (scheme 0) */
    double sumS = 0.0, sum_lnS = 0.0, sum_dS_dS0 = 0.0, sum_dS_dsig = 0.0;
    int alive = 1, alive_bb = 1;
    const double lnB = log(B);
    double margin = -INFINITY, margin_bb = -INFINITY;

    for (int i = 0; i < n; ++i) {
        double Z = 0.0;
        for (int c = 0; c < coarsen; ++c) Z += ns_next(&ns);
        Z /= sqrt((double)coarsen);
        double x_prev = x;
        if (scheme == 0) {
            x = x + (r - 0.5 * sig * sig) * dt + sig * sdt * Z;
            S = exp(x);
            if (extras) {
                dx_dsig = dx_dsig - sig * dt + sdt * Z;
                dS_dS0 = S / S0;
                dS_dsig = S * dx_dsig;
            }
        } else {
            double f = 1.0 + r * dt + sig * sdt * Z;
            dS_dsig = dS_dsig * f + S * sdt * Z;
            S = S * f;
            dS_dS0 = dS_dS0 * f;
            x = log(S);
        }
        sumS += S;
        sum_lnS += log(S);
        if (!(S < B)) alive = 0;
        if (!extras) continue;
        sum_dS_dS0 += dS_dS0;
        sum_dS_dsig += dS_dsig;
        if (log(S) - lnB > margin) margin = log(S) - lnB;
        if (scheme == 0) {
            uint32_t w[4];
            orc_block_words(seed, tag + 5u, path, (uint64_t)i / 4, w);
            double U = orc_uniform(w[i % 4]);
            double d = x_prev - x;
            double m = 0.5 * (x_prev + x + sqrt(d * d - 2.0 * dt * sig * sig * log(U)));
            if (!(m < lnB)) alive_bb = 0;
            if (m - lnB > margin_bb) margin_bb = m - lnB;
        }
    }
    double A = sumS / n;
    double G = exp(sum_lnS / n);
    double call = pos(S - K);
    o[0] = disc * call;
    o[1] = disc * pos(A - K);
    o[2] = disc * pos(G - K);
    o[3] = alive ? disc * call : 0.0;
    o[8] = disc * S;
    if (!extras) {
        o[4] = o[5] = o[6] = o[7] = o[9] = o[10] = o[11] = NAN;
        return;
    }
    o[4] = S > K ? disc * dS_dS0 : 0.0;
    o[5] = S > K ? disc * dS_dsig : 0.0;
    o[6] = A > K ? disc * sum_dS_dS0 / n : 0.0;
    o[7] = A > K ? disc * sum_dS_dsig / n : 0.0;
    o[9] = (scheme == 0 && alive_bb) ? disc * call : 0.0;
    o[10] = margin;
    o[11] = margin_bb;
}

int orc_gbm_channels(void) { return GBM_CH; }

/* prm = {S0, r, sigma, T, K, B}; every channel. */
void orc_gbm(const double *prm, int n_steps, int scheme, int coarsen,
             uint64_t seed, uint32_t tag, uint64_t path0, uint64_t n_paths,
             double *out)
{
#pragma omp parallel for schedule(static)
    for (long long p = 0; p < (long long)n_paths; ++p)
        gbm_one_path(prm, n_steps, scheme, coarsen, seed, tag,
                     path0 + (uint64_t)p, 1, out + (uint64_t)p * GBM_CH);
}

/* The same paths with the payoff channels only (0-3 and 8; the rest NaN). */
void orc_gbm_payoffs(const double *prm, int n_steps, int scheme, int coarsen,
                     uint64_t seed, uint32_t tag, uint64_t path0,
                     uint64_t n_paths, double *out)
{
#pragma omp parallel for schedule(static)
    for (long long p = 0; p < (long long)n_paths; ++p)
        gbm_one_path(prm, n_steps, scheme, coarsen, seed, tag,
                     path0 + (uint64_t)p, 0, out + (uint64_t)p * GBM_CH);
}

/* ------------------------------------------------------------------------ */
/* 6. Heston stochastic volatility (stochastic volatility is named in Sec.   */
/*    I-A.1 and Sec. II-A.1 as the same computation pattern), discretised by */
/*    full-truncation Euler on (ln S, v):                                    */
/*      v+ = max(v, 0)                                                       */
/*      x += (r - v+/2) dt + sqrt(v+ dt) Zs                                  */
/*      v += kappa (theta - v+) dt + xi sqrt(v+ dt) Z1                       */
/*      Zs = rho Z1 + sqrt(1 - rho^2) Z2                                     */
/*    Step i uses normals k = 2i (Z1) and k = 2i+1 (Z2).                     */
/*    Channels (discounted):                                                 */
/*      0 European call        1 arithmetic Asian call (mean of S_1..S_n)    */
/*      2 d/dS0 of 0           3 d/dv0 of 0                                  */
/*      4 d/dS0 of 1           5 d/dv0 of 1                                  */
/*      6 e^{-rT} S_n                                                        */
/*    Tangents in forward mode; the derivative of sqrt(v+) at v <= 0 is 0.   */
/* ------------------------------------------------------------------------ */
#define HES_CH 7

static void heston_one_path(const double *prm, int n, uint64_t seed,
                            uint32_t tag, uint64_t path, double *o)
{
    const double S0 = prm[0], v0 = prm[1], kap = prm[2], th = prm[3];
    const double xi = prm[4], rho = prm[5], r = prm[6], T = prm[7], K = prm[8];
    const double dt = T / n, disc = exp(-r * T);
    const double rho_c = sqrt(1.0 - rho * rho);
    normal_stream ns;
    ns_init(&ns, seed, tag, path);

    double x = log(S0), v = v0;
    double dx_dS0 = 1.0 / S0;                /* d x_i / d S0 (constant) */
    double dx_dv0 = 0.0, dv_dv0 = 1.0;       /* tangents w.r.t. v0 */
    double S = S0, sumS = 0.0, sum_dS0 = 0.0, sum_dv0 = 0.0;
    for (int i = 0; i < n; ++i) {
        double Z1 = ns_next(&ns);
        double Z2 = ns_next(&ns);
        double Zs = rho * Z1 + rho_c * Z2;
        double vp = pos(v);
        double dvp = v > 0.0 ? dv_dv0 : 0.0;
        double sq = sqrt(vp * dt);
        double dsq = vp > 0.0 ? dt * dvp / (2.0 * sq) : 0.0;
        double x_new = x + (r - 0.5 * vp) * dt + sq * Zs;
        double v_new = v + kap * (th - vp) * dt + xi * sq * Z1;
        double dx_new = dx_dv0 - 0.5 * dvp * dt + dsq * Zs;
        double dv_new = dv_dv0 - kap * dvp * dt + xi * dsq * Z1;
        x = x_new; v = v_new; dx_dv0 = dx_new; dv_dv0 = dv_new;
        S = exp(x);
        sumS += S;
        sum_dS0 += S * dx_dS0;
        sum_dv0 += S * dx_dv0;
    }
    double A = sumS / n;
    o[0] = disc * pos(S - K);
    o[1] = disc * pos(A - K);
    o[2] = S > K ? disc * S * dx_dS0 : 0.0;
    o[3] = S > K ? disc * S * dx_dv0 : 0.0;
    o[4] = A > K ? disc * sum_dS0 / n : 0.0;
    o[5] = A > K ? disc * sum_dv0 / n : 0.0;
    o[6] = disc * S;
}

int orc_heston_channels(void) { return HES_CH; }

/* prm = {S0, v0, kappa, theta, xi, rho, r, T, K} */
void orc_heston(const double *prm, int n_steps, uint64_t seed, uint32_t tag,
                uint64_t path0, uint64_t n_paths, double *out)
{
#pragma omp parallel for schedule(static)
    for (long long p = 0; p < (long long)n_paths; ++p)
        heston_one_path(prm, n_steps, seed, tag, path0 + (uint64_t)p,
                        out + (uint64_t)p * HES_CH);
}

/* ------------------------------------------------------------------------ */
/* 7. Cholesky factorisation C = L L^T (lower triangular), the textbook      */
/*    column-by-column algorithm. Returns 0, or -1 if C is not positive      */
/*    definite (a pivot <= 0). The paper factors Gram matrices the same way  */
/*    in its regression workload (Sec. II-A.3) and builds correlated         */
/*    increments from a volatility matrix (Sec. II-A.2).                     */
/* ------------------------------------------------------------------------ */
int orc_cholesky(int d, const double *C, double *L)
{
    memset(L, 0, sizeof(double) * (size_t)d * (size_t)d);
    for (int j = 0; j < d; ++j) {
        double s = C[(size_t)j * d + j];
        for (int k = 0; k < j; ++k) s -= L[(size_t)j * d + k] * L[(size_t)j * d + k];
        if (!(s > 0.0)) return -1;
        double ljj = sqrt(s);
        L[(size_t)j * d + j] = ljj;
        for (int i = j + 1; i < d; ++i) {
            double t = C[(size_t)i * d + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * d + k] * L[(size_t)j * d + k];
            L[(size_t)i * d + j] = t / ljj;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 8. Basket of d correlated GBM assets (Sec. II-A.2; basket call of         */
/*    Sec. VI-A.2), log-Euler per asset:                                     */
/*      x_a += (r - sigma_a^2/2) dt + sigma_a sqrt(dt) (L Z_i)_a             */
/*    with Z_i the d normals k = i*d + a of the step and L the lower         */
/*    Cholesky factor of the correlation matrix.                             */
/*    Channels (discounted):                                                 */
/*      0 basket call (sum_a w_a S_{n,a} - K)+                               */
/*      1 geometric basket call (exp(sum_a w_a x_{n,a}) - K)+                */
/*      2 pathwise d/dS0 of asset 0 of channel 0                             */
/* ------------------------------------------------------------------------ */
#define BSK_CH 3

int orc_basket_channels(void) { return BSK_CH; }

static void basket_paths(int d, const double *S0, const double *sigma, const double *L,
                         const double *w, double r, double T, double K, int n_steps,
                         uint64_t seed, uint32_t tag, uint64_t path0, uint64_t n_paths,
                         const uint32_t *V, const uint32_t *shift, double *out);

void orc_basket(int d, const double *S0, const double *sigma, const double *L,
                const double *w, double r, double T, double K, int n_steps,
                uint64_t seed, uint32_t tag, uint64_t path0, uint64_t n_paths,
                double *out)
{
    basket_paths(d, S0, sigma, L, w, r, T, K, n_steps, seed, tag, path0, n_paths,
                 NULL, NULL, out);
}

static void basket_paths(int d, const double *S0, const double *sigma, const double *L,
                         const double *w, double r, double T, double K, int n_steps,
                         uint64_t seed, uint32_t tag, uint64_t path0, uint64_t n_paths,
                         const uint32_t *V, const uint32_t *shift, double *out)
{
    const double dt = T / n_steps, sdt = sqrt(dt), disc = exp(-r * T);
#pragma omp parallel
    {
        double *x = (double *)malloc(sizeof(double) * (size_t)d);
        double *Z = (double *)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(static)
        for (long long p = 0; p < (long long)n_paths; ++p) {
            normal_stream ns;
            ns_init(&ns, seed, tag, path0 + (uint64_t)p);
            ns.V = V;
            ns.shift = shift;
            for (int a = 0; a < d; ++a) x[a] = log(S0[a]);
            for (int i = 0; i < n_steps; ++i) {
                for (int a = 0; a < d; ++a) Z[a] = ns_next(&ns);
                for (int a = 0; a < d; ++a) {
                    double dW = 0.0;
                    for (int b = 0; b <= a; ++b) dW += L[(size_t)a * d + b] * Z[b];
                    x[a] += (r - 0.5 * sigma[a] * sigma[a]) * dt + sigma[a] * sdt * dW;
                }
            }
            double basket = 0.0, geo = 0.0;
            for (int a = 0; a < d; ++a) {
                basket += w[a] * exp(x[a]);
                geo += w[a] * x[a];
            }
            double *o = out + (uint64_t)p * BSK_CH;
            o[0] = disc * pos(basket - K);
            o[1] = disc * pos(exp(geo) - K);
            o[2] = basket > K ? disc * w[0] * exp(x[0]) / S0[0] : 0.0;
        }
        free(x);
        free(Z);
    }
}

/* ------------------------------------------------------------------------ */
/* 8b. Portfolio profit and loss for the risk metrics of Sec. VI-B.1: the    */
/*    d correlated GBM assets of section 8 under the real-world measure      */
/*    (drift mu_a in place of r), log-Euler over the horizon T in n steps.   */
/*    The portfolio holds q_k European calls of strike m_k S0_a on every     */
/*    asset a (k = 0..ns-1), expiring at the horizon:                        */
/*      PnL = sum_a sum_k q_k (S_{T,a} - m_k S0_a)^+  -  V0,                 */
/*    V0 the Black-Scholes value at time 0 (rate r, volatility sigma_a) of   */
/*    the same holdings. No discounting of the horizon value.                */
/* ------------------------------------------------------------------------ */
double orc_bs_call(double S, double K, double r, double sig, double T)
{
    const double sq = sig * sqrt(T);
    const double d1 = (log(S / K) + (r + 0.5 * sig * sig) * T) / sq;
    const double d2 = d1 - sq;
    const double N1 = 0.5 * erfc(-d1 / sqrt(2.0));
    const double N2 = 0.5 * erfc(-d2 / sqrt(2.0));
    return S * N1 - K * exp(-r * T) * N2;
}

double orc_portfolio_premium(int d, const double *S0, const double *sigma, int ns,
                             const double *m, const double *q, double r, double T)
{
    double v = 0.0;
    for (int a = 0; a < d; ++a)
        for (int k = 0; k < ns; ++k)
            v += q[k] * orc_bs_call(S0[a], m[k] * S0[a], r, sigma[a], T);
    return v;
}

void orc_portfolio_pnl(int d, const double *S0, const double *sigma, const double *mu,
                       const double *L, int ns, const double *m, const double *q,
                       double r, double T, int n_steps, uint64_t seed, uint32_t tag,
                       uint64_t path0, uint64_t n_paths, double *out)
{
    const double dt = T / n_steps, sdt = sqrt(dt);
    const double V0 = orc_portfolio_premium(d, S0, sigma, ns, m, q, r, T);
#pragma omp parallel
    {
        double *x = (double *)malloc(sizeof(double) * (size_t)d);
        double *Z = (double *)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(static)
        for (long long p = 0; p < (long long)n_paths; ++p) {
            normal_stream ns_;
            ns_init(&ns_, seed, tag, path0 + (uint64_t)p);
            for (int a = 0; a < d; ++a) x[a] = log(S0[a]);
            for (int i = 0; i < n_steps; ++i) {
                for (int a = 0; a < d; ++a) Z[a] = ns_next(&ns_);
                for (int a = 0; a < d; ++a) {
                    double dW = 0.0;
                    for (int b = 0; b <= a; ++b) dW += L[(size_t)a * d + b] * Z[b];
                    x[a] += (mu[a] - 0.5 * sigma[a] * sigma[a]) * dt + sigma[a] * sdt * dW;
                }
            }
            double v = 0.0;
            for (int a = 0; a < d; ++a) {
                const double S = exp(x[a]);
                for (int k = 0; k < ns; ++k) v += q[k] * pos(S - m[k] * S0[a]);
            }
            out[p] = v - V0;
        }
        free(x);
        free(Z);
    }
}

/* ------------------------------------------------------------------------ */
/* 9. Learned martingale control variate on the Heston Asian call.           */
/*    A small network Delta_theta(t, state) is a hedge ratio; the hedge     */
/*    P&L  H = sum_j Delta(t_j, phi_j) (St_{j+1} - St_j),  St_i = e^{-r t_i}  */
/*    S_i, has zero mean for any weights because St is a martingale under   */
/*    the log-Euler step. The estimator averages Y = payoff - H (Eq. 3      */
/*    applied to Y). With rebalancing every m steps the hedge is held from  */
/*    step j*m to (j+1)*m.                                                   */
/*    Network 4 -> 64 -> 64 -> 1, tanh after the two hidden layers.         */
/*    Parameters, flat: W1[64][4], b1[64], W2[64][64], b2[64], W3[64], b3.   */
/*    Features phi_i = (t_i/T, ln(S_i/K), v_i/theta, Abar_i/K - 1), Abar_i  */
/*    the running mean of S_1..S_i (Abar_0 = S0).                            */
/* ------------------------------------------------------------------------ */
#define MLP_H 64
#define MLP_NPARAM (MLP_H * 4 + MLP_H + MLP_H * MLP_H + MLP_H + MLP_H + 1)

int orc_mlp_nparam(void) { return MLP_NPARAM; }

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3;
    int bf16;    /* round the operands of the two matrix products to bfloat16 */
} mlp_view;

/* The mixed-precision matrix product of the paper's matrix units (Sec. III,
 * Sec. V-A): operands in bfloat16, products accumulated in higher
 * precision. A value is rounded to single precision and then to its top 16
 * bits, to nearest with ties to even. */
static double bf16_round(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, sizeof(u));
    if ((u & 0x7f800000u) == 0x7f800000u) return x;     /* inf, nan */
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, sizeof(f));
    return f;
}

static mlp_view mlp_split(const double *th)
{
    mlp_view m;
    m.W1 = th;
    m.b1 = m.W1 + MLP_H * 4;
    m.W2 = m.b1 + MLP_H;
    m.b2 = m.W2 + MLP_H * MLP_H;
    m.W3 = m.b2 + MLP_H;
    m.b3 = m.W3 + MLP_H;
    m.bf16 = 0;
    return m;
}

/* Forward pass; keeps the hidden activations for the backward pass. */
static double mlp_forward(const mlp_view *m, const double phi[4],
                          double h1[MLP_H], double h2[MLP_H])
{
    const int r = m->bf16;
    double x[4], a1[MLP_H];
    for (int f = 0; f < 4; ++f) x[f] = r ? bf16_round(phi[f]) : phi[f];
    for (int u = 0; u < MLP_H; ++u) {
        double s = r ? bf16_round(m->b1[u]) : m->b1[u];
        for (int f = 0; f < 4; ++f) s += (r ? bf16_round(m->W1[u * 4 + f]) : m->W1[u * 4 + f]) * x[f];
        h1[u] = tanh(s);
        a1[u] = r ? bf16_round(h1[u]) : h1[u];
    }
    for (int u = 0; u < MLP_H; ++u) {
        double s = m->b2[u];
        for (int q = 0; q < MLP_H; ++q)
            s += (r ? bf16_round(m->W2[u * MLP_H + q]) : m->W2[u * MLP_H + q]) * a1[q];
        h2[u] = tanh(s);
    }
    double out = m->b3[0];
    for (int u = 0; u < MLP_H; ++u) out += m->W3[u] * h2[u];
    return out;
}

/* Backward pass of g * Delta with respect to every parameter, accumulated
 * into grad (same flat layout). */
static void mlp_backward(const mlp_view *m, const double phi[4],
                         const double h1[MLP_H], const double h2[MLP_H],
                         double g, double *grad)
{
    double *gW1 = grad, *gb1 = gW1 + MLP_H * 4, *gW2 = gb1 + MLP_H;
    double *gb2 = gW2 + MLP_H * MLP_H, *gW3 = gb2 + MLP_H, *gb3 = gW3 + MLP_H;
    double d2[MLP_H], d1[MLP_H];
    gb3[0] += g;
    for (int u = 0; u < MLP_H; ++u) {
        gW3[u] += g * h2[u];
        d2[u] = g * m->W3[u] * (1.0 - h2[u] * h2[u]);
    }
    for (int u = 0; u < MLP_H; ++u) {
        gb2[u] += d2[u];
        for (int q = 0; q < MLP_H; ++q) gW2[u * MLP_H + q] += d2[u] * h1[q];
    }
    for (int q = 0; q < MLP_H; ++q) {
        double s = 0.0;
        for (int u = 0; u < MLP_H; ++u) s += m->W2[u * MLP_H + q] * d2[u];
        d1[q] = s * (1.0 - h1[q] * h1[q]);
    }
    for (int u = 0; u < MLP_H; ++u) {
        gb1[u] += d1[u];
        for (int f = 0; f < 4; ++f) gW1[u * 4 + f] += d1[u] * phi[f];
    }
}

/* Simulates one Heston path and its hedge. Returns the discounted Asian
 * payoff in *pay and the hedge P&L in *H. When grad != NULL it also adds
 * g_up * dH/dtheta to grad (g_up is the upstream derivative of the loss
 * with respect to H of this path). */
static void heston_cv_path(const double *prm, int n, int m_every,
                           const mlp_view *net, uint64_t seed, uint32_t tag,
                           uint64_t path, double *pay, double *H,
                           double g_up, double *grad)
{
    const double S0 = prm[0], v0 = prm[1], kap = prm[2], th = prm[3];
    const double xi = prm[4], rho = prm[5], r = prm[6], T = prm[7], K = prm[8];
    const double dt = T / n, disc = exp(-r * T);
    const double rho_c = sqrt(1.0 - rho * rho);
    normal_stream ns;
    ns_init(&ns, seed, tag, path);
    double x = log(S0), v = v0, S = S0, sumS = 0.0, Abar = S0;
    double hedge = 0.0, Hsum = 0.0;
    double St_open = S0;             /* discounted S where the hedge opened */
    double phi_open[4], h1[MLP_H], h2[MLP_H];
    for (int i = 0; i < n; ++i) {
        if (i % m_every == 0) {
            phi_open[0] = (i * dt) / T;
            phi_open[1] = log(S / K);
            phi_open[2] = v / th;
            phi_open[3] = Abar / K - 1.0;
            hedge = mlp_forward(net, phi_open, h1, h2);
            St_open = exp(-r * i * dt) * S;
        }
        double Z1 = ns_next(&ns);
        double Z2 = ns_next(&ns);
        double Zs = rho * Z1 + rho_c * Z2;
        double vp = pos(v);
        double sq = sqrt(vp * dt);
        x = x + (r - 0.5 * vp) * dt + sq * Zs;
        v = v + kap * (th - vp) * dt + xi * sq * Z1;
        S = exp(x);
        sumS += S;
        Abar = sumS / (i + 1);
        if ((i + 1) % m_every == 0 || i + 1 == n) {
            double dSt = exp(-r * (i + 1) * dt) * S - St_open;
            Hsum += hedge * dSt;
            if (grad) mlp_backward(net, phi_open, h1, h2, g_up * dSt, grad);
        }
    }
    *pay = disc * pos(sumS / n - K);
    *H = Hsum;
}

/* Per-path (payoff, H, payoff - H); bf16 = 1 evaluates the network with
 * bfloat16 matrix-product operands. */
void orc_heston_cv(const double *prm, int n_steps, int m_every,
                   const double *theta, uint64_t seed, uint32_t tag,
                   uint64_t path0, uint64_t n_paths, int bf16, double *out /* n x 3 */)
{
    mlp_view net = mlp_split(theta);
    net.bf16 = bf16;
#pragma omp parallel for schedule(static)
    for (long long p = 0; p < (long long)n_paths; ++p) {
        double pay, H;
        heston_cv_path(prm, n_steps, m_every, &net, seed, tag,
                       path0 + (uint64_t)p, &pay, &H, 0.0, NULL);
        out[3 * p] = pay;
        out[3 * p + 1] = H;
        out[3 * p + 2] = pay - H;
    }
}

double orc_bf16_round(double x) { return bf16_round(x); }

/* Network output alone, for a list of feature vectors (n x 4). */
void orc_mlp_eval(const double *theta, uint64_t n, const double *phi, int bf16,
                  double *out)
{
    mlp_view net = mlp_split(theta);
    net.bf16 = bf16;
    double h1[MLP_H], h2[MLP_H];
    for (uint64_t i = 0; i < n; ++i) out[i] = mlp_forward(&net, phi + 4 * i, h1, h2);
}

/* Training loss over a batch of B paths and its gradient:
 *   L(theta) = (1/B) sum_b (Y_b - Ybar)^2,  Y_b = payoff_b - H_b(theta).
 *   dL/dtheta = (2/B) sum_b (Y_b - Ybar) dY_b/dtheta
 *             = sum_b [-(2/B)(Y_b - Ybar)] dH_b/dtheta.
 * The first pass gets Ybar, the second accumulates the gradient. Paths are
 * path0 .. path0+B-1 of stream `tag`. */
double orc_cv_loss_grad(const double *prm, int n_steps, int m_every,
                        const double *theta, uint64_t seed, uint32_t tag,
                        uint64_t path0, uint64_t B, double *grad)
{
    mlp_view net = mlp_split(theta);
    double *Y = (double *)malloc(sizeof(double) * B);
#pragma omp parallel for schedule(static)
    for (long long b = 0; b < (long long)B; ++b) {
        double pay, H;
        heston_cv_path(prm, n_steps, m_every, &net, seed, tag,
                       path0 + (uint64_t)b, &pay, &H, 0.0, NULL);
        Y[b] = pay - H;
    }
    double Ybar = 0.0;
    for (uint64_t b = 0; b < B; ++b) Ybar += Y[b];
    Ybar /= (double)B;
    double loss = 0.0;
    for (uint64_t b = 0; b < B; ++b) loss += (Y[b] - Ybar) * (Y[b] - Ybar);
    loss /= (double)B;
    if (grad) {
        memset(grad, 0, sizeof(double) * MLP_NPARAM);
        /* Serial in b: the gradient is a sum over paths in path order. */
        for (uint64_t b = 0; b < B; ++b) {
            double pay, H;
            double g_up = -(2.0 / (double)B) * (Y[b] - Ybar);
            heston_cv_path(prm, n_steps, m_every, &net, seed, tag,
                           path0 + b, &pay, &H, g_up, grad);
        }
    }
    free(Y);
    return loss;
}

/* ------------------------------------------------------------------------ */
/* 11. Sobol' low-discrepancy points with a random digital shift (the        */
/*    quasi-random generator of Sec. IV-B and the Sobol' experiment of       */
/*    Sec. VI-D), written from Sobol's construction:                         */
/*    - dimension 0: the van der Corput sequence (direction integers         */
/*      m_i = 1);                                                            */
/*    - dimension j >= 1: the j-th primitive polynomial over GF(2),          */
/*      p = x^s + a_1 x^(s-1) + ... + a_(s-1) x + 1, taken in order of       */
/*      degree and then of its bit pattern, with initial direction integers  */
/*      m_i = 2 (h mod 2^(i-1)) + 1 for i = 1..s, h = SplitMix64(64 j + i)   */
/*      (odd and below 2^i, as the construction requires; the Joe-Kuo       */
/*      table is not available), and for i > s                              */
/*        m_i = m_(i-s) xor 2^s m_(i-s) xor sum_k a_k 2^k m_(i-k)             */
/*    - direction word of bit b of the point index: V_b = m_(b+1) 2^(31-b);  */
/*    - coordinate of point p in dimension j: the xor of V_b over the set    */
/*      bits b of p, a 32-bit fraction.                                      */
/*    Randomisation: word j of a point is xored with shift_j, word (j mod 4) */
/*    of Philox block (floor(j/4), replicate, tag) -- a random digital shift */
/*    per replicate; the shifted words then go through the same uniform and  */
/*    Box-Muller map as Philox words (normal k uses dimension k).            */
/* ------------------------------------------------------------------------ */
static uint64_t smix64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

/* a * b mod p in GF(2)[x], deg p = s, deg a, b < s. */
static uint32_t gf2_mulmod(uint32_t a, uint32_t b, uint32_t p, int s)
{
    uint32_t r = 0;
    while (b) {
        if (b & 1u) r ^= a;
        b >>= 1;
        a <<= 1;
        if (a & (1u << s)) a ^= p;
    }
    return r;
}

static uint32_t gf2_powx(uint64_t e, uint32_t p, int s)
{
    uint32_t result = 1u, base = (s == 1) ? (2u ^ p) : 2u;   /* x mod p */
    while (e) {
        if (e & 1u) result = gf2_mulmod(result, base, p, s);
        base = gf2_mulmod(base, base, p, s);
        e >>= 1;
    }
    return result;
}

/* p (degree s, constant term 1) is primitive when x has order 2^s - 1. */
static int gf2_primitive(uint32_t p, int s)
{
    const uint64_t order = (1ull << s) - 1;
    if (gf2_powx(order, p, s) != 1u) return 0;
    uint64_t n = order;
    for (uint64_t q = 2; q * q <= n; ++q) {
        if (n % q) continue;
        while (n % q == 0) n /= q;
        if (gf2_powx(order / q, p, s) == 1u) return 0;
    }
    if (n > 1 && gf2_powx(order / n, p, s) == 1u) return 0;
    return 1;
}

/* First n primitive polynomials (bit patterns including x^s and 1) and their
 * degrees. Returns n, or the number found up to degree 24. */
int orc_sobol_polys(int n, int *deg, uint32_t *poly)
{
    int found = 0;
    for (int s = 1; s <= 24 && found < n; ++s)
        for (uint32_t c = (1u << s) | 1u; c < (2u << s) && found < n; c += 2)
            if (gf2_primitive(c, s)) {
                deg[found] = s;
                poly[found] = c;
                ++found;
            }
    return found;
}

void orc_sobol_dirs(int n_dims, uint32_t *V)
{
    int *deg = (int *)malloc(sizeof(int) * (size_t)(n_dims > 1 ? n_dims : 1));
    uint32_t *poly = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n_dims > 1 ? n_dims : 1));
    if (n_dims > 1) orc_sobol_polys(n_dims - 1, deg, poly);
    for (int j = 0; j < n_dims; ++j) {
        uint64_t m[33];
        if (j == 0) {
            for (int i = 1; i <= 32; ++i) m[i] = 1;
        } else {
            const int s = deg[j - 1];
            const uint32_t p = poly[j - 1];
            for (int i = 1; i <= s && i <= 32; ++i) {
                const uint64_t h = smix64(64ull * (uint64_t)j + (uint64_t)i);
                m[i] = 2 * (h % (1ull << (i - 1))) + 1;
            }
            for (int i = s + 1; i <= 32; ++i) {
                uint64_t v = m[i - s] ^ (m[i - s] << s);
                for (int k = 1; k < s; ++k)
                    if ((p >> (s - k)) & 1u) v ^= m[i - k] << k;
                m[i] = v;
            }
        }
        for (int b = 0; b < 32; ++b) V[(size_t)j * 32 + b] = (uint32_t)(m[b + 1] << (31 - b));
    }
    free(deg);
    free(poly);
}

uint32_t orc_sobol_word(const uint32_t *V, int dim, uint64_t point)
{
    uint32_t x = 0;
    for (int b = 0; b < 32; ++b)
        if ((point >> b) & 1u) x ^= V[(size_t)dim * 32 + b];
    return x;
}

void orc_qmc_shifts(uint64_t seed, uint32_t tag, uint64_t replicate, int n_dims,
                    uint32_t *shift)
{
    for (int j = 0; j < n_dims; j += 4) {
        uint32_t w[4];
        orc_block_words(seed, tag, replicate, (uint64_t)(j / 4), w);
        for (int t = 0; t < 4 && j + t < n_dims; ++t) shift[j + t] = w[t];
    }
}

/* The basket of section 8 on shifted Sobol' points: point index = path. */
void orc_basket_qmc(int d, const double *S0, const double *sigma, const double *L,
                    const double *w, double r, double T, double K, int n_steps,
                    uint64_t seed, uint32_t tag, uint64_t replicate, uint64_t path0,
                    uint64_t n_paths, double *out)
{
    const int n_dims = ((n_steps * d + 3) / 4) * 4;
    uint32_t *V = (uint32_t *)malloc(sizeof(uint32_t) * 32 * (size_t)n_dims);
    uint32_t *sh = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n_dims);
    orc_sobol_dirs(n_dims, V);
    orc_qmc_shifts(seed, tag, replicate, n_dims, sh);
    basket_paths(d, S0, sigma, L, w, r, T, K, n_steps, seed, tag, path0, n_paths, V, sh, out);
    free(V);
    free(sh);
}

/* ------------------------------------------------------------------------ */
/* 12. Longstaff-Schwartz regression for callable (Bermudan) options        */
/*    (Sec. II-A.3; the American max-option experiment of Sec. VI-C).       */
/*    Model: d <= 4 correlated GBM assets with continuous dividend yield q,   */
/*    log-Euler per asset as in section 8 with drift r - q:                   */
/*      x_a += (r - q - sigma_a^2/2) dt + sigma_a sqrt(dt) (L Z_i)_a          */
/*    Exercise dates t_j = j T / M (j = 1..M), `spd` Euler steps between     */
/*    consecutive dates (dt = T / (M spd)); step i uses normals i*d + a.      */
/*    State y_a = S_a / K. Payoffs f (equal weights 1/d):                   */
/*      1 max-call    (max_a S_a - K)+                                        */
/*      2 basket put  (K - mean_a S_a)+                                       */
/*      3 basket call (mean_a S_a - K)+                                       */
/*    Dynamic programming on realised cash flows: every path carries its      */
/*    discounted cash flow C (at first e^{-rT} f(t_M)). For j = M-1 .. 1 the  */
/*    cash flows of the paths in the money at t_j (f > 0) are projected on    */
/*    the features psi(y(t_j)) by least squares, solving the normal          */
/*    equations (sum psi psi^T) beta = sum psi C through a Cholesky          */
/*    factorisation of the Gram matrix; an in-the-money path whose           */
/*    discounted exercise value e^{-r t_j} f is at least the fitted           */
/*    continuation psi . beta exercises: C = e^{-r t_j} f. The price is the   */
/*    mean of C over all paths (an averaging reduction, as the paper ends    */
/*    the method); t = 0 is not an exercise date.                            */
/*    Features: every monomial of y_1..y_d of total degree <= deg, by degree, */
/*    then by the nondecreasing index tuple; for the max-call with d >= 2    */
/*    the payoff f / K is appended (on the in-the-money set the basket       */
/*    payoffs are affine in y, so there it would duplicate degree 1).        */
/*    A date with fewer in-the-money paths than features, or whose Gram      */
/*    matrix has a Cholesky pivot <= 1e-12 times its diagonal entry, gets no */
/*    regression and no exercise (beta row NaN).                             */
/* ------------------------------------------------------------------------ */
#define LSM_MAXB 12

static double lsm_payoff(int kind, int d, const double *y)
{
    double m = y[0], s = 0.0;
    for (int a = 0; a < d; ++a) {
        if (y[a] > m) m = y[a];
        s += y[a];
    }
    s /= d;
    if (kind == 1) return pos(m - 1.0);
    if (kind == 2) return pos(1.0 - s);
    return pos(s - 1.0);
}

/* Number of features, and their index triples (index d stands for 1,
 * index d+1 for f/K). */
static int lsm_features(int d, int deg, int kind, int idx[][3])
{
    int n = 0;
    idx[n][0] = d; idx[n][1] = d; idx[n][2] = d; ++n;
    if (deg >= 1)
        for (int a = 0; a < d; ++a) { idx[n][0] = a; idx[n][1] = d; idx[n][2] = d; ++n; }
    if (deg >= 2)
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b) { idx[n][0] = a; idx[n][1] = b; idx[n][2] = d; ++n; }
    if (deg >= 3)
        for (int a = 0; a < d; ++a)
            for (int b = a; b < d; ++b)
                for (int c = b; c < d; ++c) { idx[n][0] = a; idx[n][1] = b; idx[n][2] = c; ++n; }
    if (kind == 1 && d >= 2) { idx[n][0] = d + 1; idx[n][1] = d; idx[n][2] = d; ++n; }
    return n;
}

int orc_lsm_n_features(int d, int deg, int kind)
{
    int idx[64][3];
    if (d < 1 || d > 4 || deg < 0 || deg > 3) return -1;
    return lsm_features(d, deg, kind, idx);
}

static void lsm_psi(int d, int nf, int idx[][3], const double *y, double fK, double *psi)
{
    double v[6];
    for (int a = 0; a < d; ++a) v[a] = y[a];
    v[d] = 1.0;
    v[d + 1] = fK;
    for (int k = 0; k < nf; ++k) psi[k] = v[idx[k][0]] * v[idx[k][1]] * v[idx[k][2]];
}

/* Solves G x = b (G symmetric positive definite, n x n) by Cholesky; -1 when a
 * pivot is <= 1e-12 times the diagonal entry it comes from. */
static int lsm_solve(int n, const double *G, const double *b, double *x)
{
    double Lc[LSM_MAXB * LSM_MAXB], y[LSM_MAXB];
    for (int j = 0; j < n; ++j) {
        double s = G[j * n + j];
        for (int k = 0; k < j; ++k) s -= Lc[j * n + k] * Lc[j * n + k];
        if (!(s > 1e-12 * G[j * n + j])) return -1;
        Lc[j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double t = G[i * n + j];
            for (int k = 0; k < j; ++k) t -= Lc[i * n + k] * Lc[j * n + k];
            Lc[i * n + j] = t / Lc[j * n + j];
        }
    }
    for (int i = 0; i < n; ++i) {
        double t = b[i];
        for (int k = 0; k < i; ++k) t -= Lc[i * n + k] * y[k];
        y[i] = t / Lc[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double t = y[i];
        for (int k = i + 1; k < n; ++k) t -= Lc[k * n + i] * x[k];
        x[i] = t / Lc[i * n + i];
    }
    return 0;
}

/* y[(p * M + (j-1)) * d + a] = S_a(t_j) / K for paths path0 .. path0+n-1. */
static void lsm_paths(int d, const double *S0, const double *sigma, const double *L,
                      double r, double q, double T, double K, int M, int spd,
                      uint64_t seed, uint32_t tag, uint64_t path0, uint64_t n, double *y)
{
    const double dt = T / ((double)M * spd), sdt = sqrt(dt);
#pragma omp parallel for schedule(static)
    for (long long p = 0; p < (long long)n; ++p) {
        double x[4], Z[4];
        normal_stream ns;
        ns_init(&ns, seed, tag, path0 + (uint64_t)p);
        for (int a = 0; a < d; ++a) x[a] = log(S0[a] / K);
        for (int j = 1; j <= M; ++j) {
            for (int s = 0; s < spd; ++s) {
                for (int a = 0; a < d; ++a) Z[a] = ns_next(&ns);
                for (int a = 0; a < d; ++a) {
                    double dW = 0.0;
                    for (int b = 0; b <= a; ++b) dW += L[a * d + b] * Z[b];
                    x[a] += (r - q - 0.5 * sigma[a] * sigma[a]) * dt + sigma[a] * sdt * dW;
                }
            }
            for (int a = 0; a < d; ++a) y[((uint64_t)p * M + (j - 1)) * d + a] = exp(x[a]);
        }
    }
}

static void mean_se(const double *v, uint64_t n, double *out)
{
    double s = 0.0;
    for (uint64_t i = 0; i < n; ++i) s += v[i];
    const double m = s / (double)n;
    double ss = 0.0;
    for (uint64_t i = 0; i < n; ++i) ss += (v[i] - m) * (v[i] - m);
    out[0] = m;
    out[1] = n > 1 ? sqrt(ss / (double)(n - 1) / (double)n) : NAN;
}

/* In-sample Longstaff-Schwartz. res = {price, std_err, european, european_se}
 * (european: exercise at t_M only, same paths). beta [M][nf], row j-1 for date
 * j (row M-1 and rows without regression NaN); n_itm [M]. Optional (NULL):
 * C [n] discounted cash flows, ex [n] exercise date (0 = never), cont [n][M]
 * fitted continuation (NaN where not evaluated), yout [n][M][d]. Returns nf,
 * or -1 on bad arguments. */
int orc_lsm(int d, const double *S0, const double *sigma, const double *L, double r,
            double q, double T, int kind, double K, int M, int spd, int deg,
            uint64_t seed, uint32_t tag, uint64_t path0, uint64_t n, double *res,
            double *beta, int64_t *n_itm, double *C, int32_t *ex, double *cont, double *yout)
{
    int idx[64][3];
    if (d < 1 || d > 4 || M < 1 || spd < 1 || n < 1 || kind < 1 || kind > 3) return -1;
    const int nf = lsm_features(d, deg, kind, idx);
    if (nf > LSM_MAXB - 1) return -1;
    double *y = yout ? yout : (double *)malloc(sizeof(double) * n * (size_t)M * d);
    double *c = (double *)malloc(sizeof(double) * n);
    int32_t *e = (int32_t *)malloc(sizeof(int32_t) * n);
    lsm_paths(d, S0, sigma, L, r, q, T, K, M, spd, seed, tag, path0, n, y);
    if (cont)
        for (uint64_t i = 0; i < n * (uint64_t)M; ++i) cont[i] = NAN;
    for (int i = 0; i < M * nf; ++i) beta[i] = NAN;
    for (int j = 0; j < M; ++j) n_itm[j] = 0;
    const double discT = exp(-r * T);
    for (uint64_t p = 0; p < n; ++p) {
        const double f = K * lsm_payoff(kind, d, y + (p * M + (M - 1)) * d);
        c[p] = discT * f;
        e[p] = f > 0.0 ? M : 0;
        if (f > 0.0) n_itm[M - 1]++;
    }
    mean_se(c, n, res + 2);
    for (int j = M - 1; j >= 1; --j) {
        const double dj = exp(-r * T * j / M);
        double G[LSM_MAXB * LSM_MAXB] = {0}, b[LSM_MAXB] = {0}, psi[LSM_MAXB], bj[LSM_MAXB];
        int64_t m = 0;
        for (uint64_t p = 0; p < n; ++p) {
            const double *yp = y + (p * M + (j - 1)) * d;
            const double f = lsm_payoff(kind, d, yp);
            if (!(f > 0.0)) continue;
            ++m;
            lsm_psi(d, nf, idx, yp, f, psi);
            for (int u = 0; u < nf; ++u) {
                for (int v = 0; v < nf; ++v) G[u * nf + v] += psi[u] * psi[v];
                b[u] += psi[u] * c[p];
            }
        }
        n_itm[j - 1] = m;
        if (m < nf || lsm_solve(nf, G, b, bj) != 0) continue;
        for (int u = 0; u < nf; ++u) beta[(j - 1) * nf + u] = bj[u];
        for (uint64_t p = 0; p < n; ++p) {
            const double *yp = y + (p * M + (j - 1)) * d;
            const double f = lsm_payoff(kind, d, yp);
            if (!(f > 0.0)) continue;
            lsm_psi(d, nf, idx, yp, f, psi);
            double h = 0.0;
            for (int u = 0; u < nf; ++u) h += psi[u] * bj[u];
            if (cont) cont[p * M + (j - 1)] = h;
            if (dj * K * f >= h) {
                c[p] = dj * K * f;
                e[p] = j;
            }
        }
    }
    mean_se(c, n, res);
    if (C) memcpy(C, c, sizeof(double) * n);
    if (ex) memcpy(ex, e, sizeof(int32_t) * n);
    if (!yout) free(y);
    free(c);
    free(e);
    return nf;
}

/* Out-of-sample estimate: the exercise rule of a fitted beta [M][nf] applied
 * to independent paths (stream `tag`): each path exercises at the first date
 * j < M where it is in the money, the row of beta is not NaN and
 * e^{-r t_j} f >= psi . beta_j, else at t_M when in the money. res = {price,
 * std_err}; Y [n] and ex [n] optional. */
int orc_lsm_oos(int d, const double *S0, const double *sigma, const double *L, double r,
                double q, double T, int kind, double K, int M, int spd, int deg,
                const double *beta, uint64_t seed, uint32_t tag, uint64_t path0, uint64_t n,
                double *res, double *Y, int32_t *ex)
{
    int idx[64][3];
    if (d < 1 || d > 4 || M < 1 || spd < 1 || n < 1 || kind < 1 || kind > 3) return -1;
    const int nf = lsm_features(d, deg, kind, idx);
    if (nf > LSM_MAXB - 1) return -1;
    double *y = (double *)malloc(sizeof(double) * n * (size_t)M * d);
    double *v = (double *)malloc(sizeof(double) * n);
    lsm_paths(d, S0, sigma, L, r, q, T, K, M, spd, seed, tag, path0, n, y);
    for (uint64_t p = 0; p < n; ++p) {
        int e = 0;
        double val = 0.0;
        for (int j = 1; j <= M; ++j) {
            const double *yp = y + (p * M + (j - 1)) * d;
            const double f = lsm_payoff(kind, d, yp);
            if (!(f > 0.0)) continue;
            const double dj = exp(-r * T * j / M);
            if (j == M) {
                e = M;
                val = dj * K * f;
                break;
            }
            if (isnan(beta[(j - 1) * nf])) continue;
            double psi[LSM_MAXB], h = 0.0;
            lsm_psi(d, nf, idx, yp, f, psi);
            for (int u = 0; u < nf; ++u) h += psi[u] * beta[(j - 1) * nf + u];
            if (dj * K * f >= h) {
                e = j;
                val = dj * K * f;
                break;
            }
        }
        v[p] = val;
        if (ex) ex[p] = e;
    }
    mean_se(v, n, res);
    if (Y) memcpy(Y, v, sizeof(double) * n);
    free(y);
    free(v);
    return nf;
}

/* Bermudan price on a binomial lattice (Cox-Ross-Rubinstein), an independent
 * route to the value LSM estimates: per asset u = e^{sigma sqrt(h)}, 1/u, up
 * probability (e^{(r-q)h} - 1/u) / (u - 1/u), h = T / (M nt); for d = 2 the
 * two assets are independent and the lattice is the product of their trees.
 * Backward induction discounts by e^{-rh} per step and takes the maximum
 * with the payoff at the steps j nt (j = 1..M). d = 1 or 2; -1 otherwise. */
double orc_lsm_lattice(int d, const double *S0, const double *sigma, double r, double q,
                       double T, int kind, double K, int M, int nt)
{
    if (d < 1 || d > 2 || M < 1 || nt < 1 || kind < 1 || kind > 3) return -1.0;
    const int N = M * nt;
    const double h = T / N, disc = exp(-r * h);
    double u[2], pu[2];
    for (int a = 0; a < d; ++a) {
        u[a] = exp(sigma[a] * sqrt(h));
        pu[a] = (exp((r - q) * h) - 1.0 / u[a]) / (u[a] - 1.0 / u[a]);
    }
    const size_t W = (size_t)N + 1;
    double *V = (double *)malloc(sizeof(double) * (d == 2 ? W * W : W));
    double y[2];
    /* node (i1, i2) at step n: S_a = S0_a u_a^(2 i_a - n) */
    for (size_t i1 = 0; i1 <= (size_t)N; ++i1) {
        y[0] = S0[0] / K * pow(u[0], 2.0 * (double)i1 - N);
        if (d == 1) {
            V[i1] = K * lsm_payoff(kind, 1, y);
            continue;
        }
        for (size_t i2 = 0; i2 <= (size_t)N; ++i2) {
            y[1] = S0[1] / K * pow(u[1], 2.0 * (double)i2 - N);
            V[i1 * W + i2] = K * lsm_payoff(kind, 2, y);
        }
    }
    for (int n = N - 1; n >= 0; --n) {
        const int ex_step = (n > 0 && n % nt == 0);
        for (int i1 = 0; i1 <= n; ++i1) {
            if (d == 1) {
                double v = disc * (pu[0] * V[i1 + 1] + (1.0 - pu[0]) * V[i1]);
                if (ex_step) {
                    y[0] = S0[0] / K * pow(u[0], 2.0 * i1 - n);
                    const double f = K * lsm_payoff(kind, 1, y);
                    if (f > v) v = f;
                }
                V[i1] = v;
                continue;
            }
            for (int i2 = 0; i2 <= n; ++i2) {
                const double up = pu[0] * (pu[1] * V[(i1 + 1) * W + i2 + 1]
                                           + (1.0 - pu[1]) * V[(i1 + 1) * W + i2]);
                const double dn = (1.0 - pu[0]) * (pu[1] * V[i1 * W + i2 + 1]
                                                   + (1.0 - pu[1]) * V[i1 * W + i2]);
                double v = disc * (up + dn);
                if (ex_step) {
                    y[0] = S0[0] / K * pow(u[0], 2.0 * i1 - n);
                    y[1] = S0[1] / K * pow(u[1], 2.0 * i2 - n);
                    const double f = K * lsm_payoff(kind, 2, y);
                    if (f > v) v = f;
                }
                V[i1 * W + i2] = v;
            }
        }
    }
    const double out = V[0];
    free(V);
    return out;
}
