/*
 * PHIA CPU oracle -- TEST INFRASTRUCTURE ONLY (see phia_oracle.h).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC.
 * No fast-math: every float operation below is one IEEE binary32 operation
 * with round-to-nearest-even, and every fused multiply-add is an explicit
 * fmaf, so the results are fixed by the specification and not by the compiler.
 *
 * Paper passages followed (Wang et al., arXiv 2407.10205):
 *   Eq. 2          Ising energy over i<j pairs plus local fields.
 *   Eq. 6          quasi-gradient I_i = sum_j J_ij sgn(x_j) + h_i.
 *   Eq. 5, Eq. 8   dv/dt = beta * d sgn(x)/dx * I - x with the tanh surrogate
 *                  d/dx tanh(gamma x) = gamma (1 - tanh^2(gamma x)).
 *   App. A, A3     x drawn from g(x), the standard normal density.
 *   App. A, A7     x <- x + eps v, then v <- v - eps grad_x H at the new x.
 *   Sec. 2.1       spins read out as s = sgn(x).
 *   App. B, Tab. 3 state 5: keep the best configuration found so far.
 */
#include "phia_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x64-10: two 64x64->128 multiplies per round, Weyl key bumps.  */
/* ------------------------------------------------------------------ */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL;

void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------ */
/* Elementary functions, FP32, written from their power series.        */
/* ------------------------------------------------------------------ */
static float f_from_bits(uint32_t b) { float f; memcpy(&f, &b, 4); return f; }
static uint32_t bits_from_f(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

/* ln 2 split so that LN2_HI is the float nearest ln 2 and LN2_LO the float
 * nearest the remainder ln 2 - LN2_HI. */
#define O_LN2_HI  0.693147182464599609375f
#define O_LN2_LO  (-1.9046542999577e-09f)
#define O_LOG2E   1.44269504088896340736f
#define O_SQRT2   1.41421356237309504880f
#define O_TWO_PI  6.28318530717958647692f

/* e^y, y <= 0.  Reduction y = k ln2 + r, |r| <= ln2/2 (Cody-Waite with the
 * split constant), then the degree-7 Taylor polynomial of e^r in Horner form,
 * then an exact scaling by 2^k.  Below -80 the value is taken as 0. */
float oracle_exp_nonpos(float y)
{
    if (!(y >= -80.0f)) return 0.0f;
    float kf = rintf(y * O_LOG2E);
    float r = fmaf(-kf, O_LN2_HI, y);
    r = fmaf(-kf, O_LN2_LO, r);
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    int k = (int)kf;                              /* in [-116, 0] */
    float scale = f_from_bits((uint32_t)(k + 127) << 23);
    return p * scale;
}

/* ln u for a normal u in (0, 1).  u = m 2^e with m folded into
 * (sqrt(1/2), sqrt(2)], t = (m-1)/(m+1), ln m = 2 atanh t =
 * 2t (1 + t^2/3 + t^4/5 + t^6/7 + t^8/9), ln u = e ln2 + ln m. */
float oracle_ln_unit(float u)
{
    uint32_t b = bits_from_f(u);
    int e = (int)((b >> 23) & 0xffu) - 127;
    float m = f_from_bits((b & 0x007fffffu) | 0x3f800000u);
    if (m > O_SQRT2) {
        m = m * 0.5f;
        e += 1;
    }
    float t = (m - 1.0f) / (m + 1.0f);
    float t2 = t * t;
    float P = fmaf(t2, 1.0f / 9.0f, 1.0f / 7.0f);
    P = fmaf(P, t2, 1.0f / 5.0f);
    P = fmaf(P, t2, 1.0f / 3.0f);
    float tt = t + t;
    float lnm = fmaf(tt * t2, P, tt);
    float ef = (float)e;
    return fmaf(ef, O_LN2_HI, fmaf(ef, O_LN2_LO, lnm));
}

/* cos and sin of 2 pi u for u in (0, 1).  k = rint(4u), r = u - k/4 in
 * [-1/8, 1/8] (exact), theta = 2 pi r in [-pi/4, pi/4]; Taylor series of sin
 * to theta^9 and cos to theta^10, then a rotation by k quarter turns. */
void oracle_sincos_2pi(float u, float* c, float* s)
{
    float kf = rintf(4.0f * u);
    float r = fmaf(kf, -0.25f, u);
    float th = r * O_TWO_PI;
    float t2 = th * th;
    float sp = fmaf(t2, 1.0f / 362880.0f, -(1.0f / 5040.0f));
    sp = fmaf(sp, t2, 1.0f / 120.0f);
    sp = fmaf(sp, t2, -(1.0f / 6.0f));
    float sn = fmaf(th * t2, sp, th);
    float cp = fmaf(t2, -(1.0f / 3628800.0f), 1.0f / 40320.0f);
    cp = fmaf(cp, t2, -(1.0f / 720.0f));
    cp = fmaf(cp, t2, 1.0f / 24.0f);
    cp = fmaf(cp, t2, -0.5f);
    float cs = fmaf(t2, cp, 1.0f);
    switch (((int)kf) & 3) {
    case 0: *c = cs;  *s = sn;  break;
    case 1: *c = -sn; *s = cs;  break;
    case 2: *c = -cs; *s = -sn; break;
    default: *c = sn; *s = -cs; break;
    }
}

/* sech^2(u) = 1 - tanh^2(u) = 4t / (1+t)^2 with t = e^{-2|u|}.  The
 * reciprocal y of q = 1 + t in [1, 2] starts from the line 24/17 - 8q/17
 * (relative error at most 1/17 on [1, 2]) and takes three Newton steps
 * y <- y + y (1 - q y), each squaring the relative error; then
 * sech^2 = (4t) y^2.  No division. */
float oracle_sech2(float u)
{
    /* sech^2 u = 4t / (1 + t)^2 with t = e^{-2|u|}.  t4 = 4t comes from the
     * exponential above with every Taylor coefficient times 4 (an exact
     * power-of-two scaling of each Horner step) and the scale applied by
     * ldexp; -2|u| is clamped at -80, so t4 stays a normal number and
     * sech^2 u = sech^2 40 for |u| >= 40.  1/q, q = 1 + t in [1, 2]: the
     * quadratic (32 q^2 - 144 q + 210)/99, whose relative error 1 - q y
     * is T3(2q - 3)/99 (at most 1/99), then two Newton steps. */
    float a = fabsf(u);
    float y = fmaxf(-(a + a), -80.0f);
    float kf = rintf(y * O_LOG2E);
    float r = fmaf(-kf, O_LN2_HI, y);
    r = fmaf(-kf, O_LN2_LO, r);
    float p = 4.0f / 5040.0f;
    p = fmaf(p, r, 4.0f / 720.0f);
    p = fmaf(p, r, 4.0f / 120.0f);
    p = fmaf(p, r, 4.0f / 24.0f);
    p = fmaf(p, r, 4.0f / 6.0f);
    p = fmaf(p, r, 2.0f);
    p = fmaf(p, r, 4.0f);
    p = fmaf(p, r, 4.0f);
    float t4 = ldexpf(p, (int)kf);
    float q = fmaf(t4, 0.25f, 1.0f);
    float z = fmaf(fmaf(32.0f / 99.0f, q, -144.0f / 99.0f), q, 210.0f / 99.0f);
    for (int it = 0; it < 2; ++it) {
        float e = fmaf(-q, z, 1.0f);
        z = fmaf(z, e, z);
    }
    return t4 * (z * z);
}

/* POLY2 derivative mode: the FPGA replaces Eq. 8's sech^2 by a quadratic
 * polynomial (Sec. 2.3; its coefficients are not given).  Reading: the
 * truncated parabola d(u) = max(0, 1 - u^2 / 2.25), which equals sech^2 at 0
 * and has the same integral over the real line (4 * 1.5 / 3 = 2).  Op order:
 * t = u*u; q = fma(-t, 4/9, 1); d = q > 0 ? q : 0. */
float oracle_poly2(float u)
{
    float t = u * u;
    float q = fmaf(-t, 4.0f / 9.0f, 1.0f);
    return q > 0.0f ? q : 0.0f;
}

float oracle_uniform(uint32_t w)
{
    return (float)(2u * (w >> 9) + 1u) * 0x1p-24f;
}

/* Counter-based standard normal draw number i of stream (seed, tag, r, round):
 * Philox4x64-10 with key (seed, 0) and counter (i/8, round, r, tag); the four
 * 64-bit outputs give eight 32-bit words (low half first); draw i uses word
 * pair p = (i mod 8)/2 in a Box-Muller transform, cosine branch for even i. */
float oracle_gauss(uint64_t seed, uint32_t tag, uint64_t r, uint64_t round, uint64_t i)
{
    uint64_t ctr[4] = { i >> 3, round, r, (uint64_t)tag };
    uint64_t key[2] = { seed, 0 };
    uint64_t out[4];
    oracle_philox4x64_10(ctr, key, out);
    unsigned p = (unsigned)((i & 7u) >> 1);
    uint32_t wa = (uint32_t)out[p];
    uint32_t wb = (uint32_t)(out[p] >> 32);
    float ua = oracle_uniform(wa);
    float ub = oracle_uniform(wb);
    float rho = sqrtf(-2.0f * oracle_ln_unit(ua));
    float c, s;
    oracle_sincos_2pi(ub, &c, &s);
    return (i & 1u) ? rho * s : rho * c;
}

/* ------------------------------------------------------------------ */
/* Energies and fields                                                 */
/* ------------------------------------------------------------------ */
int64_t oracle_energy(int N, const int32_t* J, const int32_t* h, const int8_t* s)
{
    int64_t e = 0;
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j)
            e -= (int64_t)J[(int64_t)i * N + j] * s[i] * s[j];
    for (int i = 0; i < N; ++i)
        e -= (int64_t)h[i] * s[i];
    return e;
}

void oracle_local_field(int N, const int32_t* J, const int32_t* h, const int8_t* s, int32_t* I)
{
    for (int i = 0; i < N; ++i) {
        int64_t acc = h[i];
        for (int j = 0; j < N; ++j)
            acc += (int64_t)J[(int64_t)i * N + j] * s[j];
        I[i] = (int32_t)acc;
    }
}

double oracle_energy_f64(int N, const double* J, const double* h, const int8_t* s)
{
    double e = 0.0;
    for (int i = 0; i < N; ++i)
        for (int j = i + 1; j < N; ++j)
            e -= J[(int64_t)i * N + j] * (double)(s[i] * s[j]);
    for (int i = 0; i < N; ++i)
        e -= h[i] * (double)s[i];
    return e;
}

int64_t oracle_bruteforce(int N, const int32_t* J, const int32_t* h, int8_t* s_best)
{
    if (N < 1 || N > 24) return INT64_MAX;
    int8_t* s = (int8_t*)malloc((size_t)N);
    int64_t best = INT64_MAX;
    uint64_t count = 1ull << N;
    for (uint64_t m = 0; m < count; ++m) {
        for (int i = 0; i < N; ++i) s[i] = ((m >> i) & 1u) ? -1 : 1;
        int64_t e = oracle_energy(N, J, h, s);
        if (e < best) {
            best = e;
            if (s_best) memcpy(s_best, s, (size_t)N);
        }
    }
    free(s);
    return best;
}

/* ------------------------------------------------------------------ */
/* Packing onto the fixed-point grid                                   */
/* ------------------------------------------------------------------ */
static int on_grid(double v, int f)
{
    double t = ldexp(v, f);
    return t == nearbyint(t);
}

int oracle_pack(int N, const double* J, const double* h, int frac_bits, int quantize,
                int32_t* J_int, int32_t* h_int, int* f_out)
{
    if (N < 1 || !J || frac_bits > 15) return -1;
    for (int i = 0; i < N; ++i) {
        if (J[(int64_t)i * N + i] != 0.0) return -3;
        for (int j = 0; j < N; ++j) {
            double a = J[(int64_t)i * N + j];
            if (!isfinite(a)) return -1;
            if (a != J[(int64_t)j * N + i]) return -2;
        }
    }
    if (h)
        for (int i = 0; i < N; ++i)
            if (!isfinite(h[i])) return -1;
    int f = frac_bits;
    if (f < 0) {
        for (f = 0; f <= 15; ++f) {
            int ok = 1;
            for (int64_t t = 0; ok && t < (int64_t)N * N; ++t) ok = on_grid(J[t], f);
            for (int i = 0; ok && h && i < N; ++i) ok = on_grid(h[i], f);
            if (ok) break;
        }
        if (f > 15) {
            if (!quantize) return -4;
            f = 15;
        }
    }
    for (int64_t t = 0; t < (int64_t)N * N; ++t) {
        double a = ldexp(J[t], f);
        double q = nearbyint(a);
        if (!quantize && q != a) return -4;
        if (fabs(q) > 2147483647.0) return -4;
        J_int[t] = (int32_t)q;
    }
    for (int i = 0; i < N; ++i) {
        double a = h ? ldexp(h[i], f) : 0.0;
        double q = nearbyint(a);
        if (!quantize && q != a) return -4;
        if (fabs(q) > 2147483647.0) return -4;
        h_int[i] = (int32_t)q;
    }
    if (f_out) *f_out = f;
    return 0;
}

void oracle_beta_linear(float b0, float b1, int64_t T, float* out)
{
    for (int64_t k = 0; k < T; ++k) {
        double b = (double)b0;
        if (T > 1) b = (double)b0 + (((double)b1 - (double)b0) * (double)k) / (double)(T - 1);
        out[k] = (float)b;
    }
}

/* ------------------------------------------------------------------ */
/* The sweep                                                           */
/* ------------------------------------------------------------------ */
enum { TAG_X = 0, TAG_V = 1, TAG_MH = 2 };

/* State of the accept/reject step of one replica (App. A, Table 3 state 4). */
typedef struct {
    int enable;
    float up, down;   /* factors of lam after an accepted / a rejected trajectory */
    float* x0;        /* [N] x at the start of the current trajectory              */
    int64_t* Estart;  /* energy of sgn x0, INT64_MIN before the first one is known */
    int64_t* Qstart;  /* quantised x.x + v.v at the start of the trajectory        */
    float* lam;       /* multiplier of beta                                        */
    int32_t* acc;     /* accepted trajectories                                     */
    int32_t* dec;     /* decided trajectories                                      */
    int8_t* trace;    /* optional: outcome of trajectory m (1 accept, 0 reject,
                         -1 taken without a decision), indexed m - m_first         */
    int64_t m_first;
} mh_ctx;

/* x_i^2 + v_i^2 on the grid 2^-24, capped at 2^46 grid units (2^22), as int64:
 * the squares are exact in double, their sum rounds once. */
static int64_t kinetic_units(float x, float v)
{
    double t = ((double)x * (double)x + (double)v * (double)v) * 0x1p24;
    return (t < 0x1p46) ? (int64_t)nearbyint(t) : ((int64_t)1 << 46);
}

static int64_t kinetic_sum(int N, const float* x, const float* v)
{
    int64_t q = 0;
    for (int i = 0; i < N; ++i) q += kinetic_units(x[i], v[i]);
    return q;
}

/* End of trajectory m = k/L - 1 at the start of step k (k a positive multiple
 * of L): accept its end point (x, v) with probability min(1, exp(-dH)), where
 * H(x, v) = beta E(sgn x) + x.x/2 + v.v/2 (App. A) with the beta of the
 * trajectory's last step times lam; otherwise return x to the trajectory's
 * start.  The first trajectory starts from the initial draw, whose energy is
 * never evaluated: it is taken without a decision.  lam is then multiplied by
 * up or down (Table 3, state 4), clamped to [2^-10, 2^10]. */
static void metropolis(const mh_ctx* m, int N, float sigma, int64_t rr, int64_t k, int64_t L,
                       const float* betas, uint64_t seed, int64_t Eend, float* x, const float* v)
{
    const int64_t traj = k / L - 1;
    int8_t outcome = -1;
    if (*m->Estart != INT64_MIN) {
        const double beta = (double)betas[k - 1] * (double)*m->lam;
        const double dE = (double)(Eend - *m->Estart);
        const double dQ = (double)(kinetic_sum(N, x, v) - *m->Qstart) * 0x1p-25;
        const double dH = fma(beta * (double)sigma, dE, dQ);
        uint64_t ctr[4] = {0, (uint64_t)traj, (uint64_t)rr, TAG_MH}, key[2] = {seed, 0}, out[4];
        oracle_philox4x64_10(ctr, key, out);
        const float lnu = oracle_ln_unit(oracle_uniform((uint32_t)out[0]));
        outcome = ((double)lnu < -dH) ? 1 : 0;
        float lam = *m->lam * (outcome ? m->up : m->down);
        lam = fminf(fmaxf(lam, 0x1p-10f), 0x1p10f);
        *m->lam = lam;
        *m->acc += outcome;
        *m->dec += 1;
    }
    if (outcome == 0)
        memcpy(x, m->x0, sizeof(float) * (size_t)N);
    else
        *m->Estart = Eend;
    if (m->trace && traj >= m->m_first) m->trace[traj - m->m_first] = outcome;
}

/* Momentum update of A7's second line at the current x with step size h_eps:
 * v <- v + h_eps (c sech^2(gamma x) I - x), c = beta gamma sigma (times lam). */
static void kick(int N, float c, float h_eps, float gamma, int deriv, const float* x, const int32_t* I, float* v)
{
    for (int i = 0; i < N; ++i) {
        float d = deriv ? oracle_poly2(gamma * x[i]) : oracle_sech2(gamma * x[i]);
        float p = c * d;
        float g = fmaf(p, (float)I[i], -x[i]);
        v[i] = fmaf(h_eps, g, v[i]);
    }
}

static void anneal_one(int N, const int32_t* J, const int32_t* h, float sigma,
                       int64_t rr, int64_t k0, int64_t k1, const float* betas,
                       float eps, float gamma, int64_t L, uint64_t seed, int init, int deriv, int ikick,
                       float* x, float* v, int64_t* bestE, int8_t* bestS, int64_t* bestStep,
                       int64_t* Etrace, int8_t* s, int32_t* I, const mh_ctx* mh, int64_t* Elast)
{
    if (init) {
        /* App. A, A3: x ~ g(x), the standard normal. */
        for (int i = 0; i < N; ++i) x[i] = oracle_gauss(seed, TAG_X, (uint64_t)rr, 0, (uint64_t)i);
        for (int i = 0; i < N; ++i) v[i] = 0.0f;
        *bestE = INT64_MAX;
        *bestStep = -1;
        memset(bestS, 0, (size_t)N);
        if (mh) {
            *mh->Estart = INT64_MIN;
            *mh->Qstart = 0;
            *mh->lam = 1.0f;
            *mh->acc = 0;
            *mh->dec = 0;
            memcpy(mh->x0, x, sizeof(float) * (size_t)N);
        }
    }
    for (int64_t k = k0; k < k1; ++k) {
        if (k % L == 0) {
            /* Accept/reject of the trajectory that ended with step k - 1. */
            if (mh && k > 0) metropolis(mh, N, sigma, rr, k, L, betas, seed, *Elast, x, v);
            /* Momentum drawn afresh at the start of every round of L steps. */
            for (int i = 0; i < N; ++i)
                v[i] = oracle_gauss(seed, TAG_V, (uint64_t)rr, (uint64_t)(k / L), (uint64_t)i);
            if (mh) {
                memcpy(mh->x0, x, sizeof(float) * (size_t)N);
                *mh->Qstart = kinetic_sum(N, x, v);
            }
            /* Table 3, state 2 (initial-kick variant): the trajectory's first
             * momentum update is half a kick at its start point, with the field
             * of the current spins and this step's beta; the drift-kick steps
             * that follow then form a leapfrog (velocities at half steps). */
            if (ikick) {
                for (int i = 0; i < N; ++i) s[i] = (x[i] >= 0.0f) ? 1 : -1;
                oracle_local_field(N, J, h, s, I);
                kick(N, (betas[k] * gamma) * sigma, 0.5f * eps, gamma, deriv, x, I, v);
            }
        }
        /* A7, first line: drift with the current momentum. */
        for (int i = 0; i < N; ++i) x[i] = fmaf(eps, v[i], x[i]);
        /* Spin readout s = sgn x, with sgn(+0) = sgn(-0) = +1. */
        for (int i = 0; i < N; ++i) s[i] = (x[i] >= 0.0f) ? 1 : -1;
        /* Eq. 6: quasi-gradient. */
        oracle_local_field(N, J, h, s, I);
        /* Eq. 2 through the field: sum_i s_i (I_i + h_i) = 2 sum_{i<j} J s s + 2 sum h s. */
        int64_t two_e = 0;
        for (int i = 0; i < N; ++i) two_e += (int64_t)s[i] * ((int64_t)I[i] + h[i]);
        int64_t E = -(two_e / 2);
        *Elast = E;
        if (Etrace) Etrace[k - k0] = E;
        /* Table 3, state 5: best-so-far, strict improvement keeps the earliest. */
        if (E < *bestE) {
            *bestE = E;
            *bestStep = k;
            memcpy(bestS, s, (size_t)N);
        }
        /* A7, second line, with Eq. 5 and Eq. 8:
         * v <- v + eps (beta gamma sech^2(gamma x) sigma I - x)
         * (POLY2 mode: the quadratic in place of sech^2). */
        float c = (betas[k] * gamma) * sigma;
        if (mh) c = c * *mh->lam;
        kick(N, c, eps, gamma, deriv, x, I, v);
    }
}

int oracle_anneal_ex(int N, const int32_t* J, const int32_t* h, int frac_bits,
                     int R, int64_t r0, int64_t k0, int64_t k1, const float* betas,
                     float eps, float gamma, int64_t L, uint64_t seed, int init, int deriv, int ikick,
                     float* x, float* v, int64_t* bestE, int8_t* bestS, int64_t* bestStep,
                     int64_t* Etrace, int threads, const oracle_mh* mh)
{
    if (N < 1 || R < 0 || k0 < 0 || k1 < k0 || L < 1 || frac_bits < 0 || frac_bits > 30) return -1;
    if (deriv != 0 && deriv != 1) return -1;
    if (ikick != 0 && ikick != 1) return -1;
    if (ikick && mh && mh->enable) return -1;
    if (init && k0 != 0) return -1;
    if (mh && !mh->enable) mh = NULL;
    if (mh && (!mh->x0 || !mh->Estart || !mh->Qstart || !mh->Elast || !mh->lam || !mh->acc || !mh->dec))
        return -1;
    if (mh && !(mh->up > 0.0f && mh->down > 0.0f)) return -1;
    float sigma = ldexpf(1.0f, -frac_bits);
    if (threads < 1) threads = 1;
    /* decisions at k in [max(k0, L), k1) with k % L == 0, trajectories k/L - 1 */
    const int64_t kd0 = (k0 < L ? L : k0 + (L - k0 % L) % L);
    const int64_t m_first = kd0 / L - 1;
    const int64_t nd = (k1 > kd0) ? (k1 - 1 - kd0) / L + 1 : 0;
    int fail = 0;
#ifdef _OPENMP
#pragma omp parallel num_threads(threads)
#endif
    {
        int8_t* s = (int8_t*)malloc((size_t)N);
        int32_t* I = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
        if (!s || !I) fail = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 1)
#endif
        for (int r = 0; r < R; ++r) {
            if (!s || !I) continue;
            int64_t elast_local = 0;
            int64_t* Elast = &elast_local;
            mh_ctx ctx, *pc = NULL;
            if (mh) {
                ctx.enable = 1;
                ctx.up = mh->up;
                ctx.down = mh->down;
                ctx.x0 = mh->x0 + (int64_t)r * N;
                ctx.Estart = mh->Estart + r;
                ctx.Qstart = mh->Qstart + r;
                ctx.lam = mh->lam + r;
                ctx.acc = mh->acc + r;
                ctx.dec = mh->dec + r;
                ctx.trace = mh->trace ? mh->trace + (int64_t)r * nd : NULL;
                ctx.m_first = m_first;
                Elast = mh->Elast + r;
                pc = &ctx;
            }
            anneal_one(N, J, h, sigma, r0 + r, k0, k1, betas, eps, gamma, L, seed, init, deriv, ikick,
                       x + (int64_t)r * N, v + (int64_t)r * N, bestE + r,
                       bestS + (int64_t)r * N, bestStep + r,
                       Etrace ? Etrace + (int64_t)r * (k1 - k0) : NULL, s, I, pc, Elast);
        }
        free(s);
        free(I);
    }
    return fail ? -1 : 0;
}

int oracle_anneal_mh(int N, const int32_t* J, const int32_t* h, int frac_bits,
                     int R, int64_t r0, int64_t k0, int64_t k1, const float* betas,
                     float eps, float gamma, int64_t L, uint64_t seed, int init, int deriv,
                     float* x, float* v, int64_t* bestE, int8_t* bestS, int64_t* bestStep,
                     int64_t* Etrace, int threads, const oracle_mh* mh)
{
    return oracle_anneal_ex(N, J, h, frac_bits, R, r0, k0, k1, betas, eps, gamma, L, seed, init, deriv, 0,
                            x, v, bestE, bestS, bestStep, Etrace, threads, mh);
}

int oracle_anneal(int N, const int32_t* J, const int32_t* h, int frac_bits,
                  int R, int64_t r0, int64_t k0, int64_t k1, const float* betas,
                  float eps, float gamma, int64_t L, uint64_t seed, int init, int deriv,
                  float* x, float* v, int64_t* bestE, int8_t* bestS, int64_t* bestStep,
                  int64_t* Etrace, int threads)
{
    return oracle_anneal_ex(N, J, h, frac_bits, R, r0, k0, k1, betas, eps, gamma, L, seed, init, deriv, 0,
                            x, v, bestE, bestS, bestStep, Etrace, threads, NULL);
}

int oracle_argmin(int R, const int64_t* bestE)
{
    int best = -1;
    for (int r = 0; r < R; ++r)
        if (best < 0 || bestE[r] < bestE[best]) best = r;
    return best;
}
