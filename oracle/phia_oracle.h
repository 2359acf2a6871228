/*
 * PHIA CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU reference of the gradient-based
 * Hamiltonian Monte Carlo Ising annealer (Wang et al., "Parallel Ising
 * Annealer via Gradient-based Hamiltonian Monte Carlo").  Only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code with the device library: every routine here is written
 * from the paper and from the numeric specification of the sweep (FP32 op
 * order, counter-based Gaussian stream), never from the device sources.
 *
 * Conventions: J is a full symmetric N x N matrix of integers (units of
 * sigma = 2^-f) with a zero diagonal, h is a length-N integer vector in the
 * same units, spins are int8 +1/-1, energies are exact int64 in sigma units.
 */
#ifndef PHIA_ORACLE_H
#define PHIA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x64-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void oracle_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Elementary FP32 functions of the sweep specification. */
float oracle_exp_nonpos(float y);            /* e^y for y <= 0, 0 below -80          */
float oracle_ln_unit(float u);               /* ln u for normal u in (0, 1)           */
void  oracle_sincos_2pi(float u, float* c, float* s); /* cos, sin of 2*pi*u, u in (0,1) */
float oracle_sech2(float u);                 /* 1 - tanh^2(u), the Eq. 8 factor      */
float oracle_poly2(float u);                 /* max(0, 1 - u^2/2.25), POLY2 mode     */
float oracle_uniform(uint32_t w);            /* (2*(w>>9)+1) * 2^-24                  */
float oracle_gauss(uint64_t seed, uint32_t tag, uint64_t r, uint64_t round, uint64_t i);

/* Eq. 2 energy (double loop over i<j), Eq. 6 local field, FP64 energy. */
int64_t oracle_energy(int N, const int32_t* J, const int32_t* h, const int8_t* s);
void    oracle_local_field(int N, const int32_t* J, const int32_t* h, const int8_t* s, int32_t* I);
double  oracle_energy_f64(int N, const double* J, const double* h, const int8_t* s);

/* Exhaustive ground state over all 2^N configurations (N <= 24).  Ties keep the
 * lowest enumeration index m, where bit i of m set means s_i = -1. */
int64_t oracle_bruteforce(int N, const int32_t* J, const int32_t* h, int8_t* s_best);

/* Fixed-point packing of real couplings onto the grid sigma = 2^-f.
 * frac_bits < 0 picks the smallest f in [0, 15] on which every value lies.
 * quantize = 0 rejects off-grid values; 1 rounds half to even.
 * Returns 0 or a negative code: -1 bad argument, -2 not symmetric,
 * -3 nonzero diagonal, -4 off grid / out of int32 range.  *f_out gets f. */
int oracle_pack(int N, const double* J, const double* h, int frac_bits, int quantize,
                int32_t* J_int, int32_t* h_int, int* f_out);

/* Linear inverse-temperature table: beta_k = b0 + ((b1 - b0) * k) / (T - 1), in
 * double, rounded once to float (T == 1 gives b0). */
void oracle_beta_linear(float b0, float b1, int64_t T, float* out);

/* The annealing sweep.  Runs steps k0 <= k < k1 for replicas r0 .. r0+R-1.
 * init = 1 draws x from the stream and resets the best-so-far records
 * (requires k0 == 0); init = 0 continues from the given x, v and records.
 * betas has at least k1 entries (indexed by absolute step k).
 * Etrace (optional) receives E_k for every replica and step: [R][k1-k0].
 * threads: OpenMP threads over replicas (<= 0 means 1).
 * deriv: 0 TANH (sech^2 of Eq. 8), 1 POLY2 (oracle_poly2 in its place).
 * Returns 0, or -1 on a bad argument. */
int oracle_anneal(int N, const int32_t* J, const int32_t* h, int frac_bits,
                  int R, int64_t r0, int64_t k0, int64_t k1, const float* betas,
                  float eps, float gamma, int64_t L, uint64_t seed, int init, int deriv,
                  float* x, float* v, int64_t* bestE, int8_t* bestS, int64_t* bestStep,
                  int64_t* Etrace, int threads);

/* Accept/reject step at the end of every trajectory of L steps (App. A,
 * Table 3 state 4), with a multiplier lam of beta driven by its outcomes.
 * Arrays are per replica ([R], x0 [R][N]) and carry the state from one call to
 * the next; init = 1 resets them.  trace (optional) receives the outcome of
 * every trajectory decided in this call, [R][number of multiples of L in
 * [max(k0, L), k1)]: 1 accepted, 0 rejected, -1 taken without a decision. */
typedef struct {
    int32_t enable;
    float up, down;   /* lam *= up after an acceptance, *= down after a rejection */
    float* x0;
    int64_t* Estart;
    int64_t* Qstart;
    int64_t* Elast;   /* energy of the last step run                               */
    float* lam;
    int32_t* acc;
    int32_t* dec;
    int8_t* trace;
} oracle_mh;

int oracle_anneal_mh(int N, const int32_t* J, const int32_t* h, int frac_bits,
                     int R, int64_t r0, int64_t k0, int64_t k1, const float* betas,
                     float eps, float gamma, int64_t L, uint64_t seed, int init, int deriv,
                     float* x, float* v, int64_t* bestE, int8_t* bestS, int64_t* bestStep,
                     int64_t* Etrace, int threads, const oracle_mh* mh);

/* Both of the above, plus ikick = 1: the initial-kick variant of Table 3,
 * state 2 -- after every momentum draw, half a kick (step eps / 2) at the
 * current x with the field of its spins and the step's beta, so that the
 * drift-kick steps of each trajectory form a leapfrog.  ikick with an
 * enabled accept/reject step is rejected (-1). */
int oracle_anneal_ex(int N, const int32_t* J, const int32_t* h, int frac_bits,
                     int R, int64_t r0, int64_t k0, int64_t k1, const float* betas,
                     float eps, float gamma, int64_t L, uint64_t seed, int init, int deriv, int ikick,
                     float* x, float* v, int64_t* bestE, int8_t* bestS, int64_t* bestStep,
                     int64_t* Etrace, int threads, const oracle_mh* mh);

/* Lowest best energy over R replicas; ties take the lowest replica index. */
int oracle_argmin(int R, const int64_t* bestE);

#ifdef __cplusplus
}
#endif
#endif
