// Device helpers shared by the sweep kernels of the PHIA library (gfx950):
// block-shared Box-Muller draws of the momentum stream, the kick of one
// element (Eq. 5, Eq. 7-8, App. A A7), wave reductions, and the pieces of the
// accept/reject step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phia_devmath.h"

namespace phia {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Momentum draws happen once every L steps; a real call keeps the unrolled
// sweep loops from holding many Philox states live at once.
// Block-shared momentum draws.  One Philox block of the momentum stream,
// (replica, columns 8 c8 .. 8 c8 + 7), yields the draws of those 8 columns;
// each of its four 64-bit words gives two of them by Box-Muller exactly as
// dev_gauss computes them (gc: the cosine draw of the even column, gs: the
// sine draw of the odd one).
__device__ __forceinline__ void gauss_pair(uint64_t word, float& gc, float& gs)
{
    const float ua = dev_uniform(static_cast<uint32_t>(word));
    const float ub = dev_uniform(static_cast<uint32_t>(word >> 32));
    const float rho = sqrtf(-2.0f * dev_ln_unit(ua));
    float c, sn;
    dev_sincos_2pi(ub, c, sn);
    gc = rho * c;
    gs = rho * sn;
}

// Draws 4 half .. 4 half + 3 of the block (pairs 2 half and 2 half + 1).
__device__ __forceinline__ void gauss_block_half(uint64_t seed, uint64_t replica, uint64_t round, uint64_t c8, int half,
                                                 float (&g)[4])
{
    const u64x4 o = dev_philox(c8, round, replica, kTagV, seed, 0);
    gauss_pair(half ? o.w[2] : o.w[0], g[0], g[1]);
    gauss_pair(half ? o.w[3] : o.w[1], g[2], g[3]);
}

// All 8 draws of the block, g[i & 7] = draw i.
__device__ __forceinline__ void gauss_block(uint64_t seed, uint64_t replica, uint64_t round, uint64_t c8,
                                            float (&g)[8])
{
    const u64x4 o = dev_philox(c8, round, replica, kTagV, seed, 0);
#pragma unroll
    for (int p = 0; p < 4; ++p) gauss_pair(o.w[p], g[2 * p], g[2 * p + 1]);
}

// Value v of lane `src` (all lanes of the wave active).
__device__ __forceinline__ float lane_read(int src, float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src * 4, __builtin_bit_cast(int, v)));
}

__device__ __attribute__((noinline)) float gauss_v(uint64_t seed, uint64_t replica, uint64_t round, int i)
{
    return dev_gauss(seed, kTagV, replica, round, static_cast<uint64_t>(i));
}

// DERIV 0: sech^2 (Eq. 8); 1: the POLY2 quadratic.  Callers branch on the
// (uniform) mode outside their element loops so that the elements of a lane
// interleave.
template <int DERIV>
__device__ __forceinline__ float kick_t(float x, float v, int I, float ck, float eps, float gamma)
{
    const float u = gamma * x;
    const float d = DERIV ? dev_poly2(u) : dev_sech2(u);
    const float p = ck * d;
    const float g = __builtin_fmaf(p, static_cast<float>(I), -x);
    return __builtin_fmaf(eps, g, v);
}

// The same kick with the field already in FP32 (If == (float)I exactly:
// integer fields below 2^24 in magnitude).
template <int DERIV>
__device__ __forceinline__ float kick_tf(float x, float v, float If, float ck, float eps, float gamma)
{
    const float u = gamma * x;
    const float d = DERIV ? dev_poly2(u) : dev_sech2(u);
    const float p = ck * d;
    const float g = __builtin_fmaf(p, If, -x);
    return __builtin_fmaf(eps, g, v);
}

// row_sum16_dpp for FP32 values that are integers below 2^24 in magnitude
// (every partial sum is then exact, so the order does not matter).
__device__ __forceinline__ float dpp_f_b1(float a)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, a), 0xb1, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_f_4e(float a)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, a), 0x4e, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_f_141(float a)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, a), 0x141, 0xf, 0xf, false));
}
__device__ __forceinline__ float row_sum16_dpp_f(float v)
{
    v += dpp_f_b1(v);   // quad_perm [1,0,3,2]
    v += dpp_f_4e(v);   // quad_perm [2,3,0,1]
    v += dpp_f_141(v);  // row_half_mirror
    v += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x140, 0xf, 0xf, true));
    return v;
}

__device__ __forceinline__ float kick(float x, float v, int I, float ck, float eps, float gamma, int deriv)
{
    const float u = gamma * x;
    const float d = deriv ? dev_poly2(u) : dev_sech2(u);
    const float p = ck * d;
    const float g = __builtin_fmaf(p, static_cast<float>(I), -x);
    return __builtin_fmaf(eps, g, v);
}

// Sum over the 16 lanes of a DPP row (lanes sharing lane / 16), result in
// every lane of the row.  All 64 lanes must be active.
__device__ __forceinline__ int row_sum16_dpp(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
    v += __builtin_amdgcn_update_dpp(0, v, 0x4e, 0xf, 0xf, false);   // quad_perm [2,3,0,1]
    v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xf, 0xf, false);  // row_half_mirror
    v += __builtin_amdgcn_mov_dpp(v, 0x140, 0xf, 0xf, true);          // row_mirror (every lane has a source)
    return v;
}

__device__ __forceinline__ int wave_sum16(int v)
{
    // sum over the 16 lanes that share lane / 16
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    return v;
}

__device__ __forceinline__ int wave_sum64(int v)
{
    v = wave_sum16(v);
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    return v;
}

// Accept/reject at the end of every trajectory of L steps (App. A: H(x, v) =
// beta E(sgn x) + x.x/2 + v.v/2; Table 3, state 4: acceptance and temperature).
constexpr uint32_t kTagMH = 2;

// x^2 + v^2 on the grid 2^-24, capped at 2^46 grid units: the squares are exact
// in double and their sum rounds once, so sums over a replica are exact int64
// and independent of the order of summation.
__device__ __forceinline__ long long kin_units(float x, float v)
{
    const double t = (static_cast<double>(x) * static_cast<double>(x) +
                      static_cast<double>(v) * static_cast<double>(v)) * 0x1p24;
    return t < 0x1p46 ? static_cast<long long>(__builtin_rint(t)) : (1ll << 46);
}

// Outcome of trajectory `traj` of stream replica rs: 1 accepted, 0 rejected,
// -1 taken without a decision (start energy Es not known: the first
// trajectory starts from the initial draw).  Ee: energy at its end, dq: change
// of the kinetic units over all columns, beta: inverse temperature of its last
// step, lam: the replica's beta multiplier.  Accept iff ln u < -dH with
// dH = beta lam sigma (Ee - Es) + dq 2^-25 in double and u the first uniform
// of the stream's accept/reject counter (0, traj, rs, tag 2).
__device__ __forceinline__ int mh_outcome(uint64_t seed, uint64_t rs, int64_t traj, int64_t Es, int64_t Ee,
                                          int64_t dq, float beta, float lam, float sigma)
{
    if (Es == INT64_MIN) return -1;
    const double bl = static_cast<double>(beta) * static_cast<double>(lam);
    const double dE = static_cast<double>(Ee - Es);
    const double dQ = static_cast<double>(dq) * 0x1p-25;
    const double dH = __builtin_fma(bl * static_cast<double>(sigma), dE, dQ);
    const u64x4 o = dev_philox(0, static_cast<uint64_t>(traj), rs, kTagMH, seed, 0);
    const float lnu = dev_ln_unit(dev_uniform(static_cast<uint32_t>(o.w[0])));
    return (static_cast<double>(lnu) < -dH) ? 1 : 0;
}

// beta multiplier after an outcome, clamped to [2^-10, 2^10].
__device__ __forceinline__ float mh_lambda(float lam, int outcome, float up, float down)
{
    if (outcome < 0) return lam;
    const float l = lam * (outcome ? up : down);
    return fminf(fmaxf(l, 0x1p-10f), 0x1p10f);
}

__device__ __forceinline__ long long wave_sum16_i64(long long v)
{
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    return v;
}

}  // namespace phia
