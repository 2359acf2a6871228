// VALU sweeps of the PHIA library for gfx950 (k_sweep_valu).
//
// A workgroup of VT threads (256; 1024 for FORMs 0 and 2 above Np = 256)
// owns RB replicas and all of their columns for the whole launch: thread t
// keeps x and v of columns i = t + VT c (c < CPT) of every replica in
// registers, the spins of the current step go to LDS, and J.s + h (Eq. 6)
// runs on the vector ALUs in one of three forms:
//
//   FORM 0 (FP32 path): FP32 couplings [Np][Np] row-major, one FMA per
//          coupling against spins stored as +-1.0f.  The plain sweep.
//   FORM 1 (int8 couplings, few replicas): the int8 fragment layout of the
//          matrix-core sweeps, read by rows: thread i takes the 16-byte runs
//          J[i][16 q .. 16 q + 15] (the lanes of a wave read 256-byte runs)
//          and v_dot4 multiplies four couplings by four int8 spins at once.
//          With few replicas J.s is a matrix-vector product per step and a
//          step is bound by its latency: J sits in LDS when it fits (Np <=
//          384), so no step waits on L2, and no 16-row matrix tile is padded.
//   FORM 2 (ELL path): sparse couplings as D slots per row, [D][Np] words
//          (column index in the low 16 bits, the integer coupling in the
//          high 16), padding slots zero; each slot gathers one spin byte from
//          LDS.  Work per step is proportional to the nonzeros, not N^2.
//
// Every product and sum is an exact integer, so all forms give the same
// field, and the step (refresh, drift, readout, J.s + h, exact energy,
// records, kick; Sec. 2.1, App. A A7, Table 3) is the one of the other
// sweeps bit for bit.  MH adds the accept/reject step of App. A (Table 3,
// state 4) at the end of every trajectory; a.ikick the initial-kick variant
// of Table 3, state 2 (half a kick after every momentum draw).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "phia_devmath.h"
#include "phia_devsweep.h"
#include "phia_internal.h"

namespace phia {

namespace {

constexpr int kVT = 256;  // threads per workgroup of the int8 and ELL forms
// The FP32 and ELL forms take 1024 threads above Np = 256 (one column each
// up to Np = 1024): four waves per SIMD hide the latency of their coupling
// rows (L2) and spin gathers (LDS), where one wave per SIMD with up to 16
// columns per thread waits on them.  Up to Np = 256 one column per thread
// needs only 256.
constexpr int kVtWide = 1024;

// J.s of this thread's columns for every replica of the block (FORM 1):
// fragments [Np/16][Np/64][64][16], lane l of fragment (cb, kb) holding
// J[16 cb + l % 16][64 kb + 16 (l / 16) + t].
template <int CPT, int RB, int VT>
__device__ __forceinline__ void dot_i8(const int8_t* __restrict__ J8, const int8_t* sS8, int Np, int tid,
                                       int (&acc)[RB][CPT])
{
    const int nkb = Np / 64;
    for (int kb = 0; kb < nkb; ++kb) {
        v4i s[RB][4];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int g = 0; g < 4; ++g) s[r][g] = *reinterpret_cast<const v4i*>(sS8 + r * Np + kb * 64 + 16 * g);
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int i = tid + VT * c;
            if (i >= Np) continue;
            const v4i* src = reinterpret_cast<const v4i*>(
                J8 + ((static_cast<size_t>(i >> 4) * nkb + kb) * 64 + (i & 15)) * 16);
            v4i w[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) w[g] = src[16 * g];
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int t = 0; t < 4; ++t) acc[r][c] = __builtin_amdgcn_sdot4(w[g][t], s[r][g][t], acc[r][c], false);
        }
    }
}

// J.s by ELL gathers (FORM 2): slot d of row i is E[d Np + i].
template <int CPT, int RB, int VT>
__device__ __forceinline__ void dot_ell(const int32_t* __restrict__ E, const int8_t* sS8, int Np, int D, int tid,
                                        int (&acc)[RB][CPT])
{
    int d = 0;
    for (; d + 4 <= D; d += 4) {
        int32_t w[4][CPT];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int i = tid + VT * c;
                w[u][c] = (i < Np) ? E[static_cast<size_t>(d + u) * Np + i] : 0;
            }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int j = w[u][c] & 0xffff, val = w[u][c] >> 16;
#pragma unroll
                for (int r = 0; r < RB; ++r) acc[r][c] += val * static_cast<int>(sS8[r * Np + j]);
            }
    }
    for (; d < D; ++d)
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int i = tid + VT * c;
            const int32_t w = (i < Np) ? E[static_cast<size_t>(d) * Np + i] : 0;
            const int j = w & 0xffff, val = w >> 16;
#pragma unroll
            for (int r = 0; r < RB; ++r) acc[r][c] += val * static_cast<int>(sS8[r * Np + j]);
        }
}

// J.s by FP32 multiply-adds (FORM 0), eight rows of J in flight per thread.
template <int CPT, int RB, int VT>
__device__ __forceinline__ void dot_f32(const float* __restrict__ J, const float* sSf, int N, int Np, int tid,
                                        int (&I)[RB][CPT])
{
    float acc[RB][CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c)
#pragma unroll
        for (int r = 0; r < RB; ++r) acc[r][c] = 0.0f;
    int j = 0;
    for (; j + 8 <= N; j += 8) {
        float jv[8][CPT];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int i = tid + VT * c;
                jv[u][c] = (i < Np) ? J[static_cast<int64_t>(j + u) * Np + i] : 0.0f;
            }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            float sj[RB];
#pragma unroll
            for (int r = 0; r < RB; ++r) sj[r] = sSf[r * Np + j + u];
#pragma unroll
            for (int c = 0; c < CPT; ++c)
#pragma unroll
                for (int r = 0; r < RB; ++r) acc[r][c] = __builtin_fmaf(jv[u][c], sj[r], acc[r][c]);
        }
    }
    for (; j < N; ++j) {
        float sj[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) sj[r] = sSf[r * Np + j];
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int i = tid + VT * c;
            const float jv = (i < Np) ? J[static_cast<int64_t>(j) * Np + i] : 0.0f;
#pragma unroll
            for (int r = 0; r < RB; ++r) acc[r][c] = __builtin_fmaf(jv, sj[r], acc[r][c]);
        }
    }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int c = 0; c < CPT; ++c) I[r][c] = static_cast<int>(acc[r][c]);
}

}  // namespace

// JL (FORM 1): the int8 couplings are copied to LDS once per launch, after
// the spins, and every step reads them there.
template <int FORM, int CPT, int RB, bool MH, bool JL, int VT>
__global__ void __launch_bounds__(VT) k_sweep_valu(SweepArgs a)
{
    // spins of the current step: [RB][Np] +-1.0f (FORM 0) or +-1 int8
    extern __shared__ __align__(16) unsigned char sRaw[];
    float* sSf = reinterpret_cast<float*>(sRaw);
    int8_t* sS8 = reinterpret_cast<int8_t*>(sRaw);
    int8_t* sJ8 = reinterpret_cast<int8_t*>(sRaw + valu_jl_offset(RB, a.Np));
    __shared__ int64_t sPart[RB][VT / 64];
    __shared__ int64_t sBest[RB];
    __shared__ int sImp[RB];
    // accept/reject bookkeeping (MH only)
    __shared__ int64_t mEs[RB], mQ0[RB], mEl[RB];
    __shared__ long long mPart[RB][VT / 64];
    __shared__ float mLam[RB];
    __shared__ int mOut[RB], mAcc[RB], mDec[RB];
    constexpr bool mh = MH;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int Np = a.Np, N = a.N;
    const int64_t rb0 = static_cast<int64_t>(blockIdx.x) * RB;

    float x[RB][CPT], v[RB][CPT];
    int hc[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int i = tid + VT * c;
        hc[c] = (i < Np) ? a.h[i] : 0;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const bool ok = (rb0 + r < a.R) && (i < Np);
            x[r][c] = ok ? a.x[(rb0 + r) * Np + i] : 0.0f;
            v[r][c] = ok ? a.v[(rb0 + r) * Np + i] : 0.0f;
        }
    }
    if constexpr (JL) {
        const uint4* src = static_cast<const uint4*>(a.J);
        uint4* dst = reinterpret_cast<uint4*>(sJ8);
        const int n16 = Np * Np / 16;
        for (int u = tid; u < n16; u += VT) dst[u] = src[u];
    }
    int64_t bstep = -1;
    if (tid < RB) {
        const bool ok = rb0 + tid < a.R;
        sBest[tid] = ok ? a.bestE[rb0 + tid] : INT64_MAX;
        bstep = ok ? a.bestStep[rb0 + tid] : -1;
        if (mh) {
            const int64_t gq = rb0 + tid;
            mEs[tid] = ok ? a.mhE[gq * 2] : INT64_MIN;
            mEl[tid] = ok ? a.mhE[gq * 2 + 1] : 0;
            mQ0[tid] = ok ? a.mhQ[gq] : 0;
            mLam[tid] = ok ? a.lam[gq] : 1.0f;
            mAcc[tid] = ok ? a.mhc[gq * 2] : 0;
            mDec[tid] = ok ? a.mhc[gq * 2 + 1] : 0;
        }
    }
    __syncthreads();
    float lamr[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) lamr[r] = mh ? mLam[r] : 1.0f;
    // kinetic units of this thread's elements of row r, summed into mPart[r][wave]
    auto kin_rows = [&]() {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            long long q = 0;
#pragma unroll
            for (int c = 0; c < CPT; ++c) q += kin_units(x[r][c], v[r][c]);
            q = wave_sum16_i64(q);
            q += __shfl_xor(q, 16, 64);
            q += __shfl_xor(q, 32, 64);
            if (lane == 0) mPart[r][wave] = q;
        }
    };

    // J.s of the spins in LDS (no field yet)
    auto js = [&](int (&I)[RB][CPT]) {
        if constexpr (FORM == 0) {
            dot_f32<CPT, RB, VT>(static_cast<const float*>(a.J), sSf, N, Np, tid, I);
        } else {
#pragma unroll
            for (int r = 0; r < RB; ++r)
#pragma unroll
                for (int c = 0; c < CPT; ++c) I[r][c] = 0;
            if constexpr (FORM == 1)
                dot_i8<CPT, RB, VT>(JL ? sJ8 : static_cast<const int8_t*>(a.J), sS8, Np, tid, I);
            else
                dot_ell<CPT, RB, VT>(static_cast<const int32_t*>(a.J), sS8, Np, a.ell_d, tid, I);
        }
    };
    // spins of the current x into LDS
    auto put_spins = [&]() {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int i = tid + VT * c;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const bool pos = x[r][c] >= 0.0f;
                if (i < Np) {
                    if (FORM == 0)
                        sSf[r * Np + i] = pos ? 1.0f : -1.0f;
                    else
                        sS8[r * Np + i] = pos ? 1 : -1;
                }
            }
        }
    };
    // Kick of every element by step size he with the field I (mode branch
    // outside the element loops).
    auto kick_all = [&](const int (&I)[RB][CPT], float ck, float he) {
        auto body = [&](auto mode) {
#pragma unroll
            for (int c = 0; c < CPT; ++c)
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    v[r][c] = kick_t<decltype(mode)::value>(x[r][c], v[r][c], I[r][c], ck * lamr[r], he, a.gamma);
        };
        if (a.deriv)
            body(std::integral_constant<int, 1>{});
        else
            body(std::integral_constant<int, 0>{});
    };

    for (int64_t k = a.k0; k < a.k1; ++k) {
        if (k % a.L == 0) {
            if (mh && k > 0) {
                // End of trajectory k / L - 1 (energy of step k - 1 in mEl): one
                // decision per replica; a rejected end point returns x to the
                // trajectory's start.
                kin_rows();
                __syncthreads();
                if (tid < RB) {
                    const int64_t gq = rb0 + tid;
                    int out = 1;
                    if (gq < a.R) {
                        int64_t qe = 0;
#pragma unroll
                        for (int w = 0; w < VT / 64; ++w) qe += mPart[tid][w];
                        out = mh_outcome(a.seed, static_cast<uint64_t>(a.r_base + gq), k / a.L - 1, mEs[tid],
                                         mEl[tid], qe - mQ0[tid], a.btab[k - 1], mLam[tid], a.sigma);
                        if (out != 0) mEs[tid] = mEl[tid];
                        mLam[tid] = mh_lambda(mLam[tid], out, a.mh_up, a.mh_down);
                        if (out >= 0) {
                            mAcc[tid] += out;
                            mDec[tid] += 1;
                        }
                    }
                    mOut[tid] = out;
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < RB; ++r) {
                    lamr[r] = mLam[r];
                    if (mOut[r] == 0 && rb0 + r < a.R)
#pragma unroll
                        for (int c = 0; c < CPT; ++c) {
                            const int i = tid + VT * c;
                            if (i < Np) x[r][c] = a.x0[(rb0 + r) * Np + i];
                        }
                }
            }
            const uint64_t rnd = static_cast<uint64_t>(k / a.L);
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int i = tid + VT * c;
#pragma unroll
                for (int r = 0; r < RB; ++r)
                    v[r][c] = (i < N && rb0 + r < a.R) ? gauss_v(a.seed, a.r_base + rb0 + r, rnd, i) : 0.0f;
            }
            if (mh) {
                // Start of a trajectory: x snapshot and kinetic units (summed
                // into mQ0 after the next barrier).
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int i = tid + VT * c;
#pragma unroll
                    for (int r = 0; r < RB; ++r)
                        if (rb0 + r < a.R && i < Np) a.x0[(rb0 + r) * Np + i] = x[r][c];
                }
                kin_rows();
            }
            if (a.ikick) {
                // Table 3, state 2 (initial-kick variant): the trajectory's
                // first momentum update is half a kick at its start point,
                // with the field of the current spins and this step's beta.
                put_spins();
                __syncthreads();
                int Ih[RB][CPT];
                js(Ih);
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int c = 0; c < CPT; ++c) Ih[r][c] += hc[c];
                kick_all(Ih, a.ctab[k], 0.5f * a.eps);
                __syncthreads();  // the spins are read before the drift rewrites them
            }
        }
        // Drift and readout; padded columns keep x = 0 and read +1, which
        // meets only zero couplings.
#pragma unroll
        for (int c = 0; c < CPT; ++c)
#pragma unroll
            for (int r = 0; r < RB; ++r) x[r][c] = __builtin_fmaf(a.eps, v[r][c], x[r][c]);
        put_spins();
        __syncthreads();

        int I[RB][CPT];
        js(I);

        // Field, and the row energy partials s (I + h) of step k.
        int part[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            part[r] = 0;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                const int i = tid + VT * c;
                I[r][c] += hc[c];
                const int s = (x[r][c] >= 0.0f) ? 1 : -1;
                if (i < N) part[r] += s * (I[r][c] + hc[c]);
            }
            const int ws = wave_sum64(part[r]);
            if (lane == 0) sPart[r][wave] = ws;
        }
        __syncthreads();
        if (tid < RB) {
            int64_t tot = 0;
#pragma unroll
            for (int w = 0; w < VT / 64; ++w) tot += sPart[tid][w];
            const int64_t E = -(tot / 2);
            if (mh) {
                mEl[tid] = E;
                if (k % a.L == 0) {
                    int64_t q0 = 0;
#pragma unroll
                    for (int w = 0; w < VT / 64; ++w) q0 += mPart[tid][w];
                    mQ0[tid] = q0;
                }
            }
            const bool ok = rb0 + tid < a.R;
            if (ok && a.etrace) a.etrace[(rb0 + tid) * a.T + k] = E;
            const int imp = ok && (E < sBest[tid]);
            if (imp) {
                sBest[tid] = E;
                bstep = k;
            }
            sImp[tid] = imp;
        }
        __syncthreads();
        // Records (Table 3, state 5): the spins of an improved replica.
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (sImp[r]) {
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    const int i = tid + VT * c;
                    if (i < N) a.bestS[(rb0 + r) * Np + i] = (x[r][c] >= 0.0f) ? 1 : -1;
                }
            }
        }
        // Kick (A7, second line).
        kick_all(I, a.ctab[k], a.eps);
    }

#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int i = tid + VT * c;
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            if (rb0 + r < a.R && i < Np) {
                a.x[(rb0 + r) * Np + i] = x[r][c];
                a.v[(rb0 + r) * Np + i] = v[r][c];
            }
        }
    }
    if (tid < RB && rb0 + tid < a.R) {
        a.bestE[rb0 + tid] = sBest[tid];
        a.bestStep[rb0 + tid] = bstep;
        if (mh) {
            const int64_t gq = rb0 + tid;
            a.mhE[gq * 2] = mEs[tid];
            a.mhE[gq * 2 + 1] = mEl[tid];
            a.mhQ[gq] = mQ0[tid];
            a.lam[gq] = mLam[tid];
            a.mhc[gq * 2] = mAcc[tid];
            a.mhc[gq * 2 + 1] = mDec[tid];
        }
    }
}

namespace {

template <int FORM, int CPT, int RB, bool MH, bool JL, int VT = kVT>
hipError_t launch_valu_cpt(const SweepArgs& a, size_t lds, hipStream_t st)
{
    const auto kern = k_sweep_valu<FORM, CPT, RB, MH, JL, VT>;
    // dynamic LDS above the default limit must be allowed per kernel
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    const unsigned blocks = static_cast<unsigned>((a.R + RB - 1) / RB);
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(VT), lds, st, a);
    return hipGetLastError();
}

template <int FORM, int RB, bool MH, bool JL>
hipError_t launch_valu_t(const SweepArgs& a, hipStream_t st)
{
    const size_t lds = valu_lds_bytes(FORM, RB, a.Np, JL);
    if constexpr (FORM == kValuFp32 || FORM == kValuEll) {
        if (a.Np <= kVT) return launch_valu_cpt<FORM, 1, RB, MH, JL>(a, lds, st);
        const int cpt = (a.Np + kVtWide - 1) / kVtWide;
        if (cpt <= 1) return launch_valu_cpt<FORM, 1, RB, MH, JL, kVtWide>(a, lds, st);
        if (cpt <= 2) return launch_valu_cpt<FORM, 2, RB, MH, JL, kVtWide>(a, lds, st);
        if (cpt <= 4) return launch_valu_cpt<FORM, 4, RB, MH, JL, kVtWide>(a, lds, st);
        return hipErrorInvalidValue;  // Np <= 4096
    }
    const int cpt = (a.Np + kVT - 1) / kVT;
    if (cpt <= 1) return launch_valu_cpt<FORM, 1, RB, MH, JL>(a, lds, st);
    if (cpt <= 2) return launch_valu_cpt<FORM, 2, RB, MH, JL>(a, lds, st);
    if constexpr (JL) {
        return hipErrorInvalidValue;  // J in LDS: Np <= 384
    } else {
        if (cpt <= 4) return launch_valu_cpt<FORM, 4, RB, MH, JL>(a, lds, st);
        if (cpt <= 8) return launch_valu_cpt<FORM, 8, RB, MH, JL>(a, lds, st);
        if (cpt <= 16) return launch_valu_cpt<FORM, 16, RB, MH, JL>(a, lds, st);
        return hipErrorInvalidValue;
    }
}

}  // namespace

size_t valu_lds_bytes(int form, int rb, int Np, bool jl)
{
    const size_t spins = static_cast<size_t>(rb) * Np * (form == kValuFp32 ? sizeof(float) : 1);
    return jl ? valu_jl_offset(rb, Np) + static_cast<size_t>(Np) * Np : spins;
}

bool valu_variant(int form, int rb, int mh, bool jl)
{
    switch (form) {
    case kValuFp32: return rb == kFp32Rows && !jl;
    case kValuDot8: return (rb == 1 || rb == 2) && !mh;
    case kValuEll: return (rb == 1 || rb == 4) && !jl;
    default: return false;
    }
}

hipError_t launch_sweep_valu(int form, int rb, bool jl, const SweepArgs& a, hipStream_t st)
{
    if (!valu_variant(form, rb, a.mh, jl) || a.Np > kValuMaxNp) return hipErrorInvalidValue;
    if (jl && valu_lds_bytes(form, rb, a.Np, true) > static_cast<size_t>(kLdsMax)) return hipErrorInvalidValue;
    if (form == kValuFp32) return a.mh ? launch_valu_t<kValuFp32, kFp32Rows, true, false>(a, st)
                                       : launch_valu_t<kValuFp32, kFp32Rows, false, false>(a, st);
    if (form == kValuDot8) {
        if (jl) return rb == 1 ? launch_valu_t<kValuDot8, 1, false, true>(a, st)
                               : launch_valu_t<kValuDot8, 2, false, true>(a, st);
        return rb == 1 ? launch_valu_t<kValuDot8, 1, false, false>(a, st)
                       : launch_valu_t<kValuDot8, 2, false, false>(a, st);
    }
    if (rb == 1) return a.mh ? launch_valu_t<kValuEll, 1, true, false>(a, st)
                             : launch_valu_t<kValuEll, 1, false, false>(a, st);
    return a.mh ? launch_valu_t<kValuEll, 4, true, false>(a, st) : launch_valu_t<kValuEll, 4, false, false>(a, st);
}

}  // namespace phia
