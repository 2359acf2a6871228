// HIP kernels of the PHIA sweep for gfx950 (MI355X).
//
// One step k of the sweep, for every replica r and spin i at once
// (Wang et al., Sec. 2.1 Eq. 5-8 and App. A A7):
//   if k mod L == 0: v_i ~ N(0, 1)                      (momentum refresh)
//   x_i <- x_i + eps v_i ;  s_i = sgn x_i, sgn(0) = +1   (drift, readout)
//   I_i = sum_j J_ij s_j + h_i                            (Eq. 6, exact int32)
//   E   = -(sum_i s_i (I_i + h_i)) / 2                    (Eq. 2, exact int64)
//   best-so-far record of (E, s)                          (App. B, Table 3)
//   v_i <- v_i + eps (c_k sech^2(gamma x_i) I_i - x_i),   c_k = beta_k gamma sigma
//
// Optionally, at every k > 0 with k mod L == 0, the trajectory that just
// ended is accepted or rejected with H(x, v) = beta E + x.x/2 + v.v/2
// (App. A; App. B, Table 3, state 4), and a per-replica multiplier of beta
// follows the outcomes.
//
// Kernels:
//   k_init         x ~ N(0, I) (App. A, A3), records and accept/reject
//                  state reset.
//   k_sweep_mfma   J.s on matrix cores: int8 x int8 -> int32
//                  (v_mfma_i32_16x16x64_i8) or two BF16 planes J = 256 hi + lo
//                  with FP32 accumulation (v_mfma_f32_16x16x32_bf16).  A
//                  workgroup owns 16*MT replicas and a slice of the columns,
//                  its J slice in LDS or streamed from L2.  When J is too
//                  large for one CU, G workgroups split the columns and swap
//                  the new spins of their slices every step through tagged
//                  64-bit words (bounded polls; partial energies ride along
//                  one step late).  x, v and the accumulators stay in VGPRs
//                  in the MFMA output layout, so the kick is fused with J.s.
//                  Batch mode: one work item (instance, replica block) per
//                  workgroup from a table; with GROUP, several column-split
//                  instances in one cooperative launch.  MH: the accept/reject
//                  step.  INC (column split, J streamed): J.s kept across
//                  steps and updated over the column blocks whose signs
//                  changed, I(k) = I(k-1) + J (s(k) - s(k-1)), exact.
//   k_sweep_pp     the column-split int8 sweep with two 16-replica sub-blocks
//                  per workgroup on two wave teams one phase apart, so the
//                  exchange of one sub-block hides behind the compute of the
//                  other; int8 or FP4 matrix-core operands.
//   k_argmin       lowest best energy over replicas (lowest index on ties).
//   k_energy_f64   FP64 Eq. 2 energy of one configuration.
//   k_fmath_eval   the elementary functions, for bit-exact checks.
#include <stdint.h>

#include <type_traits>

#include "phia_devmath.h"
#include "phia_devsweep.h"
#include "phia_internal.h"

namespace phia {

// ------------------------------------------------------------------ init --
__global__ void __launch_bounds__(256) k_init(SweepArgs a)
{
    const int64_t total = static_cast<int64_t>(a.R) * a.Np;
    for (int64_t idx = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; idx < total;
         idx += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int64_t r = idx / a.Np;
        const int i = static_cast<int>(idx - r * a.Np);
        a.x[idx] = (i < a.N) ? dev_gauss(a.seed, kTagX, a.r_base + r, 0, i) : 0.0f;
        a.v[idx] = 0.0f;
        a.bestS[idx] = 0;
        if (i == 0) {
            a.bestE[r] = INT64_MAX;
            a.bestStep[r] = -1;
            if (a.mh) {
                a.mhE[r * 2] = INT64_MIN;
                a.mhE[r * 2 + 1] = 0;
                a.lam[r] = 1.0f;
                a.mhc[r * 2] = 0;
                a.mhc[r * 2 + 1] = 0;
                const int G = a.G > 1 ? a.G : 1;
                for (int g = 0; g < G; ++g) a.mhQ[r * G + g] = 0;
            }
        }
    }
}

hipError_t launch_init(const SweepArgs& a, hipStream_t st)
{
    const int64_t total = static_cast<int64_t>(a.R) * a.Np;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_init, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// --------------------------------------------------------- MFMA sweep --
// LDS carve-up of one workgroup, shared with the host launch code.
struct LdsPlan {
    uint32_t j_off, s_off, s_bytes, p_off, e_off, b_off, k_off, misc_off, mh_off, u_off, l_off, total;
};

// Accept/reject bookkeeping of a replica block in LDS, 56 bytes per replica:
// int64 [5][rows] (start energy, own kinetic units at the start, own kinetic
// units at the end, summed energy partials, summed kinetic change), then
// float [rows] beta multiplier and int32 [3][rows] (outcome, accepted, decided).
constexpr uint32_t kMhLdsPerRow = 56u;

__host__ __device__ inline uint32_t esz_of(int path) { return path == kPathI8 ? 1u : 2u; }
__host__ __device__ inline uint32_t cb_bytes(int path, int Np)
{
    return static_cast<uint32_t>(Np) * 16u * (path == kPathI8 ? 1u : 4u);
}

// inc: LDS of the flip-incremental field update (the changed column blocks
// as a bit mask [ceil(Np/1024)] uint64 and one list of changed column blocks
// per wave [kWaves][inc_list_len(Np)] uint16, at least 64 entries).
__host__ __device__ inline uint32_t inc_list_len(int Np)
{
    const uint32_t ncb = static_cast<uint32_t>(Np) / 16u;
    return ncb > 64u ? ncb : 64u;
}

__host__ __device__ inline LdsPlan lds_plan(int path, int mt, int Np, int cbs_max, int j_lds, int mh = 0, int inc = 0)
{
    LdsPlan p;
    const uint32_t rows = 16u * mt;
    p.j_off = 0;
    p.s_off = j_lds ? static_cast<uint32_t>(cbs_max) * cb_bytes(path, Np) : 0u;
    p.s_bytes = rows * (static_cast<uint32_t>(Np) * esz_of(path) + 16u);
    p.p_off = p.s_off + 2u * p.s_bytes;
    p.e_off = p.p_off + 3u * rows * 8u;
    p.b_off = p.e_off + 2u * rows * 8u;  // [2][RB] best energies (parity buffers)
    p.k_off = p.b_off + 2u * rows * 8u;  // [RB] step of the best energy
    p.misc_off = p.k_off + rows * 8u;
    p.mh_off = p.misc_off + 16u;
    const uint32_t ncb = static_cast<uint32_t>(Np) / 16u;
    p.u_off = p.mh_off + (mh ? rows * kMhLdsPerRow : 0u);
    p.l_off = p.u_off + (inc ? ((ncb + 63u) / 64u * 8u + 15u) & ~15u : 0u);
    p.total = p.l_off + (inc ? (static_cast<uint32_t>(kWaves) * inc_list_len(Np) * 2u + 15u) & ~15u : 0u);
    return p;
}

// Poll a tagged exchange word until its upper 32 bits equal seq.  Gives up
// after kSpinLimit polls (or when another workgroup has already given up),
// raising the device error word and the workgroup's abort flag; the caller
// then leaves the sweep, so every wave of the grid terminates.
__device__ __forceinline__ uint64_t await_tag(const uint64_t* p, uint32_t seq, int32_t* err, int* abort_flag)
{
    uint32_t polls = 0;
    for (;;) {
        const uint64_t w = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (static_cast<uint32_t>(w >> 32) == seq) return w;
        ++polls;
        if (polls > kSpinLimit ||
            ((polls & 255u) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *abort_flag = 1;
            return w;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Unpack one 16-bit sign word (bit t set: spin +1) into 16 int8 or 16 bf16
// spins of an S row.
template <int ESZ>
__device__ __forceinline__ void unpack_signs(uint32_t w, unsigned char* dst)
{
    if (ESZ == 1) {
        uint32_t d[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint32_t n = (w >> (4 * t)) & 0xfu;
            const uint32_t m = (n * 0x00204081u) & 0x01010101u;  // bit i -> byte i
            d[t] = 0xffffffffu - 0xfeu * m;                      // 0x01 or 0xff per byte
        }
        *reinterpret_cast<uint4*>(dst) = uint4{d[0], d[1], d[2], d[3]};
    } else {
        uint32_t d[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const uint32_t n = (w >> (2 * t)) & 3u;
            const uint32_t m = (n & 1u) | ((n & 2u) << 15);      // bit i -> half i
            d[t] = 0xbf80bf80u - 0x8000u * m;                    // bf16 +1 / -1
        }
        uint4* q = reinterpret_cast<uint4*>(dst);
        q[0] = uint4{d[0], d[1], d[2], d[3]};
        q[1] = uint4{d[4], d[5], d[6], d[7]};
    }
}

// Quasi-gradient of one wave: NCW column blocks (16 columns each) for the MT
// row tiles of the block, I = S . J^T + h on matrix cores.  Jw points at the
// wave's first column block; the next one is kWaves blocks further.  The
// operands of k-block kb+1 are loaded while the products of kb issue.
template <int PATH, int MT, int CBW, int NCW>
__device__ __forceinline__ void quasi_gradient(const unsigned char* S, uint32_t srow, const unsigned char* Jw,
                                               size_t cw_stride, int Np, int lane, int lr, int lg,
                                               const int (&hreg)[CBW], int (&I)[MT][CBW][4])
{
    if (PATH == kPathI8) {
        const int nkb = Np / 64;
        v4i acc[MT][NCW];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw) acc[mt][cw] = v4i{0, 0, 0, 0};
        v4i An[MT], Bn[NCW];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            An[mt] = *reinterpret_cast<const v4i*>(S + (mt * 16 + lr) * srow + 16 * lg);
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) Bn[cw] = *reinterpret_cast<const v4i*>(Jw + cw * cw_stride + lane * 16);
        for (int kb = 0; kb < nkb; ++kb) {
            v4i A[MT], B[NCW];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) A[mt] = An[mt];
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw) B[cw] = Bn[cw];
            if (kb + 1 < nkb) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    An[mt] = *reinterpret_cast<const v4i*>(S + (mt * 16 + lr) * srow + (kb + 1) * 64 + 16 * lg);
#pragma unroll
                for (int cw = 0; cw < NCW; ++cw)
                    Bn[cw] = *reinterpret_cast<const v4i*>(Jw + cw * cw_stride + (kb + 1) * 1024 + lane * 16);
            }
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    acc[mt][cw] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[mt], B[cw], acc[mt][cw], 0, 0, 0);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw)
#pragma unroll
                for (int j = 0; j < 4; ++j) I[mt][cw][j] = acc[mt][cw][j] + hreg[cw];
    } else {
        const int nkc = Np / 32;
        v4f ahi[MT][NCW], alo[MT][NCW];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw) {
                ahi[mt][cw] = v4f{0.f, 0.f, 0.f, 0.f};
                alo[mt][cw] = v4f{0.f, 0.f, 0.f, 0.f};
            }
        v4i An[MT], Hn[NCW], Ln[NCW];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            An[mt] = *reinterpret_cast<const v4i*>(S + (mt * 16 + lr) * srow + 16 * lg);
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) {
            Hn[cw] = *reinterpret_cast<const v4i*>(Jw + cw * cw_stride + lane * 16);
            Ln[cw] = *reinterpret_cast<const v4i*>(Jw + cw * cw_stride + 1024 + lane * 16);
        }
        for (int kc = 0; kc < nkc; ++kc) {
            v4i A[MT], H[NCW], Lo[NCW];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) A[mt] = An[mt];
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw) {
                H[cw] = Hn[cw];
                Lo[cw] = Ln[cw];
            }
            if (kc + 1 < nkc) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    An[mt] = *reinterpret_cast<const v4i*>(S + (mt * 16 + lr) * srow + (kc + 1) * 64 + 16 * lg);
#pragma unroll
                for (int cw = 0; cw < NCW; ++cw) {
                    const unsigned char* b = Jw + cw * cw_stride + static_cast<size_t>(kc + 1) * 2048 + lane * 16;
                    Hn[cw] = *reinterpret_cast<const v4i*>(b);
                    Ln[cw] = *reinterpret_cast<const v4i*>(b + 1024);
                }
            }
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw) {
                const v8bf Bh = __builtin_bit_cast(v8bf, H[cw]);
                const v8bf Bl = __builtin_bit_cast(v8bf, Lo[cw]);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const v8bf Am = __builtin_bit_cast(v8bf, A[mt]);
                    ahi[mt][cw] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am, Bh, ahi[mt][cw], 0, 0, 0);
                    alo[mt][cw] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Am, Bl, alo[mt][cw], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    I[mt][cw][j] = 256 * static_cast<int>(ahi[mt][cw][j]) + static_cast<int>(alo[mt][cw][j]) + hreg[cw];
    }
}

// Dispatch on the wave's column-block count (uniform in the wave).
template <int PATH, int MT, int CBW>
__device__ __forceinline__ void quasi_gradient_w(int ncw, const unsigned char* S, uint32_t srow,
                                                 const unsigned char* Jw, size_t cws, int Np, int lane, int lr,
                                                 int lg, const int (&hreg)[CBW], int (&I)[MT][CBW][4])
{
    if (CBW >= 4 && ncw >= 4)
        quasi_gradient<PATH, MT, CBW, (CBW >= 4 ? 4 : 1)>(S, srow, Jw, cws, Np, lane, lr, lg, hreg, I);
    else if (CBW >= 3 && ncw == 3)
        quasi_gradient<PATH, MT, CBW, (CBW >= 3 ? 3 : 1)>(S, srow, Jw, cws, Np, lane, lr, lg, hreg, I);
    else if (CBW >= 2 && ncw == 2)
        quasi_gradient<PATH, MT, CBW, (CBW >= 2 ? 2 : 1)>(S, srow, Jw, cws, Np, lane, lr, lg, hreg, I);
    else if (ncw >= 1)
        quasi_gradient<PATH, MT, CBW, 1>(S, srow, Jw, cws, Np, lane, lr, lg, hreg, I);
}

// Flip-incremental field update (int8 path, one row tile): acc += J[:, F] dS_F
// over the column blocks F listed in `list` (nf entries), where dS = S_new -
// S_old is -2, 0 or +2 per spin.  The k range of one MFMA holds four listed
// blocks, one per lane group, and a lane's 16 coupling bytes of a block are
// contiguous in the fragment-major layout, so the loads stay 16-byte vectors.
// Integer arithmetic keeps acc equal to the full product J s bit for bit.
template <int CBW, int NCW>
__device__ __forceinline__ void quasi_gradient_inc(const unsigned char* Sn, const unsigned char* So, uint32_t srow,
                                                   const unsigned char* Jw, size_t cw_stride, const uint16_t* list,
                                                   int nf, int lr, int lg, v4i (&acc)[CBW])
{
    const int nvk = (nf + 3) >> 2;
    auto load = [&](int vk, v4i& d, v4i (&B)[NCW]) {
        const int e = 4 * vk + lg;
        const bool ok = e < nf;
        const int c = ok ? list[e] : 0;
        const v4i sn = *reinterpret_cast<const v4i*>(Sn + lr * srow + 16 * c);
        const v4i so = *reinterpret_cast<const v4i*>(So + lr * srow + 16 * c);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            // bytes are 0x01 (+1) or 0xff (-1): 2 s_new per byte where the sign changed
            const uint32_t n = static_cast<uint32_t>(sn[t]), o = static_cast<uint32_t>(so[t]);
            d[t] = ok ? static_cast<int>(((n << 1) & 0xfefefefeu) & (n ^ o)) : 0;
        }
        const size_t off = static_cast<size_t>(c >> 2) * 1024 + static_cast<size_t>(((c & 3) * 16 + lr) * 16);
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) B[cw] = *reinterpret_cast<const v4i*>(Jw + cw * cw_stride + off);
    };
    if (nvk == 0) return;
    v4i dn, Bn[NCW];
    load(0, dn, Bn);
    for (int vk = 0; vk < nvk; ++vk) {
        const v4i d = dn;
        v4i B[NCW];
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) B[cw] = Bn[cw];
        if (vk + 1 < nvk) load(vk + 1, dn, Bn);
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) acc[cw] = __builtin_amdgcn_mfma_i32_16x16x64_i8(d, B[cw], acc[cw], 0, 0, 0);
    }
}

// BF16 hi/lo form of quasi_gradient_inc: a 32-wide k chunk holds two listed
// column blocks (lane groups 0-1 and 2-3 take their halves); dS = +-2 or 0
// is exact in bf16, and the hi and lo planes of each incremental step start
// from zero, so acc += 256 hi + lo stays the exact integer J s.
template <int CBW, int NCW>
__device__ __forceinline__ void quasi_gradient_inc_bf16(const unsigned char* Sn, const unsigned char* So,
                                                        uint32_t srow, const unsigned char* Jw, size_t cw_stride,
                                                        const uint16_t* list, int nf, int lr, int lg,
                                                        v4i (&acc)[CBW])
{
    const int nvk = (nf + 1) >> 1;
    const int h = lg & 1;
    auto load = [&](int vk, v4i& d, v4i (&H)[NCW], v4i (&Lo)[NCW]) {
        const int e = 2 * vk + (lg >> 1);
        const bool ok = e < nf;
        const int c = ok ? list[e] : 0;
        const v4i sn = *reinterpret_cast<const v4i*>(Sn + lr * srow + 32 * c + 16 * h);
        const v4i so = *reinterpret_cast<const v4i*>(So + lr * srow + 32 * c + 16 * h);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            // halves are 0x3f80 (+1) or 0xbf80 (-1): +-2 (0x4000 / 0xc000) where the sign changed
            const uint32_t n = static_cast<uint32_t>(sn[t]), o = static_cast<uint32_t>(so[t]);
            const uint32_t m = ((n ^ o) >> 15) * 0xffffu;
            d[t] = ok ? static_cast<int>(((n & 0x80008000u) | 0x40004000u) & m) : 0;
        }
        const size_t off = static_cast<size_t>(c >> 1) * 2048 +
                           static_cast<size_t>(((2 * (c & 1) + h) * 16 + lr) * 16);
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) {
            H[cw] = *reinterpret_cast<const v4i*>(Jw + cw * cw_stride + off);
            Lo[cw] = *reinterpret_cast<const v4i*>(Jw + cw * cw_stride + off + 1024);
        }
    };
    if (nvk == 0) return;
    v4f ahi[NCW], alo[NCW];
#pragma unroll
    for (int cw = 0; cw < NCW; ++cw) {
        ahi[cw] = v4f{0.f, 0.f, 0.f, 0.f};
        alo[cw] = v4f{0.f, 0.f, 0.f, 0.f};
    }
    v4i dn, Hn[NCW], Ln[NCW];
    load(0, dn, Hn, Ln);
    for (int vk = 0; vk < nvk; ++vk) {
        const v8bf A = __builtin_bit_cast(v8bf, dn);
        v4i H[NCW], Lo[NCW];
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) {
            H[cw] = Hn[cw];
            Lo[cw] = Ln[cw];
        }
        if (vk + 1 < nvk) load(vk + 1, dn, Hn, Ln);
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) {
            ahi[cw] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(v8bf, H[cw]), ahi[cw], 0, 0, 0);
            alo[cw] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, __builtin_bit_cast(v8bf, Lo[cw]), alo[cw], 0, 0, 0);
        }
    }
#pragma unroll
    for (int cw = 0; cw < NCW; ++cw)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            acc[cw][j] += 256 * static_cast<int>(ahi[cw][j]) + static_cast<int>(alo[cw][j]);
}

// One column block and one row tile per wave: registers are capped at 128 so two
// workgroups share a CU and hide each other's exchange latency.
// BATCH: each workgroup runs one work item of a table, with the J placement
// chosen per item: one replica block of one instance and all of its columns,
// or (with GROUP) one member of one group of a column-split instance, so that
// one cooperative launch carries several instances.
// INC: the field is kept in registers across steps and updated by the
// flip-incremental product over the column blocks whose signs changed in any
// replica of the block, or recomputed in full when too many changed.
template <int PATH, int MT, int CBW, bool GROUP, bool JLDS, bool TRACE, bool BATCH = false, bool MH = false,
          bool INC = false>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(CBW == 1 && MT == 1 ? 4 : 2)))
k_sweep_mfma(SweepArgs args)
{
    SweepArgs a = BATCH ? args.table[blockIdx.x] : args;
    if (BATCH && a.seedp) a.seed = *a.seedp;
    const bool jl = BATCH ? (a.j_lds != 0) : JLDS;
    constexpr int RB = 16 * MT;
    constexpr int ESZ = (PATH == kPathI8) ? 1 : 2;
    constexpr int NE = MT * CBW * 4;  // owned elements per lane
    static_assert(NE <= 32, "previous-sign mask holds 32 elements");
    static_assert(!INC || (MT == 1 && GROUP && !BATCH), "flip-incremental variant: one row tile, column split");
    extern __shared__ __align__(16) unsigned char lds[];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lg = lane >> 4;
    const int Np = a.Np, N = a.N;

    int group = BATCH ? a.block : static_cast<int>(blockIdx.x), member = 0;
    const int G = GROUP ? a.G : 1;
    if (GROUP && BATCH) {
        member = a.member;
    } else if (GROUP) {
        if (a.xcd_map) {
            const int w = blockIdx.x, pos = w >> 3;
            member = pos % G;
            group = (pos / G) * 8 + (w & 7);
        } else {
            member = blockIdx.x % G;
            group = blockIdx.x / G;
        }
    }
    const int cb0 = member * a.ncb / G;
    const int cb1 = (member + 1) * a.ncb / G;
    const int cbs = cb1 - cb0;
    const int cbs_max = (a.ncb + G - 1) / G;
    constexpr bool mh = MH;  // accept/reject step (App. A, Table 3 state 4)
    const LdsPlan P = lds_plan(PATH, MT, Np, cbs_max, jl ? 1 : 0, mh ? 1 : 0, INC ? 1 : 0);
    const uint32_t srow = static_cast<uint32_t>(Np) * ESZ + 16u;  // S row stride, bytes
    const uint32_t cbb = cb_bytes(PATH, Np);
    unsigned char* sJ = lds + P.j_off;
    int64_t* sP = reinterpret_cast<int64_t*>(lds + P.p_off);   // [3][RB] partial energies
    int64_t* sE = reinterpret_cast<int64_t*>(lds + P.e_off);   // [2][RB] member-summed partials
    int64_t* sB = reinterpret_cast<int64_t*>(lds + P.b_off);   // [2][RB] best energies
    int64_t* sK = reinterpret_cast<int64_t*>(lds + P.k_off);   // [RB] step of the best
    int* sAbort = reinterpret_cast<int*>(lds + P.misc_off);
    // accept/reject bookkeeping (used only when mh)
    int64_t* mEs = reinterpret_cast<int64_t*>(lds + P.mh_off);  // energy at the trajectory start
    int64_t* mQ0 = mEs + RB;      // member's kinetic units at the trajectory start
    int64_t* mQe = mEs + 2 * RB;  // member's kinetic units at the trajectory end
    int64_t* mTE = mEs + 3 * RB;  // energy partials of the trajectory's last step, summed
    int64_t* mTQ = mEs + 4 * RB;  // kinetic change, summed over the group
    float* mLam = reinterpret_cast<float*>(mEs + 5 * RB);
    int* mOut = reinterpret_cast<int*>(mLam + RB);
    int* mAcc = mOut + RB;
    int* mDec = mAcc + RB;
    // flip-incremental bookkeeping (used only when INC)
    const int ncbk = a.ncb;
    uint64_t* sM = reinterpret_cast<uint64_t*>(lds + P.u_off);  // bit c: a sign of block c changed
    uint16_t* sLw = reinterpret_cast<uint16_t*>(lds + P.l_off) + wave * inc_list_len(Np);  // this wave's list

    const unsigned char* Jg = static_cast<const unsigned char*>(a.J) + static_cast<size_t>(cb0) * cbb;
    if (jl) {
        const uint32_t nvec = static_cast<uint32_t>(cbs) * cbb / 16u;
        const uint4* src = reinterpret_cast<const uint4*>(Jg);
        uint4* dst = reinterpret_cast<uint4*>(sJ);
        for (uint32_t q = tid; q < nvec; q += kThreads) dst[q] = src[q];
    }
    if (tid == 0) *sAbort = 0;
    // column blocks of this wave: c = wave + kWaves * cw for cw < ncw
    const int ncw = wave < cbs ? min(CBW, (cbs - wave + kWaves - 1) / kWaves) : 0;

    int col[CBW], hreg[CBW];
    bool cval[CBW];
#pragma unroll
    for (int cw = 0; cw < CBW; ++cw) {
        const int c = wave + kWaves * cw;
        cval[cw] = c < cbs;
        col[cw] = (cb0 + c) * 16 + lr;
        hreg[cw] = (cval[cw] && col[cw] < Np) ? a.h[col[cw]] : 0;
    }
    const float eps = a.eps, gamma = a.gamma;
    const int nsteps = static_cast<int>(a.k1 - a.k0);
    const uint32_t seq_stride = static_cast<uint32_t>(nsteps + 1);
    // first momentum refresh at or after k0
    const int64_t ref0 = a.k0 + (a.L - a.k0 % a.L) % a.L;
    int iter = 0;

    for (int blk = group; blk < a.nblocks; blk += a.ngroups, ++iter) {
        const int64_t rb0 = static_cast<int64_t>(blk) * RB;
        float x[MT][CBW][4], v[MT][CBW][4];
        bool rval[MT][4];
        for (int q = tid; q < RB; q += kThreads) {
            const bool ok = rb0 + q < a.R;
            sB[q] = sB[RB + q] = ok ? a.bestE[rb0 + q] : INT64_MAX;
            sK[q] = ok ? a.bestStep[rb0 + q] : -1;
            if (mh) {
                const int64_t gq = rb0 + q;
                mEs[q] = ok ? a.mhE[gq * 2] : INT64_MIN;
                mQ0[q] = ok ? a.mhQ[gq * G + member] : 0;
                mQe[q] = mTE[q] = mTQ[q] = 0;
                mLam[q] = ok ? a.lam[gq] : 1.0f;
                mAcc[q] = ok ? a.mhc[gq * 2] : 0;
                mDec[q] = ok ? a.mhc[gq * 2 + 1] : 0;
            }
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t gr = rb0 + mt * 16 + 4 * lg + j;
                rval[mt][j] = gr < a.R;
#pragma unroll
                for (int cw = 0; cw < CBW; ++cw) {
                    const bool ok = rval[mt][j] && cval[cw];
                    x[mt][cw][j] = ok ? a.x[gr * Np + col[cw]] : 0.0f;
                    v[mt][cw][j] = ok ? a.v[gr * Np + col[cw]] : 0.0f;
                }
            }
        // Best configuration of the owned elements as sign bits (bit set:
        // spin +1), same bit layout as pm; written back once per launch.
        uint32_t bestbits = 0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int cw = 0; cw < CBW; ++cw) {
                    const int64_t gr = rb0 + mt * 16 + 4 * lg + j;
                    if (rval[mt][j] && cval[cw] && col[cw] < N && a.bestS[gr * Np + col[cw]] > 0)
                        bestbits |= 1u << ((mt * CBW + cw) * 4 + j);
                }
        for (int q = tid; q < 3 * RB; q += kThreads) sP[q] = 0;
        __syncthreads();
        float lamr[MT][4];  // beta multiplier of each held row
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) lamr[mt][j] = mh ? mLam[mt * 16 + 4 * lg + j] : 1.0f;

        uint32_t pm = 0;  // signs of step k-1, bit (mt*CBW + cw)*4 + j
        v4i accI[CBW];    // INC: J s of the current step (no field), exact
#pragma unroll
        for (int cw = 0; cw < CBW; ++cw) accI[cw] = v4i{0, 0, 0, 0};
        uint32_t n_inc = 0, n_full = 0;  // INC: steps by kind (uniform in the workgroup)
        uint64_t n_kb = 0;               // INC: k blocks of the incremental products
        bool aborted = false;
        int64_t next_ref = ref0;
        uint64_t round = static_cast<uint64_t>(ref0 / a.L);
        int r3 = static_cast<int>(a.k0 % 3);  // k mod 3
        for (int s = 0; s <= nsteps; ++s) {
            const int64_t k = a.k0 + s;
            const bool last = (s == nsteps);  // closing pass: records of step k1-1 only
            const int par = static_cast<int>(k & 1);
            const int r3p = (r3 == 0) ? 2 : r3 - 1, r3n = (r3 == 2) ? 0 : r3 + 1;
            unsigned char* S = lds + P.s_off + par * P.s_bytes;
            pm = 0;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int cw = 0; cw < CBW; ++cw)
#pragma unroll
                    for (int j = 0; j < 4; ++j)
                        if (x[mt][cw][j] >= 0.0f) pm |= 1u << ((mt * CBW + cw) * 4 + j);
            if (!last) {
                if (k == next_ref) {
                    if (mh && k > 0) {
                        // End of trajectory k / L - 1: the member's kinetic units
                        // at its end, then the energy of step k - 1 and the
                        // kinetic change summed over the group, one decision
                        // per replica, and a rejected end point returns x to
                        // the trajectory's start.
                        __syncthreads();  // partial energies of step k - 1 complete
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                long long q = 0;
#pragma unroll
                                for (int cw = 0; cw < CBW; ++cw)
                                    if (cval[cw]) q += kin_units(x[mt][cw][j], v[mt][cw][j]);
                                q = wave_sum16_i64(q);
                                if (lr == 0)
                                    atomicAdd(reinterpret_cast<unsigned long long*>(mQe + mt * 16 + 4 * lg + j),
                                              static_cast<unsigned long long>(q));
                            }
                        __syncthreads();
                        if (GROUP) {
                            const uint32_t mseq = a.seq_base + static_cast<uint32_t>(iter) * seq_stride +
                                                  static_cast<uint32_t>(s) + 1u;
                            const uint64_t mtag = static_cast<uint64_t>(mseq) << 32;
                            const size_t gslot = static_cast<size_t>(par) * a.ngroups + group;
                            uint64_t* Mb = a.mhbuf + gslot * static_cast<size_t>(G) * RB * 4;
                            if (tid < RB) {
                                const uint64_t e = static_cast<uint64_t>(s > 0 ? sP[r3p * RB + tid] : 0);
                                const uint64_t d = static_cast<uint64_t>(mQe[tid] - mQ0[tid]);
                                uint64_t* dst = Mb + (static_cast<size_t>(member) * RB + tid) * 4;
                                __hip_atomic_store(dst, mtag | (e & 0xffffffffu), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                                __hip_atomic_store(dst + 1, mtag | (e >> 32), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                                __hip_atomic_store(dst + 2, mtag | (d & 0xffffffffu), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                                __hip_atomic_store(dst + 3, mtag | (d >> 32), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                            }
                            for (int q = tid; q < G * RB; q += kThreads) {
                                const uint64_t* src = Mb + static_cast<size_t>(q) * 4;
                                uint64_t w[4];
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    w[u] = __hip_atomic_load(src + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
                                for (int u = 0; u < 4; ++u)
                                    if (static_cast<uint32_t>(w[u] >> 32) != mseq)
                                        w[u] = await_tag(src + u, mseq, a.err, sAbort);
                                const uint64_t e = (w[0] & 0xffffffffu) | ((w[1] & 0xffffffffu) << 32);
                                const uint64_t d = (w[2] & 0xffffffffu) | ((w[3] & 0xffffffffu) << 32);
                                atomicAdd(reinterpret_cast<unsigned long long*>(mTE + q % RB),
                                          static_cast<unsigned long long>(e));
                                atomicAdd(reinterpret_cast<unsigned long long*>(mTQ + q % RB),
                                          static_cast<unsigned long long>(d));
                            }
                        } else if (tid < RB) {
                            mTE[tid] = s > 0 ? sP[r3p * RB + tid] : 0;
                            mTQ[tid] = mQe[tid] - mQ0[tid];
                        }
                        __syncthreads();
                        if (GROUP && *sAbort) {
                            aborted = true;
                            break;
                        }
                        if (tid < RB) {
                            const int64_t gq = rb0 + tid;
                            int out = 1;
                            if (gq < a.R) {
                                // energy of step k - 1: summed partials, or stored by
                                // the previous launch when k is its first step
                                const int64_t Ee = s > 0 ? -(mTE[tid] / 2) : a.mhE[gq * 2 + 1];
                                out = mh_outcome(a.seed, static_cast<uint64_t>(a.r_base + gq), k / a.L - 1,
                                                 mEs[tid], Ee, mTQ[tid], a.btab[k - 1], mLam[tid], a.sigma);
                                if (out != 0) mEs[tid] = Ee;
                                mLam[tid] = mh_lambda(mLam[tid], out, a.mh_up, a.mh_down);
                                if (out >= 0) {
                                    mAcc[tid] += out;
                                    mDec[tid] += 1;
                                }
                            }
                            mOut[tid] = out;
                            mQ0[tid] = mQe[tid] = mTE[tid] = mTQ[tid] = 0;
                        }
                        __syncthreads();
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const int row = mt * 16 + 4 * lg + j;
                                lamr[mt][j] = mLam[row];
                                if (mOut[row] == 0 && rval[mt][j]) {
                                    const int64_t gr = rb0 + row;
#pragma unroll
                                    for (int cw = 0; cw < CBW; ++cw)
                                        if (cval[cw]) x[mt][cw][j] = a.x0[gr * Np + col[cw]];
                                }
                            }
                    }
                    // Momentum refresh: one Gaussian per owned element, moved
                    // into the register-resident v afterwards.  The wave's
                    // elements (16 replicas x 16 columns per tile and column
                    // block) fill 32 MT CBW Philox blocks of 8 columns each.
                    // In the column-split sweep (also its table launches)
                    // with two tiles or column blocks per wave that is one
                    // block per lane (two passes of that with the four column
                    // blocks per wave of the int8 batch sweep): every block is
                    // generated once and each element reads its draw from the
                    // lane that made it.  Elsewhere (where the extra
                    // registers would cost occupancy) a rolled loop draws per
                    // element.
                    float vn[NE];
                    if constexpr ((GROUP && MT * CBW == 2) ||
                                  (PATH == kPathI8 && BATCH && !GROUP && !MH && MT == 1 && CBW == 4)) {
                        // pass h covers tiles/column blocks u = 2 h, 2 h + 1;
                        // lane L: u = 2 h + (L >> 5), replica row (L >> 1) & 15,
                        // 8-column half L & 1 (all 8 draws)
                        const int q = lr & 7;
#pragma unroll
                        for (int h = 0; h < MT * CBW / 2; ++h) {
                        const int u = 2 * h + (lane >> 5), mtl = u / CBW, cwl = u % CBW;
                        float g[8];
                        gauss_block(a.seed, a.r_base + rb0 + mtl * 16 + ((lane >> 1) & 15), round,
                                    static_cast<uint64_t>(cb0 + wave + kWaves * cwl) * 2 + (lane & 1), g);
#pragma unroll
                        for (int e = 8 * h; e < 8 * h + 8; ++e) {
                            const int mt = e / (CBW * 4), cw = (e >> 2) % CBW, j = e & 3;
                            const int src = ((mt * CBW + cw) & 1) * 32 + 2 * (4 * lg + j) + (lr >> 3);
                            float t = 0.0f;
#pragma unroll
                            for (int r = 0; r < 8; ++r) {
                                const float tr = lane_read(src, g[r]);
                                t = q == r ? tr : t;
                            }
                            const int c = wave + kWaves * cw;
                            const int64_t gr = rb0 + mt * 16 + 4 * lg + j;
                            vn[e] = (c < cbs && gr < a.R && (cb0 + c) * 16 + lr < N) ? t : 0.0f;
                        }
                        }
                    } else {
#pragma unroll 1
                        for (int e = 0; e < NE; ++e) {
                            const int mt = e / (CBW * 4), cw = (e >> 2) % CBW, j = e & 3;
                            const int c = wave + kWaves * cw;
                            const int cl = (cb0 + c) * 16 + lr;
                            const int64_t gr = rb0 + mt * 16 + 4 * lg + j;
                            const bool ok = c < cbs && gr < a.R && cl < N;
                            vn[e] = ok ? dev_gauss(a.seed, kTagV, a.r_base + gr, round, cl) : 0.0f;
                        }
                    }
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int cw = 0; cw < CBW; ++cw)
#pragma unroll
                            for (int j = 0; j < 4; ++j) v[mt][cw][j] = vn[(mt * CBW + cw) * 4 + j];
                    next_ref += a.L;
                    ++round;
                    if (mh) {
                        // Start of a trajectory: x snapshot and the member's
                        // kinetic units with the fresh momentum.
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const int64_t gr = rb0 + mt * 16 + 4 * lg + j;
                                long long q = 0;
#pragma unroll
                                for (int cw = 0; cw < CBW; ++cw)
                                    if (cval[cw]) {
                                        q += kin_units(x[mt][cw][j], v[mt][cw][j]);
                                        if (rval[mt][j]) a.x0[gr * Np + col[cw]] = x[mt][cw][j];
                                    }
                                q = wave_sum16_i64(q);
                                if (lr == 0)
                                    atomicAdd(reinterpret_cast<unsigned long long*>(mQ0 + mt * 16 + 4 * lg + j),
                                              static_cast<unsigned long long>(q));
                            }
                    }
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int cw = 0; cw < CBW; ++cw) {
                        if (!cval[cw]) continue;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            x[mt][cw][j] = __builtin_fmaf(eps, v[mt][cw][j], x[mt][cw][j]);
                            if (GROUP) continue;  // spins reach S through the exchange
                            const int row = mt * 16 + 4 * lg + j;
                            const bool pos = x[mt][cw][j] >= 0.0f;
                            if (ESZ == 1)
                                S[row * srow + col[cw]] = pos ? 1 : 0xff;
                            else
                                reinterpret_cast<uint16_t*>(S + row * srow)[col[cw]] = pos ? 0x3f80 : 0xbf80;
                        }
                    }
            }

            if (GROUP) {
                // Exchange through agent-coherent relaxed 64-bit atomics (sc1
                // accesses, no L2 write-back or invalidate).  Every word carries
                // the 32-bit sequence number of the step it belongs to, so a
                // reader polls the data itself: one publish and one gather per
                // step, and a stale value is never taken as current.
                const uint32_t seq = a.seq_base + static_cast<uint32_t>(iter) * seq_stride +
                                     static_cast<uint32_t>(s) + 1u;
                const uint64_t tag = static_cast<uint64_t>(seq) << 32;
                const size_t gslot = static_cast<size_t>(par) * a.ngroups + group;
                uint64_t* X = a.xbits + gslot * RB * static_cast<size_t>(a.ncb);
                uint64_t* Pb = a.pbuf + gslot * static_cast<size_t>(G) * RB * 2;
                if (!last) {
                    // One 16-bit sign word per (replica, 16-column block): the
                    // wave's MT*CBW*4 ballots are wave-uniform, and each
                    // publishing lane selects its own with a short select
                    // chain, so every lane stores one word with a single
                    // unbranched instruction (no staging, no per-ballot branch).
                    // With INC every word also carries, in bit 16, whether any
                    // sign of its column block changed in any replica of the
                    // block since step k-1 (pm holds those signs).
                    constexpr int NB = MT * CBW * 4;
                    uint64_t bal[NB];
                    uint32_t lchg = 0;  // INC: bit cw set when one of this lane's signs of block cw changed
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int cw = 0; cw < CBW; ++cw)
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                const bool pos = x[mt][cw][j] >= 0.0f;
                                bal[(mt * CBW + cw) * 4 + j] = __ballot(pos);
                                if (INC) {
                                    const uint32_t was = (pm >> ((mt * CBW + cw) * 4 + j)) & 1u;
                                    lchg |= ((pos ? 1u : 0u) ^ was) << cw;
                                }
                            }
                    uint32_t chg = 0;  // INC: bit cw set when column block cw changed in any replica
                    if (INC) {
#pragma unroll
                        for (int cw = 0; cw < CBW; ++cw)
                            chg |= (__ballot((lchg >> cw) & 1u) != 0 ? 1u : 0u) << cw;
                    }
                    // lane -> (ballot bi = lane / 4, row group g = lane % 4)
                    constexpr int NW = NB * 4;
                    if (lane < NW) {
                        const int bi = lane >> 2, g = lane & 3;
                        const int mt = bi / (CBW * 4), cw = (bi >> 2) % CBW, j = bi & 3;
                        const int c = wave + kWaves * cw;
                        uint64_t b = bal[0];
#pragma unroll
                        for (int t = 1; t < NB; ++t) b = bi == t ? bal[t] : b;
                        const uint64_t w = ((b >> (16 * g)) & 0xffffu) |
                                           (INC ? static_cast<uint64_t>((chg >> cw) & 1u) << 16 : 0u);
                        const int row = mt * 16 + 4 * g + j;
                        if (c < cbs)
                            __hip_atomic_store(X + row * a.ncb + cb0 + c, tag | w, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                if (tid < RB) sE[par * RB + tid] = 0;  // last read two steps ago
                __syncthreads();  // sP of step k-1 complete, sE[par] cleared
                if (s > 0 && tid < RB) {
                    const uint64_t e = static_cast<uint64_t>(sP[r3p * RB + tid]);
                    uint64_t* dst = Pb + (static_cast<size_t>(member) * RB + tid) * 2;
                    __hip_atomic_store(dst, tag | (e & 0xffffffffu), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(dst + 1, tag | (e >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                // Gather every sign word of the block (own columns included)
                // into S, and the members' partial energies of step k-1 into
                // sE[par].  All of a thread's loads are issued before any is
                // inspected: one memory round trip.
                const int nw = last ? 0 : RB * a.ncb;
                bool chg_cb = false;  // INC: changed flag of block tid (words q < ncb are row 0's)
                for (int base = 0; base < nw; base += kThreads * kGatherWords) {
                    uint64_t wv[kGatherWords];
#pragma unroll
                    for (int u = 0; u < kGatherWords; ++u) {
                        const int q = base + u * kThreads + tid;
                        wv[u] = (q < nw) ? __hip_atomic_load(X + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : tag;
                    }
#pragma unroll
                    for (int u = 0; u < kGatherWords; ++u) {
                        const int q = base + u * kThreads + tid;
                        if (q >= nw) continue;
                        uint64_t w = wv[u];
                        if (static_cast<uint32_t>(w >> 32) != seq) w = await_tag(X + q, seq, a.err, sAbort);
                        const int row = q / a.ncb, cb = q - row * a.ncb;
                        unpack_signs<ESZ>(static_cast<uint32_t>(w) & 0xffffu, S + row * srow + cb * 16 * ESZ);
                        if (INC && q < a.ncb) chg_cb = ((w >> 16) & 1u) != 0;
                    }
                }
                if (INC) {
                    // words 0 .. ncb-1 (row 0, all blocks) are thread tid's first
                    // word, so each wave's ballot is 64 blocks of the mask
                    const uint64_t fb = __ballot(chg_cb);
                    if (lane == 0 && wave * 64 < ncbk) sM[wave] = fb;
                }
                if (s > 0) {
                    const int np = G * RB;
                    for (int q = tid; q < np; q += kThreads) {
                        const uint64_t* src = Pb + static_cast<size_t>(q) * 2;
                        uint64_t lo = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        uint64_t hi = __hip_atomic_load(src + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (static_cast<uint32_t>(lo >> 32) != seq) lo = await_tag(src, seq, a.err, sAbort);
                        if (static_cast<uint32_t>(hi >> 32) != seq) hi = await_tag(src + 1, seq, a.err, sAbort);
                        const uint64_t e = (lo & 0xffffffffu) | ((hi & 0xffffffffu) << 32);
                        atomicAdd(reinterpret_cast<unsigned long long*>(sE + par * RB + (q % RB)),
                                  static_cast<unsigned long long>(e));
                    }
                }
                __syncthreads();
                if (*sAbort) {
                    aborted = true;
                    break;
                }
            } else {
                __syncthreads();
            }

            // Records of step k-1 (App. B, Table 3, state 5).  Every lane that
            // holds a row takes the same decision from the previous record
            // (parity buffer par^1); in wave 0 one lane per row writes the new
            // record into buffer par.
            if (s > 0) {
                const int64_t* tot = GROUP ? sE + par * RB : sP + r3p * RB;
                const int64_t* prev = sB + (par ^ 1) * RB;
                int64_t* next = sB + par * RB;
                int64_t Ev[MT][4], Bv[MT][4];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {  // all reads before any write
                        const int row = mt * 16 + 4 * lg + j;
                        Ev[mt][j] = -(tot[row] / 2);
                        Bv[mt][j] = prev[row];
                    }
                if constexpr (GROUP) {
                    uint32_t impm = 0;  // bit mt 4 + j: row mt 16 + 4 lg + j improved
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const bool imp = Ev[mt][j] < Bv[mt][j];
                            impm |= (imp ? 1u : 0u) << (mt * 4 + j);
                            // replace this row's bits of the record by the signs of step k-1
                            uint32_t rowmask = 0;
#pragma unroll
                            for (int cw = 0; cw < CBW; ++cw) rowmask |= 1u << ((mt * CBW + cw) * 4 + j);
                            if (imp) bestbits = (bestbits & ~rowmask) | (pm & rowmask);
                        }
                    // lane lr < 4 MT of each row group of wave 0 writes row
                    // (lr >> 2) 16 + 4 lg + (lr & 3): one masked block of stores
                    if (wave == 0 && lr < 4 * MT) {
                        const int t = lr, row = (t >> 2) * 16 + 4 * lg + (t & 3);
                        int64_t E = Ev[0][0], B = Bv[0][0];
                        bool rv = rval[0][0];
#pragma unroll
                        for (int u = 1; u < 4 * MT; ++u) {
                            E = t == u ? Ev[u >> 2][u & 3] : E;
                            B = t == u ? Bv[u >> 2][u & 3] : B;
                            rv = t == u ? rval[u >> 2][u & 3] : rv;
                        }
                        const bool imp = (impm >> t) & 1u;
                        next[row] = imp ? E : B;
                        if (imp) sK[row] = k - 1;
                        if (TRACE && member == 0 && rv) a.etrace[(rb0 + row) * a.T + (k - 1)] = E;
                        if (mh && last && member == 0 && rv) a.mhE[(rb0 + row) * 2 + 1] = E;
                    }
                } else {
                    // one workgroup per replica block: lane 0 of each row group
                    // writes its rows one by one (fewer registers, so two
                    // workgroups share a CU)
                    const bool writer = (wave == 0 && lr == 0);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int row = mt * 16 + 4 * lg + j;
                            const int64_t E = Ev[mt][j];
                            const int64_t B = Bv[mt][j];
                            const bool imp = E < B;
                            if (writer) {
                                next[row] = imp ? E : B;
                                if (imp) sK[row] = k - 1;
                            }
                            if (TRACE && member == 0 && writer && rval[mt][j])
                                a.etrace[(rb0 + row) * a.T + (k - 1)] = E;
                            if (mh && last && member == 0 && writer && rval[mt][j])
                                a.mhE[(rb0 + row) * 2 + 1] = E;
                            uint32_t rowmask = 0;
#pragma unroll
                            for (int cw = 0; cw < CBW; ++cw) rowmask |= 1u << ((mt * CBW + cw) * 4 + j);
                            if (imp) bestbits = (bestbits & ~rowmask) | (pm & rowmask);
                        }
                }
            }
            if (last) break;
            if (tid < RB) sP[r3n * RB + tid] = 0;
            const float ck = a.ctab[k];

            // Quasi-gradient on matrix cores (columns of this wave only).
            int I[MT][CBW][4] = {};
            bool incr = false;
            if constexpr (INC) {
                // Column blocks whose signs changed in any replica since step
                // k-1, compacted in order into this wave's list; the
                // incremental product runs when it needs at most 2/3 of the
                // full product's k blocks (one of its k blocks costs about
                // 1.5 of the full product's: two spin reads and scattered
                // coupling blocks).
                if (s > 0) {
                    int nf = 0;
                    for (int c0 = 0; c0 < ncbk; c0 += 64) {
                        const uint64_t b = sM[c0 >> 6];  // bits past the last block are clear
                        const int pos = nf + static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                                                 static_cast<uint32_t>(b >> 32),
                                                 __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(b), 0u)));
                        if ((b >> lane) & 1u) sLw[pos] = static_cast<uint16_t>(c0 + lane);
                        nf += __popcll(b);
                    }
                    incr = 3 * ((nf + 3) >> 2) <= 2 * (Np / 64);  // 64-wide k blocks on both paths
                    n_inc += incr ? 1u : 0u;
                    n_kb += incr ? static_cast<uint64_t>((nf + 3) >> 2) : 0u;
                    if (incr) {
                        __builtin_amdgcn_wave_barrier();
                        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                        const unsigned char* So = lds + P.s_off + (par ^ 1) * P.s_bytes;
                        const unsigned char* Jw = Jg + static_cast<size_t>(wave) * cbb;
                        const size_t cws = static_cast<size_t>(kWaves) * cbb;
                        if (PATH == kPathI8) {
                            if (CBW >= 2 && ncw >= 2)
                                quasi_gradient_inc<CBW, (CBW >= 2 ? 2 : 1)>(S, So, srow, Jw, cws, sLw, nf, lr, lg,
                                                                            accI);
                            else if (ncw >= 1)
                                quasi_gradient_inc<CBW, 1>(S, So, srow, Jw, cws, sLw, nf, lr, lg, accI);
                        } else {
                            if (CBW >= 2 && ncw >= 2)
                                quasi_gradient_inc_bf16<CBW, (CBW >= 2 ? 2 : 1)>(S, So, srow, Jw, cws, sLw, nf, lr,
                                                                                 lg, accI);
                            else if (ncw >= 1)
                                quasi_gradient_inc_bf16<CBW, 1>(S, So, srow, Jw, cws, sLw, nf, lr, lg, accI);
                        }
#pragma unroll
                        for (int cw = 0; cw < CBW; ++cw)
#pragma unroll
                            for (int j = 0; j < 4; ++j) I[0][cw][j] = accI[cw][j] + hreg[cw];
                    }
                }
            }
            if (!incr) {
                const size_t cws = static_cast<size_t>(kWaves) * cbb;
                if (jl)
                    quasi_gradient_w<PATH, MT, CBW>(ncw, S, srow, sJ + static_cast<size_t>(wave) * cbb, cws, Np, lane,
                                                    lr, lg, hreg, I);
                else
                    quasi_gradient_w<PATH, MT, CBW>(ncw, S, srow, Jg + static_cast<size_t>(wave) * cbb, cws, Np, lane,
                                                    lr, lg, hreg, I);
                if constexpr (INC) {
                    ++n_full;
#pragma unroll
                    for (int cw = 0; cw < CBW; ++cw)
#pragma unroll
                        for (int j = 0; j < 4; ++j) accI[cw][j] = I[0][cw][j] - hreg[cw];
                }
            }

            // The kick of the owned elements (mode branch outside the loops),
            // then the partial energies of step k.
            auto kick_all = [&](auto mode) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int cw = 0; cw < CBW; ++cw) {
                        if (!cval[cw]) continue;
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            v[mt][cw][j] = kick_t<decltype(mode)::value>(x[mt][cw][j], v[mt][cw][j], I[mt][cw][j],
                                                                        ck * lamr[mt][j], eps, gamma);
                    }
            };
            if (a.deriv)
                kick_all(std::integral_constant<int, 1>{});
            else
                kick_all(std::integral_constant<int, 0>{});
            int psum[MT][4];  // row sums over the 16 columns of each row group
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    int part = 0;
#pragma unroll
                    for (int cw = 0; cw < CBW; ++cw) {
                        if (!cval[cw]) continue;
                        const int sg = (x[mt][cw][j] >= 0.0f) ? 1 : -1;
                        if (col[cw] < N) part += sg * (I[mt][cw][j] + hreg[cw]);
                    }
                    psum[mt][j] = row_sum16_dpp(part);
                }
            // Lane lr < 4 MT of each row group adds row (lr >> 2) 16 + 4 lg + (lr & 3).
            if (lr < 4 * MT) {
                int v = psum[0][0];
#pragma unroll
                for (int t = 1; t < 4 * MT; ++t) v = lr == t ? psum[t >> 2][t & 3] : v;
                atomicAdd(reinterpret_cast<unsigned long long*>(sP + r3 * RB + (lr >> 2) * 16 + 4 * lg + (lr & 3)),
                          static_cast<unsigned long long>(static_cast<int64_t>(v)));
            }
            r3 = r3n;
        }
        if (aborted) return;

#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!rval[mt][j]) continue;
                const int64_t gr = rb0 + mt * 16 + 4 * lg + j;
#pragma unroll
                for (int cw = 0; cw < CBW; ++cw)
                    if (cval[cw]) {
                        a.x[gr * Np + col[cw]] = x[mt][cw][j];
                        a.v[gr * Np + col[cw]] = v[mt][cw][j];
                        if (col[cw] < N)
                            a.bestS[gr * Np + col[cw]] = ((bestbits >> ((mt * CBW + cw) * 4 + j)) & 1u) ? 1 : -1;
                    }
            }
        if (INC && member == 0 && tid == 0 && a.incstat) {
            atomicAdd(reinterpret_cast<unsigned long long*>(a.incstat), static_cast<unsigned long long>(n_inc));
            atomicAdd(reinterpret_cast<unsigned long long*>(a.incstat + 1), static_cast<unsigned long long>(n_full));
            atomicAdd(reinterpret_cast<unsigned long long*>(a.incstat + 2), static_cast<unsigned long long>(n_kb));
        }
        __syncthreads();
        if (member == 0) {
            // Final records sit in the buffer written by the closing pass (k1).
            const int64_t* fin = sB + (a.k1 & 1) * RB;
            for (int q = tid; q < RB; q += kThreads)
                if (rb0 + q < a.R) {
                    a.bestE[rb0 + q] = fin[q];
                    a.bestStep[rb0 + q] = sK[q];
                }
        }
        if (mh)
            for (int q = tid; q < RB; q += kThreads) {
                const int64_t gq = rb0 + q;
                if (gq >= a.R) continue;
                a.mhQ[gq * G + member] = mQ0[q];
                if (member == 0) {
                    a.mhE[gq * 2] = mEs[q];
                    a.lam[gq] = mLam[q];
                    a.mhc[gq * 2] = mAcc[q];
                    a.mhc[gq * 2 + 1] = mDec[q];
                }
            }
        __syncthreads();
    }
}

// ------------------------------------------ interleaved group sweep --
// Column-split int8 sweep in which every workgroup carries two 16-replica
// sub-blocks whose steps alternate.  The spins a sub-block publishes travel
// to the other members of its group while the workgroup computes the other
// sub-block, so the exchange latency hides behind matrix-core and kick work.
// Host-checked requirements: at most kWaves column blocks per member (wave w
// owns column block cb0 + w of both sub-blocks), Np / 16 <= 32 * NU,
// 32 * max_i(sum_j |J_ij| + |h_i|) < 2^23 (a 16-column partial energy fits 24
// bits) and 2 N max_i(...) < 2^31 (a row's energy sum fits int32).  With
// NKB > 0 (FP4 operands: NKB blocks of 128 k positions; int8: Np <= 64 NKB)
// a wave keeps its column block of J in VGPRs as NKB MFMA operand fragments
// for the whole launch; with NKB = 0 the member's int8 J slice sits in LDS,
// or (JG) each product reads it from global memory and both teams share the
// product of the computing one.
//
// Exchange word of (sub-block, replica row, column block), 64 bits:
//   [63:40] low 24 bits of the publication's sequence number (tag)
//   [39:16] sum over the block's 16 columns of s_i (I_i + h_i) of the
//           previous step, signed 24-bit
//   [15:0]  spins, bit t set: spin +1
// Publication q (q = 0 .. nsteps) of a sub-block carries the spins of step
// k0 + q and the partial energies of step k0 + q - 1; the last one (q =
// nsteps) repeats the spins of step k1 - 1, which nothing reads.  Sequence
// numbers of consecutive publications are consecutive (also across replica
// block iterations and launches), and publication seq lives in the slot of
// parity seq & 1: a slot is rewritten two publications later, after every
// member has read it.
struct PpPlan {
    uint32_t j_off, s_off, s_bytes, e_off, b_off, k_off, misc_off, part_off, total;
};

// S row stride: Np bytes, or 64 NKB bytes when the MFMA loop reads NKB
// k blocks unconditionally (bytes past Np meet zero J fragments), plus 16.
__host__ __device__ inline uint32_t pp_srow(int Np, int nkb_regs)
{
    return static_cast<uint32_t>(nkb_regs > 0 ? 64 * nkb_regs : Np) + 16u;
}

// FP4 operands: NKB blocks of 128 k positions, 64 bytes of spins each.
__host__ __device__ inline uint32_t pp_srow_fp4(int nkb_regs) { return 64u * nkb_regs + 16u; }

// LDS of the interleaved sweep.  int8 operands: J slice in LDS unless
// nkb_regs > 0 (VGPR fragments) or jg (J streamed from global memory, the
// L2 of the member's XCD).  FP4 operands: J always in VGPRs (nkb_regs
// fragments per wave, zero past the packed ones).  Without a J slice LDS
// holds the spins and the records only.
__host__ __device__ inline PpPlan pp_plan(int Np, int cbs_max, int nkb_regs, bool fp4 = false, bool jg = false)
{
    PpPlan p;
    p.j_off = 0;
    p.s_off = (fp4 || nkb_regs > 0 || jg) ? 0u : static_cast<uint32_t>(cbs_max) * cb_bytes(kPathI8, Np);
    p.s_bytes = 16u * (fp4 ? pp_srow_fp4(nkb_regs) : pp_srow(Np, nkb_regs));
    p.e_off = p.s_off + 2u * p.s_bytes;  // [2][16] energies of the previous step
    p.b_off = p.e_off + 2u * 16u * 8u;   // [2 sub-blocks][2 parities][16] best energies
    p.k_off = p.b_off + 4u * 16u * 8u;   // [2][16] step of the best energy
    p.misc_off = p.k_off + 2u * 16u * 8u;
    p.part_off = p.misc_off + 16u;  // jg: [8 waves][64 lanes] partial products of the gathering team
    p.total = p.part_off + (jg ? static_cast<uint32_t>(kWaves) * 64u * 16u : 0u);
    return p;
}


// Gather mapping: thread t reads the words of replica row t / 32, column
// blocks t % 32 + 32 u, u < NU; a column block past the end reads the last
// one instead (a valid word, ignored afterwards), so every load is issued
// unconditionally.  off[u] is the word's index in the sub-block's array.
template <int NU>
__device__ __forceinline__ void pp_issue(const uint64_t* Xs, const int (&off)[NU], uint64_t (&w)[NU])
{
#pragma unroll
    for (int u = 0; u < NU; ++u) w[u] = __hip_atomic_load(Xs + off[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NU>
__device__ __forceinline__ uint32_t pp_stale(uint32_t tag, const uint64_t (&w)[NU])
{
    uint32_t m = 0;
#pragma unroll
    for (int u = 0; u < NU; ++u)
        if (static_cast<uint32_t>(w[u] >> 40) != tag) m |= 1u << u;
    return m;
}

// Re-read the words that still carry an older tag until all are current.
// The loop is uniform over the wave.  Returns false after kSpinLimit polls
// or once another workgroup has raised the device error word (then this
// one raises it too).
template <int NU>
__device__ __forceinline__ bool pp_complete(const uint64_t* Xs, const int (&off)[NU], uint32_t tag, uint64_t (&w)[NU],
                                            int32_t* err)
{
    uint32_t stale = pp_stale<NU>(tag, w);
    uint32_t polls = 0;
    while (__any(stale != 0)) {
        ++polls;
        if (polls > kSpinLimit ||
            ((polls & 255u) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
#pragma unroll
        for (int u = 0; u < NU; ++u)
            if ((stale >> u) & 1u) w[u] = __hip_atomic_load(Xs + off[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        stale = pp_stale<NU>(tag, w);
    }
    return true;
}

// The products below run transposed, D = J_slice . S^T: the J fragments are
// the A operand and the spins the B operand (both MFMA operands take row
// lane % 16 and k chunk lane / 16, so the same registers serve either
// side).  Lane (lr, lg) then receives replica lr, columns 4 lg .. 4 lg + 3 of
// the wave's column block: a lane holds one replica, which makes its
// records, its partial energy and its share of the published spins local.
constexpr int kPpDepth = 4;

// J fragments in VGPRs.  The S operands of kPpDepth k blocks are in flight
// ahead of the products; k blocks at or past the packed ones read S padding
// against zero J fragments and add nothing.
template <int NKB>
__device__ __forceinline__ v4i quasi_gradient_regj(const unsigned char* S, uint32_t srow, const v4i (&jr)[NKB], int lr,
                                                   int lg)
{
    const unsigned char* row = S + lr * srow + 16 * lg;
    v4i B[kPpDepth];
#pragma unroll
    for (int d = 0; d < kPpDepth && d < NKB; ++d) B[d] = *reinterpret_cast<const v4i*>(row + d * 64);
    v4i acc = v4i{0, 0, 0, 0};
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
        const v4i cur = B[kb % kPpDepth];
        if (kb + kPpDepth < NKB) B[kb % kPpDepth] = *reinterpret_cast<const v4i*>(row + (kb + kPpDepth) * 64);
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(jr[kb], cur, acc, 0, 0, 0);
    }
    return acc;
}

// The wave's column block of J in LDS (fragment-major, nkb blocks of
// 1 KiB), one k block in flight ahead of the product.
__device__ __forceinline__ v4i quasi_gradient_ldsj(const unsigned char* S, uint32_t srow, const unsigned char* Jw,
                                                   int nkb, int lane, int lr, int lg)
{
    const unsigned char* row = S + lr * srow + 16 * lg;
    const unsigned char* jl = Jw + lane * 16;
    v4i sn = *reinterpret_cast<const v4i*>(row), jn = *reinterpret_cast<const v4i*>(jl);
    v4i acc = v4i{0, 0, 0, 0};
    for (int kb = 0; kb < nkb; ++kb) {
        const v4i s = sn, j = jn;
        if (kb + 1 < nkb) {
            sn = *reinterpret_cast<const v4i*>(row + (kb + 1) * 64);
            jn = *reinterpret_cast<const v4i*>(jl + (kb + 1) * 1024);
        }
        acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(j, s, acc, 0, 0, 0);
    }
    return acc;
}

// The wave's column block of J read from global memory (fragment-major, nkb
// blocks of 1 KiB, served by L2 after the first pass): D fragments in
// flight ahead of the products keep the L2-to-CU fill busy.  The steady
// state loads unconditionally (a conditionally written fragment makes the
// compiler wait for every load at the join); the last fewer than 2 D blocks
// come from the ring and, if needed, one more batch.
constexpr int kPpJgDepth = 4;

template <int D>
__device__ __forceinline__ v4i quasi_gradient_gj(const unsigned char* S, uint32_t srow, const unsigned char* Jg,
                                                 int nkb, int lane, int lr, int lg)
{
    const unsigned char* row = S + lr * srow + 16 * lg;
    const unsigned char* jl = Jg + lane * 16;
    v4i jb[D];
#pragma unroll
    for (int d = 0; d < D; ++d) jb[d] = *reinterpret_cast<const v4i*>(jl + min(d, nkb - 1) * 1024);
    v4i acc = v4i{0, 0, 0, 0};
    int kb = 0;
    for (; kb + 2 * D <= nkb; kb += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            // consume the fragment, then reload its registers (no copy at the
            // loop edge, so the loads stay in flight across iterations)
            const v4i sv = *reinterpret_cast<const v4i*>(row + (kb + d) * 64);
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(jb[d], sv, acc, 0, 0, 0);
            jb[d] = *reinterpret_cast<const v4i*>(jl + (kb + D + d) * 1024);
        }
    }
    if (kb + D < nkb) {  // blocks kb + D .. nkb - 1 (fewer than D)
        v4i jc[D];
#pragma unroll
        for (int d = 0; d < D; ++d) jc[d] = *reinterpret_cast<const v4i*>(jl + min(kb + D + d, nkb - 1) * 1024);
#pragma unroll
        for (int d = 0; d < D; ++d)
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(jb[d], *reinterpret_cast<const v4i*>(row + (kb + d) * 64),
                                                        acc, 0, 0, 0);
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (kb + D + d < nkb)
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                    jc[d], *reinterpret_cast<const v4i*>(row + (kb + D + d) * 64), acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (kb + d < nkb)
                acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                    jb[d], *reinterpret_cast<const v4i*>(row + (kb + d) * 64), acc, 0, 0, 0);
    }
    return acc;
}

// One byte of sign bits as 8 FP4 (E2M1) spins, +1.0 = 0x2 and -1.0 = 0xA:
// the nibbles hold spins 0 4 1 5 2 6 3 7 (the packed J uses the same order
// along k).  The 24-bit multiplies keep the expansion at full VALU rate (the
// compiler would otherwise fold the nibble shift into a 32-bit multiply).
__device__ __forceinline__ uint32_t fp4_byte(uint32_t b)
{
    const uint32_t lo = __umul24(b & 0xfu, 0x00204081u) & 0x01010101u;  // bit i -> bit 8 i
    const uint32_t hi = __umul24(b >> 4, 0x00204081u) & 0x01010101u;
    return 0xaaaaaaaau ^ ((lo | (hi << 4)) << 3);  // clears bit 3 of the nibbles of -1 spins
}

// The product with FP4 operands and FP32 accumulation
// (v_mfma_scale_f32_16x16x128_f8f6f4, scales 1.0): every product and partial
// sum is an integer below 2^24, so the result is exact.  J fragments in
// VGPRs (NKB blocks of 128 k positions; zero past the packed ones), the S
// operands of kPpDepth k blocks in flight ahead of the products; even and
// odd k blocks go to two accumulators (two independent MFMA chains).
template <int NKB>
__device__ __forceinline__ v4f quasi_gradient_fp4(const unsigned char* S, uint32_t srow, const v4i (&jr)[NKB], int lr,
                                                  int lg)
{
    const unsigned char* row = S + lr * srow + 16 * lg;
    v4i B[kPpDepth];
#pragma unroll
    for (int d = 0; d < kPpDepth && d < NKB; ++d) B[d] = *reinterpret_cast<const v4i*>(row + d * 64);
    v4f acc0 = v4f{0.0f, 0.0f, 0.0f, 0.0f}, acc1 = v4f{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
        const v4i ca = jr[kb], cb = B[kb % kPpDepth];
        if (kb + kPpDepth < NKB) B[kb % kPpDepth] = *reinterpret_cast<const v4i*>(row + (kb + kPpDepth) * 64);
        const v8i a8 = v8i{ca[0], ca[1], ca[2], ca[3], 0, 0, 0, 0};
        const v8i b8 = v8i{cb[0], cb[1], cb[2], cb[3], 0, 0, 0, 0};
        if (kb & 1)
            acc1 = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, acc1, 4, 4, 0, 127, 0, 127);
        else
            acc0 = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, b8, acc0, 4, 4, 0, 127, 0, 127);
    }
    return acc0 + acc1;
}

// Sum over the four lanes l, l ^ 16, l ^ 32, l ^ 48 (the lanes of one replica
// in the transposed products), in each of them.  The gfx950 lane swaps
// exchange rows 2i + 1 of the first operand with rows 2i of the second
// (permlane16), then the upper half of the first with the lower half of the
// second (permlane32); applied to two copies of v, the two outputs add up to
// v[l] + v[partner] in every lane.  VALU only: no LDS round trip queued
// behind the other waves' operand reads.  Written in assembly so that the
// two copies stay two registers (the compiler may otherwise take one output
// for the other); the nop covers the VALU-write-to-permlane-read hazard.
// The whole wave must be active.
__device__ __forceinline__ uint32_t replica_sum_u(uint32_t v)
{
    uint32_t a = v, b = v;
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(a), "+v"(b));
    v = a + b;
    a = v;
    b = v;
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
    return a + b;
}

// Sixteen waves: team 0 (waves 0-7) owns sub-block 0, team 1 (waves 8-15)
// sub-block 1; wave w of a team owns column block cb0 + w.  Each team
// alternates between gathering its sub-block's spins (and the previous
// step's energies) and computing one step of it; the teams are one phase
// apart, so in every phase one team computes while the other waits for the
// exchange, and a workgroup barrier closes each phase.
constexpr int kPpWaves = 16;
constexpr int kPpThreads = 64 * kPpWaves;

template <int NU, int NKB, bool FP4 = false, bool JG = false>
__global__ void __launch_bounds__(kPpThreads) __attribute__((amdgpu_waves_per_eu(4))) k_sweep_pp(SweepArgs a)
{
    static_assert(!FP4 || NKB > 0, "FP4 operands need the unrolled k loop");
    static_assert(!JG || (NKB == 0 && !FP4), "streamed J: int8 operands, runtime k loop");
    constexpr bool JREG = NKB > 0;  // J fragments in VGPRs (always for FP4)
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: team and column block in SGPRs
    const int team = wave >> 3, tw = wave & 7, tt = tid & 511;
    const int lr = lane & 15, lg = lane >> 4;
    const int Np = a.Np, N = a.N, ncb = a.ncb, G = a.G;
    int group, member;
    if (a.xcd_map) {
        const int w = blockIdx.x, pos = w >> 3;
        member = pos % G;
        group = (pos / G) * 8 + (w & 7);
    } else {
        member = blockIdx.x % G;
        group = blockIdx.x / G;
    }
    const int cb0 = member * ncb / G, cb1 = (member + 1) * ncb / G, cbs = cb1 - cb0;
    const PpPlan P = pp_plan(Np, (ncb + G - 1) / G, NKB, FP4, JG);
    const uint32_t srow = FP4 ? pp_srow_fp4(NKB) : pp_srow(Np, NKB);
    const int nkb = FP4 ? (Np + 127) / 128 : Np / 64;  // packed k blocks
    const uint32_t cbb = FP4 ? static_cast<uint32_t>(nkb) * 1024u : cb_bytes(kPathI8, Np);
    unsigned char* sJ = lds + P.j_off;
    unsigned char* S = lds + P.s_off + team * P.s_bytes;
    // Energies in int32: the host admits this kernel only when
    // 2 N max_i(sum_j |J_ij| + |h_i|) < 2^31, which bounds every row sum.
    int32_t* sEt = reinterpret_cast<int32_t*>(lds + P.e_off) + team * 16;
    int32_t* sBall = reinterpret_cast<int32_t*>(lds + P.b_off);
    int32_t* sB = sBall + team * 32;  // [parity][16]
    int64_t* sKall = reinterpret_cast<int64_t*>(lds + P.k_off);
    int64_t* sK = sKall + team * 16;
    int* sAbort = reinterpret_cast<int*>(lds + P.misc_off);
    v4i* sPart = reinterpret_cast<v4i*>(lds + P.part_off);
    const bool cval = tw < cbs;  // this wave owns a column block
    const int cblk = cb0 + tw;
    const int col0 = cblk * 16 + 4 * lg;  // the lane's columns col0 .. col0 + 3 (of replica lr)
    // J of the wave's column block: VGPR fragments (fragment-major, nkb
    // packed blocks of 1 KiB per column block, zero past them), the member's
    // int8 slice in LDS, or (JG) read from global memory at every product.
    v4i jr[JREG ? NKB : 1];
    const unsigned char* Jw = static_cast<const unsigned char*>(a.J) + static_cast<size_t>(cblk) * cbb;
    if (JG) {
    } else if (JREG) {
#pragma unroll
        for (int kb = 0; kb < (JREG ? NKB : 1); ++kb)
            jr[kb] = (cval && kb < nkb) ? *reinterpret_cast<const v4i*>(Jw + kb * 1024 + lane * 16)
                                        : v4i{0, 0, 0, 0};
    } else {
        const uint32_t nvec = static_cast<uint32_t>(cbs) * cbb / 16u;
        const uint4* src = reinterpret_cast<const uint4*>(static_cast<const unsigned char*>(a.J) +
                                                          static_cast<size_t>(cb0) * cbb);
        uint4* dst = reinterpret_cast<uint4*>(sJ);
        for (uint32_t q = tid; q < nvec; q += kPpThreads) dst[q] = src[q];
    }
    if (tid == 0) *sAbort = 0;

    // Fields of the lane's columns in FP32 (|h| < 2^18, exact), and which of
    // them are real (col < N; padded columns have zero couplings and field).
    float hf[4];
    uint32_t creal = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        hf[j] = cval ? static_cast<float>(a.h[col0 + j]) : 0.0f;
        if (cval && col0 + j < N) creal |= 1u << j;
    }
    const int grow = tt >> 5, gc0 = tt & 31;
    const float eps = a.eps, gamma = a.gamma;
    const int nsteps = static_cast<int>(a.k1 - a.k0);
    const uint32_t seq_stride = static_cast<uint32_t>(nsteps + 1);
    const int64_t ref0 = a.k0 + (a.L - a.k0 % a.L) % a.L;
    const size_t plane = static_cast<size_t>(16) * ncb;
    int goff[NU];  // gather: word indices of this thread
#pragma unroll
    for (int u = 0; u < NU; ++u) goff[u] = grow * ncb + min(gc0 + 32 * u, ncb - 1);
    const int poff = lr * ncb + cblk;  // publication: the word of replica row lr (lanes lg == 0)
    int iter = 0;

    for (int blk = group; blk < a.nblocks; blk += a.ngroups, ++iter) {
        const int64_t rb0 = static_cast<int64_t>(blk) * 32;
        const int64_t tb0 = rb0 + team * 16;  // first replica of this team's sub-block
        // word array of this team's sub-block for publication seq
        auto xs = [&](uint32_t seq) -> uint64_t* {
            return a.xbits + ((static_cast<size_t>(seq & 1u) * a.ngroups + group) * 2 + team) * plane;
        };
        for (int q = tid; q < 32; q += kPpThreads) {
            const int sb = q >> 4, r = q & 15;
            const bool ok = rb0 + q < a.R;
            const int64_t b = ok ? a.bestE[rb0 + q] : INT64_MAX;
            const int32_t b32 = b > INT32_MAX ? INT32_MAX : static_cast<int32_t>(b);  // INT32_MAX: no record yet
            sBall[(sb * 2 + 0) * 16 + r] = b32;
            sBall[(sb * 2 + 1) * 16 + r] = b32;
            sKall[q] = ok ? a.bestStep[rb0 + q] : -1;
        }
        const int64_t gr = tb0 + lr;  // the lane's replica
        const bool rok = cval && gr < a.R;
        float x[4], v[4];
        uint32_t bestbits = 0, pm = 0;
        if (rok) {
            const float4 xx = *reinterpret_cast<const float4*>(a.x + gr * Np + col0);
            const float4 vv = *reinterpret_cast<const float4*>(a.v + gr * Np + col0);
            const uint32_t bs = *reinterpret_cast<const uint32_t*>(a.bestS + gr * Np + col0);
            x[0] = xx.x, x[1] = xx.y, x[2] = xx.z, x[3] = xx.w;
            v[0] = vv.x, v[1] = vv.y, v[2] = vv.z, v[3] = vv.w;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (((creal >> j) & 1u) && static_cast<int8_t>((bs >> (8 * j)) & 0xffu) > 0) bestbits |= 1u << j;
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = v[j] = 0.0f;
        }

        const uint32_t seq0 = a.seq_base + static_cast<uint32_t>(iter) * seq_stride + 1u;
        int64_t next_ref = ref0;
        uint64_t round = static_cast<uint64_t>(ref0 / a.L);
        uint64_t w[NU];

        // Momentum refresh of the lane's four elements (draws of `round`):
        // columns 4 lg .. 4 lg + 3 of the column block are the half lg & 1 of
        // the Philox block of (replica, 8-column group 2 cblk + (lg >> 1)),
        // so every lane draws its own elements.
        auto refresh = [&]() {
            float g[4];
            gauss_block_half(a.seed, a.r_base + gr, round, static_cast<uint64_t>(cblk) * 2 + (lg >> 1), lg & 1, g);
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = (((creal >> j) & 1u) && gr < a.R) ? g[j] : 0.0f;
        };
        auto signs4 = [&]() {
            uint32_t m = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (x[j] >= 0.0f) m |= 1u << j;
            return m;
        };
        // Word of replica lr: the 16 spins of the column block gathered from
        // the four lanes of the replica, and the partial energy qi.  Called
        // with the whole wave active.
        auto publish = [&](uint64_t* X, int qi, uint32_t tag) {
            const uint32_t m = replica_sum_u(signs4() << (4 * lg));  // disjoint bits: the sum is the OR
            const uint64_t word = (static_cast<uint64_t>(tag) << 40) |
                                  (static_cast<uint64_t>(static_cast<uint32_t>(qi) & 0xffffffu) << 16) | m;
            if (lg == 0) __hip_atomic_store(X + poff, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };

        // Publication q: spins of step k0 + q and partial energies of step
        // k0 + q - 1 of this team's sub-block; read into S (q < nsteps) and
        // the energies (q > 0).  Returns false when the wait gave up.
        float ck_next = 0.0f;  // c_k of the next compute phase, loaded with its gather
        auto gather = [&](int q) {
            const uint32_t seq = seq0 + static_cast<uint32_t>(q);
            if (q < nsteps) ck_next = a.ctab[a.k0 + q];
            const uint64_t* X = xs(seq);
            pp_issue<NU>(X, goff, w);
            const bool ok = pp_complete<NU>(X, goff, seq & 0xffffffu, w, a.err);
            int psum = 0;
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int c = gc0 + 32 * u;
                if (c < ncb) {
                    const uint32_t lo = static_cast<uint32_t>(w[u]);
                    if (q < nsteps) {
                        if (FP4)
                            *reinterpret_cast<uint2*>(S + grow * srow + c * 8) =
                                uint2{fp4_byte(lo & 0xffu), fp4_byte((lo >> 8) & 0xffu)};
                        else
                            unpack_signs<1>(lo & 0xffffu, S + grow * srow + c * 16);
                    }
                    psum += static_cast<int32_t>(static_cast<uint32_t>(w[u] >> 16) << 8) >> 8;
                }
            }
            if (q > 0) {
                // Row total over the 32 lanes of the replica row: DPP row
                // sums, then row r - 1 added into rows 1 and 3.  The total
                // is even (J symmetric, h counted twice); its negative half
                // is the energy (Eq. 2).
                int t = row_sum16_dpp(psum);
                t += __builtin_amdgcn_update_dpp(0, t, 0x142, 0xa, 0xf, false);  // row_bcast:15
                if (gc0 == 31) sEt[grow] = -(t >> 1);
            }
            return ok;
        };

        // Step k0 + s and its publication s + 1 (s < nsteps), then the
        // records of step k0 + s - 1.
        auto compute = [&](int s, v4i jg_acc) {
            const int64_t k = a.k0 + s;
            const bool closing = (s == nsteps);
            const float ck = ck_next;
            v4f facc = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            v4i iacc = v4i{0, 0, 0, 0};
            if (!closing && cval) {
                if (FP4)
                    facc = quasi_gradient_fp4<(JREG ? NKB : 1)>(S, srow, jr, lr, lg);
                else if (JREG)
                    iacc = quasi_gradient_regj<(JREG ? NKB : 1)>(S, srow, jr, lr, lg);
                else if (JG)
                    iacc = jg_acc;  // computed by both teams before the mid-phase barrier
                else
                    iacc = quasi_gradient_ldsj(S, srow, sJ + static_cast<size_t>(tw) * cbb, nkb, lane, lr, lg);
            }
            // The records of step k - 1 wait until after the publication:
            // the next gather of every member waits on the words, nothing
            // waits on the records within the phase.
            const uint32_t pm_prev = pm;
            auto records = [&]() {
                if (s > 0) {  // App. B, Table 3, state 5: the records of replica lr
                    const int par = static_cast<int>(k & 1);
                    const int32_t Ev = sEt[lr], Bv = sB[(par ^ 1) * 16 + lr];
                    const bool imp = Ev < Bv;
                    if (imp) bestbits = pm_prev;
                    if (tw == 0 && lg == 0) {
                        sB[par * 16 + lr] = imp ? Ev : Bv;
                        if (imp) sK[lr] = k - 1;
                    }
                }
            };
            if (closing || !cval) {
                records();
                return;
            }
            // I = J s + h and s (I + h) in FP32: integers below 2^24 (host
            // check), so every sum is exact.
            float If[4], q = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float f = FP4 ? facc[j] : static_cast<float>(iacc[j]);
                If[j] = f + hf[j];
                const float e = If[j] + hf[j];
                q += (x[j] >= 0.0f) ? e : -e;
            }
            const int qi = static_cast<int>(replica_sum_u(static_cast<uint32_t>(static_cast<int>(q))));
            if (a.deriv) {
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = kick_tf<1>(x[j], v[j], If[j], ck, eps, gamma);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = kick_tf<0>(x[j], v[j], If[j], ck, eps, gamma);
            }
            pm = signs4();
            if (s + 1 < nsteps) {
                if (k + 1 == next_ref) refresh();
#pragma unroll
                for (int j = 0; j < 4; ++j) x[j] = __builtin_fmaf(eps, v[j], x[j]);
            }
            const uint32_t seq = seq0 + static_cast<uint32_t>(s) + 1u;
            publish(xs(seq), qi, seq & 0xffffffu);
            records();
        };

        // Publication 0: the drift of step k0.
        {
            pm = signs4();
            if (a.k0 == next_ref) {
                refresh();
                next_ref += a.L;
                ++round;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) x[j] = __builtin_fmaf(eps, v[j], x[j]);
            if (cval) publish(xs(seq0), 0, seq0 & 0xffffffu);
        }
        __syncthreads();  // records initialised
        if (team == 0 && !gather(0)) *sAbort = 1;
        __syncthreads();
        // Phase ph: team ph % 2 computes, the other team gathers.
        bool aborted = false;
        int abort_seen = 0;
        const int nphase = 2 * nsteps + 2;
        for (int ph = 0; ph < nphase; ++ph) {
            if (abort_seen) {
                aborted = true;
                break;
            }
            const int abort_flag = *sAbort;  // consumed one phase later
            v4i jg_acc = v4i{0, 0, 0, 0};
            if (JG) {
                // The product of the computing team's step, split between the
                // teams: the computing team takes k blocks [0, kh), the
                // gathering team [kh, nkb) of the same column block and
                // sub-block (its spins are in LDS since the previous phase),
                // handing its partial over through LDS.  Twice the J fragments
                // in flight per CU; the gathering team polls for its words
                // after the barrier.
                const int cteam = ph & 1, sc = (ph - cteam) >> 1;
                const int kh = (nkb + 1) >> 1;
                if (sc < nsteps && cval) {
                    const unsigned char* Sc = lds + P.s_off + cteam * P.s_bytes;
                    if (team == cteam)
                        jg_acc = quasi_gradient_gj<kPpJgDepth>(Sc, srow, Jw, kh, lane, lr, lg);
                    else if (nkb > kh)
                        sPart[tw * 64 + lane] = quasi_gradient_gj<kPpJgDepth>(Sc + kh * 64, srow, Jw + kh * 1024,
                                                                              nkb - kh, lane, lr, lg);
                }
                __syncthreads();
                if (team == cteam && sc < nsteps && cval && nkb > kh) jg_acc += sPart[tw * 64 + lane];
            }
            if (team == (ph & 1)) {
                const int s = (ph - team) >> 1;
                compute(s, jg_acc);
                if (s + 1 < nsteps && a.k0 + s + 1 == next_ref) {
                    next_ref += a.L;
                    ++round;
                }
            } else {
                const int q = (team == 0) ? (ph + 1) >> 1 : ph >> 1;
                if (q <= nsteps && !gather(q)) *sAbort = 1;
            }
            __syncthreads();
            abort_seen = abort_flag;
        }
        if (aborted) return;

        if (rok) {
            *reinterpret_cast<float4*>(a.x + gr * Np + col0) = float4{x[0], x[1], x[2], x[3]};
            *reinterpret_cast<float4*>(a.v + gr * Np + col0) = float4{v[0], v[1], v[2], v[3]};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((creal >> j) & 1u) a.bestS[gr * Np + col0 + j] = ((bestbits >> j) & 1u) ? 1 : -1;
        }
        __syncthreads();
        if (member == 0) {
            const int fin = static_cast<int>(a.k1 & 1);
            for (int q = tid; q < 32; q += kPpThreads)
                if (rb0 + q < a.R) {
                    const int sb = q >> 4, r = q & 15;
                    const int32_t e = sBall[(sb * 2 + fin) * 16 + r];
                    a.bestE[rb0 + q] = e == INT32_MAX ? INT64_MAX : e;
                    a.bestStep[rb0 + q] = sKall[q];
                }
        }
        __syncthreads();
    }
}

// J fragments per wave kept in VGPRs for Np: the k-block count rounded up
// to even, up to 4 (sixteen waves leave 128 registers per lane); 0: J slice
// in LDS.
static int pp_nkb_regs(int Np)
{
    const int nkb = Np / 64;
    return nkb <= 4 ? (nkb + 1) / 2 * 2 : 0;
}

// FP4 k blocks (128 wide) of the unrolled product: ceil(Np / 128) rounded up
// to even, up to 8 (Np <= 1024).
static int pp_nkb4(int Np)
{
    const int nkb = (Np + 127) / 128;
    return nkb <= 8 ? (nkb + 1) / 2 * 2 : 0;
}

size_t sweep_pp_lds_bytes(int Np, int G, int fp4, int jg)
{
    const int ncb = Np / 16;
    if (fp4) return pp_plan(Np, (ncb + G - 1) / G, pp_nkb4(Np), true).total;
    if (jg) return pp_plan(Np, (ncb + G - 1) / G, 0, false, true).total;
    return pp_plan(Np, (ncb + G - 1) / G, pp_nkb_regs(Np)).total;
}

static const void* pp_kernel(int ncb, int fp4, int jg)
{
    const int Np = 16 * ncb;
    if (fp4) {
        switch (pp_nkb4(Np)) {
        case 2: return reinterpret_cast<const void*>(k_sweep_pp<1, 2, true>);
        case 4: return reinterpret_cast<const void*>(k_sweep_pp<1, 4, true>);
        case 6: return reinterpret_cast<const void*>(k_sweep_pp<2, 6, true>);
        case 8: return reinterpret_cast<const void*>(k_sweep_pp<2, 8, true>);
        default: return nullptr;
        }
    }
    if (jg) {  // Np <= 2048: wider gathers would spill the J ring
        if (ncb <= 32) return reinterpret_cast<const void*>(k_sweep_pp<1, 0, false, true>);
        if (ncb <= 64) return reinterpret_cast<const void*>(k_sweep_pp<2, 0, false, true>);
        if (ncb <= 128) return reinterpret_cast<const void*>(k_sweep_pp<4, 0, false, true>);
        return nullptr;
    }
    switch (pp_nkb_regs(Np)) {
    case 2: return reinterpret_cast<const void*>(k_sweep_pp<1, 2>);
    case 4: return reinterpret_cast<const void*>(k_sweep_pp<1, 4>);
    default: break;
    }
    if (ncb <= 32) return reinterpret_cast<const void*>(k_sweep_pp<1, 0>);
    if (ncb <= 64) return reinterpret_cast<const void*>(k_sweep_pp<2, 0>);
    if (ncb <= 128) return reinterpret_cast<const void*>(k_sweep_pp<4, 0>);
    return reinterpret_cast<const void*>(k_sweep_pp<8, 0>);
}

hipError_t launch_sweep_pp(const SweepArgs& a, int fp4, int jg, size_t lds, hipStream_t st)
{
    if (a.ncb < 1 || a.ncb > kPpMaxNcb) return hipErrorInvalidValue;
    const void* kern = pp_kernel(a.ncb, fp4, jg);
    if (!kern) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    SweepArgs copy = a;
    void* args[] = {&copy};
    e = hipLaunchCooperativeKernel(kern, dim3(static_cast<unsigned>(a.ngroups * a.G)), dim3(kPpThreads), args,
                                   static_cast<unsigned>(lds), st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

int max_coresident_pp(int ncb, int fp4, int jg, size_t lds)
{
    int dev = 0, cus = 0, per = 0;
    if (ncb < 1 || ncb > kPpMaxNcb) return 0;
    const void* f = pp_kernel(ncb, fp4, jg);
    if (!f) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, kPpThreads, lds) != hipSuccess) return 0;
    return per * cus;
}

// ------------------------------------------------------------ batching --
// One workgroup per instance: x ~ N(0, I), v = 0, records reset.
__global__ void __launch_bounds__(256) k_init_batch(const SweepArgs* table)
{
    SweepArgs a = table[blockIdx.x];
    if (a.seedp) a.seed = *a.seedp;
    const int64_t total = static_cast<int64_t>(a.R) * a.Np;
    for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int64_t r = idx / a.Np;
        const int i = static_cast<int>(idx - r * a.Np);
        a.x[idx] = (i < a.N) ? dev_gauss(a.seed, kTagX, a.r_base + r, 0, i) : 0.0f;
        a.v[idx] = 0.0f;
        a.bestS[idx] = 0;
        if (i == 0) {
            a.bestE[r] = INT64_MAX;
            a.bestStep[r] = -1;
            if (a.mh) {
                a.mhE[r * 2] = INT64_MIN;
                a.mhE[r * 2 + 1] = 0;
                a.lam[r] = 1.0f;
                a.mhc[r * 2] = 0;
                a.mhc[r * 2 + 1] = 0;
                const int G = a.G > 1 ? a.G : 1;
                for (int g = 0; g < G; ++g) a.mhQ[r * G + g] = 0;
            }
        }
    }
}

hipError_t launch_init_batch(const SweepArgs* dtable, int count, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_batch, dim3(static_cast<unsigned>(count)), dim3(256), 0, st, dtable);
    return hipGetLastError();
}

size_t sweep_batch_lds_bytes(int path, int Np, int j_lds, int mh)
{
    return lds_plan(path, 1, Np, Np / 16, j_lds, mh).total;
}

template <int PATH, int CBW>
static const void* batch_kernel(bool mh)
{
    return mh ? reinterpret_cast<const void*>(k_sweep_mfma<PATH, 1, CBW, false, false, false, true, true>)
              : reinterpret_cast<const void*>(k_sweep_mfma<PATH, 1, CBW, false, false, false, true, false>);
}

static const void* batch_kernel(int path, int cbw, bool mh)
{
    if (path == kPathI8) return cbw == 2 ? batch_kernel<kPathI8, 2>(mh) : batch_kernel<kPathI8, 4>(mh);
    return cbw == 2 ? batch_kernel<kPathBf16, 2>(mh) : batch_kernel<kPathBf16, 4>(mh);
}

hipError_t prepare_sweep_batch(int path, int cbw, int mh, size_t lds)
{
    return hipFuncSetAttribute(batch_kernel(path, cbw, mh != 0), hipFuncAttributeMaxDynamicSharedMemorySize,
                               static_cast<int>(lds));
}

// Items of one bucket: same path, column-block width and accept/reject mode;
// table entries describe one 16-replica block each.
hipError_t launch_sweep_batch(int path, int cbw, int mh, const SweepArgs* dtable, int nitems, size_t lds,
                              hipStream_t st)
{
    SweepArgs a{};
    a.table = dtable;
    void* args[] = {&a};
    return hipLaunchKernel(batch_kernel(path, cbw, mh != 0), dim3(static_cast<unsigned>(nitems)), dim3(kThreads),
                           args, lds, st);
}

template <int PATH, int MT, int CBW>
static const void* group_table_kernel(bool mh)
{
    if constexpr (MT == 1 && CBW == 2)
        if (mh) return reinterpret_cast<const void*>(k_sweep_mfma<PATH, MT, CBW, true, false, false, true, true>);
    return mh ? nullptr : reinterpret_cast<const void*>(k_sweep_mfma<PATH, MT, CBW, true, false, false, true>);
}

// Accept/reject runs: MT = 1, CBW = 2 only (null otherwise).
static const void* group_table_kernel(int path, int mt, int cbw, bool mh)
{
    if (path == kPathI8) {
        if (mt == 1) return cbw == 1 ? group_table_kernel<kPathI8, 1, 1>(mh) : group_table_kernel<kPathI8, 1, 2>(mh);
        return cbw == 1 ? group_table_kernel<kPathI8, 2, 1>(mh) : group_table_kernel<kPathI8, 2, 2>(mh);
    }
    if (mt == 1) return cbw == 1 ? group_table_kernel<kPathBf16, 1, 1>(mh) : group_table_kernel<kPathBf16, 1, 2>(mh);
    return cbw == 1 ? group_table_kernel<kPathBf16, 2, 1>(mh) : group_table_kernel<kPathBf16, 2, 2>(mh);
}

hipError_t launch_sweep_group_table(int path, int mt, int cbw, int mh, const SweepArgs* dtable, int nwg, size_t lds,
                                    hipStream_t st)
{
    if (mt < 1 || mt > 2 || cbw < 1 || cbw > 2 || nwg < 1) return hipErrorInvalidValue;
    const void* kern = group_table_kernel(path, mt, cbw, mh != 0);
    if (!kern) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    SweepArgs a{};
    a.table = dtable;
    void* args[] = {&a};
    e = hipLaunchCooperativeKernel(kern, dim3(static_cast<unsigned>(nwg)), dim3(kThreads), args,
                                   static_cast<unsigned>(lds), st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

int max_coresident_group_table(int path, int mt, int cbw, int mh, size_t lds)
{
    int dev = 0, cus = 0, per = 0;
    if (mt < 1 || mt > 2 || cbw < 1 || cbw > 2) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const void* f = group_table_kernel(path, mt, cbw, mh != 0);
    if (!f) return 0;
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, kThreads, lds) != hipSuccess) return 0;
    return per * cus;
}

size_t sweep_mfma_lds_bytes(int path, int mt, const SweepArgs& a)
{
    const int cbs_max = (a.ncb + a.G - 1) / a.G;
    return lds_plan(path, mt, a.Np, cbs_max, a.j_lds, a.mh, a.inc).total;
}

template <int PATH, int MT, int CBW, bool GROUP, bool JLDS, bool TRACE, bool MH, bool INC = false>
static hipError_t launch_mfma_t(const SweepArgs& a, size_t lds, hipStream_t st)
{
    const unsigned grid = static_cast<unsigned>(GROUP ? a.ngroups * a.G : a.nblocks);
    auto kern = k_sweep_mfma<PATH, MT, CBW, GROUP, JLDS, TRACE, false, MH, INC>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
    if (GROUP) {
        SweepArgs copy = a;
        void* args[] = {&copy};
        e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(grid), dim3(kThreads), args,
                                       static_cast<unsigned>(lds), st);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), lds, st, a);
    }
    return hipGetLastError();
}

template <int PATH, int MT, int CBW, bool GROUP, bool JLDS, bool TRACE>
static hipError_t launch_mfma_m(const SweepArgs& a, size_t lds, hipStream_t st)
{
    // accept/reject variants exist for MT = 1, CBW = 2 only
    if constexpr (MT == 1 && CBW == 2) {
        if constexpr (GROUP && !JLDS)
            if (a.mh && a.inc) return launch_mfma_t<PATH, MT, CBW, GROUP, JLDS, TRACE, true, true>(a, lds, st);
        if (a.mh && !a.inc) return launch_mfma_t<PATH, MT, CBW, GROUP, JLDS, TRACE, true>(a, lds, st);
    }
    if (a.mh) return hipErrorInvalidValue;
    // flip-incremental variants: one row tile, column split, J streamed
    if constexpr (MT == 1 && GROUP && !JLDS)
        if (a.inc) return launch_mfma_t<PATH, MT, CBW, GROUP, JLDS, TRACE, false, true>(a, lds, st);
    if (a.inc) return hipErrorInvalidValue;
    return launch_mfma_t<PATH, MT, CBW, GROUP, JLDS, TRACE, false>(a, lds, st);
}

template <int PATH, int MT, int CBW, bool GROUP, bool JLDS>
static hipError_t launch_mfma_tr(const SweepArgs& a, size_t lds, hipStream_t st)
{
    return a.etrace ? launch_mfma_m<PATH, MT, CBW, GROUP, JLDS, true>(a, lds, st)
                    : launch_mfma_m<PATH, MT, CBW, GROUP, JLDS, false>(a, lds, st);
}

template <int PATH, int MT, int CBW, bool GROUP>
static hipError_t launch_mfma_j(const SweepArgs& a, size_t lds, hipStream_t st)
{
    return a.j_lds ? launch_mfma_tr<PATH, MT, CBW, GROUP, true>(a, lds, st)
                   : launch_mfma_tr<PATH, MT, CBW, GROUP, false>(a, lds, st);
}

template <int PATH, int MT, int CBW>
static hipError_t launch_mfma_g(const SweepArgs& a, size_t lds, hipStream_t st)
{
    return a.G > 1 ? launch_mfma_j<PATH, MT, CBW, true>(a, lds, st) : launch_mfma_j<PATH, MT, CBW, false>(a, lds, st);
}

template <int PATH>
static hipError_t launch_mfma_p(int mt, int cbw, const SweepArgs& a, size_t lds, hipStream_t st)
{
    if (mt == 1 && cbw == 1) return launch_mfma_g<PATH, 1, 1>(a, lds, st);
    if (mt == 1 && cbw == 2) return launch_mfma_g<PATH, 1, 2>(a, lds, st);
    if (mt == 2 && cbw == 1) return launch_mfma_g<PATH, 2, 1>(a, lds, st);
    if (mt == 2 && cbw == 2) return launch_mfma_g<PATH, 2, 2>(a, lds, st);
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_mfma(int path, int mt, int cbw, const SweepArgs& a, size_t lds, hipStream_t st)
{
    if (path == kPathI8) return launch_mfma_p<kPathI8>(mt, cbw, a, lds, st);
    if (path == kPathBf16) return launch_mfma_p<kPathBf16>(mt, cbw, a, lds, st);
    return hipErrorInvalidValue;
}

template <int PATH, int MT, int CBW, bool MH>
static const void* group_kernel(int jlds, int trace)
{
    if (jlds)
        return trace ? reinterpret_cast<const void*>(k_sweep_mfma<PATH, MT, CBW, true, true, true, false, MH>)
                     : reinterpret_cast<const void*>(k_sweep_mfma<PATH, MT, CBW, true, true, false, false, MH>);
    return trace ? reinterpret_cast<const void*>(k_sweep_mfma<PATH, MT, CBW, true, false, true, false, MH>)
                 : reinterpret_cast<const void*>(k_sweep_mfma<PATH, MT, CBW, true, false, false, false, MH>);
}

template <int PATH, int CBW, bool MH = false>
static const void* group_kernel_inc(int trace)
{
    return trace ? reinterpret_cast<const void*>(k_sweep_mfma<PATH, 1, CBW, true, false, true, false, MH, true>)
                 : reinterpret_cast<const void*>(k_sweep_mfma<PATH, 1, CBW, true, false, false, false, MH, true>);
}

template <int PATH>
static const void* group_kernel_p(int mt, int cbw, int jlds, int trace, int mh, int inc)
{
    if (inc) {
        if (mt != 1 || jlds) return nullptr;
        if (mh) return cbw == 2 ? group_kernel_inc<PATH, 2, true>(trace) : nullptr;
        return cbw == 1 ? group_kernel_inc<PATH, 1>(trace) : group_kernel_inc<PATH, 2>(trace);
    }
    if (mh) return (mt == 1 && cbw == 2) ? group_kernel<PATH, 1, 2, true>(jlds, trace) : nullptr;
    return mt == 1 ? (cbw == 1 ? group_kernel<PATH, 1, 1, false>(jlds, trace)
                               : group_kernel<PATH, 1, 2, false>(jlds, trace))
                   : (cbw == 1 ? group_kernel<PATH, 2, 1, false>(jlds, trace)
                               : group_kernel<PATH, 2, 2, false>(jlds, trace));
}

// Workgroups of the group sweep variant (mt, cbw, jlds, trace, mh, inc) that
// can be resident on the device at once (0 if the variant does not exist).
int max_coresident_mfma(int path, int mt, int cbw, int jlds, int trace, int mh, int inc, size_t lds)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const void* f = path == kPathI8 ? group_kernel_p<kPathI8>(mt, cbw, jlds, trace, mh, inc)
                                    : group_kernel_p<kPathBf16>(mt, cbw, jlds, trace, mh, inc);
    if (!f) return 0;
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, kThreads, lds) != hipSuccess) return 0;
    return per * cus;
}

// ---------------------------------------------------------------- argmin --
__global__ void __launch_bounds__(256) k_argmin(const int64_t* bestE, int32_t R, int64_t* out)
{
    __shared__ int64_t sE[256];
    __shared__ int64_t sR[256];
    int64_t e = INT64_MAX, r = -1;
    for (int i = threadIdx.x; i < R; i += 256) {
        const int64_t v = bestE[i];
        if (r < 0 || v < e) {
            e = v;
            r = i;
        }
    }
    sE[threadIdx.x] = e;
    sR[threadIdx.x] = r;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const int64_t e2 = sE[threadIdx.x + w], r2 = sR[threadIdx.x + w];
            const int64_t e1 = sE[threadIdx.x], r1 = sR[threadIdx.x];
            const bool take = r2 >= 0 && (r1 < 0 || e2 < e1 || (e2 == e1 && r2 < r1));
            if (take) {
                sE[threadIdx.x] = e2;
                sR[threadIdx.x] = r2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sE[0];
        out[1] = sR[0];
    }
}

hipError_t launch_argmin(const int64_t* bestE, int32_t R, int64_t* out2, hipStream_t st)
{
    hipLaunchKernelGGL(k_argmin, dim3(1), dim3(256), 0, st, bestE, R, out2);
    return hipGetLastError();
}

// ------------------------------------------------------------ FP64 energy --
__global__ void __launch_bounds__(256) k_energy_f64(const double* J, const double* h, int32_t N, const int8_t* s,
                                                    double* out)
{
    __shared__ double sred[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < N; i += 256) {
        const double si = s[i];
        double row = 0.0;
        for (int j = i + 1; j < N; ++j) row += J[static_cast<int64_t>(i) * N + j] * s[j];
        acc += si * row + (h ? h[i] * si : 0.0);
    }
    sred[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sred[threadIdx.x] += sred[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = -sred[0];
}

hipError_t launch_energy_f64(const double* J, const double* h, int32_t N, const int8_t* s, double* out,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_energy_f64, dim3(1), dim3(256), 0, st, J, h, N, s, out);
    return hipGetLastError();
}

// ----------------------------------------------------- fmath self-check --
__global__ void __launch_bounds__(256) k_fmath_eval(int kind, const float* in, const uint64_t* in64, float* out,
                                                    int64_t n)
{
    for (int64_t q = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; q < n;
         q += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        if (kind == 0) {
            out[q] = dev_exp_nonpos(in[q]);
        } else if (kind == 1) {
            out[q] = dev_ln_unit(in[q]);
        } else if (kind == 2) {
            float c, s;
            dev_sincos_2pi(in[q], c, s);
            out[2 * q] = c;
            out[2 * q + 1] = s;
        } else if (kind == 3) {
            out[q] = dev_sech2(in[q]);
        } else if (kind == 5) {
            out[q] = dev_poly2(in[q]);
        } else {
            out[q] = dev_gauss(in64[0], static_cast<uint32_t>(in64[1 + 4 * q]), in64[2 + 4 * q], in64[3 + 4 * q],
                               in64[4 + 4 * q]);
        }
    }
}

hipError_t launch_fmath_eval(int kind, const float* in, const uint64_t* in64, float* out, int64_t n, hipStream_t st)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fmath_eval, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, kind, in, in64, out, n);
    return hipGetLastError();
}

}  // namespace phia
