// Persistent batched sweep of the PHIA library for gfx950 (k_batch_fp4).
//
// Many instances of uneven size (N <= 512) whose integer couplings are all
// FP4 (E2M1) values run in one launch: every workgroup takes work items --
// one instance's block of 32 replicas -- from a global queue ordered largest
// first, until the queue is empty, and runs each item's steps with all of
// its columns.  One step is the sweep of Sec. 2.1 / App. A A7 for every
// element at once (momentum refresh, drift, readout, J.s + h on matrix
// cores, exact energy, records, kick), exactly as the other sweep kernels
// compute it.
//
// Layout.  Eight waves; wave w owns column blocks c = w + 8 cw (16 columns
// each) of both 16-replica row tiles, with x, v and the MFMA accumulators of
// its elements in VGPRs in the 16x16 MFMA output layout (lane l: column l %
// 16, rows 4 (l / 16) + j).  The coupling slice of the instance sits in LDS
// as FP4 fragments for the whole item; the spins go to LDS as FP8 bytes
// (+1 = 0x38, -1 = 0xB8) in the k order of the FP4 fragments, and J.s runs
// on v_mfma_scale_f32_16x16x128_f8f6f4 (FP8 spins x FP4 couplings, FP32
// accumulation, scales 1): every product and partial sum is an integer
// below 2^24, so the field is exact, and it stays in FP32 for the kick and
// the energy terms (their sums are integers below 2^24 too: host-checked).
// Row energies are summed by DPP within a wave and by LDS atomics over the
// waves; the records of step k are taken
// in step k + 1 after the step's only barrier.  x is drawn here when an item
// starts a fresh anneal (no separate init kernel).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "phia_devmath.h"
#include "phia_devsweep.h"
#include "phia_internal.h"

namespace phia {

namespace {

constexpr int kBW = 8;                 // waves per workgroup
constexpr int kBT = 64 * kBW;          // threads per workgroup
constexpr uint32_t kFixedLds = 512;    // energy sums [3][32] int32, the item slot
constexpr uint32_t kSpinPlus = 0x38u;  // FP8 E4M3 +1.0
constexpr uint32_t kSpinMinus = 0xB8u; // FP8 E4M3 -1.0

__host__ __device__ inline int nkb4_of(int Np) { return (Np + 127) / 128; }
__host__ __device__ inline uint32_t srow_of(int Np) { return static_cast<uint32_t>(nkb4_of(Np)) * 128u + 16u; }
__host__ __device__ inline uint32_t jbytes_of(int Np)
{
    return static_cast<uint32_t>(Np / 16) * static_cast<uint32_t>(nkb4_of(Np)) * 1024u;
}
__host__ __device__ inline uint32_t sbytes_of(int Np) { return static_cast<uint32_t>(kBatchRows) * srow_of(Np); }

// Initial position draw (a call, so that the element loops do not hold many
// generator states at once).
__device__ __attribute__((noinline)) float gauss_x(uint64_t seed, uint64_t replica, int i)
{
    return dev_gauss(seed, kTagX, replica, 0, static_cast<uint64_t>(i));
}

// All 8 draws of one momentum block (a call for the same reason).
struct Draws8 {
    float g[8];
};
__device__ __attribute__((noinline)) Draws8 gauss_block8(uint64_t seed, uint64_t replica, uint64_t round, uint64_t c8)
{
    Draws8 d;
    gauss_block(seed, replica, round, c8, d.g);
    return d;
}

// The steps of one work item for a wave that owns NCW column blocks of an
// instance with NKB k blocks of 128 (NCW = 0: a wave without columns, which
// only keeps the workgroup's barriers).
template <int NKB, int NCW>
__device__ __attribute__((noinline)) void batch_item(const BatchInst& a, int blk, unsigned char* lds, bool dbuf, int wave,
                                           int lane)
{
    constexpr int MT = 2;
    constexpr uint32_t srow = NKB * 128u + 16u;
    constexpr uint32_t sb = kBatchRows * srow;
    const uint32_t jb = static_cast<uint32_t>(a.Np / 16) * NKB * 1024u;
    float* sE = reinterpret_cast<float*>(lds);  // [3][32] row energy sums of steps k mod 3 (exact integers)
    unsigned char* sJ = lds + kFixedLds;
    unsigned char* sS = lds + kFixedLds + jb;       // [dbuf ? 2 : 1][32][srow] FP8 spins
    const int nsteps = static_cast<int>(a.k1 - a.k0);

    if constexpr (NCW == 0) {
        for (int s = 0; s <= nsteps; ++s) {
            if (!dbuf && s > 0) __syncthreads();
            __syncthreads();
        }
        return;
    } else {
        const int lr = lane & 15, lg = lane >> 4;
        const int Np = a.Np, N = a.N;
        const int64_t rb0 = static_cast<int64_t>(blk) * kBatchRows;
        const uint64_t seed = *a.seed;
        int col[NCW];
        float hf[NCW], h2f[NCW];
        bool creal[NCW];
#pragma unroll
        for (int cw = 0; cw < NCW; ++cw) {
            col[cw] = (wave + kBW * cw) * 16 + lr;
            creal[cw] = col[cw] < N;
            const int hv = a.h[col[cw]];
            hf[cw] = static_cast<float>(hv);
            h2f[cw] = static_cast<float>(2 * hv);
        }
        // rows of this lane: rb0 + mt 16 + 4 lg + j; bit mt 4 + j set when < R
        uint32_t rmask = 0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                rmask |= (rb0 + mt * 16 + 4 * lg + j < a.R ? 1u : 0u) << (mt * 4 + j);
        float x[MT][NCW][4], v[MT][NCW][4];
        float bE[MT][4];    // record energy (+inf: none yet)
        int32_t bK[MT][4];
        uint32_t bestbits = 0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool ok = (rmask >> (mt * 4 + j)) & 1u;
                const int64_t gr = rb0 + mt * 16 + 4 * lg + j;
                if (a.init) {
                    bE[mt][j] = __builtin_inff();
                    bK[mt][j] = -1;
                } else {
                    const int64_t b = ok ? a.bestE[gr] : INT64_MAX;
                    bE[mt][j] = b == INT64_MAX ? __builtin_inff() : static_cast<float>(b);
                    bK[mt][j] = ok ? static_cast<int32_t>(a.bestStep[gr]) : -1;
                }
#pragma unroll
                for (int cw = 0; cw < NCW; ++cw) {
                    const int64_t idx = gr * Np + col[cw];
                    if (a.init) {
                        x[mt][cw][j] = (ok && creal[cw]) ? gauss_x(seed, static_cast<uint64_t>(gr), col[cw]) : 0.0f;
                        v[mt][cw][j] = 0.0f;
                    } else {
                        x[mt][cw][j] = ok ? a.x[idx] : 0.0f;
                        v[mt][cw][j] = ok ? a.v[idx] : 0.0f;
                        if (ok && creal[cw] && a.bestS[idx] > 0) bestbits |= 1u << ((mt * NCW + cw) * 4 + j);
                    }
                }
            }
        const float eps = a.eps, gamma = a.gamma;
        const int64_t ref0 = a.k0 + (a.L - a.k0 % a.L) % a.L;
        int64_t next_ref = ref0;
        uint64_t round = static_cast<uint64_t>(ref0 / a.L);
        // byte offset of this lane's spin of row 4 lg, column block 0, in the
        // FP4 k order (columns 0 4 1 5 2 6 3 7 in each group of 8)
        const int q7 = lr & 7;
        const uint32_t sbase = 4u * lg * srow + 8u * (lr >> 3) + static_cast<uint32_t>(q7 < 4 ? 2 * q7 : 2 * q7 - 7) +
                               16u * wave;
        // signs of the step before the current one, bit (mt NCW + cw) 4 + j
        uint32_t pm = 0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int cw = 0; cw < NCW; ++cw)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (x[mt][cw][j] >= 0.0f) pm |= 1u << ((mt * NCW + cw) * 4 + j);

        int r3 = static_cast<int>(a.k0 % 3);
        for (int s = 0; s <= nsteps; ++s) {
            const int64_t k = a.k0 + s;
            const bool last = (s == nsteps);
            const int r3p = (r3 == 0) ? 2 : r3 - 1, r3n = (r3 == 2) ? 0 : r3 + 1;
            unsigned char* S = sS + (dbuf ? static_cast<uint32_t>(k & 1) * sb : 0u);
            const uint32_t pprev = pm;  // signs of step k - 1
            if (!dbuf && s > 0) __syncthreads();  // every wave has read the spins of step k - 1
            if (!last) {
                if (k == next_ref) {
                    // Momentum refresh (the draws of `round`): the wave's 2 NCW
                    // tiles fill 32 Philox blocks each; pass hp covers tiles
                    // 2 hp and 2 hp + 1, lane L generating the block of replica
                    // row (L >> 1) & 15, 8-column half L & 1 of tile
                    // 2 hp + (L >> 5), and every element reads its draw from
                    // that lane.
#pragma unroll
                    for (int hp = 0; hp < NCW; ++hp) {
                        const int u = 2 * hp + (lane >> 5), mtl = u / NCW, cwl = u % NCW;
                        const Draws8 d = gauss_block8(seed, static_cast<uint64_t>(rb0 + mtl * 16 + ((lane >> 1) & 15)),
                                                      round, static_cast<uint64_t>(wave + kBW * cwl) * 2 + (lane & 1));
                        const float* g = d.g;
#pragma unroll
                        for (int e = 8 * hp; e < 8 * hp + 8; ++e) {
                            const int mt = e / (NCW * 4), cw = (e >> 2) % NCW, j = e & 3;
                            const int src = ((mt * NCW + cw) & 1) * 32 + 2 * (4 * lg + j) + (lr >> 3);
                            float t = 0.0f;
#pragma unroll
                            for (int r = 0; r < 8; ++r) {
                                const float tr = lane_read(src, g[r]);
                                t = q7 == r ? tr : t;
                            }
                            v[mt][cw][j] = (creal[cw] && ((rmask >> (mt * 4 + j)) & 1u)) ? t : 0.0f;
                        }
                    }
                    next_ref += a.L;
                    ++round;
                }
                // Drift and readout; the spins go to LDS for the product.
                pm = 0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int cw = 0; cw < NCW; ++cw)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            x[mt][cw][j] = __builtin_fmaf(eps, v[mt][cw][j], x[mt][cw][j]);
                            const bool pos = x[mt][cw][j] >= 0.0f;
                            pm |= (pos ? 1u : 0u) << ((mt * NCW + cw) * 4 + j);
                            S[sbase + (mt * 16 + j) * srow + 128u * cw] =
                                static_cast<unsigned char>(pos ? kSpinPlus : kSpinMinus);
                        }
            }
            __syncthreads();  // spins of step k and energy sums of step k - 1 complete

            // Records of step k - 1 (App. B, Table 3, state 5): every lane that
            // holds a row takes the same decision.
            if (s > 0) {
                float E[MT][4];
                uint32_t impm = 0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const float4 t4 = *reinterpret_cast<const float4*>(sE + r3p * 32 + mt * 16 + 4 * lg);
                    const float tot[4] = {t4.x, t4.y, t4.z, t4.w};
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        E[mt][j] = -0.5f * tot[j];  // the sum is even: exact
                        if (E[mt][j] < bE[mt][j]) impm |= 1u << (mt * 4 + j);
                    }
                }
                // Late in an anneal few steps improve a record: the updates
                // run only when some row of the wave improved (uniform branch).
                if (__any(impm != 0)) {
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const bool imp = (impm >> (mt * 4 + j)) & 1u;
                            bE[mt][j] = imp ? E[mt][j] : bE[mt][j];
                            bK[mt][j] = imp ? static_cast<int32_t>(k - 1) : bK[mt][j];
                            uint32_t rowmask = 0;
#pragma unroll
                            for (int cw = 0; cw < NCW; ++cw) rowmask |= 1u << ((mt * NCW + cw) * 4 + j);
                            bestbits = imp ? ((bestbits & ~rowmask) | (pprev & rowmask)) : bestbits;
                        }
                }
            }
            if (last) break;
            if (wave == 0 && lane < 32) sE[r3n * 32 + lane] = 0.0f;  // read two steps ago
            const float ck = a.ctab[k];

            // J.s on matrix cores: FP8 spins x FP4 couplings over the k blocks.
            v4f acc[MT][NCW];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int cw = 0; cw < NCW; ++cw) acc[mt][cw] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
            {
                // Operand k order of v_mfma_scale_f32_16x16x128_f8f6f4: FP4 nibble
                // t of lane group g (the couplings) is k = 32 g + t; FP8 byte t
                // (the spins) is k = 16 g + t for t < 16 and 64 + 16 g + t - 16
                // above.  So a lane's spin operand is the 16 bytes at 16 g and
                // the 16 bytes at 64 + 16 g of the row's 128-wide k block.
                const unsigned char* arow = S + lr * srow + 16 * lg;
                const unsigned char* jl = sJ + lane * 16 + static_cast<uint32_t>(wave * NKB) * 1024u;
#pragma unroll
                for (int kb = 0; kb < NKB; ++kb) {
                    v8i A[MT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const v4i lo = *reinterpret_cast<const v4i*>(arow + mt * 16 * srow + kb * 128);
                        const v4i hi = *reinterpret_cast<const v4i*>(arow + mt * 16 * srow + kb * 128 + 64);
                        A[mt] = v8i{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                    }
#pragma unroll
                    for (int cw = 0; cw < NCW; ++cw) {
                        const v4i b = *reinterpret_cast<const v4i*>(jl + (kBW * cw * NKB + kb) * 1024u);
                        const v8i b8 = v8i{b[0], b[1], b[2], b[3], 0, 0, 0, 0};
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt)
                            acc[mt][cw] =
                                __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(A[mt], b8, acc[mt][cw], 0, 4, 0, 127,
                                                                                 0, 127);
                    }
                    // keep the operand loads of later k blocks from piling up in registers
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            float I[MT][NCW][4];  // field J s + h, an exact integer in FP32
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int cw = 0; cw < NCW; ++cw)
#pragma unroll
                    for (int j = 0; j < 4; ++j) I[mt][cw][j] = acc[mt][cw][j] + hf[cw];

            // Kick (mode branch outside the element loops).
            auto kick_all = [&](auto mode) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int cw = 0; cw < NCW; ++cw)
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            v[mt][cw][j] = kick_tf<decltype(mode)::value>(x[mt][cw][j], v[mt][cw][j], I[mt][cw][j],
                                                                         ck, eps, gamma);
            };
            if (a.deriv)
                kick_all(std::integral_constant<int, 1>{});
            else
                kick_all(std::integral_constant<int, 0>{});

            // Row energy partials s (I + h) of step k (padded columns have
            // zero couplings and field, so I + h = 0 there).
            float psum[MT][4];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    float part = 0.0f;
#pragma unroll
                    for (int cw = 0; cw < NCW; ++cw) {
                        const float ih = acc[mt][cw][j] + h2f[cw];
                        part += (x[mt][cw][j] >= 0.0f) ? ih : -ih;
                    }
                    psum[mt][j] = row_sum16_dpp_f(part);
                }
            // lane lr < 8 of each row group adds row (lr >> 2) 16 + 4 lg + (lr & 3)
            if (lr < 4 * MT) {
                float t = psum[0][0];
#pragma unroll
                for (int u = 1; u < 4 * MT; ++u) t = lr == u ? psum[u >> 2][u & 3] : t;
                atomicAdd(sE + r3 * 32 + (lr >> 2) * 16 + 4 * lg + (lr & 3), t);
            }
            r3 = r3n;
        }

        // Final state and records of the item.
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                if (!((rmask >> (mt * 4 + j)) & 1u)) continue;
                const int64_t gr = rb0 + mt * 16 + 4 * lg + j;
#pragma unroll
                for (int cw = 0; cw < NCW; ++cw) {
                    const int64_t idx = gr * Np + col[cw];
                    a.x[idx] = x[mt][cw][j];
                    a.v[idx] = v[mt][cw][j];
                    if (creal[cw]) a.bestS[idx] = ((bestbits >> ((mt * NCW + cw) * 4 + j)) & 1u) ? 1 : -1;
                }
                if (wave == 0 && lr == 0) {
                    a.bestE[gr] = bE[mt][j] == __builtin_inff() ? INT64_MAX : static_cast<int64_t>(bE[mt][j]);
                    a.bestStep[gr] = bK[mt][j];
                }
            }
    }
}

__global__ void __launch_bounds__(kBT) __attribute__((amdgpu_waves_per_eu(2)))
k_batch_fp4(const BatchInst* __restrict__ insts, const BatchItem* __restrict__ items, int nitems, int* queue,
            uint32_t lds_bytes)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    int* sItem = reinterpret_cast<int*>(lds + 3 * 32 * 4);
    for (;;) {
        if (tid == 0) *sItem = atomicAdd(queue, 1);
        __syncthreads();
        const int q = __builtin_amdgcn_readfirstlane(*sItem);
        if (q >= nitems) break;
        const BatchItem it = items[q];
        const BatchInst a = insts[it.inst];
        const int Np = a.Np, ncb = Np / 16, nkb = nkb4_of(Np);
        const uint32_t jb = jbytes_of(Np), sb = sbytes_of(Np);
        // spins double-buffered when both buffers fit the launch's LDS (else
        // one buffer and a second barrier per step)
        const bool dbuf = kFixedLds + jb + 2 * sb <= lds_bytes;
        // coupling slice into LDS, spins and energy sums cleared (k positions
        // past Np meet zero couplings but must hold a finite value)
        {
            const uint4* src = reinterpret_cast<const uint4*>(a.J4);
            uint4* dst = reinterpret_cast<uint4*>(lds + kFixedLds);
            for (uint32_t u = tid; u < jb / 16u; u += kBT) dst[u] = src[u];
            uint32_t* sz = reinterpret_cast<uint32_t*>(lds + kFixedLds + jb);
            const uint32_t nsw = (dbuf ? 2u : 1u) * sb / 4u;
            for (uint32_t u = tid; u < nsw; u += kBT) sz[u] = 0u;
            if (tid < 96) reinterpret_cast<int32_t*>(lds)[tid] = 0;
        }
        __syncthreads();
        const int ncw = wave < ncb ? (ncb - wave + kBW - 1) / kBW : 0;
        const int blk = it.block;
        // nkb = ceil(ncb / 8); a wave owns nkb or nkb - 1 column blocks
        if (nkb == 1) {
            if (ncw == 1) batch_item<1, 1>(a, blk, lds, dbuf, wave, lane);
            else batch_item<1, 0>(a, blk, lds, dbuf, wave, lane);
        } else if (nkb == 2) {
            if (ncw == 2) batch_item<2, 2>(a, blk, lds, dbuf, wave, lane);
            else batch_item<2, 1>(a, blk, lds, dbuf, wave, lane);
        } else if (nkb == 3) {
            if (ncw == 3) batch_item<3, 3>(a, blk, lds, dbuf, wave, lane);
            else batch_item<3, 2>(a, blk, lds, dbuf, wave, lane);
        } else {
            if (ncw == 4) batch_item<4, 4>(a, blk, lds, dbuf, wave, lane);
            else batch_item<4, 3>(a, blk, lds, dbuf, wave, lane);
        }
        __syncthreads();
    }
}

__global__ void k_batch_queue_reset(int* queue)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0;
}

}  // namespace

size_t batch_fp4_lds_bytes(int Np, bool double_buffered)
{
    return kFixedLds + jbytes_of(Np) + (double_buffered ? 2u : 1u) * sbytes_of(Np);
}

hipError_t launch_batch_queue_reset(int* queue, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_queue_reset, dim3(1), dim3(64), 0, st, queue);
    return hipGetLastError();
}

int batch_fp4_grid(size_t lds)
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    const void* f = reinterpret_cast<const void*>(k_batch_fp4);
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, kBT, lds) != hipSuccess) return 0;
    return per * cus;
}

hipError_t launch_batch_fp4(const BatchInst* insts, const BatchItem* items, int nitems, int* queue, size_t lds,
                            hipStream_t st)
{
    const int grid = batch_fp4_grid(lds);
    if (grid < 1) return hipErrorInvalidConfiguration;
    const int nwg = grid < nitems ? grid : (nitems > 0 ? nitems : 1);
    hipLaunchKernelGGL(k_batch_fp4, dim3(static_cast<unsigned>(nwg)), dim3(kBT), lds, st, insts, items, nitems, queue,
                       static_cast<uint32_t>(lds));
    return hipGetLastError();
}

}  // namespace phia
