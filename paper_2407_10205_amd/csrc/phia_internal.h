// Internal interface between the host runtime and the HIP kernels of the PHIA
// sweep.  Not part of the public ABI (include/phia.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace phia {

constexpr int kWaves = 8;            // waves per workgroup in the MFMA sweep
constexpr int kThreads = 64 * kWaves;
constexpr int kCbwMax = 2;           // max 16-column blocks per wave (MFMA sweep)
constexpr int kFp32Rows = 4;         // replicas per workgroup in the FP32 sweep
constexpr int kLdsMax = 160 * 1024;  // LDS bytes per workgroup on gfx950
constexpr uint32_t kSpinLimit = 1u << 21;  // bounded polls per exchange word
constexpr int kGatherWords = 8;      // exchange words in flight per thread

enum Path : int { kPathAuto = 0, kPathFp32 = 1, kPathI8 = 2, kPathBf16 = 3 };

// Arguments of one sweep launch.  Device pointers unless noted.
struct SweepArgs {
    int32_t N, Np;              // spins, padded spins (multiple of 64)
    const int32_t* h;           // [Np] fields in sigma units, zero padded
    const void* J;              // packed couplings, layout depends on the path
    const float* ctab;          // [T] c_k = (beta_k * gamma) * sigma
    float eps, gamma;
    int32_t deriv;              // 0: sech^2 (Eq. 8), 1: POLY2 quadratic
    int32_t ell_d;              // ELL slots per row (ELL path)
    int32_t ikick;              // 1: half a kick after every momentum draw (VALU sweep only)
    int64_t L;                  // momentum refresh period
    uint64_t seed;
    int64_t k0, k1;             // steps [k0, k1) of this launch
    int32_t R;                  // replicas of the problem
    int64_t r_base;             // stream replica index of replica 0
    float* x;                   // [R][Np]
    float* v;                   // [R][Np]
    int64_t* bestE;             // [R]
    int8_t* bestS;              // [R][Np]
    int64_t* bestStep;          // [R]
    int64_t* etrace;            // [R][T] energy of every step, or null
    int64_t T;                  // total steps (row length of etrace)
    // MFMA sweep geometry
    int32_t G;                  // workgroups per replica block (column split)
    int32_t ncb;                // Np / 16
    int32_t rows;               // replicas per block (16 * MT)
    int32_t nblocks;            // ceil(R / rows)
    int32_t ngroups;            // concurrently running groups
    int32_t xcd_map;            // 1: group members share blockIdx % 8
    int32_t j_lds;              // 1: J slice resident in LDS, 0: read from global
    int32_t inc;                // 1: flip-incremental field update (column split, J streamed)
    int64_t* incstat;           // [3] incremental steps, full-product steps, k blocks of the
                                //     incremental products (member 0 of every group), or null
    // group exchange (G > 1)
    uint64_t* xbits;            // [2][ngroups][rows][Np/16] tagged sign words
    uint64_t* pbuf;             // [2][ngroups][G][rows][2] (seq << 32) | 32-bit half of a partial energy
    uint32_t seq_base;          // sequence number before this launch (tags start at seq_base + 1)
    int32_t* err;               // device error word (1 = barrier timeout)
    // accept/reject at the end of every trajectory of L steps (mh != 0)
    int32_t mh;
    float mh_up, mh_down;       // beta multiplier factors after an acceptance / a rejection
    float sigma;                // 2^-f
    const float* btab;          // [T] beta_k
    float* x0;                  // [R][Np] x at the start of the current trajectory
    int64_t* mhE;               // [R][2] energy at the trajectory start (INT64_MIN: not known),
                                //        energy of the last step run
    int64_t* mhQ;               // [R][G] kinetic units of a member's columns at the trajectory start
    float* lam;                 // [R] beta multiplier
    int32_t* mhc;               // [R][2] accepted, decided trajectories
    uint64_t* mhbuf;            // [2][ngroups][G][rows][4] tagged 32-bit halves of (energy, kinetic) partials
    // batch mode: the launch argument points at one entry per workgroup
    const SweepArgs* table;     // work items (device), or null
    const uint64_t* seedp;      // batch mode: the item's seed in device memory (replaces seed), or null
    int32_t block;              // replica block (group) of this work item
    int32_t member;             // group member of this work item (table launches of the group sweep)
};

// Layout of packed couplings.
//  FP32: float [Np][Np] row-major.
//  ELL:  int32 [D][Np]: slot d of row i is (J_ij << 16) | j for the d-th
//        nonzero J_ij of row i (ascending j), zero for unused slots.
//  I8:   fragment-major int8: [Np/16 col blocks][Np/64 k blocks][64 lanes][16],
//        lane l holds J[cb*16 + l%16][kb*64 + 16*(l/16) + t], t < 16.
//  BF16: [Np/16][Np/32 k chunks][2 planes hi, lo][64 lanes][8 bf16],
//        lane l holds plane[cb*16 + l%16][kc*32 + 8*(l/16) + t], t < 8,
//        with J = 256 hi + lo, lo in [-128, 127].

hipError_t launch_init(const SweepArgs& a, hipStream_t st);
// VALU sweeps (k_sweep_valu): RB replicas and all columns per workgroup.
enum ValuForm : int { kValuFp32 = 0, kValuDot8 = 1, kValuEll = 2 };
constexpr int kValuMaxNp = 4096;  // 16 columns per thread at 256 threads, 4 at 1024
// LDS offset of the couplings of the int8 form when they reside in LDS.
__host__ __device__ inline size_t valu_jl_offset(int rb, int Np) { return (static_cast<size_t>(rb) * Np + 15) & ~size_t(15); }
size_t valu_lds_bytes(int form, int rb, int Np, bool jl);
bool valu_variant(int form, int rb, int mh, bool jl);  // a compiled (form, rows, accept/reject, J in LDS) combination
hipError_t launch_sweep_valu(int form, int rb, bool jl, const SweepArgs& a, hipStream_t st);
hipError_t launch_sweep_mfma(int path, int mt, int cbw, const SweepArgs& a, size_t lds_bytes, hipStream_t st);
size_t sweep_mfma_lds_bytes(int path, int mt, const SweepArgs& a);
hipError_t launch_argmin(const int64_t* bestE, int32_t R, int64_t* out2, hipStream_t st);
// n problems' argmins in one launch (phia_server_kernels.hip): pairs[2 j], pairs[2 j + 1] =
// (energy, replica) of problem j, errs[j] = *err[j] (0 for a null err[j]).
hipError_t launch_argmin_many(const int64_t* const* bestE, const int32_t* R, const int32_t* const* err, int n,
                              int64_t* pairs, int32_t* errs, hipStream_t st);
hipError_t launch_energy_f64(const double* J, const double* h, int32_t N, const int8_t* s,
                             double* out, hipStream_t st);
hipError_t launch_fmath_eval(int kind, const float* in, const uint64_t* in64, float* out, int64_t n,
                             hipStream_t st);
int max_coresident_mfma(int path, int mt, int cbw, int jlds, int trace, int mh, int inc, size_t lds_bytes);
// interleaved group sweep: int8 J, two 16-replica sub-blocks per workgroup
constexpr int kPpMaxNcb = 256;            // Np <= 4096
constexpr int64_t kPpMaxRowSum = 1 << 18;  // 32 * max_i(sum_j |J_ij| + |h_i|) < 2^23
size_t sweep_pp_lds_bytes(int Np, int G, int fp4, int jg);
hipError_t launch_sweep_pp(const SweepArgs& a, int fp4, int jg, size_t lds_bytes, hipStream_t st);
int max_coresident_pp(int ncb, int fp4, int jg, size_t lds_bytes);
// batch mode: 16-replica work items, one workgroup each, up to 512 columns
constexpr int kBatchMaxNp = kWaves * 4 * 16;
hipError_t launch_init_batch(const SweepArgs* dtable, int count, hipStream_t st);

// Persistent batched sweep (k_batch_fp4): every workgroup takes 32-replica
// work items from a queue until it is empty.  One entry per instance.
struct BatchInst {
    const unsigned char* J4;    // FP4 fragments [Np/16][ceil(Np/128)][64][16] (k order of the interleaved sweep)
    const int32_t* h;           // [Np] fields in sigma units, zero padded
    const float* ctab;          // [T] c_k
    const uint64_t* seed;       // the instance's seed (device)
    float* x;                   // [R][Np]
    float* v;                   // [R][Np]
    int64_t* bestE;             // [R]
    int8_t* bestS;              // [R][Np]
    int64_t* bestStep;          // [R]
    int64_t k0, k1;             // steps [k0, k1) of this launch
    int64_t L;                  // momentum refresh period
    float eps, gamma;
    int32_t N, Np, R;
    int32_t deriv;              // 0: sech^2, 1: POLY2
    int32_t init;               // 1: draw x ~ N(0, I), v = 0 and reset the records first (k0 = 0)
    int32_t pad_;
};
struct BatchItem {
    int32_t inst;               // index into the instance table
    int32_t block;              // 32-replica block of that instance
};
constexpr int kBatchRows = 32;           // replicas per work item
constexpr int kBatchFp4MaxNp = 512;      // columns of the persistent sweep (8 waves x 4 column blocks)
// LDS the persistent sweep needs for an instance of Np columns (J slice and
// spins double-buffered, or single-buffered when double does not fit).
size_t batch_fp4_lds_bytes(int Np, bool double_buffered);
hipError_t launch_batch_fp4(const BatchInst* insts, const BatchItem* items, int nitems, int* queue, size_t lds,
                            hipStream_t st);
hipError_t launch_batch_queue_reset(int* queue, hipStream_t st);
int batch_fp4_grid(size_t lds);
size_t sweep_batch_lds_bytes(int path, int Np, int j_lds, int mh);
hipError_t prepare_sweep_batch(int path, int cbw, int mh, size_t lds_bytes);
hipError_t launch_sweep_batch(int path, int cbw, int mh, const SweepArgs* dtable, int nitems, size_t lds_bytes,
                              hipStream_t st);
// column-split sweeps of several problems in one cooperative launch: one
// table entry per workgroup (problem, group, member); all of one problem's
// workgroups in the same launch
// (accept/reject runs: mt = 1, cbw = 2 only)
hipError_t launch_sweep_group_table(int path, int mt, int cbw, int mh, const SweepArgs* dtable, int nwg,
                                    size_t lds_bytes, hipStream_t st);
int max_coresident_group_table(int path, int mt, int cbw, int mh, size_t lds_bytes);

}  // namespace phia
