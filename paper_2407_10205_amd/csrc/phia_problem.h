// The opaque problem handle of include/phia.h (host-side bookkeeping).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "phia.h"
#include "phia_internal.h"

namespace phia {

// Launch geometry of the MFMA sweep (see k_sweep_mfma).
struct Geometry {
    bool ok = false;
    int kind = 0;      // 0: k_sweep_mfma; k_sweep_pp (interleaved sub-blocks) with 1: int8, 2: FP4 operands;
                       // 3: persistent batch sweep (k_batch_fp4); 4: VALU sweep (k_sweep_valu)
    int mt = 1;        // 16-replica row tiles per workgroup
    int cbw = 2;       // max 16-column blocks per wave
    int G = 1;         // workgroups splitting the columns of one replica block
    int j_lds = 1;     // J slice resident in LDS
    int rows = 16;     // replicas per block (kind 4: per workgroup)
    int nblocks = 0;   // replica blocks
    int ngroups = 0;   // groups running concurrently
    int xcd_map = 0;   // group members share blockIdx % 8 (one XCD)
    size_t lds = 0;    // dynamic LDS bytes per workgroup
    int mh = 0;        // LDS sized for the accept/reject step
    int inc = 0;       // flip-incremental field update
};

phia_status fail(phia_status st, const char* fmt, ...);
phia_status hip_fail(struct ::phia_problem* p, hipError_t e, const char* what);
void clear_error();

}  // namespace phia

#include <vector>

namespace phia {
phia_status check_usable(const ::phia_problem* p);
phia_status check_schedule(int32_t replicas, int64_t steps, const phia_schedule* s);
void kick_factors(const ::phia_problem* p, int64_t steps, const phia_schedule* s, std::vector<float>& ctab);
phia_status setup_state(::phia_problem* p, int32_t replicas, int64_t steps, const phia_schedule* s, uint64_t seed,
                        const std::vector<float>& ctab, bool& reuse, bool sync_first);
void free_state(::phia_problem* p);
hipError_t clear_exchange(::phia_problem* p);
phia_status make_resident(::phia_problem* p);
void release_resident(::phia_problem* p);
int valu_crossover(int Np);
phia_status setup_mh_geometry(::phia_problem* p);
SweepArgs sweep_args(const ::phia_problem* p);
Geometry plain_geometry(::phia_problem* p, int R, int ikick = 0);
phia_status launch_batch_chunk(::phia_problem* const* probs, int count, const int64_t* k_end, hipStream_t st,
                               SweepArgs*& dtab, size_t& cap);
phia_status launch_group_chunk(::phia_problem* const* probs, int count, const int64_t* k_end, hipStream_t st,
                               SweepArgs*& dtab, size_t& cap);
}  // namespace phia

struct phia_problem;
struct phia_batch;
namespace phia {
hipError_t batch_wait(::phia_batch* b);
void batch_forget(::phia_batch* b, ::phia_problem* p);
phia_status check_owned(const ::phia_problem* p);
}  // namespace phia
struct phia_problem {
    int dev = 0;
    hipStream_t st = nullptr;
    int N = 0, Np = 0, path = 0, f = 0;
    bool exact = true;
    int64_t maxabsJ = 0;
    int64_t maxrow = 0;  // max_i (sum_j |J_ij| + |h_i|) in units
    int ell_d = 0;       // ELL slots per row (ELL path)
    bool poisoned = false;
    // instance
    void* dJ = nullptr;
    void* dJ4 = nullptr;  // FP4 operand copy of J (interleaved sweep), or null
    int32_t* dh = nullptr;
    double* dJ64 = nullptr;
    double* dh64 = nullptr;
    int32_t* derr = nullptr;
    int64_t* dscratch = nullptr;
    size_t base_bytes = 0;
    // packed couplings and fields on the host (dropped once resident unless
    // the upload is deferred), FP64 copies only for rounded input
    std::vector<unsigned char> hJ, hJ4;
    std::vector<int32_t> hh;
    std::vector<double> hJ64, hh64;
    bool has_j4 = false;    // the couplings have an FP4 operand copy
    bool defer = false;     // uploaded at first use, released when a served request ends
    size_t jres_bytes = 0;  // device bytes of those copies when resident
    // anneal
    bool started = false, has_run = false, trace = false;
    bool one_block_kernel = false;  // restrict geometries to k_sweep_mfma (server table launches)
    int inc_mode = -1;              // flip-incremental update: -1 default, 0 off, 1 on where a variant exists
    int inc_mode_geo = -1;          // inc_mode when the current state and geometry were set up
    int64_t* dincstat = nullptr;    // [4] flip-incremental step counters of the current anneal
    int32_t R = 0;
    int64_t T = 0, k = 0, L = 1;
    float eps = 0.f, gamma = 0.f;
    int deriv = 0;  // phia_deriv of the current anneal
    int ikick = 0;  // initial-kick variant of the current anneal
    // accept/reject step of the current anneal
    int mh = 0;
    float mh_up = 1.f, mh_down = 1.f;
    float* dbtab = nullptr;     // [T] beta_k
    float* dx0 = nullptr;       // [R][Np] x at the trajectory start
    int64_t* dmhE = nullptr;    // [R][2]
    int64_t* dmhQ = nullptr;    // [R][max(1, G)]
    size_t mhQ_cap = 0;         // entries of dmhQ
    float* dlam = nullptr;      // [R]
    int32_t* dmhc = nullptr;    // [R][2]
    uint64_t* dmhbuf = nullptr; // group exchange of the decision's partial sums
    uint64_t seed = 0;
    float* dctab = nullptr;
    float* dx = nullptr;
    float* dv = nullptr;
    int64_t* dbestE = nullptr;
    int8_t* dbestS = nullptr;
    int64_t* dbestStep = nullptr;
    int64_t* detrace = nullptr;
    uint64_t* dxbits = nullptr;
    uint64_t* dpbuf = nullptr;
    uint32_t seq = 0;
    bool give_up = false;  // test hook: the device error word is raised before every sweep launch
    int32_t best_r = -1;
    size_t state_bytes = 0;
    phia::Geometry geo;
    phia::Geometry tuned;  // autotuned geometry for tuned_R replicas
    int32_t tuned_R = 0;
    struct phia_batch* batch = nullptr;  // batch plan that holds the replica state, or null
};
