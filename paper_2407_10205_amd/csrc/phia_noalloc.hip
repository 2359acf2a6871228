// Allocation-free form of phia_anneal (include/phia.h, phia_anneal_noalloc).
//
// The caller passes the device buffers of the replica state and records; the
// kernels' scratch (kick factors, the error word, the column-split exchange
// words and partial energies, the argmin result) lives in one file-scope
// device array of kScratchBytes per GPU.  Its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is handed to kernels and copies: in host code the array's
// name stands for a host-side shadow, not device memory.  No device memory
// is allocated or freed here.  Every call on one GPU shares the array and
// finds the previous call's contents, so whatever must start at zero is
// cleared by a fill kernel at the start of every call; calls that overlap on
// one GPU race on it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "phia.h"
#include "phia_internal.h"
#include "phia_problem.h"

namespace phia {

constexpr size_t kScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once).
hipError_t scratch_address(int dev, unsigned char** out)
{
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch_dev[dev]);
    return hipSuccess;
}

// Zero n 64-bit words (a kernel, so the clearing is an ordinary launch).
__global__ void __launch_bounds__(256) k_zero_words(uint64_t* p, size_t n)
{
    for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        p[i] = 0;
}

hipError_t zero_words(void* p, size_t bytes, hipStream_t st)
{
    const size_t n = bytes / 8;
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_zero_words, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st,
                       static_cast<uint64_t*>(p), n);
    return hipGetLastError();
}

size_t round256(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

}  // namespace
}  // namespace phia

using namespace phia;

extern "C" phia_status phia_anneal_noalloc(phia_problem* p, int32_t replicas, int64_t steps,
                                           const phia_schedule* s, uint64_t seed, float* x, float* v,
                                           int64_t* bestE, int8_t* bestS, int64_t* bestStep,
                                           int64_t* best_energy_units, int32_t* best_replica)
{
    clear_error();
    phia_status st = check_usable(p);
    if (st != PHIA_OK) return st;
    if ((st = check_schedule(replicas, steps, s)) != PHIA_OK) return st;
    if (s->metropolis) return fail(PHIA_EINVAL, "phia_anneal_noalloc runs without the accept/reject step");
    if (!x || !v || !bestE || !bestS || !bestStep) return fail(PHIA_EINVAL, "state and record buffers are required");
    if (!p->dJ) return fail(PHIA_ESTATE, "the couplings are not resident (a deferred upload happens at an anneal)");
    hipError_t e = hipSetDevice(p->dev);
    if (e != hipSuccess) return hip_fail(p, e, "hipSetDevice");
    unsigned char* base = nullptr;
    if ((e = scratch_address(p->dev, &base)) != hipSuccess) return hip_fail(nullptr, e, "scratch address");

    const Geometry g = plain_geometry(p, replicas, s->initial_kick ? 1 : 0);
    if (!g.ok) return fail(PHIA_ERANGE, "no kernel geometry fits N = %d on this device", p->N);
    const bool group = g.kind != 4 && g.G > 1;
    const size_t ncb = static_cast<size_t>(p->Np / 16);
    const size_t xb = group ? 2 * static_cast<size_t>(g.ngroups) * g.rows * ncb * sizeof(uint64_t) : 0;
    const size_t pb = group ? 2 * static_cast<size_t>(g.ngroups) * g.G * g.rows * 2 * sizeof(uint64_t) : 0;
    // scratch layout: error word, argmin result, kick factors, exchange words, partial energies
    const size_t err_off = 0, arg_off = 256, ctab_off = 512;
    const size_t xb_off = ctab_off + round256(sizeof(float) * static_cast<size_t>(steps));
    const size_t pb_off = xb_off + round256(xb);
    const size_t need = pb_off + round256(pb);
    if (need > kScratchBytes)
        return fail(PHIA_ERANGE, "this anneal needs %zu bytes of scratch; phia_anneal_noalloc holds %zu", need,
                    kScratchBytes);
    const int64_t iters = (g.nblocks + g.ngroups - 1) / g.ngroups;
    constexpr int64_t kChunk = int64_t(1) << 22;  // steps per launch of the interleaved sweep
    if (group) {
        // one call never restarts the exchange tags: 24 bits (interleaved
        // sweep) or 32 bits of sequence numbers must cover the whole anneal
        // (a launch of n steps takes n + 1 per pass over the replica blocks)
        const int64_t room = g.kind >= 1 ? (int64_t(1) << 24) - 2 : (int64_t(1) << 32) - 2;
        const int64_t launches = g.kind >= 1 ? (steps + kChunk - 1) / kChunk : 1;
        if (iters * (steps + launches) > room)
            return fail(PHIA_ERANGE, "%lld steps x %lld block passes exceed the exchange tags of one call",
                        static_cast<long long>(steps), static_cast<long long>(iters));
    }
    int32_t* derr = reinterpret_cast<int32_t*>(base + err_off);
    int64_t* darg = reinterpret_cast<int64_t*>(base + arg_off);
    float* dctab = reinterpret_cast<float*>(base + ctab_off);

    std::vector<float> ctab;
    kick_factors(p, steps, s, ctab);
    const hipStream_t stream = p->st;
    // the synchronous copy completes before the host table goes out of scope
    if ((e = hipMemcpy(dctab, ctab.data(), sizeof(float) * ctab.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = zero_words(derr, 256, stream)) != hipSuccess ||
        (group && (e = zero_words(base + xb_off, xb, stream)) != hipSuccess) ||
        (group && (e = zero_words(base + pb_off, pb, stream)) != hipSuccess))
        return hip_fail(p, e, "scratch set-up");

    SweepArgs a = sweep_args(p);
    a.J = g.kind == 2 ? p->dJ4 : p->dJ;
    a.ctab = dctab;
    a.eps = s->eps;
    a.gamma = s->gamma;
    a.L = s->refresh_L;
    a.deriv = s->deriv_mode;
    a.ikick = s->initial_kick ? 1 : 0;
    a.seed = seed;
    a.R = replicas;
    a.r_base = 0;
    a.x = x;
    a.v = v;
    a.bestE = bestE;
    a.bestS = bestS;
    a.bestStep = bestStep;
    a.etrace = nullptr;
    a.T = steps;
    a.G = g.G;
    a.ncb = static_cast<int32_t>(ncb);
    a.rows = g.rows;
    a.nblocks = g.nblocks;
    a.ngroups = g.ngroups;
    a.xcd_map = g.xcd_map;
    a.j_lds = g.j_lds;
    a.inc = g.inc;
    a.incstat = nullptr;
    a.xbits = group ? reinterpret_cast<uint64_t*>(base + xb_off) : nullptr;
    a.pbuf = group ? reinterpret_cast<uint64_t*>(base + pb_off) : nullptr;
    a.seq_base = 0;
    a.err = derr;
    a.mh = 0;
    a.btab = nullptr;
    a.x0 = nullptr;
    a.mhE = nullptr;
    a.mhQ = nullptr;
    a.lam = nullptr;
    a.mhc = nullptr;
    a.mhbuf = nullptr;
    a.k0 = 0;
    a.k1 = steps;

    if ((e = launch_init(a, stream)) != hipSuccess) return hip_fail(p, e, "init kernel launch");
    if (g.kind == 4) {
        e = launch_sweep_valu(p->path == PHIA_PATH_FP32 ? kValuFp32 : p->path == PHIA_PATH_ELL ? kValuEll : kValuDot8,
                              g.rows, g.j_lds != 0, a, stream);
    } else if (g.kind >= 1) {
        // launches of at most 2^22 steps, sequence numbers running on
        uint32_t seq = 0;
        for (int64_t k = 0; k < steps && e == hipSuccess;) {
            const int64_t kk = std::min<int64_t>(steps, k + kChunk);
            a.k0 = k;
            a.k1 = kk;
            a.seq_base = seq;
            e = launch_sweep_pp(a, g.kind == 2, g.kind == 1 && !g.j_lds, g.lds, stream);
            seq += static_cast<uint32_t>(iters * (kk - k + 1));
            k = kk;
        }
    } else {
        e = launch_sweep_mfma(p->path, g.mt, g.cbw, a, g.lds, stream);
    }
    if (e != hipSuccess) return hip_fail(p, e, "sweep launch");
    if ((e = launch_argmin(bestE, replicas, darg, stream)) != hipSuccess) return hip_fail(p, e, "argmin launch");
    int64_t res[2] = {0, 0};
    int32_t err = 0;
    if ((e = hipMemcpyAsync(res, darg, sizeof res, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(&err, derr, sizeof err, hipMemcpyDeviceToHost, stream)) != hipSuccess ||
        (e = stream ? hipStreamSynchronize(stream) : hipDeviceSynchronize()) != hipSuccess)
        return hip_fail(p, e, "result readback");
    if (err) {
        p->poisoned = true;
        return fail(PHIA_EDEVICE, "a workgroup-group barrier timed out (device error word %d)", err);
    }
    if (best_energy_units) *best_energy_units = res[0];
    if (best_replica) *best_replica = static_cast<int32_t>(res[1]);
    return PHIA_OK;
}
