// muca_static.hip -- production sweeps that allocate nothing, for callers that
// cannot allocate device or host memory while they run (serving loops and
// harnesses that forbid allocation).
//
// muca_production_static is muca_production on lattices and energies the
// caller owns: the same thresholds, the same kernels, the same bits.  What an
// instance keeps in its own device workspace -- the uploaded threshold table
// and the 64-bit histogram the workgroups merge into -- lives here in one
// file-scope device array, `scratch`, sized for the largest lattice
// (MUCA_MAX_L); the host copies of the tables live in static host arrays.
// Every call on a device shares that device's copy of the array: the call
// holds a process-wide lock and returns only after its device work is done,
// so two calls never use the array at once.
#include "muca.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>

#include "muca_device.h"
#include "muca_internal.h"

namespace {

constexpr uint32_t kMaxBins = MUCA_MAX_L * MUCA_MAX_L + 1;
constexpr size_t kAlign = 256;
constexpr size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
// scratch layout: the device threshold table (32 bytes per bin), then the
// merged histogram (8 bytes per bin)
constexpr size_t table_bytes(uint32_t bins) { return (size_t)bins * 4 * sizeof(uint64_t); }
constexpr size_t hist_offset(uint32_t bins) { return round_up(table_bytes(bins)); }
constexpr size_t scratch_bytes(uint32_t bins) { return hist_offset(bins) + round_up((size_t)bins * sizeof(uint64_t)); }
static_assert(scratch_bytes(kMaxBins) == MUCA_STATIC_SCRATCH_BYTES, "scratch size in muca.h");

constexpr int kMaxDevices = 64;

std::mutex g_lock;                       // held for the whole of a call
void* g_scratch[kMaxDevices];            // device address of `scratch` on each device
int g_cus[kMaxDevices];                  // compute units of each device
uint64_t g_table5[5 * (size_t)kMaxBins]; // thresholds T[k*5 + d] of the call
uint64_t g_table4[4 * (size_t)kMaxBins]; // the device form of the table, before upload

}  // namespace

// The call's threshold table and merged histogram, on every device the
// library runs on (one copy per device, held until the process ends).  In
// host code this name stands for the device array and is not its address:
// only the per-device address from hipGetSymbolAddress is handed to kernels
// and copies.
static __device__ __align__(256) unsigned char scratch[MUCA_STATIC_SCRATCH_BYTES];

namespace {

int fail(int code, const char* msg)
{
    muca_host::set_null_error(msg);
    return code;
}

int device_fail(hipError_t e, const char* what)
{
    char buf[200];
    std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorName(e));
    muca_host::set_null_error(buf);
    return MUCA_ERR_DEVICE;
}

}  // namespace

extern "C" int muca_production_static(const muca_params* p, uint64_t sweep0, uint32_t therm_sweeps,
                                      uint32_t sweeps, const double* omega, uint32_t* spins, int32_t* energies,
                                      uint64_t* hist, void* hip_stream)
{
    if (!p || !omega || !spins || !energies || !hist)
        return fail(MUCA_ERR_INVALID_ARG, "a pointer argument is NULL");
    if (p->L < 4 || p->L % 2 != 0 || p->L > MUCA_MAX_L || !muca::sweep_supported(p->L))
        return fail(MUCA_ERR_INVALID_ARG, "L must be even, 4 <= L <= 128, with a sweep kernel built for it");
    if (p->walkers == 0 || p->walkers > (1u << 30))
        return fail(MUCA_ERR_INVALID_ARG, "walkers must be in 1 .. 2^30");
    const uint32_t N = p->L * p->L;
    if (scratch_bytes(N + 1) > MUCA_STATIC_SCRATCH_BYTES)
        return fail(MUCA_ERR_INVALID_ARG, "the lattice's tables exceed the static scratch size");
    for (uint32_t k = 0; k <= N; ++k)
        if (!std::isfinite(omega[k]))
            return fail(MUCA_ERR_INVALID_ARG, "omega must be finite");
    const uint64_t total = (uint64_t)therm_sweeps + sweeps;
    if (sweep0 > (UINT64_MAX / N - total))
        return fail(MUCA_ERR_OVERFLOW, "the attempt position would wrap");
    if ((long double)p->walkers * N * (long double)total >= 18446744073709551615.0L)
        return fail(MUCA_ERR_OVERFLOW, "walkers * attempts exceeds 2^64");

    std::lock_guard<std::mutex> guard(g_lock);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return device_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(MUCA_ERR_INVALID_ARG, "device index beyond the static call's device table");
    if (!g_scratch[dev]) {
        // first call on this device (which is current): where its copy of
        // `scratch` lives, and its compute-unit count for the kernel choice
        void* ptr = nullptr;
        if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
            return device_fail(e, "hipGetSymbolAddress(scratch)");
        int cus = 0;
        if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
            return device_fail(e, "hipDeviceGetAttribute");
        g_cus[dev] = cus;
        g_scratch[dev] = ptr;
    }
    unsigned char* base = static_cast<unsigned char*>(g_scratch[dev]);

    muca_host::compute_thresholds(N, omega, g_table5);
    muca_host::CallTarget t{};
    t.L = p->L;
    t.wpad = muca::padded_walkers(p->walkers);
    t.walkers = p->walkers;
    t.seed = p->seed;
    t.flags = p->flags;
    t.cus = g_cus[dev];
    t.d_spins = spins;
    t.d_energy = energies;
    t.d_table = reinterpret_cast<uint64_t*>(base);
    t.d_hist = reinterpret_cast<unsigned long long*>(base + hist_offset(N + 1));
    t.h_table4 = g_table4;
    muca_host::Segment seg{};
    seg.sweep0 = sweep0;
    seg.n = total;
    seg.therm = therm_sweeps;
    hipStream_t stream = (hipStream_t)hip_stream;
    uint32_t launches = 0, variant = 0;
    const char* what = "";
    // the histogram is cleared by a kernel inside enqueue_call: the array
    // keeps the previous call's counts until then
    if ((e = muca_host::enqueue_call(t, g_table5, &seg, total ? 1u : 0u, stream, nullptr, nullptr, &launches,
                                     &variant, &what)) != hipSuccess)
        return device_fail(e, what);
    if ((e = hipMemcpyAsync(hist, t.d_hist, (size_t)(N + 1) * sizeof(uint64_t), hipMemcpyDeviceToHost,
                            stream)) != hipSuccess)
        return device_fail(e, "histogram download");
    if ((e = hipStreamSynchronize(stream)) != hipSuccess)
        return device_fail(e, "stream");
    uint64_t sum = 0;
    for (uint32_t k = 0; k <= N; ++k)
        sum += hist[k];
    if (sum != (uint64_t)p->walkers * N * sweeps)
        return fail(MUCA_ERR_DEVICE, "histogram sum != walkers * recorded attempts");
    return MUCA_OK;
}
