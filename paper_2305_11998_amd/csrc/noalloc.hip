// lc_sweep_noalloc: the sweep of lc_sweep with its scratch -- the cell
// coefficient table and the float32 per-group maxima -- in a static device
// array of fixed size instead of the plan's workspace, for callers that may
// not allocate while they sweep.
#include <cmath>
#include <mutex>
#include <vector>

#include "lc_internal.hpp"

namespace lc {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;     // 64 MiB per device
constexpr size_t kScratchAlign = 256;

// The device copy of this array lives at a per-device address; host code
// uses only the address returned by hipGetSymbolAddress (scratch_of), never
// the array's name.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;   // per device ordinal, filled on first use

lc_status scratch_of(void** out) {
    int dev = 0;
    LC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress of the static sweep scratch failed on device %d: %s", dev,
                      hipGetErrorString(e));
            (void)hipGetLastError();
            return LC_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LC_OK;
}

size_t round_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bytes of the coefficient table of a plan, rounded up to the alignment.
size_t coef_table_bytes(const Plan* pl) {
    const size_t rec = pl->prec == LC_F32 ? sizeof(Coef<float>) : sizeof(Coef<double>);
    return round_up((size_t)pl->rays->cells * (size_t)pl->G * rec, kScratchAlign);
}

}  // namespace
}  // namespace lc

using namespace lc;

extern "C" {

lc_status lc_sweep_noalloc(lc_plan_t plan, const double* kappa, const double* planck, double c_dt,
                           const void* state_prev, void* state_new, const double* I_in, double* I_exit,
                           void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(kappa && planck && state_prev && state_new && I_in,
           "kappa, planck, states and I_in must not be NULL");
    LC_ARG(state_prev != state_new, "state_prev and state_new must be distinct buffers");
    LC_ARG(std::isfinite(c_dt) && c_dt > 0.0, "c_dt must be finite and > 0");
    const size_t need = coef_table_bytes(pl) + 2 * (size_t)pl->G * sizeof(unsigned long long);
    LC_ARG(need <= kScratchBytes,
           "lc_sweep_noalloc needs %zu bytes of scratch (cells x G coefficient records and 2 G maxima); the "
           "static scratch holds %zu bytes -- use lc_sweep",
           need, kScratchBytes);
    void* base = nullptr;
    lc_status rc = scratch_of(&base);
    if (rc) return rc;
    if (validation_on()) {                       // the plan's check slot: allocated with the plan
        rc = validate_inputs(pl, kappa, planck, (int64_t)pl->G * pl->rays->cells, I_in,
                             static_cast<hipStream_t>(stream));
        if (rc) return rc;
    }
    SweepScratch ws;
    ws.coef = base;
    ws.gmax = reinterpret_cast<unsigned long long*>(static_cast<char*>(base) + coef_table_bytes(pl));
    return launch_sweep(pl, kappa, planck, c_dt, state_prev, state_new, I_in, I_exit,
                        static_cast<hipStream_t>(stream), nullptr, &ws);
}

}  // extern "C"
