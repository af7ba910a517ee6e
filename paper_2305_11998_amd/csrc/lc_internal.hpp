// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/lc.h"

namespace lc {

void set_error(const char* fmt, ...);

// Every device allocation of the library goes through lc_malloc, which
// refuses (hipErrorOutOfMemory, nothing allocated) any request above the
// process-wide cap set by lc_set_alloc_limit (0: no cap).
hipError_t lc_malloc(void** p, size_t bytes);

#define LC_HIP(expr)                                                          \
    do {                                                                      \
        hipError_t lc_e_ = (expr);                                            \
        if (lc_e_ != hipSuccess) {                                            \
            ::lc::set_error("%s failed: %s", #expr, hipGetErrorString(lc_e_)); \
            return LC_ERR_HIP;                                                \
        }                                                                     \
    } while (0)

#define LC_CHECK(cond, code, ...)          \
    do {                                   \
        if (!(cond)) {                     \
            ::lc::set_error(__VA_ARGS__);  \
            return (code);                 \
        }                                  \
    } while (0)

#define LC_ARG(cond, ...) LC_CHECK(cond, LC_ERR_ARG, __VA_ARGS__)

constexpr uint32_t kRaysMagic = 0x4c435259u;   // "LCRY"
constexpr uint32_t kPlanMagic = 0x4c43504cu;   // "LCPL"
constexpr uint32_t kBatchMagic = 0x4c434254u;  // "LCBT"
constexpr int kMaxPol = 8;
constexpr int kMaxPolUnroll16 = 4;               // sweep_unroll 16: float32 plans with n_pol up to this
constexpr int kSplitUnroll = 4;                  // load chunk of the split sweep; split lengths are multiples
constexpr int kBlock = 256;                    // threads per block of the streaming kernels
constexpr int kWave = 64;                      // lanes per wavefront (gfx9)
constexpr int kDirW = 10;                      // per-direction weight record, see dirw_index

// Per (pair a, traversal d, polar p) record, float64:
//   [0] omega, [1] omega Ox, [2] omega Oy, [3] omega Ox Ox, [4] omega Ox Oy,
//   [5] omega Oy Oy, [6] omega Oz Oz, [7] Ox, [8] Oy, [9] 1/sin(zeta)
inline size_t dirw_index(int a, int d, int p, int n_pol) {
    return ((size_t)(a * 2 + d) * n_pol + p) * kDirW;
}

struct Rays {
    uint32_t magic = 0;
    int nx = 0, ny = 0;
    double lx = 0, ly = 0, hx = 0, hy = 0;
    int n_az = 0, n_pol = 0, n_pairs = 0, nb = 0, cells = 0, mode = 0;
    double h_moc = 0;
    int64_t n_rays = 0, n_seg = 0;
    int max_seg = 0;
    bool sym = false;                 // mu[p] == -mu[P-1-p] for every p
    std::vector<double> phi, mu, omega, inv_sinz, cphi, sphi;
    std::vector<int> ray_off;         // host copy [n_pairs + 1]
    std::vector<int> seg_off;         // host copy [n_rays + 1]
    std::vector<double> dirw;         // host copy of d_dirw
    // device geometry
    int* d_ray_off = nullptr;         // [n_pairs + 1]
    int* d_seg_off = nullptr;         // [n_rays + 1]
    int* d_face = nullptr;            // [n_rays][2] entry, exit face of the forward traversal
    double* d_v = nullptr;            // [n_rays] centreline offsets
    double* d_width = nullptr;        // [n_rays]
    double* d_pts = nullptr;          // [n_rays][4] entry x, y, exit x, y
    int* d_cell = nullptr;            // [n_seg]
    double* d_len = nullptr;          // [n_seg]
    int* d_csr_off = nullptr;         // [cells * n_pairs + 1], index cell * n_pairs + a
    int* d_csr_ray = nullptr;         // [n_seg] global ray k of the entry
    int2* d_csr_t = nullptr;          // [n_seg] position of the segment in the d = 0 and d = 1 traversal
    double* d_csr_w = nullptr;        // [n_seg] A_j / sum of A over C(i, m)
    float* d_csr_w32 = nullptr;
    int2* d_seg32 = nullptr;          // [n_seg] sweep record {cell, bits of the float32 length}
    int4* d_seg64 = nullptr;          // [n_seg] sweep record {cell, 0, low and high words of the float64 length}
    int* d_bmap = nullptr;            // [nb][n_pairs][2][2] first, end global ray leaving through b; -1 = incoming
    double* d_dirw = nullptr;         // [n_pairs][2][n_pol][kDirW]
    // interior-face crossing lists, built on request (lc_plan_enable_faces):
    // x-faces first ((nx-1) * ny, row-major), then y-faces (nx * (ny-1))
    int64_t n_fent = 0;               // crossings over all pairs
    int* d_fcsr_off = nullptr;        // [n_ifaces * n_pairs + 1], index face * n_pairs + a
    int* d_fcsr_ray = nullptr;        // [n_fent] global ray k
    int2* d_fcsr_t = nullptr;         // [n_fent] {s, nk - s}: steps of the segments entered there (d = 0, 1)
    double* d_fcsr_w = nullptr;       // [n_fent] w_k / sum of w over the (face, pair) list
    float* d_fcsr_w32 = nullptr;
    std::vector<void*> owned;         // every device allocation above
};

struct Plan;

// Global (address space 1) pointers: device code loads through them so that
// the compiler emits global rather than flat memory instructions even where a
// pointer comes from an argument record in memory.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<const T> as_global(const T* p) { return (gptr<const T>)p; }
template <typename T> __device__ __forceinline__ gptr<T> as_global_w(T* p) { return (gptr<T>)p; }

// Cell record of eq. (11): kappa_t and the emission kappa B / kappa_t; the
// remaining coefficient 1/(c dt kappa_t) is formed in the sweep.
template <typename T> struct alignas(2 * sizeof(T)) Coef { T kt, a; };

struct GraphEntry {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec = nullptr;
};

struct Plan {
    uint32_t magic = 0;
    Rays* rays = nullptr;
    int G = 0;
    int prec = 0;
    size_t hdr_bytes = 0;             // state header (per-group scale exponents)
    size_t value_bytes = 0;
    void* d_coef = nullptr;           // [cells][G] {kappa_t, kappa B / kappa_t}
    unsigned long long* d_gmax = nullptr;  // [2][G] per-group maxima of |B| and of |I_in| (float32 scale)
    unsigned long long* d_check = nullptr; // first invalid input index (validation mode)
    int sweep_unroll = 0;             // steps whose loads are issued together (1, 2, 4, 8 or 16)
    int moments_entries = 0;          // C(i, m) entries per list in the moment pipeline (1..4)
    // State layout: the lanes (k, g) of pair a, g fastest, are cut into
    // bundles of 64 (one wavefront each).  For traversal d and bundle B the
    // values [t][lane][p] (t = step along the traversal, padded to the
    // longest characteristic of the bundle) are contiguous at
    // d * half_elems + bun_base[B].
    int64_t n_bun = 0;                // bundles over all pairs
    std::vector<int> bun_off;         // [n_pairs + 1] first bundle of each pair
    std::vector<int> bun_len_h;       // [n_bun] steps of each bundle
    std::vector<int64_t> bun_base_h;  // [n_bun] element offset within one traversal half
    int64_t half_elems = 0;
    int* d_bun_off = nullptr;
    int* d_bun_len = nullptr;
    int64_t* d_bun_base = nullptr;
    unsigned* d_ent_off = nullptr;    // [n_seg][4] state lane records (P values each) and float32 weight of each C(i, m) entry
    unsigned* d_fent_off = nullptr;   // [n_fent][4] the same for the interior-face crossings (on request)
    unsigned* d_bun_rec = nullptr;    // [n_bun] first lane record of each bundle
    int tile_w = 1, tile_h = 1;       // cell tile of the moments kernel
    // gathers split over azimuth pairs (lc_plan_set_moment_split): bit 0 the
    // cell and face moments, bit 1 the boundary factors; per-pair partial
    // sums in d_mom_part, combined in pair order by a second kernel
    int mom_split = 0;
    void* d_mom_part = nullptr;
    size_t mom_part_bytes = 0;
    int64_t sweep_blocks = 0;         // blocks of one sweep launch
    size_t sweep_lds = 0;             // LDS reserved per sweep block (caps the blocks per CU)
    // split sweep (lc_plan_set_split): traversals cut into chunks of
    // split_len steps; items {wavefront, chunk} of the transfer pass (the
    // first n_split1) then of the sweep pass; transfer records per wavefront
    int split_len = 0;
    int2* d_split_items = nullptr;
    int64_t n_split1 = 0, n_split_items = 0;
    int64_t* d_cbase = nullptr;       // [2 n_bun + 1] first transfer record of each wavefront
    void* d_carry = nullptr;          // [records][n_pol][64] {A, B} pairs of the state type
    std::vector<GraphEntry> graphs;   // captured lc_step sequences
    hipStream_t capture = nullptr;    // stream used only to record graphs
    bool profile = false;             // record events around the main kernels
    bool capturing = false;           // inside lc_step capture: never record events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_sweep, ev_mom;
};

// Validation mode (lc_set_validation): when on, the sweep entry points check
// kappa and planck (n_mat values each) and I_in for values that are not
// finite or are negative before any launch; LC_ERR_ARG names the first.
bool validation_on();
lc_status validate_inputs(Plan* pl, const double* kappa, const double* planck, int64_t n_mat, const double* I_in,
                          hipStream_t st);

// Event pair around one kernel launch when the plan records timings.
lc_status prof_begin(Plan* pl, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, hipStream_t st);
lc_status prof_end(Plan* pl, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, hipStream_t st);

inline Rays* as_rays(lc_rays_t r) {
    Rays* p = reinterpret_cast<Rays*>(r);
    return (p && p->magic == kRaysMagic) ? p : nullptr;
}
inline Plan* as_plan(lc_plan_t r) {
    Plan* p = reinterpret_cast<Plan*>(r);
    return (p && p->magic == kPlanMagic) ? p : nullptr;
}

// device allocation owned by a vector of pointers (freed together)
template <typename T>
lc_status dalloc(std::vector<void*>& owned, T** out, size_t n) {
    void* p = nullptr;
    size_t bytes = n ? n * sizeof(T) : sizeof(T);
    hipError_t e = lc_malloc(&p, bytes);
    if (e != hipSuccess) {
        set_error("hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
        (void)hipGetLastError();
        return LC_ERR_ALLOC;
    }
    owned.push_back(p);
    *out = static_cast<T*>(p);
    return LC_OK;
}

// Scratch of one sweep given by the caller instead of the plan's: the
// coefficient table [cells][G] and the float32 per-group maxima [2][G].
// With it the sweep runs whole traversals and records no timing events.
struct SweepScratch {
    void* coef = nullptr;
    unsigned long long* gmax = nullptr;
};

// Internal launchers (stream-ordered, no allocation, no synchronisation).
lc_status launch_sweep(Plan* pl, const double* kappa, const double* planck, double c_dt,
                       const void* state_prev, void* state_new, const double* I_in,
                       double* I_exit, hipStream_t st, void* point = nullptr,
                       const SweepScratch* ws = nullptr);
lc_status launch_moments(Plan* pl, const void* state, const double* I_exit, const double* I_in,
                         double c, double* E, double* F, double* f, double* bnd, hipStream_t st);
lc_status launch_state_fill(Plan* pl, const double* field, void* state, hipStream_t st);
lc_status launch_state_export(Plan* pl, const void* state, double* out, hipStream_t st);
lc_status launch_state_import(Plan* pl, const double* in, void* state, hipStream_t st);
lc_status build_geometry(Rays* r, hipStream_t st);
lc_status plan_init_sweep(Plan* pl);
lc_status plan_set_split(Plan* pl, int len);
void plan_free_split(Plan* pl);
lc_status plan_init_moments(Plan* pl);
lc_status plan_set_moment_split(Plan* pl, int mode);
lc_status plan_enable_faces(Plan* pl, hipStream_t st);
lc_status launch_face_moments(Plan* pl, const void* point, const void* state, double c, double* E, double* F,
                              double* f, hipStream_t st);

// Batched form: argument records (built on the host, copied to the device)
// and launchers of the persistent kernels.
size_t sweep_args_bytes();
size_t coef_args_bytes();
size_t mom_args_bytes();
size_t bnd_args_bytes();
void make_batch_args(Plan* pl, double c_dt, void* state_a, void* state_b, const double* I_in, double* I_exit,
                     void* sweep_out2);
void make_coef_args(Plan* pl, double c_dt, const double* kappa, const double* planck, int64_t stride,
                    void* state_a, void* state_b, const double* I_in, unsigned long long* gmax,
                    unsigned long long* gmax_in, int64_t max_blk_off, int64_t coef_blk_off, int64_t g_off, void* out,
                    int64_t* n_max_blocks, int64_t* n_coef_blocks);
lc_status launch_prologue(Plan* pl, const double* kappa, const double* planck, double c_dt,
                          const void* state_prev, void* state_new, const double* I_in, hipStream_t st,
                          void* coef, unsigned long long* gmax);
void make_moment_args(Plan* pl, const void* state, const double* I_exit, const double* I_in, double c,
                      double* E, double* F, double* f, double* bnd, int64_t bnd_blk_off, void* mom_out,
                      void* bnd_out);
int64_t moment_tiles(const Plan* pl);
int moment_tile_waves(const Plan* pl);
lc_status launch_prologue_batch(int prec, const void* coef_args, int n, int64_t max_blocks_all,
                                int64_t coef_blocks_all, int max_G, unsigned long long* gmax, int64_t n_gmax, int t,
                                hipStream_t st);
lc_status launch_zero_counters(int* c, int n, hipStream_t st);
// The sweep form without per-polar-slot branches: a mirror-symmetric polar
// set whose size is a power of two (so it fills its polar bound exactly).
inline bool sweep_full(const Rays* r) { return r->sym && (r->n_pol & (r->n_pol - 1)) == 0; }
lc_status sweep_lds_bytes(size_t* lds);
lc_status sweep_batch_grid(int prec, int pm, int unroll, bool full, size_t lds, int* grid);
lc_status launch_sweep_batch(int prec, int pm, int unroll, bool full, size_t lds, int grid, const void* args,
                             const int2* items, const int64_t* qb, int* counters, hipStream_t st);
lc_status launch_moments_batch(int prec, int pm, int ent, const void* args, const int2* items, int64_t n_items,
                               hipStream_t st);
lc_status launch_boundary_batch(const void* args, int n, int64_t blocks, hipStream_t st);
lc_status build_face_lists(Rays* r, hipStream_t st);
inline int64_t n_interior_faces(const Rays* r) { return (int64_t)(r->nx - 1) * r->ny + (int64_t)r->nx * (r->ny - 1); }
lc_status launch_grey_closures_dims(int cells, int G, const double* E, const double* F, const double* f,
                                    const double* kappa, const double* planck, double* out, hipStream_t st);
lc_status launch_grey_closures(const Plan* pl, const double* E, const double* F, const double* f,
                               const double* kappa, const double* planck, double* out, hipStream_t st);

// Device pointers to the values of a state buffer (after its header).
inline const void* state_values(const Plan* pl, const void* s) {
    return static_cast<const char*>(s) + pl->hdr_bytes;
}
inline void* state_values(const Plan* pl, void* s) { return static_cast<char*>(s) + pl->hdr_bytes; }


}  // namespace lc
