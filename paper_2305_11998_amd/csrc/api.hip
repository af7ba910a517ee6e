// Host side of the C ABI: argument validation, handle lifetime, plans and the
// graph-captured time step.  Every entry point checks its arguments before any
// HIP call and reports failures as status codes.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <limits>

#include "lc_internal.hpp"

namespace lc {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

namespace {

void free_rays(Rays* r) {
    if (!r) return;
    for (void* p : r->owned) (void)hipFree(p);
    r->owned.clear();
    r->magic = 0;
    delete r;
}

void clear_events(Plan* pl) {
    for (auto* v : {&pl->ev_sweep, &pl->ev_mom}) {
        for (auto& e : *v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        v->clear();
    }
}

void free_plan(Plan* pl) {
    if (!pl) return;
    clear_events(pl);
    for (auto& g : pl->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (pl->capture) (void)hipStreamDestroy(pl->capture);
    if (pl->d_coef) (void)hipFree(pl->d_coef);
    if (pl->d_gmax) (void)hipFree(pl->d_gmax);
    if (pl->d_check) (void)hipFree(pl->d_check);
    if (pl->d_bun_off) (void)hipFree(pl->d_bun_off);
    if (pl->d_bun_len) (void)hipFree(pl->d_bun_len);
    if (pl->d_bun_base) (void)hipFree(pl->d_bun_base);
    if (pl->d_ent_off) (void)hipFree(pl->d_ent_off);
    if (pl->d_fent_off) (void)hipFree(pl->d_fent_off);
    if (pl->d_bun_rec) (void)hipFree(pl->d_bun_rec);
    if (pl->d_mom_part) (void)hipFree(pl->d_mom_part);
    plan_free_split(pl);
    pl->magic = 0;
    delete pl;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

std::atomic<uint64_t> g_alloc_cap{0};
std::atomic<int> g_validate{0};

// Smallest index i < n with a[i] not finite or negative (atomicMin over the
// index: the same answer however the threads are scheduled).
__global__ void k_first_invalid(const double* __restrict__ a, int64_t n, unsigned long long* first) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = a[i];
        if (!(std::isfinite(v) && v >= 0.0)) atomicMin(first, (unsigned long long)i);
    }
}

}  // namespace

hipError_t lc_malloc(void** p, size_t bytes) {
    const uint64_t cap = g_alloc_cap.load();
    if (cap && bytes > cap) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

bool validation_on() { return g_validate.load() != 0; }

lc_status validate_inputs(Plan* pl, const double* kappa, const double* planck, int64_t n_mat, const double* I_in,
                          hipStream_t st) {
    const Rays* r = pl->rays;
    const struct {
        const double* a;
        int64_t n;
        const char* name;
    } arrays[3] = {{kappa, n_mat, "kappa"},
                   {planck, n_mat, "planck"},
                   {I_in, (int64_t)r->nb * r->n_az * r->n_pol * pl->G, "I_in"}};
    for (const auto& x : arrays) {
        const unsigned long long none = ~0ull;
        LC_HIP(hipMemcpyAsync(pl->d_check, &none, sizeof(none), hipMemcpyHostToDevice, st));
        const int64_t blocks = std::min<int64_t>((x.n + 255) / 256, 4096);
        hipLaunchKernelGGL(k_first_invalid, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, x.a, x.n,
                           pl->d_check);
        LC_HIP(hipGetLastError());
        unsigned long long first = none;
        LC_HIP(hipMemcpyAsync(&first, pl->d_check, sizeof(first), hipMemcpyDeviceToHost, st));
        LC_HIP(hipStreamSynchronize(st));
        LC_ARG(first == none, "%s[%llu] is not finite or is negative", x.name, first);
    }
    return LC_OK;
}

lc_status prof_begin(Plan* pl, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, hipStream_t st) {
    if (!pl->profile || pl->capturing) return LC_OK;
    hipEvent_t a = nullptr, b = nullptr;
    LC_HIP(hipEventCreate(&a));
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        set_error("hipEventCreate failed: %s", hipGetErrorString(e));
        return LC_ERR_HIP;
    }
    v.push_back({a, b});
    LC_HIP(hipEventRecord(a, st));
    return LC_OK;
}

lc_status prof_end(Plan* pl, std::vector<std::pair<hipEvent_t, hipEvent_t>>& v, hipStream_t st) {
    if (!pl->profile || pl->capturing || v.empty()) return LC_OK;
    LC_HIP(hipEventRecord(v.back().second, st));
    return LC_OK;
}

}  // namespace lc

using namespace lc;

extern "C" {

lc_status lc_set_alloc_limit(uint64_t bytes) {
    g_alloc_cap.store(bytes);
    return LC_OK;
}

lc_status lc_set_validation(int32_t enable) {
    g_validate.store(enable != 0);
    return LC_OK;
}

int32_t lc_version(void) { return 1 * 10000 + 4 * 100 + 0; }

const char* lc_last_error(void) { return g_err; }

lc_status lc_build_rays(const lc_grid* grid, const lc_quad* quad, double h_moc, int32_t mode,
                        void* stream, lc_rays_t* out) {
    g_err[0] = 0;
    LC_ARG(out, "out is NULL");
    *out = nullptr;
    LC_ARG(grid && quad, "grid or quad is NULL");
    LC_ARG(grid->nx >= 1 && grid->ny >= 1, "nx, ny must be >= 1 (got %d, %d)", grid->nx, grid->ny);
    LC_ARG(finite_pos(grid->lx) && finite_pos(grid->ly), "lx, ly must be finite and > 0");
    LC_ARG((int64_t)grid->nx * grid->ny < (1 << 28), "grid too large");
    LC_ARG(quad->phi && quad->mu && quad->omega, "quadrature arrays must not be NULL");
    LC_ARG(quad->n_az >= 2 && quad->n_az % 2 == 0, "n_az must be even and >= 2 (got %d)", quad->n_az);
    LC_ARG(quad->n_pol >= 1 && quad->n_pol <= kMaxPol, "n_pol must be in 1..%d (got %d)", kMaxPol,
           quad->n_pol);
    LC_ARG(finite_pos(h_moc), "h_moc must be finite and > 0");
    LC_ARG(mode == LC_RAYS_UNIFORM || mode == LC_RAYS_TUBES, "unknown ray mode %d", mode);
    const int n_az = quad->n_az, P = quad->n_pol, half = n_az / 2;
    for (int p = 0; p < P; ++p)
        LC_ARG(std::isfinite(quad->mu[p]) && std::fabs(quad->mu[p]) < 1.0, "|mu[%d]| must be < 1", p);
    for (int m = 0; m < n_az * P; ++m)
        LC_ARG(std::isfinite(quad->omega[m]), "omega[%d] is not finite", m);
    for (int a = 0; a < n_az; ++a) {
        LC_ARG(std::isfinite(quad->phi[a]), "phi[%d] is not finite", a);
        const double c = std::cos(quad->phi[a]), s = std::sin(quad->phi[a]);
        LC_ARG(std::fabs(c) >= 1e-12 && std::fabs(s) >= 1e-12,
               "azimuth %d is parallel to a grid axis", a);
    }
    for (int a = 0; a < half; ++a)
        LC_ARG(std::fabs(quad->phi[a + half] - (quad->phi[a] + M_PI)) <= 1e-12,
               "phi[%d] must equal phi[%d] + pi", a + half, a);
    // segments per characteristic are at most nx + ny - 1; keep int32 indices
    {
        double W = grid->lx + grid->ly;
        double rays_bound = (double)half * (std::ceil(W / h_moc) + 1.0);
        LC_ARG(rays_bound * (grid->nx + grid->ny) < 2.0e9,
               "characteristic grid too large for 32-bit segment indices");
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    Rays* r = new (std::nothrow) Rays();
    LC_CHECK(r, LC_ERR_ALLOC, "host allocation failed");
    r->magic = kRaysMagic;
    r->nx = grid->nx;
    r->ny = grid->ny;
    r->lx = grid->lx;
    r->ly = grid->ly;
    r->hx = grid->lx / grid->nx;
    r->hy = grid->ly / grid->ny;
    r->n_az = n_az;
    r->n_pol = P;
    r->n_pairs = half;
    r->nb = 2 * (grid->nx + grid->ny);
    r->cells = grid->nx * grid->ny;
    r->mode = mode;
    r->h_moc = h_moc;
    r->phi.assign(quad->phi, quad->phi + n_az);
    r->mu.assign(quad->mu, quad->mu + P);
    r->omega.assign(quad->omega, quad->omega + n_az * P);
    r->inv_sinz.resize(P);
    r->sym = true;
    for (int p = 0; p < P; ++p) {
        r->inv_sinz[p] = 1.0 / std::sqrt(1.0 - r->mu[p] * r->mu[p]);
        if (r->mu[p] != -r->mu[P - 1 - p]) r->sym = false;
    }
    r->cphi.resize(half);
    r->sphi.resize(half);
    for (int a = 0; a < half; ++a) {
        r->cphi[a] = std::cos(r->phi[a]);
        r->sphi[a] = std::sin(r->phi[a]);
    }
    r->dirw.assign((size_t)half * 2 * P * kDirW, 0.0);
    for (int a = 0; a < half; ++a)
        for (int d = 0; d < 2; ++d)
            for (int p = 0; p < P; ++p) {
                const int az = a + d * half;
                const double sz = std::sqrt(1.0 - r->mu[p] * r->mu[p]);
                const double ox = sz * std::cos(r->phi[az]), oy = sz * std::sin(r->phi[az]);
                const double oz = r->mu[p];
                const double w = r->omega[az * P + p];
                double* rec = &r->dirw[dirw_index(a, d, p, P)];
                rec[0] = w;
                rec[1] = w * ox;
                rec[2] = w * oy;
                rec[3] = w * ox * ox;
                rec[4] = w * ox * oy;
                rec[5] = w * oy * oy;
                rec[6] = w * oz * oz;
                rec[7] = ox;
                rec[8] = oy;
                rec[9] = 1.0 / sz;
            }
    lc_status rc = build_geometry(r, st);
    if (rc == LC_OK) rc = dalloc(r->owned, &r->d_dirw, r->dirw.size());

    if (rc == LC_OK) {
        hipError_t e = hipMemcpy(r->d_dirw, r->dirw.data(), r->dirw.size() * sizeof(double),
                                 hipMemcpyHostToDevice);

        if (e != hipSuccess) {
            set_error("hipMemcpy failed: %s", hipGetErrorString(e));
            rc = LC_ERR_HIP;
        }
    }
    if (rc != LC_OK) {
        free_rays(r);
        return rc;
    }
    *out = reinterpret_cast<lc_rays_t>(r);
    return LC_OK;
}

lc_status lc_rays_free(lc_rays_t rays) {
    if (!rays) return LC_OK;
    Rays* r = as_rays(rays);
    LC_CHECK(r, LC_ERR_STATE, "invalid rays handle");
    free_rays(r);
    return LC_OK;
}

lc_status lc_rays_info(lc_rays_t rays, lc_rays_info_t* info) {
    Rays* r = as_rays(rays);
    LC_CHECK(r, LC_ERR_STATE, "invalid rays handle");
    LC_ARG(info, "info is NULL");
    info->n_rays = r->n_rays;
    info->n_segments = r->n_seg;
    info->n_pairs = r->n_pairs;
    info->n_az = r->n_az;
    info->n_pol = r->n_pol;
    info->n_cells = r->cells;
    info->n_faces = r->nb;
    info->max_seg_per_ray = r->max_seg;
    info->mode = r->mode;
    info->h_moc = r->h_moc;
    return LC_OK;
}

lc_status lc_rays_export(lc_rays_t rays, int32_t* ray_off, int32_t* seg_off, int32_t* cell, double* len,
                         double* width, int32_t* face) {
    Rays* r = as_rays(rays);
    LC_CHECK(r, LC_ERR_STATE, "invalid rays handle");
    if (ray_off) std::memcpy(ray_off, r->ray_off.data(), (r->n_pairs + 1) * sizeof(int32_t));
    if (seg_off) LC_HIP(hipMemcpy(seg_off, r->d_seg_off, (r->n_rays + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (cell) LC_HIP(hipMemcpy(cell, r->d_cell, r->n_seg * sizeof(int32_t), hipMemcpyDeviceToHost));
    if (len) LC_HIP(hipMemcpy(len, r->d_len, r->n_seg * sizeof(double), hipMemcpyDeviceToHost));
    if (width) LC_HIP(hipMemcpy(width, r->d_width, r->n_rays * sizeof(double), hipMemcpyDeviceToHost));
    if (face) LC_HIP(hipMemcpy(face, r->d_face, 2 * r->n_rays * sizeof(int32_t), hipMemcpyDeviceToHost));
    return LC_OK;
}

lc_status lc_plan_create(lc_rays_t rays, int32_t G, int32_t prec, lc_plan_t* out) {
    g_err[0] = 0;
    LC_ARG(out, "out is NULL");
    *out = nullptr;
    Rays* r = as_rays(rays);
    LC_CHECK(r, LC_ERR_STATE, "invalid rays handle");
    LC_ARG(G >= 1 && G <= 4096, "G must be in 1..4096 (got %d)", G);
    LC_ARG(prec == LC_F64 || prec == LC_F32, "unknown precision %d", prec);
    Plan* pl = new (std::nothrow) Plan();
    LC_CHECK(pl, LC_ERR_ALLOC, "host allocation failed");
    pl->magic = kPlanMagic;
    pl->rays = r;
    pl->G = G;
    pl->prec = prec;
    pl->hdr_bytes = ((size_t)G * sizeof(int32_t) + 255) / 256 * 256;
    pl->sweep_unroll = prec == LC_F32 ? 4 : 2;
    pl->moments_entries = 3;
    lc_status rc = plan_init_sweep(pl);
    pl->value_bytes = (size_t)pl->half_elems * 2 * (prec == LC_F32 ? 4 : 8);
    hipError_t e = hipSuccess;
    if (rc == LC_OK) {
        const size_t coef_bytes = (size_t)r->cells * G * (prec == LC_F32 ? 8 : 16);
        const size_t nbun = (size_t)pl->n_bun;
        e = lc_malloc(&pl->d_coef, coef_bytes);
        if (e == hipSuccess)
            e = lc_malloc(reinterpret_cast<void**>(&pl->d_gmax), 2 * (size_t)G * sizeof(unsigned long long));
        if (e == hipSuccess) e = lc_malloc(reinterpret_cast<void**>(&pl->d_check), sizeof(unsigned long long));
        if (e == hipSuccess) e = lc_malloc(reinterpret_cast<void**>(&pl->d_bun_off), pl->bun_off.size() * sizeof(int));
        if (e == hipSuccess) e = lc_malloc(reinterpret_cast<void**>(&pl->d_bun_len), std::max<size_t>(nbun, 1) * sizeof(int));
        if (e == hipSuccess) e = lc_malloc(reinterpret_cast<void**>(&pl->d_bun_base), std::max<size_t>(nbun, 1) * sizeof(int64_t));
        if (e == hipSuccess)
            e = hipMemcpy(pl->d_bun_off, pl->bun_off.data(), pl->bun_off.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pl->d_bun_len, pl->bun_len_h.data(), nbun * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pl->d_bun_base, pl->bun_base_h.data(), nbun * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->capture, hipStreamNonBlocking);
        if (e != hipSuccess) {
            set_error("plan allocation failed: %s", hipGetErrorString(e));
            (void)hipGetLastError();
            rc = LC_ERR_ALLOC;
        }
    }
    if (rc == LC_OK) rc = plan_init_moments(pl);
    if (rc != LC_OK) {
        free_plan(pl);
        return rc;
    }
    *out = reinterpret_cast<lc_plan_t>(pl);
    return LC_OK;
}

lc_status lc_plan_free(lc_plan_t plan) {
    if (!plan) return LC_OK;
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    free_plan(pl);
    return LC_OK;
}

size_t lc_state_bytes(lc_plan_t plan) {
    Plan* pl = as_plan(plan);
    if (!pl) {
        set_error("invalid plan handle");
        return 0;
    }
    return pl->hdr_bytes + pl->value_bytes;
}

lc_status lc_state_fill(lc_plan_t plan, const double* field, void* state, void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(field && state, "field and state must not be NULL");
    return launch_state_fill(pl, field, state, static_cast<hipStream_t>(stream));
}

lc_status lc_state_export(lc_plan_t plan, const void* state, double* out, void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(state && out, "state and out must not be NULL");
    return launch_state_export(pl, state, out, static_cast<hipStream_t>(stream));
}

lc_status lc_state_import(lc_plan_t plan, const double* in, void* state, void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(state && in, "in and state must not be NULL");
    return launch_state_import(pl, in, state, static_cast<hipStream_t>(stream));
}

lc_status lc_sweep(lc_plan_t plan, const double* kappa, const double* planck, double c_dt,
                   const void* state_prev, void* state_new, const double* I_in, double* I_exit,
                   void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(kappa && planck && state_prev && state_new && I_in,
           "kappa, planck, states and I_in must not be NULL");
    LC_ARG(state_prev != state_new, "state_prev and state_new must be distinct buffers");
    LC_ARG(finite_pos(c_dt), "c_dt must be finite and > 0");
    if (validation_on()) {
        lc_status rc = validate_inputs(pl, kappa, planck, (int64_t)pl->G * pl->rays->cells, I_in,
                                       static_cast<hipStream_t>(stream));
        if (rc) return rc;
    }
    return launch_sweep(pl, kappa, planck, c_dt, state_prev, state_new, I_in, I_exit,
                        static_cast<hipStream_t>(stream));
}

lc_status lc_moments(lc_plan_t plan, const void* state, const double* I_exit, const double* I_in,
                     double c, double* E, double* F, double* f, double* bnd, void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(state, "state must not be NULL");
    LC_ARG(finite_pos(c), "c must be finite and > 0");
    LC_ARG(!bnd || (I_exit && I_in), "boundary factors need I_exit and I_in");
    return launch_moments(pl, state, I_exit, I_in, c, E, F, f, bnd, static_cast<hipStream_t>(stream));
}

lc_status lc_plan_enable_faces(lc_plan_t plan, void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    return plan_enable_faces(pl, static_cast<hipStream_t>(stream));
}

lc_status lc_sweep_points(lc_plan_t plan, const double* kappa, const double* planck, double c_dt,
                          const void* state_prev, void* state_new, const double* I_in, double* I_exit,
                          void* points, void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(kappa && planck && state_prev && state_new && I_in && points,
           "kappa, planck, states, I_in and points must not be NULL");
    LC_ARG(state_prev != state_new && points != state_prev && points != state_new,
           "state_prev, state_new and points must be distinct buffers");
    LC_ARG(finite_pos(c_dt), "c_dt must be finite and > 0");
    if (validation_on()) {
        lc_status rc = validate_inputs(pl, kappa, planck, (int64_t)pl->G * pl->rays->cells, I_in,
                                       static_cast<hipStream_t>(stream));
        if (rc) return rc;
    }
    return launch_sweep(pl, kappa, planck, c_dt, state_prev, state_new, I_in, I_exit,
                        static_cast<hipStream_t>(stream), points);
}

lc_status lc_face_moments(lc_plan_t plan, const void* points, const void* state, double c, double* E, double* F,
                          double* f, void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(points && state, "points and state must not be NULL");
    LC_ARG(finite_pos(c), "c must be finite and > 0");
    return launch_face_moments(pl, points, state, c, E, F, f, static_cast<hipStream_t>(stream));
}

lc_status lc_grey_closures(lc_plan_t plan, const double* E, const double* F, const double* f,
                           const double* kappa, const double* planck, double* out, void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(E && F && f && kappa && planck && out, "E, F, f, kappa, planck and out must not be NULL");
    return launch_grey_closures(pl, E, F, f, kappa, planck, out, static_cast<hipStream_t>(stream));
}

lc_status lc_grey_closures_dims(int32_t cells, int32_t G, const double* E, const double* F, const double* f,
                                const double* kappa, const double* planck, double* out, void* stream) {
    LC_ARG(cells >= 1 && G >= 1, "cells and G must be >= 1 (got %d, %d)", cells, G);
    LC_ARG(E && F && f && kappa && planck && out, "E, F, f, kappa, planck and out must not be NULL");
    return launch_grey_closures_dims(cells, G, E, F, f, kappa, planck, out, static_cast<hipStream_t>(stream));
}

lc_status lc_step(lc_plan_t plan, int32_t n_steps, const double* kappa, const double* planck,
                  int64_t material_stride, double c_dt, double c, void* state_a, void* state_b,
                  const double* I_in, double* I_exit, double* E, double* F, double* f, double* bnd,
                  void* stream) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(n_steps >= 1, "n_steps must be >= 1");
    LC_ARG(kappa && planck && state_a && state_b && I_in, "kappa, planck, states and I_in must not be NULL");
    LC_ARG(state_a != state_b, "state_a and state_b must be distinct buffers");
    LC_ARG(material_stride >= 0, "material_stride must be >= 0");
    LC_ARG(finite_pos(c_dt) && finite_pos(c), "c_dt and c must be finite and > 0");
    LC_ARG(!bnd || I_exit, "boundary factors need I_exit");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (validation_on()) {
        lc_status rc = validate_inputs(pl, kappa, planck,
                                       (int64_t)(n_steps - 1) * material_stride + (int64_t)pl->G * pl->rays->cells,
                                       I_in, st);
        if (rc) return rc;
    }
    uint64_t cdt_bits, c_bits;
    std::memcpy(&cdt_bits, &c_dt, 8);
    std::memcpy(&c_bits, &c, 8);
    std::vector<uintptr_t> key = {(uintptr_t)n_steps, (uintptr_t)kappa, (uintptr_t)planck,
                                  (uintptr_t)material_stride, (uintptr_t)cdt_bits, (uintptr_t)c_bits,
                                  (uintptr_t)state_a, (uintptr_t)state_b, (uintptr_t)I_in,
                                  (uintptr_t)I_exit, (uintptr_t)E, (uintptr_t)F, (uintptr_t)f,
                                  (uintptr_t)bnd};
    hipGraphExec_t exec = nullptr;
    for (auto& g : pl->graphs)
        if (g.key == key) exec = g.exec;
    if (!exec) {
        LC_HIP(hipStreamBeginCapture(pl->capture, hipStreamCaptureModeThreadLocal));
        pl->capturing = true;
        lc_status rc = LC_OK;
        for (int t = 0; t < n_steps && rc == LC_OK; ++t) {
            void* prev = (t % 2 == 0) ? state_a : state_b;
            void* next = (t % 2 == 0) ? state_b : state_a;
            rc = launch_sweep(pl, kappa + t * material_stride, planck + t * material_stride, c_dt, prev,
                              next, I_in, I_exit, pl->capture);
            if (rc == LC_OK)                          // every step forms its moments
                rc = launch_moments(pl, next, I_exit, I_in, c, E, F, f, bnd, pl->capture);
        }
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(pl->capture, &graph);
        pl->capturing = false;
        if (rc != LC_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        LC_CHECK(e == hipSuccess && graph, LC_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        LC_CHECK(e == hipSuccess, LC_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
        if (pl->graphs.size() >= 8) {
            (void)hipGraphExecDestroy(pl->graphs.front().exec);
            pl->graphs.erase(pl->graphs.begin());
        }
        pl->graphs.push_back({key, exec});
    }
    LC_HIP(hipGraphLaunch(exec, st));
    return LC_OK;
}

lc_status lc_plan_set_tuning(lc_plan_t plan, const lc_tuning_t* t) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(t, "tuning is NULL");
    LC_ARG(t->sweep_unroll == 1 || t->sweep_unroll == 2 || t->sweep_unroll == 4 || t->sweep_unroll == 8 ||
               t->sweep_unroll == 16,
           "sweep_unroll must be 1, 2, 4, 8 or 16");
    LC_ARG(t->sweep_unroll != 16 || (pl->prec == LC_F32 && pl->rays->n_pol <= kMaxPolUnroll16),
           "sweep_unroll 16 needs LC_F32 and n_pol <= %d", kMaxPolUnroll16);
    LC_ARG(t->moments_entries >= 1 && t->moments_entries <= 4, "moments_entries must be 1, 2, 3 or 4");
    LC_HIP(hipDeviceSynchronize());   // no captured step of the plan is still running
    pl->sweep_unroll = t->sweep_unroll;
    pl->moments_entries = t->moments_entries;
    for (auto& g : pl->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    pl->graphs.clear();
    return LC_OK;
}

lc_status lc_plan_set_sweep_residency(lc_plan_t plan, int32_t capped) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(capped == 0 || capped == 1, "capped must be 0 or 1");
    size_t lds = 0;
    if (capped) {
        lc_status rc = sweep_lds_bytes(&lds);
        if (rc) return rc;
    }
    LC_HIP(hipDeviceSynchronize());   // no captured step of the plan is still running
    pl->sweep_lds = lds;
    for (auto& g : pl->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    pl->graphs.clear();
    return LC_OK;
}

lc_status lc_plan_set_split(lc_plan_t plan, int32_t chunk_steps) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(chunk_steps >= 0 && chunk_steps % kSplitUnroll == 0 && chunk_steps <= (1 << 24),
           "chunk_steps must be 0 or a positive multiple of %d up to 2^24", kSplitUnroll);
    LC_HIP(hipDeviceSynchronize());   // no sweep in flight still reads the old records
    for (auto& g : pl->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    pl->graphs.clear();
    return plan_set_split(pl, chunk_steps);
}

lc_status lc_plan_set_moment_split(lc_plan_t plan, int32_t mode) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(mode >= -1 && mode <= 1, "mode must be -1 (automatic), 0 (whole) or 1 (split)");
    LC_HIP(hipDeviceSynchronize());   // no captured step of the plan is still running
    for (auto& g : pl->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    pl->graphs.clear();
    return plan_set_moment_split(pl, mode);
}

lc_status lc_plan_get_moment_split(lc_plan_t plan, int32_t* mode) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(mode, "mode is NULL");
    *mode = pl->mom_split;
    return LC_OK;
}

lc_status lc_plan_get_tuning(lc_plan_t plan, lc_tuning_t* t) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(t, "tuning is NULL");
    t->sweep_unroll = pl->sweep_unroll;
    t->moments_entries = pl->moments_entries;
    return LC_OK;
}

lc_status lc_plan_profile(lc_plan_t plan, int32_t enable) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    pl->profile = enable != 0;
    return LC_OK;
}

lc_status lc_plan_profile_read(lc_plan_t plan, double* out) {
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_ARG(out, "out is NULL");
    double acc[4] = {0, 0, 0, 0};
    int q = 0;
    for (auto* v : {&pl->ev_sweep, &pl->ev_mom}) {
        for (auto& e : *v) {
            LC_HIP(hipEventSynchronize(e.second));
            float ms = 0.f;
            LC_HIP(hipEventElapsedTime(&ms, e.first, e.second));
            acc[q] += ms;
            acc[q + 1] += 1;
        }
        q += 2;
    }
    clear_events(pl);
    for (int i = 0; i < 4; ++i) out[i] = acc[i];
    return LC_OK;
}

}  // extern "C"
