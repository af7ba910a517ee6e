// Per-segment state buffers: initial fill from a cell field (eq. (2)) and
// export in the canonical [j][d][p][g] float64 order.  A float32 state keeps a
// per-group power-of-two exponent in its header; values are stored divided by
// 2^e (an exact rescaling).
#include <cmath>

#include "lc_internal.hpp"

namespace lc {
namespace {

__global__ void k_field_scale(const double* __restrict__ field, int cells, int* e) {
    __shared__ double sh[kBlock];
    const int g = blockIdx.x;
    double m = 0.0;
    for (int i = threadIdx.x; i < cells; i += kBlock) m = fmax(m, fabs(field[(int64_t)g * cells + i]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) e[g] = (sh[0] > 0.0 && isfinite(sh[0])) ? ilogb(sh[0]) + 1 : 0;
}

template <typename T>
__global__ void k_fill(const double* __restrict__ field, const int* __restrict__ cell, int cells,
                       int64_t n, int PG2, int G, const int* __restrict__ e, T* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = i / PG2;
    const int g = (int)(i % G);
    double v = field[(int64_t)g * cells + cell[j]];
    if (sizeof(T) == 4) v = ldexp(v, -e[g]);
    out[i] = (T)v;
}

template <typename T>
__global__ void k_export(const T* __restrict__ in, int64_t n, int G, const int* __restrict__ e,
                         double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = (double)in[i];
    if (sizeof(T) == 4) v = ldexp(v, e[i % G]);
    out[i] = v;
}

__global__ void k_zero_int(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

lc_status launch_state_fill(Plan* pl, const double* field, void* state, hipStream_t st) {
    Rays* r = pl->rays;
    const int G = pl->G;
    const int64_t n = r->n_seg * 2 * r->n_pol * G;
    int* e = static_cast<int*>(state);
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    if (pl->prec == LC_F32) {
        hipLaunchKernelGGL(k_field_scale, dim3(G), dim3(kBlock), 0, st, field, r->cells, e);
        hipLaunchKernelGGL(k_fill<float>, dim3(nb), dim3(kBlock), 0, st, field, r->d_cell, r->cells, n,
                           2 * r->n_pol * G, G, e, static_cast<float*>(state_values(pl, state)));
    } else {
        hipLaunchKernelGGL(k_zero_int, dim3((G + kBlock - 1) / kBlock), dim3(kBlock), 0, st, e, G);
        hipLaunchKernelGGL(k_fill<double>, dim3(nb), dim3(kBlock), 0, st, field, r->d_cell, r->cells, n,
                           2 * r->n_pol * G, G, e, static_cast<double*>(state_values(pl, state)));
    }
    LC_HIP(hipGetLastError());
    return LC_OK;
}

lc_status launch_state_export(Plan* pl, const void* state, double* out, hipStream_t st) {
    Rays* r = pl->rays;
    const int G = pl->G;
    const int64_t n = r->n_seg * 2 * r->n_pol * G;
    const int* e = static_cast<const int*>(state);
    const unsigned nb = (unsigned)((n + kBlock - 1) / kBlock);
    if (pl->prec == LC_F32)
        hipLaunchKernelGGL(k_export<float>, dim3(nb), dim3(kBlock), 0, st,
                           static_cast<const float*>(state_values(pl, state)), n, G, e, out);
    else
        hipLaunchKernelGGL(k_export<double>, dim3(nb), dim3(kBlock), 0, st,
                           static_cast<const double*>(state_values(pl, state)), n, G, e, out);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

}  // namespace lc
