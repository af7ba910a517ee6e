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

struct SlotArgs {
    const int* bun_off;
    const int* bun_len;
    const int64_t* bun_base;
    const int* ray_off;
    const int* seg_off;
    const int* cell;
    int n_pairs, G, P, cells;
    int64_t n_bun, half;
};

__device__ __forceinline__ int find_pair(const int* __restrict__ off, int n, int64_t v) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// Visit every slot of the bundle (d, B) = block; fn(slot, j, g, p) with
// j = -1 for padding slots.
template <typename Fn>
__device__ void for_slots(const SlotArgs& A, Fn fn) {
    const int64_t w = blockIdx.x;
    const int d = w >= A.n_bun ? 1 : 0;
    const int64_t B = w - (d ? A.n_bun : 0);
    const int a = find_pair(A.bun_off, A.n_pairs, B);
    const int r0 = A.ray_off[a], Ka = A.ray_off[a + 1] - r0;
    const int64_t base = (int64_t)d * A.half + A.bun_base[B];
    const int64_t n = (int64_t)A.bun_len[B] * A.P * kWave;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {      // i = (t * 64 + lane) * P + p
        const int p = (int)(i % A.P);
        const int64_t tl = i / A.P;
        const int lane = (int)(tl & (kWave - 1));
        const int t = (int)(tl / kWave);
        const int f = (int)(B - A.bun_off[a]) * kWave + lane;
        const int kl = f / A.G, g = f - kl * A.G;
        int j = -1;
        if (kl < Ka) {
            const int k = r0 + kl;
            const int s0 = A.seg_off[k], nk = A.seg_off[k + 1] - s0;
            if (t < nk) j = s0 + (d == 0 ? t : nk - 1 - t);
        }
        fn(base + i, j, d, g, p);
    }
}

template <typename T>
__global__ void k_fill(SlotArgs A, const double* __restrict__ field, const int* __restrict__ e, T* out) {
    for_slots(A, [&](int64_t slot, int j, int d, int g, int p) {
        (void)d;
        (void)p;
        double v = 0.0;
        if (j >= 0) {
            v = field[(int64_t)g * A.cells + A.cell[j]];
            if (sizeof(T) == 4) v = ldexp(v, -e[g]);
        }
        out[slot] = (T)v;
    });
}

template <typename T>
__global__ void k_export(SlotArgs A, const T* __restrict__ in, const int* __restrict__ e, double* out) {
    for_slots(A, [&](int64_t slot, int j, int d, int g, int p) {
        if (j < 0) return;
        double v = (double)in[slot];
        if (sizeof(T) == 4) v = ldexp(v, e[g]);
        out[(((int64_t)j * 2 + d) * A.P + p) * A.G + g] = v;
    });
}

template <typename T>
__global__ void k_import(SlotArgs A, const double* __restrict__ in, const int* __restrict__ e, T* out) {
    for_slots(A, [&](int64_t slot, int j, int d, int g, int p) {
        double v = 0.0;
        if (j >= 0) {
            v = in[(((int64_t)j * 2 + d) * A.P + p) * A.G + g];
            if (sizeof(T) == 4) v = ldexp(v, -e[g]);
        }
        out[slot] = (T)v;
    });
}

// Per-group largest magnitude of canonical values [rows][G] (rows =
// segments x 2 x polar angles): block maxima in LDS, then integer atomics
// on the bit patterns of the non-negative doubles (order-independent).
__global__ void k_canon_max(const double* __restrict__ in, int64_t rows, int G, int64_t rows_per_block,
                            unsigned long long* gmax) {
    extern __shared__ unsigned long long sm[];
    for (int g = threadIdx.x; g < G; g += blockDim.x) sm[g] = 0ull;
    __syncthreads();
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = r0 + rows_per_block < rows ? r0 + rows_per_block : rows;
    for (int64_t i = r0 * G + threadIdx.x; i < r1 * G; i += blockDim.x) {
        const double v = fabs(in[i]);
        atomicMax(&sm[i % G], (unsigned long long)__double_as_longlong(v));
    }
    __syncthreads();
    for (int g = threadIdx.x; g < G; g += blockDim.x)
        if (sm[g]) atomicMax(&gmax[g], sm[g]);
}

__global__ void k_scale_from_max(const unsigned long long* gmax, int G, int* e) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const double m = __longlong_as_double((long long)gmax[g]);
    e[g] = (m > 0.0 && isfinite(m)) ? ilogb(m) + 1 : 0;
}

__global__ void k_zero_u64s(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void k_zero_int(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

namespace {
SlotArgs slot_args(Plan* pl) {
    Rays* r = pl->rays;
    SlotArgs A{};
    A.bun_off = pl->d_bun_off;
    A.bun_len = pl->d_bun_len;
    A.bun_base = pl->d_bun_base;
    A.ray_off = r->d_ray_off;
    A.seg_off = r->d_seg_off;
    A.cell = r->d_cell;
    A.n_pairs = r->n_pairs;
    A.G = pl->G;
    A.P = r->n_pol;
    A.cells = r->cells;
    A.n_bun = pl->n_bun;
    A.half = pl->half_elems;
    return A;
}
}  // namespace

lc_status launch_state_fill(Plan* pl, const double* field, void* state, hipStream_t st) {
    Rays* r = pl->rays;
    const int G = pl->G;
    int* e = static_cast<int*>(state);
    const SlotArgs A = slot_args(pl);
    const unsigned nb = (unsigned)(2 * pl->n_bun);
    if (pl->prec == LC_F32) {
        float* v = static_cast<float*>(state_values(pl, state));
        hipLaunchKernelGGL(k_field_scale, dim3(G), dim3(kBlock), 0, st, field, r->cells, e);
        hipLaunchKernelGGL(k_fill<float>, dim3(nb), dim3(kBlock), 0, st, A, field, e, v);
    } else {
        double* v = static_cast<double*>(state_values(pl, state));
        hipLaunchKernelGGL(k_zero_int, dim3((G + kBlock - 1) / kBlock), dim3(kBlock), 0, st, e, G);
        hipLaunchKernelGGL(k_fill<double>, dim3(nb), dim3(kBlock), 0, st, A, field, e, v);
    }
    LC_HIP(hipGetLastError());
    return LC_OK;
}

lc_status launch_state_import(Plan* pl, const double* in, void* state, hipStream_t st) {
    Rays* r = pl->rays;
    const int G = pl->G;
    int* e = static_cast<int*>(state);
    const SlotArgs A = slot_args(pl);
    const unsigned nb = (unsigned)(2 * pl->n_bun);
    const unsigned gb = (unsigned)((G + kBlock - 1) / kBlock);
    if (pl->prec == LC_F32) {
        const int64_t rows = r->n_seg * 2 * r->n_pol;
        const int64_t rpb = 1024;
        const int64_t blocks = (rows + rpb - 1) / rpb;
        LC_CHECK(blocks < INT32_MAX, LC_ERR_UNSUPPORTED, "state too large to import");
        hipLaunchKernelGGL(k_zero_u64s, dim3(gb), dim3(kBlock), 0, st, pl->d_gmax, G);
        if (blocks > 0)
            hipLaunchKernelGGL(k_canon_max, dim3((unsigned)blocks), dim3(kBlock), (size_t)G * sizeof(unsigned long long),
                               st, in, rows, G, rpb, pl->d_gmax);
        hipLaunchKernelGGL(k_scale_from_max, dim3(gb), dim3(kBlock), 0, st, pl->d_gmax, G, e);
        hipLaunchKernelGGL(k_import<float>, dim3(nb), dim3(kBlock), 0, st, A, in, e,
                           static_cast<float*>(state_values(pl, state)));
    } else {
        hipLaunchKernelGGL(k_zero_int, dim3(gb), dim3(kBlock), 0, st, e, G);
        hipLaunchKernelGGL(k_import<double>, dim3(nb), dim3(kBlock), 0, st, A, in, e,
                           static_cast<double*>(state_values(pl, state)));
    }
    LC_HIP(hipGetLastError());
    return LC_OK;
}

lc_status launch_state_export(Plan* pl, const void* state, double* out, hipStream_t st) {
    const int* e = static_cast<const int*>(state);
    const SlotArgs A = slot_args(pl);
    const unsigned nb = (unsigned)(2 * pl->n_bun);
    if (pl->prec == LC_F32)
        hipLaunchKernelGGL(k_export<float>, dim3(nb), dim3(kBlock), 0, st, A,
                           static_cast<const float*>(state_values(pl, state)), e, out);
    else
        hipLaunchKernelGGL(k_export<double>, dim3(nb), dim3(kBlock), 0, st, A,
                           static_cast<const double*>(state_values(pl, state)), e, out);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

}  // namespace lc
