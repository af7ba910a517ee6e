// Prologue of a transport step: the cell coefficients of eq. (11) and, in
// float32, the per-group power-of-two scale of the new state.
//
// Two launches, both reading their inputs once with coalesced loads:
//   * k_group_max: the largest |B| and |I_in| of every group, reduced in LDS
//     and merged with integer atomics on the bit patterns of non-negative
//     doubles (whose order is the order of the values), so the result is
//     exact and independent of scheduling.  The incoming intensities do not
//     change within one call, so their maxima are taken at its first step
//     only and kept apart for the later ones;
//   * k_coef: per tile of cells x groups, reads kappa and B in their
//     [G][cells] layout, forms (kappa_t, a) and writes the [cells][G] table
//     through an LDS transpose; it also derives the new exponents.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "lc_internal.hpp"

namespace lc {
namespace {

constexpr int kMaxChunk = 8192;   // elements per block of k_group_max
constexpr int kCoefTile = 1024;   // cells x groups per block of k_coef

struct CoefArgs {
    const double* kappa;     // step t at kappa + t * stride, [G][cells]
    const double* planck;
    int64_t stride;
    double c_dt;
    int cells, G;
    int64_t n_in;            // nb * M rows of G
    const double* I_in;
    const int* e_state[2];   // headers of state_a, state_b
    void* coef;              // Coef<T> [cells][G]
    unsigned long long* gmax;// [G] maxima of |B| as bit patterns (zeroed before the step)
    unsigned long long* gmax_in; // [G] maxima of |I_in| (zeroed before the first step of a call)
    int gt, ct;              // k_coef tile: gt groups x ct cells
    int64_t pl_blocks;       // k_group_max blocks over B (the rest cover I_in)
    int64_t max_blk_off;     // first block of this problem in a batched k_group_max
    int64_t coef_blk_off;    // first block of this problem in a batched k_coef
    int64_t g_off;           // first entry of this problem in a batch's maxima
};

// I_in rows per block of k_group_max: about kMaxChunk values, whole rows.
__host__ __device__ __forceinline__ int64_t in_rows_per_block(int G) { return G >= kMaxChunk ? 1 : kMaxChunk / G; }

__device__ __forceinline__ unsigned long long bits_of(double v) {
    return (unsigned long long)__double_as_longlong(v);
}

// Block b of the maxima of one problem at step `step`.  Blocks below
// pl_blocks take a run of one group's B row; the others take whole rows of the
// [nb*M][G] I_in array, each thread reducing one group in registers (G up to
// the block size) before one LDS merge per thread.  Values that are not
// finite are skipped.
__device__ __forceinline__ void group_max_block(const CoefArgs& A, int64_t b, int step, int t,
                                                unsigned long long* smax) {
    const int G = A.G;
    if (b < A.pl_blocks) {
        const int64_t per_g = (A.cells + kMaxChunk - 1) / kMaxChunk;
        const int g = (int)(b / per_g);
        const int64_t i0 = (b - (int64_t)g * per_g) * kMaxChunk;
        const int64_t i1 = min((int64_t)A.cells, i0 + kMaxChunk);
        const double* row = A.planck + (int64_t)step * A.stride + (int64_t)g * A.cells;
        // eight independent loads in flight per thread
        double m = 0.0;
        for (int64_t ib = i0 + t; ib < i1; ib += 8 * kBlock) {
            double v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int64_t i = ib + (int64_t)j * kBlock;
                v[j] = i < i1 ? fabs(row[i]) : 0.0;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (isfinite(v[j])) m = fmax(m, v[j]);
        }
        for (int o = kWave / 2; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
        if ((t & (kWave - 1)) == 0 && m > 0.0) atomicMax(&A.gmax[g], bits_of(m));
        return;
    }
    if (step > 0) return;              // I_in maxima: taken at the first step of the call
    for (int g = t; g < G; g += kBlock) smax[g] = 0ull;
    __syncthreads();
    // rows [r0, r1) of the [nb*M][G] I_in array
    const int64_t rpb = in_rows_per_block(G);
    const int64_t r0 = (b - A.pl_blocks) * rpb;
    const int64_t r1 = min(A.n_in, r0 + rpb);
    if (G <= kBlock) {
        // thread t keeps the maximum of group t % G over every R-th row
        const int R = kBlock / G;
        if (t < R * G) {
            const int g = t % G;
            double m = 0.0;
            for (int64_t rb = r0 + t / G; rb < r1; rb += 8 * (int64_t)R) {
                double v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int64_t r = rb + (int64_t)j * R;
                    v[j] = r < r1 ? fabs(A.I_in[r * G + g]) : 0.0;
                }
#pragma unroll
                for (int j = 0; j < 8; ++j)
                    if (isfinite(v[j])) m = fmax(m, v[j]);
            }
            if (m > 0.0) atomicMax(&smax[g], bits_of(m));
        }
    } else {
        for (int64_t r = r0; r < r1; ++r)
            for (int g = t; g < G; g += kBlock) {
                const double v = fabs(A.I_in[r * G + g]);
                if (isfinite(v) && v > 0.0) atomicMax(&smax[g], bits_of(v));
            }
    }
    __syncthreads();
    for (int q = t; q < G; q += kBlock)
        if (smax[q]) atomicMax(&A.gmax_in[q], smax[q]);
}

// Block b of the coefficients of one problem: groups [g0, g0 + gt) of cells
// [c0, c0 + ct).  Step t reads state (t even ? a : b) and writes the other.
template <typename T>
__device__ __forceinline__ void coef_block(const CoefArgs& A, int64_t b, int step, int t, char* lds) {
    const int G = A.G, cells = A.cells;
    const int g_tiles = (G + A.gt - 1) / A.gt;
    const int64_t ctile = b / g_tiles;
    const int g0 = (int)(b - ctile * g_tiles) * A.gt;
    const int64_t c0 = ctile * A.ct;
    const int ng = min(A.gt, G - g0);
    const int nc = (int)min((int64_t)A.ct, cells - c0);
    int* s_e = reinterpret_cast<int*>(lds);
    Coef<T>* sc = reinterpret_cast<Coef<T>*>(lds + ((size_t)kCoefTile * sizeof(int)));
    if (sizeof(T) == 4) {
        const int* e_prev = A.e_state[step & 1];
        int* e_new = const_cast<int*>(A.e_state[(step + 1) & 1]);
        for (int q = t; q < ng; q += kBlock) {
            int e = e_prev[g0 + q];
            const unsigned long long mb = max(A.gmax[g0 + q], A.gmax_in[g0 + q]);
            const double m = __longlong_as_double((long long)mb);
            if (m > 0.0 && isfinite(m)) e = max(e, ilogb(m) + 1);
            s_e[q] = e;
            if (c0 == 0) e_new[g0 + q] = e;
        }
        __syncthreads();
    }
    const double* kap = A.kappa + (int64_t)step * A.stride;
    const double* pla = A.planck + (int64_t)step * A.stride;
    const double inv_cdt = 1.0 / A.c_dt;
    for (int idx = t; idx < ng * nc; idx += kBlock) {
        const int q = idx / nc;
        const int c = idx - q * nc;
        const int64_t li = (int64_t)(g0 + q) * cells + c0 + c;
        const double k = kap[li];
        const double kt = k + inv_cdt;
        double a = k * pla[li] / kt;
        if (sizeof(T) == 4) a = ldexp(a, -s_e[q]);
        Coef<T> r;
        r.kt = (T)kt;
        r.a = (T)a;
        sc[c * ng + q] = r;
    }
    __syncthreads();
    Coef<T>* out = static_cast<Coef<T>*>(A.coef);
    for (int idx = t; idx < ng * nc; idx += kBlock) {
        const int c = idx / ng;
        const int q = idx - c * ng;
        out[(c0 + c) * G + g0 + q] = sc[idx];
    }
}

__global__ __launch_bounds__(kBlock) void k_group_max(CoefArgs A) {
    extern __shared__ unsigned long long smax[];
    group_max_block(A, blockIdx.x, 0, threadIdx.x, smax);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coef(CoefArgs A, int step) {
    extern __shared__ char lds[];
    coef_block<T>(A, blockIdx.x, step, threadIdx.x, lds);
}

__device__ __forceinline__ int find_block(const CoefArgs* __restrict__ P, int n, int64_t v, bool coef) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((coef ? P[mid].coef_blk_off : P[mid].max_blk_off) <= v) lo = mid; else hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kBlock) void k_group_max_batch(const CoefArgs* __restrict__ P, int n, int step) {
    extern __shared__ unsigned long long smax[];
    const int q = find_block(P, n, blockIdx.x, false);
    group_max_block(P[q], blockIdx.x - P[q].max_blk_off, step, threadIdx.x, smax);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coef_batch(const CoefArgs* __restrict__ P, int n, int step) {
    extern __shared__ char lds[];
    const int q = find_block(P, n, blockIdx.x, true);
    coef_block<T>(P[q], blockIdx.x - P[q].coef_blk_off, step, threadIdx.x, lds);
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <typename T> size_t coef_lds() { return (size_t)kCoefTile * sizeof(int) + (size_t)kCoefTile * sizeof(Coef<T>); }

CoefArgs coef_args(const Plan* pl, double c_dt, const double* kappa, const double* planck, int64_t stride,
                   const void* state_a, const void* state_b, const double* I_in, unsigned long long* gmax,
                   unsigned long long* gmax_in) {
    const Rays* r = pl->rays;
    CoefArgs C{};
    C.kappa = kappa;
    C.planck = planck;
    C.stride = stride;
    C.c_dt = c_dt;
    C.cells = r->cells;
    C.G = pl->G;
    C.n_in = (int64_t)r->nb * r->n_az * r->n_pol;
    C.I_in = I_in;
    C.e_state[0] = static_cast<const int*>(state_a);
    C.e_state[1] = static_cast<const int*>(state_b);
    C.coef = pl->d_coef;
    C.gmax = gmax;
    C.gmax_in = gmax_in;
    C.gt = std::min(pl->G, kCoefTile);
    C.ct = std::max(1, kCoefTile / C.gt);
    C.pl_blocks = (int64_t)pl->G * ((r->cells + kMaxChunk - 1) / kMaxChunk);
    return C;
}

int64_t max_blocks(const CoefArgs& C) {
    const int64_t rpb = in_rows_per_block(C.G);
    return C.pl_blocks + (C.n_in + rpb - 1) / rpb;
}
int64_t coef_blocks(const CoefArgs& C) {
    return ((int64_t)C.cells + C.ct - 1) / C.ct * ((C.G + C.gt - 1) / C.gt);
}

}  // namespace

size_t coef_args_bytes() { return sizeof(CoefArgs); }

// Prologue of one problem (lc_sweep / lc_step): the float32 scale of the new
// state in its header, then the coefficient table.
lc_status launch_prologue(Plan* pl, const double* kappa, const double* planck, double c_dt,
                          const void* state_prev, void* state_new, const double* I_in, hipStream_t st,
                          void* coef, unsigned long long* gmax) {
    const bool f32 = pl->prec == LC_F32;
    // the kernels index the state headers by step parity: step 0 reads e_state[0]
    // gmax holds the |B| maxima, then the |I_in| maxima; a single step is
    // the first of its call, so both are formed
    CoefArgs C = coef_args(pl, c_dt, kappa, planck, 0, state_prev, state_new, I_in, gmax, gmax + pl->G);
    C.coef = coef;
    if (f32) {
        hipLaunchKernelGGL(k_zero_u64, dim3(blocks_for(2 * (int64_t)pl->G)), dim3(kBlock), 0, st, gmax,
                           2 * (int64_t)pl->G);
        hipLaunchKernelGGL(k_group_max, dim3((unsigned)max_blocks(C)), dim3(kBlock),
                           (size_t)pl->G * sizeof(unsigned long long), st, C);
        hipLaunchKernelGGL(k_coef<float>, dim3((unsigned)coef_blocks(C)), dim3(kBlock), coef_lds<float>(), st, C, 0);
    } else {
        hipLaunchKernelGGL(k_coef<double>, dim3((unsigned)coef_blocks(C)), dim3(kBlock), coef_lds<double>(), st, C,
                           0);
    }
    LC_HIP(hipGetLastError());
    return LC_OK;
}

// Host record of one problem of a batch; returns its block counts.
void make_coef_args(Plan* pl, double c_dt, const double* kappa, const double* planck, int64_t stride,
                    void* state_a, void* state_b, const double* I_in, unsigned long long* gmax,
                    unsigned long long* gmax_in, int64_t max_blk_off, int64_t coef_blk_off, int64_t g_off, void* out,
                    int64_t* n_max_blocks, int64_t* n_coef_blocks) {
    CoefArgs C = coef_args(pl, c_dt, kappa, planck, stride, state_a, state_b, I_in, gmax + g_off, gmax_in + g_off);
    C.max_blk_off = max_blk_off;
    C.coef_blk_off = coef_blk_off;
    C.g_off = g_off;
    *n_max_blocks = max_blocks(C);
    *n_coef_blocks = coef_blocks(C);
    std::memcpy(out, &C, sizeof(C));
}

// Prologue of step t of a batch.  gmax holds the |B| maxima of every
// problem (n_gmax entries) followed by their |I_in| maxima, which are
// cleared and formed at the first step of a call only.
lc_status launch_prologue_batch(int prec, const void* coef_args, int n, int64_t max_blocks_all,
                                int64_t coef_blocks_all, int max_G, unsigned long long* gmax, int64_t n_gmax, int t,
                                hipStream_t st) {
    const CoefArgs* P = static_cast<const CoefArgs*>(coef_args);
    if (prec == LC_F32) {
        const int64_t nz = t == 0 ? 2 * n_gmax : n_gmax;
        hipLaunchKernelGGL(k_zero_u64, dim3(blocks_for(nz)), dim3(kBlock), 0, st, gmax, nz);
        hipLaunchKernelGGL(k_group_max_batch, dim3((unsigned)max_blocks_all), dim3(kBlock),
                           (size_t)max_G * sizeof(unsigned long long), st, P, n, t);
        hipLaunchKernelGGL(k_coef_batch<float>, dim3((unsigned)coef_blocks_all), dim3(kBlock), coef_lds<float>(), st,
                           P, n, t);
    } else {
        hipLaunchKernelGGL(k_coef_batch<double>, dim3((unsigned)coef_blocks_all), dim3(kBlock), coef_lds<double>(),
                           st, P, n, t);
    }
    LC_HIP(hipGetLastError());
    return LC_OK;
}

}  // namespace lc
