// Cell-local grey closures of the effective grey problem, eq. (8)-(9), and
// the Planck-weighted mean opacity of eq. (5a), formed from the multigroup
// cell moments of a sweep.  A wavefront takes 8 consecutive cells, 8 lanes
// to a cell; lane j of a cell sums the groups j, j + 8, j + 16, ... in
// increasing order, and the 8 partial sums are combined by a fixed butterfly
// -- deterministic, no atomics.  With this split both layouts are read in
// whole 64-byte sectors: a cell's 8 consecutive groups of the cell-major
// moments, and 8 consecutive cells of one group row of the [G][cells]
// opacity and Planck source.
#include <cmath>

#include "lc_internal.hpp"

namespace lc {
namespace {

struct GreyArgs {
    int cells, G;
    const double* E;        // [cells][G]
    const double* F;        // [cells][2][G]
    const double* f;        // [cells][4][G]
    const double* kappa;    // [G][cells]
    const double* planck;   // [G][cells]
    double* out;            // [13][cells]
};

constexpr int kLanesPerCell = 8;
constexpr int kGreyFields = 13;

// Sum over the 8 lanes of a cell; every one of them gets the total.
__device__ __forceinline__ double cell_sum(double v) {
#pragma unroll
    for (int o = 1; o < kLanesPerCell; o <<= 1) v += __shfl_xor(v, o);
    return v;
}

__global__ __launch_bounds__(kBlock) void k_grey_closures(GreyArgs A) {
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t i = t / kLanesPerCell;                  // cell
    const int j = (int)(t % kLanesPerCell);               // first group of this lane
    const bool live = i < A.cells;                        // all 8 lanes of a cell agree
    const int G = A.G;
    const size_t cells = (size_t)A.cells;
    const int64_t ic = live ? i : 0;
    const gptr<const double> E = as_global(A.E + (size_t)ic * G);
    const gptr<const double> Fx = as_global(A.F + (size_t)ic * 2 * G);
    const gptr<const double> Fy = Fx + G;
    const gptr<const double> f = as_global(A.f + (size_t)ic * 4 * G);
    const gptr<const double> kap = as_global(A.kappa + ic);
    const gptr<const double> B = as_global(A.planck + ic);
    enum { sE, sB, sFx, sFy, sk, skE, skB, saFx, saFy, skFx, skFy, sfxx, sfxy, sfyy, sfzz, kSums };
    double v[kSums];
#pragma unroll
    for (int q = 0; q < kSums; ++q) v[q] = 0.0;
    const int g0 = live ? j : G;
    for (int g = g0; g < G; g += kLanesPerCell) {
        const double e = E[g], fx = Fx[g], fy = Fy[g];
        const double k = kap[g * cells], b = B[g * cells];
        v[sE] += e;
        v[sB] += b;
        v[sFx] += fx;
        v[sFy] += fy;
        v[sk] += k;
        v[skE] += k * e;
        v[skB] += k * b;
        v[saFx] += fabs(fx);
        v[saFy] += fabs(fy);
        v[skFx] += k * fabs(fx);
        v[skFy] += k * fabs(fy);
#pragma unroll
        for (int c = 0; c < 4; ++c) v[sfxx + c] += f[(size_t)c * G + g] * e;
    }
#pragma unroll
    for (int q = 0; q < kSums; ++q) v[q] = cell_sum(v[q]);
    // averages; a zero denominator takes the documented fallback
    const double kB_raw = v[sB] > 0.0 ? v[skB] / v[sB] : 0.0;
    const double kE = v[sE] > 0.0 ? v[skE] / v[sE] : (v[sB] > 0.0 ? kB_raw : v[sk] / G);
    const double kB = v[sB] > 0.0 ? kB_raw : kE;
    const double kFx = v[saFx] > 0.0 ? v[skFx] / v[saFx] : kE;
    const double kFy = v[saFy] > 0.0 ? v[skFy] / v[saFy] : kE;
    double ex = 0.0, ey = 0.0;                            // sum_g (kappa_g - K_R,aa) F_a,g
    for (int g = g0; g < G; g += kLanesPerCell) {
        const double k = kap[g * cells];
        ex += (k - kFx) * Fx[g];
        ey += (k - kFy) * Fy[g];
    }
    ex = cell_sum(ex);
    ey = cell_sum(ey);
    if (!live) return;
    const double sum_E = v[sE];
    const double iso[4] = {1.0 / 3, 0.0, 1.0 / 3, 1.0 / 3};
    double r[16] = {sum_E, v[sFx], v[sFy], kE, kB, kFx, kFy, sum_E > 0.0 ? ex / sum_E : 0.0,
                    sum_E > 0.0 ? ey / sum_E : 0.0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int c = 0; c < 4; ++c) r[9 + c] = sum_E > 0.0 ? v[sfxx + c] / sum_E : iso[c];
    // lane j of the cell stores fields j and j + 8: each field row gets 8
    // consecutive cells from a wavefront
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int c = 0; c < kLanesPerCell; ++c)
        if (j == c) {
            a0 = r[c];
            a1 = r[c + kLanesPerCell];
        }
    const gptr<double> o = as_global_w(A.out + i);
    o[(size_t)j * cells] = a0;
    if (j + kLanesPerCell < kGreyFields) o[(size_t)(j + kLanesPerCell) * cells] = a1;
}

}  // namespace

lc_status launch_grey_closures(const Plan* pl, const double* E, const double* F, const double* f,
                               const double* kappa, const double* planck, double* out, hipStream_t st) {
    return launch_grey_closures_dims(pl->rays->cells, pl->G, E, F, f, kappa, planck, out, st);
}

lc_status launch_grey_closures_dims(int cells, int G, const double* E, const double* F, const double* f,
                                    const double* kappa, const double* planck, double* out, hipStream_t st) {
    GreyArgs A;
    A.cells = cells;
    A.G = G;
    A.E = E;
    A.F = F;
    A.f = f;
    A.kappa = kappa;
    A.planck = planck;
    A.out = out;
    const int64_t threads = (int64_t)A.cells * kLanesPerCell;
    hipLaunchKernelGGL(k_grey_closures, dim3((unsigned)((threads + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, A);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

}  // namespace lc
