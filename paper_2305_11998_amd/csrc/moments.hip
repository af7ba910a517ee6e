// Angular moments of the swept state, eq. (7), (14)-(16), and boundary
// factors.  Each lane owns one (cell, group) -- or (boundary face, group) --
// and gathers its segments in a fixed order (the cell-major lists built with
// the characteristic grid), so the sums are deterministic and need no atomics.
// The float32 form accumulates with compensated (Kahan) sums and divides in
// float64.
#include <cmath>

#include "lc_internal.hpp"

namespace lc {
namespace {

struct MomArgs {
    const int* csr_off;
    const int* csr_ray;     // ray of each entry
    const int2* csr_t;      // its step in the d = 0 and d = 1 traversal
    const void* csr_w;      // double or float
    const int* ray_off;
    const int* bun_off;
    const int64_t* bun_base;
    int64_t half;
    const double* dirw;     // [n_pairs][2][P][kDirW]
    const void* state;      // values
    const int* e;           // per-group exponents of the state (float32 only)
    int cells, G, n_pairs;
    double inv_c;
    double* E;
    double* F;
    double* f;
};

template <typename T> struct Acc;
template <> struct Acc<double> {
    double s = 0.0;
    __device__ void add(double v) { s += v; }
    __device__ double value() const { return s; }
};
template <> struct Acc<float> {
    float s = 0.f, c = 0.f;
    __device__ void add(float v) {        // Kahan summation
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ double value() const { return (double)s - (double)c; }
};

template <typename T, int P>
__global__ __launch_bounds__(kBlock) void k_cell_moments(MomArgs A) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = A.G;
    if (lane >= (int64_t)A.cells * G) return;
    const int cell = (int)(lane / G);
    const int g = (int)(lane - (int64_t)cell * G);
    const T* __restrict__ st = static_cast<const T*>(A.state);
    const T* __restrict__ cw = static_cast<const T*>(A.csr_w);
    Acc<T> acc[7];
    for (int a = 0; a < A.n_pairs; ++a) {
        const int e0 = A.csr_off[(size_t)cell * A.n_pairs + a];
        const int e1 = A.csr_off[(size_t)cell * A.n_pairs + a + 1];
        const int r0 = A.ray_off[a];
        const int b0 = A.bun_off[a];
        T Iim[2 * P];
#pragma unroll
        for (int q = 0; q < 2 * P; ++q) Iim[q] = (T)0;
        for (int e = e0; e < e1; ++e) {
            const int k = A.csr_ray[e];
            const int2 tt = A.csr_t[e];
            const T w = cw[e];
            // bundle-major state: lane f = (k - r0) G + g of bundle b0 + f / 64
            const int f = (k - r0) * G + g;
            const T* row = st + (size_t)A.bun_base[b0 + f / kWave] + (f & (kWave - 1));
            const T* r0p = row + (size_t)tt.x * P * kWave;
            const T* r1p = row + (size_t)A.half + (size_t)tt.y * P * kWave;
#pragma unroll
            for (int p = 0; p < P; ++p) {
                Iim[p] += w * __builtin_nontemporal_load(r0p + p * kWave);
                Iim[P + p] += w * __builtin_nontemporal_load(r1p + p * kWave);
            }
        }
#pragma unroll
        for (int q = 0; q < 2 * P; ++q) {
            const double* dw = A.dirw + ((size_t)a * 2 * P + q) * kDirW;   // q = d * P + p
#pragma unroll
            for (int c = 0; c < 7; ++c) acc[c].add((T)dw[c] * Iim[q]);
        }
    }
    double sc = 1.0;
    if (sizeof(T) == 4) sc = ldexp(1.0, A.e[g]);
    const double Phi = acc[0].value() * sc;
    const size_t o = (size_t)g * A.cells + cell;
    if (A.E) A.E[o] = Phi * A.inv_c;
    if (A.F) {
        A.F[((size_t)g * 2 + 0) * A.cells + cell] = acc[1].value() * sc;
        A.F[((size_t)g * 2 + 1) * A.cells + cell] = acc[2].value() * sc;
    }
    if (A.f) {
        const bool z = Phi == 0.0;
        const double inv = z ? 0.0 : 1.0 / Phi;
        A.f[((size_t)g * 4 + 0) * A.cells + cell] = z ? 1.0 / 3 : acc[3].value() * sc * inv;
        A.f[((size_t)g * 4 + 1) * A.cells + cell] = z ? 0.0 : acc[4].value() * sc * inv;
        A.f[((size_t)g * 4 + 2) * A.cells + cell] = z ? 1.0 / 3 : acc[5].value() * sc * inv;
        A.f[((size_t)g * 4 + 3) * A.cells + cell] = z ? 1.0 / 3 : acc[6].value() * sc * inv;
    }
}

struct BndArgs {
    const int* bmap;        // [nb][n_pairs][2][2]
    const double* width;
    const double* dirw;
    const double* I_exit;   // [n_rays][2][P][G]
    const double* I_in;     // [nb][M][G]
    int nx, ny, nb, G, n_pairs, n_az, P;
    double* bnd;            // [G][nb][8]
};

// Boundary factors per (face b, group g): the outgoing intensity of a
// direction is the width-weighted mean exit intensity of the characteristics
// leaving through b; incoming directions take I_in.
__global__ __launch_bounds__(kBlock) void k_boundary(BndArgs A) {
    const int lane = blockIdx.x * blockDim.x + threadIdx.x;
    const int G = A.G;
    if (lane >= A.nb * G) return;
    const int b = lane / G;
    const int g = lane - b * G;
    const int P = A.P;
    const int M = A.n_az * P;
    double nxv = 0, nyv = 0;
    if (b < A.ny) nxv = -1;
    else if (b < 2 * A.ny) nxv = 1;
    else if (b < 2 * A.ny + A.nx) nyv = -1;
    else nyv = 1;
    double Pp = 0, Jp = 0, Pm = 0, Jm = 0, S = 0, Sxx = 0, Sxy = 0, Syy = 0, wo = 0, wodn = 0;
    for (int a = 0; a < A.n_pairs; ++a) {
        for (int d = 0; d < 2; ++d) {
            const int* bm = A.bmap + ((size_t)(b * A.n_pairs + a) * 2 + d) * 2;
            const int k0 = bm[0], k1 = bm[1];
            double wsum = 0.0;
            if (k0 >= 0)
                for (int k = k0; k < k1; ++k) wsum += A.width[k];
            for (int p = 0; p < P; ++p) {
                const double* dw = A.dirw + ((size_t)(a * 2 + d) * P + p) * kDirW;
                const double om = dw[0];
                const double odn = dw[7] * nxv + dw[8] * nyv;
                double I;
                if (k0 >= 0) {
                    double acc = 0.0;
                    for (int k = k0; k < k1; ++k)
                        acc += A.width[k] * A.I_exit[((size_t)(2 * k + d) * P + p) * G + g];
                    I = acc / wsum;
                    Pp += om * I;
                    Jp += om * odn * I;
                    wo += om;
                    wodn += om * odn;
                } else {
                    const int m = (a + d * (A.n_az >> 1)) * P + p;
                    I = A.I_in[((size_t)b * M + m) * G + g];
                    Pm += om * I;
                    Jm += om * fabs(odn) * I;
                }
                S += om * I;
                Sxx += dw[3] * I;
                Sxy += dw[4] * I;
                Syy += dw[5] * I;
            }
        }
    }
    double* out = A.bnd + ((size_t)g * A.nb + b) * 8;
    out[0] = Pp;
    out[1] = Jp;
    out[2] = Pm;
    out[3] = Jm;
    out[4] = Pp > 0.0 ? Jp / Pp : wodn / wo;
    const bool z = S == 0.0;
    out[5] = z ? 1.0 / 3 : Sxx / S;
    out[6] = z ? 0.0 : Sxy / S;
    out[7] = z ? 1.0 / 3 : Syy / S;
}

template <typename T>
lc_status launch_cell_moments_p(int P, const MomArgs& A, hipStream_t st) {
    const int64_t lanes = (int64_t)A.cells * A.G;
    dim3 grid((unsigned)((lanes + kBlock - 1) / kBlock)), block(kBlock);
    switch (P) {
        case 1: hipLaunchKernelGGL((k_cell_moments<T, 1>), grid, block, 0, st, A); break;
        case 2: hipLaunchKernelGGL((k_cell_moments<T, 2>), grid, block, 0, st, A); break;
        case 3: hipLaunchKernelGGL((k_cell_moments<T, 3>), grid, block, 0, st, A); break;
        case 4: hipLaunchKernelGGL((k_cell_moments<T, 4>), grid, block, 0, st, A); break;
        case 5: hipLaunchKernelGGL((k_cell_moments<T, 5>), grid, block, 0, st, A); break;
        case 6: hipLaunchKernelGGL((k_cell_moments<T, 6>), grid, block, 0, st, A); break;
        case 7: hipLaunchKernelGGL((k_cell_moments<T, 7>), grid, block, 0, st, A); break;
        case 8: hipLaunchKernelGGL((k_cell_moments<T, 8>), grid, block, 0, st, A); break;
        default:
            set_error("n_pol = %d not supported (1..8)", P);
            return LC_ERR_UNSUPPORTED;
    }
    LC_HIP(hipGetLastError());
    return LC_OK;
}

}  // namespace

lc_status launch_moments(Plan* pl, const void* state, const double* I_exit, const double* I_in,
                         double c, double* E, double* F, double* f, double* bnd, hipStream_t st) {
    Rays* r = pl->rays;
    const bool f32 = pl->prec == LC_F32;
    if (E || F || f) {
        MomArgs A{};
        A.csr_off = r->d_csr_off;
        A.csr_ray = r->d_csr_ray;
        A.csr_t = r->d_csr_t;
        A.ray_off = r->d_ray_off;
        A.bun_off = pl->d_bun_off;
        A.bun_base = pl->d_bun_base;
        A.half = pl->half_elems;
        A.csr_w = f32 ? static_cast<const void*>(r->d_csr_w32) : static_cast<const void*>(r->d_csr_w);
        A.dirw = r->d_dirw;
        A.state = state_values(pl, state);
        A.e = static_cast<const int*>(state);
        A.cells = r->cells;
        A.G = pl->G;
        A.n_pairs = r->n_pairs;
        A.inv_c = 1.0 / c;
        A.E = E;
        A.F = F;
        A.f = f;
        lc_status rc = prof_begin(pl, pl->ev_mom, st);
        if (rc) return rc;
        rc = f32 ? launch_cell_moments_p<float>(r->n_pol, A, st)
                 : launch_cell_moments_p<double>(r->n_pol, A, st);
        if (rc) return rc;
        rc = prof_end(pl, pl->ev_mom, st);
        if (rc) return rc;
    }
    if (bnd) {
        BndArgs B{};
        B.bmap = r->d_bmap;
        B.width = r->d_width;
        B.dirw = r->d_dirw;
        B.I_exit = I_exit;
        B.I_in = I_in;
        B.nx = r->nx;
        B.ny = r->ny;
        B.nb = r->nb;
        B.G = pl->G;
        B.n_pairs = r->n_pairs;
        B.n_az = r->n_az;
        B.P = r->n_pol;
        B.bnd = bnd;
        const int lanes = r->nb * pl->G;
        hipLaunchKernelGGL(k_boundary, dim3((lanes + kBlock - 1) / kBlock), dim3(kBlock), 0, st, B);
        LC_HIP(hipGetLastError());
    }
    return LC_OK;
}

}  // namespace lc
