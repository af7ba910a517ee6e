// One backward-Euler time step of the multilevel quasidiffusion (MLQD)
// method on the Fleck-Cummings test material: the transport equation by
// long characteristics (eq. (10)-(13)) closes the multigroup LOQD equations
// (eq. (4)) through the cell and face Eddington tensors and the boundary
// factors; their solution closes the effective grey problem (eq. (5)-(6),
// averages of eq. (8)-(9)), whose temperature feeds the opacities and
// Planck functions of the next iteration.
//
// Iterations (T^(0) = T^{n-1}): an outer (transport) iteration sweeps from
// the state of step n-1 with kappa_g, B_g of T^(s) and forms the closures;
// inner (low-order) iterations then, with those closures fixed, evaluate
// kappa_g, B_g at the newest temperature, solve the multigroup equations,
// form the grey coefficients and solve the grey problem: one pass T ->
// Phi(T), until Phi(T) differs from T by at most eps (relative, every cell).
// The next inner iterate comes from Anderson mixing of the last passes on
// x = log T (g(x) = log Phi(e^x), r = g(x) - x; x <- g - dG gamma with gamma
// minimising |r - dF gamma| over the last `depth` differences of residuals
// dF and of map values dG); the mixing changes only the speed, not the
// fixed point.  The outer iteration ends when the temperature and the grey
// cell energy change by at most eps between transport sweeps.
//
// Material: kappa_g(T) = 27/nu_g^3 (1 - e^(-nu_g/T)) at each group's
// representative frequency, B_g(T) = (a_R c T^4 / 4 pi)(15/pi^4) times the
// integral of x^3/(e^x - 1) over the group's [nu_{g-1}/T, nu_g/T]: a
// Bernoulli series below x = 2, the exponential tail series
// sum_n e^(-n x)(x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4) above, so that no
// difference of large integrals is formed in the Wien tail.
#include <algorithm>
#include <cmath>
#include <vector>

#include "lc_internal.hpp"
#include "loqd_internal.hpp"

namespace lc {

constexpr uint32_t kMlqdMagic = 0x4c434d51u;   // "LCMQ"
constexpr int kMlqdBlock = 256;
constexpr int kBern = 41;                      // series terms k = 0 .. 40
constexpr int kMaxDepth = 8;                   // Anderson history
constexpr int kMaxDots = kMaxDepth * (kMaxDepth + 1) / 2 + kMaxDepth;
constexpr double kMPi = 3.14159265358979323846;

struct Mlqd {
    uint32_t magic = 0;
    lc_plan_t plan = nullptr;
    Plan* pl = nullptr;
    int G = 0, N = 0, nint = 0, nf = 0, nb = 0, nblk = 0;
    double c = 0, c_v = 0, a_R = 0, pref = 0;
    size_t state_bytes = 0;
    lc_loqd_t mg = nullptr, grey = nullptr;
    double* d_nu = nullptr;       // [G]
    double* d_edges = nullptr;    // [G + 1]
    double* d_bern = nullptr;     // [kBern] B_k / (k! (k + 3)), the Planck series coefficients
    double* d_kappa = nullptr;    // [G][N]
    double* d_planck = nullptr;   // [G][N]
    void* d_points = nullptr;     // a state-sized buffer
    double* d_exit = nullptr;     // [n_rays][2][n_pol][G]
    double* d_f = nullptr;        // [N][4][G]
    double* d_bnd = nullptr;      // [G][nb][8]
    double* d_ff = nullptr;       // [nint][4][G]
    // grey coefficients
    double *d_sigma = nullptr, *d_src = nullptr, *d_ep = nullptr, *d_kE = nullptr, *d_kB = nullptr;
    double *d_ks = nullptr, *d_es = nullptr, *d_fp = nullptr, *d_fc = nullptr, *d_ffg = nullptr, *d_bc = nullptr;
    // grey solution and temperature iterates
    double *d_Eg = nullptr, *d_Egf = nullptr, *d_Fgf = nullptr, *d_Eg_old = nullptr;
    double *d_Ts = nullptr, *d_Tl = nullptr, *d_Tn = nullptr;
    double* d_part = nullptr;     // [nblk][2] block maxima
    // Anderson mixing of the inner iteration on x = log T
    int depth = 3;
    double *d_x = nullptr, *d_gx = nullptr, *d_rprev = nullptr, *d_gprev = nullptr;   // [N]
    double *d_dF = nullptr, *d_dG = nullptr;  // [kMaxDepth][N]
    double* d_dots = nullptr;                 // [nblk][kMaxDots] block partial sums
    double* h_read = nullptr;                 // pinned host copy of d_part or d_dots
    std::vector<void*> owned;
};

inline Mlqd* as_mlqd(lc_mlqd_t h) {
    Mlqd* p = reinterpret_cast<Mlqd*>(h);
    return (p && p->magic == kMlqdMagic) ? p : nullptr;
}

namespace {

// int_0^x t^3/(e^t - 1) dt = sum_k c_k x^(k+3), c_k = B_k / (k! (k+3)), x < 2
__device__ double planck_series(double x, const double* __restrict__ c) {
    double s = 0.0, xp = x * x * x;
    for (int k = 0; k < kBern; ++k) {
        s += c[k] * xp;
        xp *= x;
    }
    return s;
}

// int_x^inf t^3/(e^t - 1) dt = sum_n e^(-n x) (x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4),
// x >= 2 (0 at infinity), 25 terms, smallest first.  e^(-n x) is formed as
// the n-th power of e^(-x) (relative error below 3e-15 for n <= 25) and the
// powers of 1/n are constants, so a term costs no exponential or division.
__device__ double planck_tail(double x) {
    if (!std::isfinite(x)) return 0.0;
    constexpr int kTail = 25;
    const double x2 = x * x, x3 = x2 * x;
    const double q = exp(-x);
    double qn[kTail];
    qn[0] = q;
#pragma unroll
    for (int n = 1; n < kTail; ++n) qn[n] = qn[n - 1] * q;
    double s = 0.0;
#pragma unroll
    for (int n = kTail; n >= 1; --n) {
        constexpr double one = 1.0;
        const double r = one / n, r2 = r * r;
        s += qn[n - 1] * (x3 * r + 3.0 * x2 * r2 + 6.0 * x * (r2 * r) + 6.0 * (r2 * r2));
    }
    return s;
}

__device__ double group_integral(double x1, double x2, const double* b) {
    const double total = kMPi * kMPi * kMPi * kMPi / 15.0;
    if (x1 >= 2.0) return planck_tail(x1) - planck_tail(x2);
    if (x2 < 2.0) return planck_series(x2, b) - planck_series(x1, b);
    return (total - planck_tail(x2)) - planck_series(x1, b);
}

__global__ void k_fc_material(int G, int N, const double* __restrict__ nu, const double* __restrict__ edges,
                              const double* __restrict__ bern, double pref, const double* __restrict__ T,
                              double* kappa, double* planck) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int g = blockIdx.y;
    if (i >= N || g >= G) return;
    const double t = T[i], v = nu[g];
    const size_t gi = (size_t)g * N + i;
    kappa[gi] = 27.0 / (v * v * v) * -expm1(-v / t);
    const double t2 = t * t;
    planck[gi] = pref * t2 * t2 * group_integral(edges[g] / t, edges[g + 1] / t, bern);
}

// Per block: rel = 1: max |a - b| / |a|; rel = 0: max |a - b| and max |a|.
// Not finite -> infinity.
__global__ void k_change(int n, const double* __restrict__ a, const double* __restrict__ b, int rel, double* part) {
    __shared__ double s0[kMlqdBlock], s1[kMlqdBlock];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double d = 0.0, m = 0.0;
    if (i < n) {
        const double x = a[i], y = b[i];
        d = rel ? fabs(x - y) / fabs(x) : fabs(x - y);
        m = fabs(x);
        if (!std::isfinite(d)) d = INFINITY;
    }
    s0[threadIdx.x] = d;
    s1[threadIdx.x] = m;
    __syncthreads();
    for (int w = kMlqdBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + w]);
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

__global__ void k_log(int n, const double* __restrict__ T, double* x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = log(T[i]);
}

// T = T2 = exp(x): the pass's temperature, and the Newton iterate that
// starts from it.
__global__ void k_exp(int n, const double* __restrict__ x, double* T, double* T2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) T[i] = T2[i] = exp(x[i]);
}

// After a pass: g = log Phi, r = g - x; with a previous pass, the history
// column `slot` takes dF = r - r_prev, dG = g - g_prev; then r_prev = r,
// g_prev = g.  Also the pass's change, as k_change with rel = 1 on
// (Phi, T): per block max |Phi - T| / |Phi| and max |Phi|.
__global__ void k_aa_update(int n, const double* __restrict__ Tn, const double* __restrict__ Tl,
                            const double* __restrict__ x, double* gx, double* rprev, double* gprev, double* dF,
                            double* dG, int have_prev, double* part) {
    __shared__ double s0[kMlqdBlock], s1[kMlqdBlock];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double d = 0.0, m = 0.0;
    if (i < n) {
        const double a = Tn[i];
        const double g = log(a), r = g - x[i];
        if (have_prev) {
            dF[i] = r - rprev[i];
            dG[i] = g - gprev[i];
        }
        gx[i] = g;
        rprev[i] = r;
        gprev[i] = g;
        d = fabs(a - Tl[i]) / fabs(a);
        m = fabs(a);
        if (!std::isfinite(d)) d = INFINITY;
    }
    s0[threadIdx.x] = d;
    s1[threadIdx.x] = m;
    __syncthreads();
    for (int w = kMlqdBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + w]);
            s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

// Block partial sums of dF_a . dF_b (a <= b < h, row-major upper triangle)
// then dF_a . r (a < h); r = rprev (the newest residual).
__global__ void k_aa_dots(int n, int h, const double* __restrict__ dF, const double* __restrict__ r, double* part) {
    __shared__ double sm[kMlqdBlock];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nd = h * (h + 1) / 2 + h;
    int a = 0, b = 0;
    for (int d = 0; d < nd; ++d) {
        const double* u = dF + (size_t)a * n;
        const double* v = d < h * (h + 1) / 2 ? dF + (size_t)b * n : r;
        sm[threadIdx.x] = i < n ? u[i] * v[i] : 0.0;
        __syncthreads();
        for (int w = kMlqdBlock / 2; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(size_t)blockIdx.x * kMaxDots + d] = sm[0];
        __syncthreads();
        if (d < h * (h + 1) / 2) {            // next pair of the triangle, then a = 0.. for dF . r
            if (++b == h) b = ++a;
            if (a == h) a = 0;
        } else {
            ++a;
        }
    }
}

// x = g - sum_k gamma_k dG_k
__global__ void k_aa_mix(int n, int h, const double* __restrict__ gx, const double* __restrict__ dG, double g0,
                         double g1, double g2, double g3, double g4, double g5, double g6, double g7, double* x) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double gam[kMaxDepth] = {g0, g1, g2, g3, g4, g5, g6, g7};
    double v = gx[i];
    for (int k = 0; k < h; ++k) v -= gam[k] * dG[(size_t)k * n + i];
    x[i] = v;
}

// Planck series coefficients c_k = b_k / (k + 3), k = 0..40, from
// b_k = B_k / k! (B_1 = -1/2): b_1 = -1/2, b_odd = 0 beyond,
// b_2m = (-1)^(m+1) 2 zeta(2m) / (2 pi)^(2m).
std::vector<double> planck_series_coefficients() {
    std::vector<double> b(kBern, 0.0);
    b[0] = 1.0;
    b[1] = -0.5;
    const double two_pi = 2.0 * kMPi;
    for (int m = 1; 2 * m < kBern; ++m) {
        double zeta;
        if (m == 1) {
            zeta = kMPi * kMPi / 6.0;
        } else if (m == 2) {
            zeta = kMPi * kMPi * kMPi * kMPi / 90.0;
        } else {
            zeta = 0.0;                               // tail below 2000^(1-2m)/(2m-1) < 1e-16
            for (int n = 2000; n >= 1; --n) zeta += std::pow((double)n, -2.0 * m);
        }
        b[2 * m] = (m % 2 ? 2.0 : -2.0) * zeta / std::pow(two_pi, 2.0 * m);
    }
    for (int k = 0; k < kBern; ++k) b[k] /= (k + 3);      // the series' coefficients
    return b;
}

void free_mlqd(Mlqd* h) {
    if (!h) return;
    for (void* p : h->owned) (void)hipFree(p);
    h->owned.clear();
    if (h->h_read) (void)hipHostFree(h->h_read);
    h->h_read = nullptr;
    if (h->mg) (void)lc_loqd_free(h->mg);
    if (h->grey) (void)lc_loqd_free(h->grey);
    h->magic = 0;
    delete h;
}

lc_status material(Mlqd* h, const double* T, double* kappa, double* planck, hipStream_t st) {
    const dim3 grid((h->N + kMlqdBlock - 1) / kMlqdBlock, h->G);
    hipLaunchKernelGGL(k_fc_material, grid, dim3(kMlqdBlock), 0, st, h->G, h->N, h->d_nu, h->d_edges, h->d_bern,
                       h->pref, T, kappa, planck);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

// Per-block partials of a change (k_change or k_aa_update), read from the
// pinned buffer after the caller's wait: out[0] the change, out[1] max |a|.
void change_read(const Mlqd* h, double out[2]) {
    const double* part = h->h_read;
    out[0] = out[1] = 0.0;
    for (int k = 0; k < h->nblk; ++k) {
        out[0] = std::max(out[0], part[2 * k]);
        out[1] = std::max(out[1], part[2 * k + 1]);
    }
}

// Largest change between a and b (see k_change).  Synchronises the stream.
lc_status change(Mlqd* h, const double* a, const double* b, int rel, double out[2], hipStream_t st) {
    hipLaunchKernelGGL(k_change, dim3(h->nblk), dim3(kMlqdBlock), 0, st, h->N, a, b, rel, h->d_part);
    LC_HIP(hipGetLastError());
    LC_HIP(hipMemcpyAsync(h->h_read, h->d_part, 2 * (size_t)h->nblk * sizeof(double), hipMemcpyDeviceToHost, st));
    LC_HIP(hipStreamSynchronize(st));
    change_read(h, out);
    return LC_OK;
}

// Anderson coefficients: gamma minimising |r - dF gamma| from the normal
// equations (dF^T dF) gamma = dF^T r, by Gaussian elimination with partial
// pivoting.  False when the history is numerically rank-deficient.  The
// Gram partials (d_dots, right after the change partials d_part on the
// device and in the pinned buffer) are copied by the caller with the
// change's, and aa_gamma solves once the caller has waited.

void aa_gamma(const Mlqd* h, int hcols, double* gamma, bool* ok) {
    const int nd = hcols * (hcols + 1) / 2 + hcols;
    const double* part = h->h_read + 2 * (size_t)h->nblk;
    std::vector<double> dots(nd, 0.0);
    for (int k = 0; k < h->nblk; ++k)
        for (int d = 0; d < nd; ++d) dots[d] += part[(size_t)k * kMaxDots + d];
    double A[kMaxDepth][kMaxDepth + 1];
    int d = 0;
    for (int a = 0; a < hcols; ++a)
        for (int b = a; b < hcols; ++b, ++d) A[a][b] = A[b][a] = dots[d];
    for (int a = 0; a < hcols; ++a) A[a][hcols] = dots[d + a];
    double dmax = 0.0;
    for (int a = 0; a < hcols; ++a) dmax = std::max(dmax, A[a][a]);
    *ok = dmax > 0.0 && std::isfinite(dmax);
    for (int col = 0; col < hcols && *ok; ++col) {
        int piv = col;
        for (int r2 = col + 1; r2 < hcols; ++r2)
            if (fabs(A[r2][col]) > fabs(A[piv][col])) piv = r2;
        if (fabs(A[piv][col]) <= 1e-13 * dmax) {
            *ok = false;
            break;
        }
        for (int k = 0; k <= hcols; ++k) std::swap(A[col][k], A[piv][k]);
        for (int r2 = col + 1; r2 < hcols; ++r2) {
            const double m = A[r2][col] / A[col][col];
            for (int k = col; k <= hcols; ++k) A[r2][k] -= m * A[col][k];
        }
    }
    for (int a = hcols - 1; a >= 0 && *ok; --a) {
        double v = A[a][hcols];
        for (int k = a + 1; k < hcols; ++k) v -= A[a][k] * gamma[k];
        gamma[a] = v / A[a][a];
        *ok = std::isfinite(gamma[a]);
    }
}

}  // namespace
}  // namespace lc

using namespace lc;

extern "C" {

lc_status lc_mlqd_create(lc_plan_t plan, const double* nu, const double* edges, double c, double c_v, double a_R,
                         lc_mlqd_t* out) {
    LC_ARG(out, "out must not be NULL");
    *out = nullptr;
    Plan* pl = as_plan(plan);
    LC_CHECK(pl, LC_ERR_STATE, "invalid plan handle");
    LC_CHECK(pl->prec == LC_F64, LC_ERR_UNSUPPORTED,
             "the multilevel step needs a float64 plan: its iterations converge to tolerances far below the float32 "
             "sweep's rounding");
    LC_ARG(nu && edges, "nu and edges must not be NULL");
    LC_ARG(std::isfinite(c) && c > 0.0 && std::isfinite(c_v) && c_v > 0.0 && std::isfinite(a_R) && a_R > 0.0,
           "c, c_v and a_R must be finite and > 0");
    const int G = pl->G;
    for (int g = 0; g < G; ++g) LC_ARG(std::isfinite(nu[g]) && nu[g] > 0.0, "nu[%d] must be finite and > 0", g);
    LC_ARG(edges[0] >= 0.0 && std::isfinite(edges[0]), "edges[0] must be finite and >= 0");
    for (int g = 0; g < G; ++g)
        LC_ARG(edges[g + 1] > edges[g] && (std::isfinite(edges[g + 1]) || g == G - 1),
               "edges must increase; only the last may be infinite");
    Rays* r = pl->rays;
    Mlqd* h = new Mlqd();
    h->plan = plan;
    h->pl = pl;
    h->G = G;
    h->N = r->cells;
    h->nint = (r->nx - 1) * r->ny + r->nx * (r->ny - 1);
    h->nb = 2 * (r->nx + r->ny);
    h->nf = h->nint + h->nb;
    h->nblk = (h->N + kMlqdBlock - 1) / kMlqdBlock;
    h->c = c;
    h->c_v = c_v;
    h->a_R = a_R;
    h->pref = a_R * c / (4.0 * kMPi) * 15.0 / (kMPi * kMPi * kMPi * kMPi);
    h->state_bytes = lc_state_bytes(plan);
    const int N = h->N, nf = h->nf, nb = h->nb;
    auto fail = [&](lc_status rc) {
        free_mlqd(h);
        return rc;
    };
    lc_status rc = lc_plan_enable_faces(plan, nullptr);
    if (!rc) rc = lc_loqd_create(r->nx, r->ny, r->lx, r->ly, G, &h->mg);
    if (!rc) rc = lc_loqd_create(r->nx, r->ny, r->lx, r->ly, 1, &h->grey);
    if (rc) return fail(rc);
    (void)lc_loqd_set_warm_start(h->mg, 1);
    (void)lc_loqd_set_warm_start(h->grey, 1);
    const size_t GN = (size_t)G * N;
    std::vector<double> bern = planck_series_coefficients();
    rc = dalloc(h->owned, &h->d_nu, (size_t)G);
    if (!rc) rc = dalloc(h->owned, &h->d_edges, (size_t)G + 1);
    if (!rc) rc = dalloc(h->owned, &h->d_bern, (size_t)kBern);
    if (!rc) rc = dalloc(h->owned, &h->d_kappa, GN);
    if (!rc) rc = dalloc(h->owned, &h->d_planck, GN);
    if (!rc) rc = dalloc(h->owned, reinterpret_cast<unsigned char**>(&h->d_points), h->state_bytes);
    if (!rc) rc = dalloc(h->owned, &h->d_exit, (size_t)r->n_rays * 2 * r->n_pol * G);
    if (!rc) rc = dalloc(h->owned, &h->d_f, 4 * GN);
    if (!rc) rc = dalloc(h->owned, &h->d_bnd, (size_t)G * nb * 8);
    if (!rc) rc = dalloc(h->owned, &h->d_ff, 4 * (size_t)G * std::max(h->nint, 1));
    for (double** p : {&h->d_sigma, &h->d_src, &h->d_ep, &h->d_kE, &h->d_kB, &h->d_Eg, &h->d_Eg_old, &h->d_Ts,
                       &h->d_Tl, &h->d_Tn})
        if (!rc) rc = dalloc(h->owned, p, (size_t)N);
    if (!rc) rc = dalloc(h->owned, &h->d_ks, 4 * (size_t)N);
    if (!rc) rc = dalloc(h->owned, &h->d_es, 4 * (size_t)N);
    if (!rc) rc = dalloc(h->owned, &h->d_fc, 3 * (size_t)N);
    if (!rc) rc = dalloc(h->owned, &h->d_fp, (size_t)nf);
    if (!rc) rc = dalloc(h->owned, &h->d_ffg, 3 * (size_t)nf);
    if (!rc) rc = dalloc(h->owned, &h->d_bc, 3 * (size_t)nb);
    if (!rc) rc = dalloc(h->owned, &h->d_Egf, (size_t)nf);
    if (!rc) rc = dalloc(h->owned, &h->d_Fgf, (size_t)nf);
    if (!rc) rc = dalloc(h->owned, &h->d_part, (2 + (size_t)kMaxDots) * h->nblk);   // then d_dots
    if (!rc) h->d_dots = h->d_part + 2 * (size_t)h->nblk;
    for (double** p : {&h->d_x, &h->d_gx, &h->d_rprev, &h->d_gprev})
        if (!rc) rc = dalloc(h->owned, p, (size_t)N);
    if (!rc) rc = dalloc(h->owned, &h->d_dF, (size_t)kMaxDepth * N);
    if (!rc) rc = dalloc(h->owned, &h->d_dG, (size_t)kMaxDepth * N);
    if (!rc) {
        const size_t bytes = (size_t)h->nblk * (2 + kMaxDots) * sizeof(double);
        if (hipHostMalloc(reinterpret_cast<void**>(&h->h_read), bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            h->h_read = nullptr;
            set_error("hipHostMalloc(%zu bytes) failed", bytes);
            rc = LC_ERR_ALLOC;
        }
    }
    if (rc) return fail(rc);
    if (hipMemcpy(h->d_nu, nu, G * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_edges, edges, (G + 1) * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_bern, bern.data(), kBern * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(h->d_Egf, 0, nf * sizeof(double)) != hipSuccess ||
        hipMemset(h->d_Eg_old, 0, N * sizeof(double)) != hipSuccess) {
        set_error("HIP error uploading the material tables");
        return fail(LC_ERR_HIP);
    }
    h->magic = kMlqdMagic;
    *out = reinterpret_cast<lc_mlqd_t>(h);
    return LC_OK;
}

lc_status lc_mlqd_free(lc_mlqd_t handle) {
    if (!handle) return LC_OK;
    Mlqd* h = as_mlqd(handle);
    LC_CHECK(h, LC_ERR_STATE, "invalid MLQD handle");
    free_mlqd(h);
    return LC_OK;
}

lc_status lc_mlqd_set_acceleration(lc_mlqd_t handle, int32_t depth) {
    Mlqd* h = as_mlqd(handle);
    LC_CHECK(h, LC_ERR_STATE, "invalid MLQD handle");
    LC_ARG(depth >= 0 && depth <= kMaxDepth, "depth must be in 0..%d", kMaxDepth);
    h->depth = depth;
    return LC_OK;
}

lc_status lc_mlqd_material(lc_mlqd_t handle, const double* T, double* kappa, double* planck, void* stream) {
    Mlqd* h = as_mlqd(handle);
    LC_CHECK(h, LC_ERR_STATE, "invalid MLQD handle");
    LC_ARG(T && kappa && planck, "T, kappa and planck must not be NULL");
    return material(h, T, kappa, planck, static_cast<hipStream_t>(stream));
}

lc_status lc_mlqd_step(lc_mlqd_t handle, double c_dt, const void* state_prev, void* state_new, const double* I_in,
                       const double* T_prev, const double* E_prev, const double* F_prev, double* T, double* E_cell,
                       double* E_face, double* F_face, double* E_grey, double eps, int32_t max_outer,
                       int32_t max_inner, int32_t* outer_iters, int32_t* inner_iters, double* changes, void* stream) {
    Mlqd* h = as_mlqd(handle);
    LC_CHECK(h, LC_ERR_STATE, "invalid MLQD handle");
    LC_ARG(state_prev && state_new && I_in && T_prev && E_prev && F_prev && T && E_cell && E_face && F_face,
           "inputs and outputs must not be NULL");
    LC_ARG(state_prev != state_new, "state_prev and state_new must be distinct buffers");
    LC_ARG(std::isfinite(c_dt) && c_dt > 0.0, "c_dt must be finite and > 0");
    LC_ARG(std::isfinite(eps) && eps > 0.0, "eps must be finite and > 0");
    LC_ARG(max_outer >= 1 && max_inner >= 1, "max_outer and max_inner must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int G = h->G, N = h->N, nf = h->nf;
    const double c = h->c;
    // Inexact passes: the low-order solves of a pass stop at a residual tied
    // to the size of the last change (1e-3 of it, within [1e-13, 1e-8]), so
    // early passes, whose temperature will move much further anyway, cost
    // fewer iterations; a pass only ends the inner iteration when it was
    // solved at the tightest tolerance.
    const double rtol_min = 1e-13, rtol_max = 1e-8;
    const int max_iter = 20000;
    const double newton_tol = std::max(std::min(eps, 1e-11), 1e-13);
    double level = 1.0;
    const size_t bytesN = N * sizeof(double);
    LC_HIP(hipMemcpyAsync(h->d_Ts, T_prev, bytesN, hipMemcpyDeviceToDevice, st));
    // The first multigroup and grey solves of a step start cold, so a step's
    // result depends on its arguments alone, not on the steps the handle ran
    // before; later passes start from the previous pass's solution.
    LC_HIP(hipMemsetAsync(E_face, 0, (size_t)G * nf * sizeof(double), st));
    LC_HIP(hipMemsetAsync(h->d_Egf, 0, (size_t)nf * sizeof(double), st));
    int s = 0, inner = 0;
    double dT = INFINITY, dE = INFINITY;
    lc_status rc = LC_OK;
    auto report = [&]() {
        if (outer_iters) *outer_iters = s;
        if (inner_iters) *inner_iters = inner;
        if (changes) {
            changes[0] = dT;
            changes[1] = dE;
        }
    };
    while (s < max_outer) {
        ++s;
        // transport with the material of T^(s), closures
        rc = material(h, h->d_Ts, h->d_kappa, h->d_planck, st);
        if (!rc) rc = lc_sweep_points(h->plan, h->d_kappa, h->d_planck, c_dt, state_prev, state_new, I_in, h->d_exit,
                                      h->d_points, st);
        if (!rc) rc = lc_moments(h->plan, state_new, h->d_exit, I_in, c, nullptr, nullptr, h->d_f, h->d_bnd, st);
        if (!rc && h->nint > 0)
            rc = lc_face_moments(h->plan, h->d_points, state_new, c, nullptr, nullptr, h->d_ff, st);
        if (rc) break;
        // inner low-order iterations with these closures (Anderson mixing on log T)
        const dim3 gN(h->nblk), bN(kMlqdBlock);
        hipLaunchKernelGGL(k_log, gN, bN, 0, st, N, h->d_Ts, h->d_x);
        int hcols = 0, slot = 0;
        bool have_prev = false;
        for (int l = 0; l < max_inner; ++l) {
            ++inner;
            const double rtol = std::min(rtol_max, std::max(rtol_min, 1e-3 * level));
            const double ntol = std::max(newton_tol, 1e3 * rtol);
            hipLaunchKernelGGL(k_exp, gN, bN, 0, st, N, h->d_x, h->d_Tl, h->d_Tn);
            rc = material(h, h->d_Tl, h->d_kappa, h->d_planck, st);
            // the multigroup solve's report is checked after the grey
            // problem's first wait on the stream
            if (!rc) rc = loqd_solve(h->mg, c, c_dt, h->d_kappa, h->d_planck, E_prev, F_prev, h->d_f, h->d_ff,
                                     h->d_bnd, E_cell, E_face, F_face, rtol, max_iter, nullptr, nullptr, st, true);
            if (!rc) rc = lc_loqd_grey_coefficients(h->mg, c, c_dt, h->d_kappa, h->d_planck, E_prev, F_prev, h->d_f,
                                                    h->d_ff, h->d_bnd, E_cell, E_face, F_face, h->d_sigma, h->d_src,
                                                    h->d_ks, h->d_es, h->d_fp, h->d_fc, h->d_ffg, h->d_bc, h->d_ep,
                                                    h->d_kE, h->d_kB, st);
            if (rc) break;
            rc = lc_loqd_grey_meb(h->grey, c, c_dt, h->d_kE, h->d_kB, h->d_ep, h->d_ks, h->d_es, h->d_fp, h->d_fc,
                                  h->d_ffg, h->d_bc, T_prev, h->c_v, h->a_R, h->d_Tn, h->d_Eg, h->d_Egf, h->d_Fgf,
                                  ntol, 100, rtol, max_iter, nullptr, nullptr, nullptr, st);
            if (!rc) rc = loqd_check_deferred(h->mg, nullptr);
            if (rc) break;
            // the pass's change and the Anderson update with its Gram
            // partials are queued together and read after one wait (when the
            // pass ends the iteration, the update is simply not used: the
            // next transport iteration starts a new history)
            double ch[2];
            const bool push = have_prev && h->depth > 0;
            hipLaunchKernelGGL(k_aa_update, gN, bN, 0, st, N, h->d_Tn, h->d_Tl, h->d_x, h->d_gx, h->d_rprev,
                               h->d_gprev, h->d_dF + (size_t)slot * N, h->d_dG + (size_t)slot * N, push ? 1 : 0,
                               h->d_part);
            if (push) {
                hcols = std::min(hcols + 1, h->depth);
                slot = (slot + 1) % h->depth;
            }
            have_prev = true;
            size_t n_read = 2 * (size_t)h->nblk;
            if (hcols > 0) {
                hipLaunchKernelGGL(k_aa_dots, gN, bN, 0, st, N, hcols, h->d_dF, h->d_rprev, h->d_dots);
                n_read += (size_t)h->nblk * kMaxDots;
            }
            LC_HIP(hipGetLastError());
            LC_HIP(hipMemcpyAsync(h->h_read, h->d_part, n_read * sizeof(double), hipMemcpyDeviceToHost, st));
            LC_HIP(hipStreamSynchronize(st));
            change_read(h, ch);
            level = ch[0];
            if (ch[0] <= eps && rtol == rtol_min) break;
            double gamma[kMaxDepth] = {0, 0, 0, 0, 0, 0, 0, 0};
            bool ok = false;
            if (hcols > 0) aa_gamma(h, hcols, gamma, &ok);
            if (ok) {
                hipLaunchKernelGGL(k_aa_mix, gN, bN, 0, st, N, hcols, h->d_gx, h->d_dG, gamma[0], gamma[1], gamma[2],
                                   gamma[3], gamma[4], gamma[5], gamma[6], gamma[7], h->d_x);
            } else {
                LC_HIP(hipMemcpyAsync(h->d_x, h->d_gx, bytesN, hipMemcpyDeviceToDevice, st));
                hcols = 0;                    // a rank-deficient history starts again
                slot = 0;
            }
            LC_HIP(hipGetLastError());
        }
        std::swap(h->d_Tl, h->d_Tn);          // T^(s+1): the last pass's Phi
        if (rc) break;
        double ct[2], ce[2];
        rc = change(h, h->d_Tl, h->d_Ts, 1, ct, st);
        if (!rc) rc = change(h, h->d_Eg, h->d_Eg_old, 0, ce, st);
        if (rc) break;
        dT = ct[0];
        dE = s == 1 ? INFINITY : (ce[1] > 0.0 ? ce[0] / ce[1] : 0.0);
        level = std::max(level, dT);           // the next sweep moves the closures by about this much
        std::swap(h->d_Ts, h->d_Tl);
        LC_HIP(hipMemcpyAsync(h->d_Eg_old, h->d_Eg, bytesN, hipMemcpyDeviceToDevice, st));
        if (dT <= eps && dE <= eps) break;
    }
    if (!rc) {
        LC_HIP(hipMemcpyAsync(T, h->d_Ts, bytesN, hipMemcpyDeviceToDevice, st));
        if (E_grey) LC_HIP(hipMemcpyAsync(E_grey, h->d_Eg, bytesN, hipMemcpyDeviceToDevice, st));
        LC_HIP(hipStreamSynchronize(st));
    }
    report();
    if (rc) return rc;
    LC_CHECK(dT <= eps && dE <= eps, LC_ERR_UNSUPPORTED,
             "MLQD step: changes %.3g (T) and %.3g (E) above %.3g after %d transport iterations", dT, dE, eps, s);
    return LC_OK;
}

}  // extern "C"
