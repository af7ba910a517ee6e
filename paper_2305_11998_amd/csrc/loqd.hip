// Multigroup low-order quasidiffusion (LOQD) equations, eq. (4), for one
// backward-Euler step on the material grid, closed by the transport sweep's
// Eddington tensors (cells: eq. (7), (15); faces: eq. (16)) and the
// half-range boundary factors.
//
// Discretisation (the paper cites a second-order finite-volume scheme
// without printing it; this is the reading the library implements): cell
// and face averages of E per group; the balance (4a) integrated over each
// cell; the first moment (4b) integrated over each half cell next to a face
// (kappa_t F taken at the face, the cell tensor times E_i at the centre, the
// face tensor times E_f on the face, the cell's transverse face averages for
// the mixed term); one normal flux per interior face; the QD boundary
// condition n.F = C (c E_f - Phi^-) - J^- on boundary faces.
//
// Solution: in the balance of cell i the mixed terms of its two opposite
// faces cancel, so the cell row couples E_i only to the cell's own four
// faces and E_i is eliminated exactly:
//   E_i = (b_i - sum_k a_ik E_k) / d_i.
// What remains is a system in the face unknowns alone (at most 7 entries a
// row: the face and the other faces of its one or two cells), solved for all
// groups at once by BiCGSTAB with a Jacobi preconditioner.  Every inner
// product is a fixed-order reduction (no atomics), so results are
// deterministic.  Then E_i and the face fluxes follow from the cell rows and
// the half-cell relations.
#include <cmath>
#include <cstring>
#include <vector>

#include "lc_internal.hpp"

namespace lc {

constexpr uint32_t kLoqdMagic = 0x4c434c51u;   // "LCLQ"
constexpr int kSlots = 7;                     // entries of a face row
constexpr int kLoqdBlock = 256;
constexpr double kPi = 3.14159265358979323846;

struct Loqd {
    uint32_t magic = 0;
    int nx = 0, ny = 0, G = 0;
    double lx = 0, ly = 0, hx = 0, hy = 0;
    int N = 0, nint = 0, nb = 0, nf = 0;
    int nblk = 0;                     // reduction blocks per group vector
    // geometry (group-independent)
    int* d_cface = nullptr;           // [4][N] faces L, R, B, T of every cell
    int* d_lo = nullptr;              // [nf] cell below / left of the face, -1 outside
    int* d_hi = nullptr;              // [nf] cell above / right, -1 outside
    int* d_col = nullptr;             // [kSlots][nf] face columns of each face row (padding: the row itself)
    // per solve, per group
    double* d_dc = nullptr;           // [G][N] cell diagonal
    double* d_ac = nullptr;           // [G][4][N] cell-row coefficients of the faces L, R, B, T
    double* d_bc = nullptr;           // [G][N] cell right-hand side
    double* d_val = nullptr;          // [G][kSlots][nf]
    double* d_dinv = nullptr;         // [G][nf]
    double* d_b = nullptr;            // [G][nf]
    double* d_vec = nullptr;          // 8 vectors [G][nf]: x r rh p v s t ph
    double* d_sh = nullptr;           // [G][nf]
    double* d_part = nullptr;         // [G][nblk][2] block partial sums
    double* d_sc = nullptr;           // [G][kScal] per-group scalars
    int* d_flag = nullptr;            // [G] 1 = iterating
    std::vector<void*> owned;
};

// per-group scalars
enum { S_RHO = 0, S_ALPHA, S_OMEGA, S_BETA, S_BNORM, S_RNORM, S_TS, S_TT, S_RV, kScal };

inline Loqd* as_loqd(lc_loqd_t h) {
    Loqd* p = reinterpret_cast<Loqd*>(h);
    return (p && p->magic == kLoqdMagic) ? p : nullptr;
}

namespace {

struct Geo {
    int nx, ny, N, nint, nf, G;
    double hx, hy, c, c_dt;
    const int* cface;
    const int* lo;
    const int* hi;
    const int* col;
};

// Face tensor entry q (0 xx, 1 xy, 2 yy) of face f for group g: interior
// faces from the face moments [nint][4][G], boundary faces from the
// boundary factors [G][nb][8] (columns 5, 6, 7).
__device__ inline double face_tensor(const Geo& Q, const double* ff, const double* bnd, int g, int f, int q) {
    if (f < Q.nint) return ff[((size_t)f * 4 + q) * Q.G + g];
    const int b = f - Q.nint;
    const int nb = Q.nf - Q.nint;
    return bnd[((size_t)g * nb + b) * 8 + 5 + q];
}

// Cell rows: d_i, a_ik and b_i of
//   c kt E_i + (F_R - F_L)/hx + (F_T - F_B)/hy = 4 pi kappa B + c E_prev / c_dt
// after the half-cell relations are put in for the four fluxes.
__global__ void k_loqd_cells(Geo Q, const double* __restrict__ kappa, const double* __restrict__ planck,
                             const double* __restrict__ E_prev, const double* __restrict__ F_prev,
                             const double* __restrict__ fc, const double* __restrict__ ff,
                             const double* __restrict__ bnd, double* dc, double* ac, double* bcv) {
    const int g = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q.N) return;
    const size_t gi = (size_t)g * Q.N + i;
    const double kap = kappa[gi];
    const double kt = kap + 1.0 / Q.c_dt;
    const double fxx = fc[((size_t)i * 4 + 0) * Q.G + g];
    const double fyy = fc[((size_t)i * 4 + 2) * Q.G + g];
    const int L = Q.cface[i], R = Q.cface[Q.N + i], B = Q.cface[2 * Q.N + i], T = Q.cface[3 * Q.N + i];
    const double ex = 2.0 * Q.c / (kt * Q.hx * Q.hx);
    const double ey = 2.0 * Q.c / (kt * Q.hy * Q.hy);
    dc[gi] = Q.c * kt + 2.0 * ex * fxx + 2.0 * ey * fyy;
    const size_t a0 = (size_t)g * 4 * Q.N + i;
    ac[a0] = -ex * face_tensor(Q, ff, bnd, g, L, 0);
    ac[a0 + Q.N] = -ex * face_tensor(Q, ff, bnd, g, R, 0);
    ac[a0 + 2 * (size_t)Q.N] = -ey * face_tensor(Q, ff, bnd, g, B, 2);
    ac[a0 + 3 * (size_t)Q.N] = -ey * face_tensor(Q, ff, bnd, g, T, 2);
    const double* Fp = F_prev + (size_t)g * Q.nf;
    bcv[gi] = 4.0 * kPi * kap * planck[gi] + Q.c * E_prev[gi] / Q.c_dt -
              (Fp[R] - Fp[L]) / (kt * Q.hx * Q.c_dt) - (Fp[T] - Fp[B]) / (kt * Q.hy * Q.c_dt);
}

// Add v to the slot of column col in a face row (cols: the row's columns).
__device__ inline void put(double* row, const int* cols, int col, double v) {
    for (int s = 0; s < kSlots; ++s)
        if (cols[s] == col) {
            row[s] += v;
            return;
        }
}

// Face rows of the face system.  A face's row is the sum over its cells of
// sigma F^(cell)_f (sigma = +1 for the cell below / left, -1 above / right;
// an interior face so states that both cells give one flux), minus
// C c E_f on a boundary face, with every cell unknown replaced by its
// cell row.
__global__ void k_loqd_faces(Geo Q, const double* __restrict__ kappa, const double* __restrict__ F_prev,
                             const double* __restrict__ fc, const double* __restrict__ ff,
                             const double* __restrict__ bnd, const double* __restrict__ dc,
                             const double* __restrict__ ac, const double* __restrict__ bcv, double* val,
                             double* dinv, double* b) {
    const int g = blockIdx.y;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= Q.nf) return;
    int cols[kSlots];
    double row[kSlots];
    for (int s = 0; s < kSlots; ++s) {
        cols[s] = Q.col[(size_t)s * Q.nf + f];
        row[s] = 0.0;
    }
    double rhs = 0.0;
    const double Fp = F_prev[(size_t)g * Q.nf + f];
    for (int side = 0; side < 2; ++side) {
        const int cell = side == 0 ? Q.lo[f] : Q.hi[f];
        if (cell < 0) continue;
        const double sg = side == 0 ? 1.0 : -1.0;
        const int L = Q.cface[cell], R = Q.cface[Q.N + cell], B = Q.cface[2 * Q.N + cell],
                  T = Q.cface[3 * Q.N + cell];
        const bool xf = (f == L || f == R);
        const double hn = xf ? Q.hx : Q.hy, ht = xf ? Q.hy : Q.hx;
        const double kt = kappa[(size_t)g * Q.N + cell] + 1.0 / Q.c_dt;
        const double a = kt * hn / 2.0;
        const double fnn = fc[((size_t)cell * 4 + (xf ? 0 : 2)) * Q.G + g];
        const double gnn = face_tensor(Q, ff, bnd, g, f, xf ? 0 : 2);
        const int hiT = xf ? T : R, loT = xf ? B : L;
        const double x = Q.c * hn / (2.0 * ht) / a;
        // sigma F^(cell)_f = (c fnn E_cell - c gnn E_f) / a
        //                    - sigma x (gxy_hiT E_hiT - gxy_loT E_loT) + sigma (hn/2) Fp / (c_dt a)
        put(row, cols, f, -Q.c * gnn / a);
        put(row, cols, hiT, -sg * x * face_tensor(Q, ff, bnd, g, hiT, 1));
        put(row, cols, loT, sg * x * face_tensor(Q, ff, bnd, g, loT, 1));
        rhs -= sg * (hn / 2.0) * Fp / (Q.c_dt * a);
        // E_cell = (b_cell - sum_k a_k E_k) / d_cell
        const double beta = Q.c * fnn / a;
        const size_t gi = (size_t)g * Q.N + cell;
        const double d = dc[gi];
        const size_t a0 = (size_t)g * 4 * Q.N + cell;
        put(row, cols, L, -beta * ac[a0] / d);
        put(row, cols, R, -beta * ac[a0 + Q.N] / d);
        put(row, cols, B, -beta * ac[a0 + 2 * (size_t)Q.N] / d);
        put(row, cols, T, -beta * ac[a0 + 3 * (size_t)Q.N] / d);
        rhs -= beta * bcv[gi] / d;
    }
    if (Q.lo[f] < 0 || Q.hi[f] < 0) {                    // n.F = C (c E_f - Phi^-) - J^-
        const int nb = Q.nf - Q.nint;
        const double* bb = bnd + ((size_t)g * nb + (f - Q.nint)) * 8;
        const double C = bb[4], Pm = bb[2], Jm = bb[3];
        put(row, cols, f, -C * Q.c);
        rhs += -C * Pm - Jm;
    }
    for (int s = 0; s < kSlots; ++s) val[((size_t)g * kSlots + s) * Q.nf + f] = row[s];
    dinv[(size_t)g * Q.nf + f] = 1.0 / row[0];           // slot 0 is the face itself
    b[(size_t)g * Q.nf + f] = rhs;
}

// ---------------------------------------------------------------------------
// BiCGSTAB over all groups (vectors [G][nf]; block y = group)
// ---------------------------------------------------------------------------

struct Vecs {
    double *x, *r, *rh, *p, *v, *s, *t, *ph, *sh;
};

// Fixed-order block reduction of two values; thread 0 writes them.
__device__ inline void block_sum2(double a, double b, double* out) {
    __shared__ double sa[kLoqdBlock], sb[kLoqdBlock];
    sa[threadIdx.x] = a;
    sb[threadIdx.x] = b;
    __syncthreads();
    for (int w = kLoqdBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sa[threadIdx.x] += sa[threadIdx.x + w];
            sb[threadIdx.x] += sb[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sa[0];
        out[1] = sb[0];
    }
}

__device__ inline double spmv_row(const Geo& Q, const double* val, const double* in, int g, int f) {
    double acc = 0.0;
    for (int s = 0; s < kSlots; ++s)
        acc += val[((size_t)g * kSlots + s) * Q.nf + f] * in[(size_t)g * Q.nf + Q.col[(size_t)s * Q.nf + f]];
    return acc;
}

// r = b - A x (x given), rh = r, p = v = 0; partials of (r, r), (b, b)
__global__ void k_bi_init(Geo Q, const double* val, const double* b, Vecs V, const int* flag, double* part,
                          int nblk, int restart) {
    const int g = blockIdx.y;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0, bbv = 0.0;
    if (f < Q.nf && flag[g]) {
        const size_t k = (size_t)g * Q.nf + f;
        const double r = b[k] - (restart ? spmv_row(Q, val, V.x, g, f) : 0.0);
        if (!restart) V.x[k] = 0.0;
        V.r[k] = r;
        V.rh[k] = r;
        V.p[k] = 0.0;
        V.v[k] = 0.0;
        rr = r * r;
        bbv = b[k] * b[k];
    }
    block_sum2(rr, bbv, part + ((size_t)g * nblk + blockIdx.x) * 2);
}

// Sum the block partials of every group in a fixed order (one block per
// group), then update that group's scalars.
//   mode 0 (after init):  rho = (rh, r) = |r|^2, |b|, |r|; alpha = omega = 1
//   mode 1 (after v):     alpha = rho / (rh, v)
//   mode 2 (after t):     omega = (t, s) / (t, t)
//   mode 3 (after x, r):  beta = (rho_new / rho) (alpha / omega), rho = rho_new, |r|
__global__ void k_bi_scalars(const double* part, int nblk, double* sc, int* flag, int mode, double rtol) {
    const int g = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
        a += part[((size_t)g * nblk + k) * 2];
        b += part[((size_t)g * nblk + k) * 2 + 1];
    }
    __shared__ double sum[2];
    block_sum2(a, b, sum);
    __syncthreads();
    if (threadIdx.x != 0 || flag[g] != 1) return;
    double* S = sc + (size_t)g * kScal;
    const double A = sum[0], B = sum[1];
    if (mode == 0) {
        S[S_RHO] = A;
        S[S_RNORM] = sqrt(A);
        S[S_BNORM] = sqrt(B);
        S[S_ALPHA] = 1.0;
        S[S_OMEGA] = 1.0;
        S[S_BETA] = 0.0;
        if (S[S_RNORM] <= rtol * S[S_BNORM]) flag[g] = 0;
    } else if (mode == 1) {
        S[S_RV] = A;
        if (A == 0.0 || !std::isfinite(A)) flag[g] = -1;     // breakdown: restart
        else S[S_ALPHA] = S[S_RHO] / A;
    } else if (mode == 2) {
        S[S_TS] = A;
        S[S_TT] = B;
        S[S_OMEGA] = B > 0.0 ? A / B : 0.0;
    } else {
        S[S_RNORM] = sqrt(B);
        if (S[S_RNORM] <= rtol * S[S_BNORM]) {
            flag[g] = 0;
        } else if (A == 0.0 || S[S_OMEGA] == 0.0 || !std::isfinite(A)) {
            flag[g] = -1;                                     // breakdown: restart
        } else {
            S[S_BETA] = (A / S[S_RHO]) * (S[S_ALPHA] / S[S_OMEGA]);
            S[S_RHO] = A;
        }
    }
}

// p = r + beta (p - omega v); ph = M^-1 p
__global__ void k_bi_p(Geo Q, Vecs V, const double* dinv, const double* sc, const int* flag) {
    const int g = blockIdx.y;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= Q.nf || flag[g] != 1) return;
    const double* S = sc + (size_t)g * kScal;
    const size_t k = (size_t)g * Q.nf + f;
    const double p = V.r[k] + S[S_BETA] * (V.p[k] - S[S_OMEGA] * V.v[k]);
    V.p[k] = p;
    V.ph[k] = dinv[k] * p;
}

// out = A in; partials of (w1, out) and (out, out) when w1 given, else of (rh, out)
__global__ void k_bi_spmv(Geo Q, const double* val, const double* in, double* out, const double* w1, const double* w2,
                          const int* flag, double* part, int nblk) {
    const int g = blockIdx.y;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (f < Q.nf && flag[g] == 1) {
        const size_t k = (size_t)g * Q.nf + f;
        const double o = spmv_row(Q, val, in, g, f);
        out[k] = o;
        a = w1[k] * o;
        b = w2 ? o * o : 0.0;
    }
    block_sum2(a, b, part + ((size_t)g * nblk + blockIdx.x) * 2);
}

// s = r - alpha v; sh = M^-1 s
__global__ void k_bi_s(Geo Q, Vecs V, const double* dinv, const double* sc, const int* flag) {
    const int g = blockIdx.y;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= Q.nf || flag[g] != 1) return;
    const size_t k = (size_t)g * Q.nf + f;
    const double s = V.r[k] - sc[(size_t)g * kScal + S_ALPHA] * V.v[k];
    V.s[k] = s;
    V.sh[k] = dinv[k] * s;
}

// x += alpha ph + omega sh; r = s - omega t; partials of (rh, r) and (r, r)
__global__ void k_bi_x(Geo Q, Vecs V, const double* sc, const int* flag, double* part, int nblk) {
    const int g = blockIdx.y;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (f < Q.nf && flag[g] == 1) {
        const double* S = sc + (size_t)g * kScal;
        const size_t k = (size_t)g * Q.nf + f;
        V.x[k] += S[S_ALPHA] * V.ph[k] + S[S_OMEGA] * V.sh[k];
        const double r = V.s[k] - S[S_OMEGA] * V.t[k];
        V.r[k] = r;
        a = V.rh[k] * r;
        b = r * r;
    }
    block_sum2(a, b, part + ((size_t)g * nblk + blockIdx.x) * 2);
}

// Cell values and face fluxes from the face solution.
__global__ void k_loqd_back(Geo Q, const double* __restrict__ kappa, const double* __restrict__ F_prev,
                            const double* __restrict__ fc, const double* __restrict__ ff,
                            const double* __restrict__ bnd, const double* __restrict__ dc,
                            const double* __restrict__ ac, const double* __restrict__ bcv,
                            const double* __restrict__ xf, double* E_cell, double* E_face, double* F_face) {
    const int g = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const double* X = xf + (size_t)g * Q.nf;
    if (t < Q.nf) E_face[(size_t)g * Q.nf + t] = X[t];
    if (t < Q.N) {
        const size_t gi = (size_t)g * Q.N + t;
        const size_t a0 = (size_t)g * 4 * Q.N + t;
        double s = bcv[gi];
        for (int k = 0; k < 4; ++k) s -= ac[a0 + (size_t)k * Q.N] * X[Q.cface[(size_t)k * Q.N + t]];
        E_cell[gi] = s / dc[gi];
    }
}

__global__ void k_loqd_flux(Geo Q, const double* __restrict__ kappa, const double* __restrict__ F_prev,
                            const double* __restrict__ fc, const double* __restrict__ ff,
                            const double* __restrict__ bnd, const double* __restrict__ E_cell,
                            const double* __restrict__ E_face, double* F_face) {
    const int g = blockIdx.y;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= Q.nf) return;
    // the half-cell relation of the cell below / left of the face (above /
    // right on the domain's low boundaries)
    const bool low_side = Q.lo[f] >= 0;
    const int cell = low_side ? Q.lo[f] : Q.hi[f];
    const int L = Q.cface[cell], R = Q.cface[Q.N + cell], B = Q.cface[2 * Q.N + cell], T = Q.cface[3 * Q.N + cell];
    const bool xf = (f == L || f == R);
    const double hn = xf ? Q.hx : Q.hy, ht = xf ? Q.hy : Q.hx;
    const double kt = kappa[(size_t)g * Q.N + cell] + 1.0 / Q.c_dt;
    const double a = kt * hn / 2.0;
    const double fnn = fc[((size_t)cell * 4 + (xf ? 0 : 2)) * Q.G + g];
    const double gnn = face_tensor(Q, ff, bnd, g, f, xf ? 0 : 2);
    const int hiT = xf ? T : R, loT = xf ? B : L;
    const double* Ef = E_face + (size_t)g * Q.nf;
    const double Ec = E_cell[(size_t)g * Q.N + cell];
    const double cross = Q.c * hn / (2.0 * ht) *
                         (face_tensor(Q, ff, bnd, g, hiT, 1) * Ef[hiT] - face_tensor(Q, ff, bnd, g, loT, 1) * Ef[loT]);
    const double Fp = F_prev[(size_t)g * Q.nf + f];
    const double grad = low_side ? (Q.c * gnn * Ef[f] - Q.c * fnn * Ec) : (Q.c * fnn * Ec - Q.c * gnn * Ef[f]);
    F_face[(size_t)g * Q.nf + f] = (-grad - cross + hn / 2.0 * Fp / Q.c_dt) / a;
}

}  // namespace

namespace {

void free_loqd(Loqd* q) {
    if (!q) return;
    for (void* p : q->owned) (void)hipFree(p);
    q->owned.clear();
    q->magic = 0;
    delete q;
}

template <typename T>
lc_status upload(Loqd* q, T** dst, const std::vector<T>& src) {
    lc_status rc = dalloc(q->owned, dst, src.size());
    if (rc) return rc;
    LC_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return LC_OK;
}

}  // namespace
}  // namespace lc

using namespace lc;

extern "C" {

lc_status lc_loqd_create(int32_t nx, int32_t ny, double lx, double ly, int32_t G, lc_loqd_t* out) {
    LC_ARG(out, "out must not be NULL");
    *out = nullptr;
    LC_ARG(nx >= 1 && ny >= 1, "nx and ny must be >= 1");
    LC_ARG(std::isfinite(lx) && lx > 0.0 && std::isfinite(ly) && ly > 0.0, "lx, ly must be finite and > 0");
    LC_ARG(G >= 1 && G <= 65535, "G must be in 1..65535");
    Loqd* q = new Loqd();
    q->nx = nx; q->ny = ny; q->G = G; q->lx = lx; q->ly = ly; q->hx = lx / nx; q->hy = ly / ny;
    q->N = nx * ny;
    q->nint = (nx - 1) * ny + nx * (ny - 1);
    q->nb = 2 * (nx + ny);
    q->nf = q->nint + q->nb;
    q->nblk = (q->nf + kLoqdBlock - 1) / kLoqdBlock;
    const int N = q->N, nf = q->nf, nint = q->nint;
    // faces of each cell (L, R, B, T) and the cells of each face
    std::vector<int> cface(4 * (size_t)N), lo(nf, -1), hi(nf, -1);
    for (int iy = 0; iy < ny; ++iy)
        for (int ix = 0; ix < nx; ++ix) {
            const int i = iy * nx + ix;
            const int L = ix > 0 ? iy * (nx - 1) + ix - 1 : nint + iy;
            const int R = ix < nx - 1 ? iy * (nx - 1) + ix : nint + ny + iy;
            const int B = iy > 0 ? (nx - 1) * ny + (iy - 1) * nx + ix : nint + 2 * ny + ix;
            const int T = iy < ny - 1 ? (nx - 1) * ny + iy * nx + ix : nint + 2 * ny + nx + ix;
            cface[i] = L; cface[N + i] = R; cface[2 * (size_t)N + i] = B; cface[3 * (size_t)N + i] = T;
            hi[L] = i; lo[R] = i; hi[B] = i; lo[T] = i;
        }
    // columns of each face row: the face, then the other faces of its cells
    std::vector<int> col((size_t)kSlots * nf);
    for (int f = 0; f < nf; ++f) {
        int c[kSlots], n = 0;
        c[n++] = f;
        for (int cell : {lo[f], hi[f]}) {
            if (cell < 0) continue;
            for (int k = 0; k < 4; ++k) {
                const int e = cface[(size_t)k * N + cell];
                bool seen = false;
                for (int s = 0; s < n; ++s) seen |= c[s] == e;
                if (!seen && n < kSlots) c[n++] = e;
            }
        }
        for (int s = n; s < kSlots; ++s) c[s] = f;           // padding: zero entries on the row itself
        for (int s = 0; s < kSlots; ++s) col[(size_t)s * nf + f] = c[s];
    }
    lc_status rc = upload(q, &q->d_cface, cface);
    if (!rc) rc = upload(q, &q->d_lo, lo);
    if (!rc) rc = upload(q, &q->d_hi, hi);
    if (!rc) rc = upload(q, &q->d_col, col);
    const size_t GN = (size_t)G * N, GF = (size_t)G * nf;
    if (!rc) rc = dalloc(q->owned, &q->d_dc, GN);
    if (!rc) rc = dalloc(q->owned, &q->d_ac, 4 * GN);
    if (!rc) rc = dalloc(q->owned, &q->d_bc, GN);
    if (!rc) rc = dalloc(q->owned, &q->d_val, (size_t)kSlots * GF);
    if (!rc) rc = dalloc(q->owned, &q->d_dinv, GF);
    if (!rc) rc = dalloc(q->owned, &q->d_b, GF);
    if (!rc) rc = dalloc(q->owned, &q->d_vec, 8 * GF);
    if (!rc) rc = dalloc(q->owned, &q->d_sh, GF);
    if (!rc) rc = dalloc(q->owned, &q->d_part, (size_t)G * q->nblk * 2);
    if (!rc) rc = dalloc(q->owned, &q->d_sc, (size_t)G * kScal);
    if (!rc) rc = dalloc(q->owned, &q->d_flag, (size_t)G);
    if (rc) {
        free_loqd(q);
        return rc;
    }
    q->magic = kLoqdMagic;
    *out = reinterpret_cast<lc_loqd_t>(q);
    return LC_OK;
}

lc_status lc_loqd_free(lc_loqd_t h) {
    if (!h) return LC_OK;
    Loqd* q = as_loqd(h);
    LC_CHECK(q, LC_ERR_STATE, "invalid LOQD handle");
    free_loqd(q);
    return LC_OK;
}

lc_status lc_loqd_solve(lc_loqd_t h, double c, double c_dt, const double* kappa, const double* planck,
                        const double* E_prev, const double* F_prev, const double* f_cell, const double* f_face,
                        const double* bnd, double* E_cell, double* E_face, double* F_face, double rtol,
                        int32_t max_iter, int32_t* iters, double* resid, void* stream) {
    Loqd* q = as_loqd(h);
    LC_CHECK(q, LC_ERR_STATE, "invalid LOQD handle");
    LC_ARG(kappa && planck && E_prev && F_prev && f_cell && bnd && E_cell && E_face && F_face,
           "inputs and outputs must not be NULL");
    LC_ARG(f_face || q->nint == 0, "f_face must not be NULL when the grid has interior faces");
    LC_ARG(std::isfinite(c) && c > 0.0 && std::isfinite(c_dt) && c_dt > 0.0, "c and c_dt must be finite and > 0");
    LC_ARG(std::isfinite(rtol) && rtol > 0.0 && rtol < 1.0, "rtol must be in (0, 1)");
    LC_ARG(max_iter >= 1, "max_iter must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int G = q->G, nf = q->nf, nblk = q->nblk;
    Geo Q{q->nx, q->ny, q->N, q->nint, nf, G, q->hx, q->hy, c, c_dt, q->d_cface, q->d_lo, q->d_hi, q->d_col};
    const dim3 blk(kLoqdBlock);
    const dim3 gc((q->N + kLoqdBlock - 1) / kLoqdBlock, G), gf(nblk, G);
    const dim3 gmax((std::max(q->N, nf) + kLoqdBlock - 1) / kLoqdBlock, G);
    hipLaunchKernelGGL(k_loqd_cells, gc, blk, 0, st, Q, kappa, planck, E_prev, F_prev, f_cell, f_face, bnd, q->d_dc,
                       q->d_ac, q->d_bc);
    hipLaunchKernelGGL(k_loqd_faces, gf, blk, 0, st, Q, kappa, F_prev, f_cell, f_face, bnd, q->d_dc, q->d_ac,
                       q->d_bc, q->d_val, q->d_dinv, q->d_b);
    LC_HIP(hipGetLastError());
    const size_t GF = (size_t)G * nf;
    Vecs V{q->d_vec, q->d_vec + GF, q->d_vec + 2 * GF, q->d_vec + 3 * GF, q->d_vec + 4 * GF, q->d_vec + 5 * GF,
           q->d_vec + 6 * GF, q->d_vec + 7 * GF, q->d_sh};
    std::vector<int> flag(G, 1), hflag(G, 1);
    std::vector<double> hsc((size_t)G * kScal);
    auto set_flags = [&](const std::vector<int>& fl) -> lc_status {
        LC_HIP(hipMemcpyAsync(q->d_flag, fl.data(), G * sizeof(int), hipMemcpyHostToDevice, st));
        return LC_OK;
    };
    lc_status rc = set_flags(flag);
    if (rc) return rc;
    hipLaunchKernelGGL(k_bi_init, gf, blk, 0, st, Q, q->d_val, q->d_b, V, q->d_flag, q->d_part, nblk, 0);
    hipLaunchKernelGGL(k_bi_scalars, dim3(G), blk, 0, st, q->d_part, nblk, q->d_sc, q->d_flag, 0, rtol);
    LC_HIP(hipGetLastError());
    // (Re)start the groups selected by sel: r = b - A x, rh = r, p = v = 0;
    // returns the device flags afterwards (1 = iterating, 0 = within rtol).
    auto restart = [&](const std::vector<int>& sel, std::vector<int>& res) -> lc_status {
        lc_status r2 = set_flags(sel);
        if (r2) return r2;
        hipLaunchKernelGGL(k_bi_init, gf, blk, 0, st, Q, q->d_val, q->d_b, V, q->d_flag, q->d_part, nblk, 1);
        hipLaunchKernelGGL(k_bi_scalars, dim3(G), blk, 0, st, q->d_part, nblk, q->d_sc, q->d_flag, 0, rtol);
        LC_HIP(hipGetLastError());
        LC_HIP(hipMemcpyAsync(res.data(), q->d_flag, G * sizeof(int), hipMemcpyDeviceToHost, st));
        LC_HIP(hipStreamSynchronize(st));
        return LC_OK;
    };
    int it = 0, true_checks = 0;
    const int check_every = 8;
    std::vector<int> sel(G), res(G);
    while (true) {
        for (int k = 0; k < check_every && it < max_iter; ++k, ++it) {
            hipLaunchKernelGGL(k_bi_p, gf, blk, 0, st, Q, V, q->d_dinv, q->d_sc, q->d_flag);
            hipLaunchKernelGGL(k_bi_spmv, gf, blk, 0, st, Q, q->d_val, V.ph, V.v, V.rh, static_cast<const double*>(nullptr),
                               q->d_flag, q->d_part, nblk);
            hipLaunchKernelGGL(k_bi_scalars, dim3(G), blk, 0, st, q->d_part, nblk, q->d_sc, q->d_flag, 1, rtol);
            hipLaunchKernelGGL(k_bi_s, gf, blk, 0, st, Q, V, q->d_dinv, q->d_sc, q->d_flag);
            hipLaunchKernelGGL(k_bi_spmv, gf, blk, 0, st, Q, q->d_val, V.sh, V.t, V.s, V.t, q->d_flag, q->d_part, nblk);
            hipLaunchKernelGGL(k_bi_scalars, dim3(G), blk, 0, st, q->d_part, nblk, q->d_sc, q->d_flag, 2, rtol);
            hipLaunchKernelGGL(k_bi_x, gf, blk, 0, st, Q, V, q->d_sc, q->d_flag, q->d_part, nblk);
            hipLaunchKernelGGL(k_bi_scalars, dim3(G), blk, 0, st, q->d_part, nblk, q->d_sc, q->d_flag, 3, rtol);
        }
        LC_HIP(hipGetLastError());
        LC_HIP(hipMemcpyAsync(hflag.data(), q->d_flag, G * sizeof(int), hipMemcpyDeviceToHost, st));
        LC_HIP(hipStreamSynchronize(st));
        bool any_broken = false;
        for (int g = 0; g < G; ++g) {
            sel[g] = hflag[g] == -1 ? 1 : 0;
            any_broken |= sel[g] != 0;
        }
        if (any_broken) {                    // restart broken groups from their current x
            rc = restart(sel, res);
            if (rc) return rc;
            for (int g = 0; g < G; ++g) flag[g] = hflag[g] == 1 ? 1 : (sel[g] ? res[g] : 0);
            rc = set_flags(flag);
            if (rc) return rc;
            hflag = flag;
        }
        bool any_running = false;
        for (int g = 0; g < G; ++g) any_running |= hflag[g] == 1;
        if (any_running && it < max_iter) continue;
        // every group stopped: check the true residual b - A x and go on with
        // those above the tolerance
        if (true_checks >= 3 || it >= max_iter) break;
        ++true_checks;
        std::fill(sel.begin(), sel.end(), 1);
        rc = restart(sel, res);
        if (rc) return rc;
        bool again = false;
        for (int g = 0; g < G; ++g) again |= res[g] == 1;
        if (!again) break;
    }
    LC_HIP(hipMemcpyAsync(hsc.data(), q->d_sc, hsc.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    hipLaunchKernelGGL(k_loqd_back, gmax, blk, 0, st, Q, kappa, F_prev, f_cell, f_face, bnd, q->d_dc, q->d_ac,
                       q->d_bc, V.x, E_cell, E_face, F_face);
    hipLaunchKernelGGL(k_loqd_flux, gf, blk, 0, st, Q, kappa, F_prev, f_cell, f_face, bnd, E_cell, E_face, F_face);
    LC_HIP(hipGetLastError());
    LC_HIP(hipStreamSynchronize(st));
    if (iters) *iters = it;
    bool ok = true;
    for (int g = 0; g < G; ++g) {
        const double rel = hsc[(size_t)g * kScal + S_BNORM] > 0.0
                               ? hsc[(size_t)g * kScal + S_RNORM] / hsc[(size_t)g * kScal + S_BNORM]
                               : 0.0;
        if (resid) resid[g] = rel;
        ok &= rel <= rtol;
    }
    LC_CHECK(ok, LC_ERR_UNSUPPORTED, "LOQD solve did not reach rtol %.3g within %d iterations", rtol, max_iter);
    return LC_OK;
}

}  // extern "C"
