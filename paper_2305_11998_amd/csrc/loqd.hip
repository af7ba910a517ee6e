// Low-order quasidiffusion (LOQD) equations of the multilevel method for one
// backward-Euler step on the material grid: the multigroup equations,
// eq. (4), closed by the transport sweep's Eddington tensors (cells:
// eq. (7), (15); faces: eq. (16)) and half-range boundary factors, and the
// effective grey equations, eq. (5), closed by spectrum averages of the
// multigroup solution, eq. (8)-(9).
//
// Discretisation (the paper cites a second-order finite-volume scheme
// without printing it; this is the reading the library implements): cell
// and face averages of E per group; the balance integrated over each cell,
//   sigma_i E_i + (F_R - F_L)/hx + (F_T - F_B)/hy = source_i;
// the first moment integrated over each half cell next to a face,
//   k (h/2) F_f = -c ((f E)_high - (f E)_low) - c h/(2 h_t) (mixed term)
//                 - (h/2) eta E_f + (h/2) F^{n-1}_f / (c dt),
// with the cell tensor times E_i at the centre, the face tensor times E_f
// on the face and the cell's transverse face averages for the mixed term;
// one normal flux per interior face; n.F = C (c E_f - Phi^-) - J^- on the
// boundary.  Eq. (4): sigma = c kappa_t, source = 4 pi kappa B +
// E^{n-1}/dt, k = kappa_t, eta = 0 (kappa_t = kappa + 1/(c dt)).  Eq. (5):
// sigma = c (<kappa>_E + 1/(c dt)), source = 4 pi <kappa>_B sum_g B_g +
// E^{n-1}/dt, k = K_R + 1/(c dt) and eta per (cell, face), so that the
// multigroup equations summed over the groups are the grey ones.
//
// The effective grey problem couples eq. (5) to the grey energy balance,
// eq. (6), with eps = c_v T: per backward-Euler step
//   c_v (T - T^{n-1})/dt = c <kappa>_E E - c <kappa>_B a_R T^4,
// solved by Newton iteration on T with the spectrum averages held fixed.
// Linearising a_R T^4 about the iterate T_k turns the energy balance into
// T = alpha + beta E per cell, which enters the grey balance as an extra
// absorption and source; each iteration is one general-form solve.
//
// Solution: a cell's balance couples E_i only to the cell's own four faces,
// so E_i is eliminated exactly:  E_i = (b_i - sum_k a_ik E_k) / d_i.  What
// remains is a system in the face unknowns alone (at most 7 entries a row:
// the face and the other faces of its one or two cells), solved for all
// groups at once by BiCGSTAB with a Jacobi preconditioner: for small
// systems by one workgroup per group that runs the whole iteration in one
// launch, for large ones by grids of blocks per vector operation with the
// host checking convergence every 8 iterations.  Every inner
// product is a fixed-order reduction (no atomics), so results are
// deterministic.  Then E_i and the face fluxes follow from the cell rows and
// the half-cell relations.
#include <algorithm>
#include <cmath>
#include <vector>

#include "lc_internal.hpp"
#include "loqd_internal.hpp"

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
    // coefficients in general form, filled from multigroup inputs by lc_loqd_solve
    double* d_sigma = nullptr;        // [G][N]
    double* d_src = nullptr;          // [G][N]
    double* d_ks = nullptr;           // [G][4][N] k per side L, R, B, T
    double* d_es = nullptr;           // [G][4][N] eta per side
    double* d_fc = nullptr;           // [G][3][N] cell tensors xx, xy, yy
    double* d_ff = nullptr;           // [G][3][nf] face tensors
    double* d_bc3 = nullptr;          // [G][nb][3] C, Phi^-, J^-
    double* d_fp = nullptr;           // [G][nf] previous normal fluxes
    // elimination and face system
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
    bool warm = false;                // BiCGSTAB starts from the E_face output's contents
    int solver = 0;                   // 0 by size, 1 one workgroup per group, 2 many blocks per group
    size_t lds_max = 0;               // LDS a workgroup may hold on this device (bytes)
    double* d_report = nullptr;       // [2][G] final relative residuals, then iterations (one-workgroup solver)
    // pinned host copies of the convergence report and of the Newton change
    // partials, so that copies queued together need one wait
    double* h_report = nullptr;       // [2][G]
    double* h_part = nullptr;         // [G * nblk]
    // a one-workgroup solve whose report was queued but not yet checked
    bool pending = false;
    double pending_rtol = 0.0;
    int pending_max_iter = 0;
    std::vector<void*> owned;
    std::vector<void*> owned_host;
};

// Face systems up to this size are solved by one workgroup per group: the
// whole iteration in one launch, reductions in LDS, no host round trips.
constexpr int kSmallFaces = 16384;
constexpr int kWG = 512;

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

// The coefficients of one group in general form (device pointers).
struct Gen {
    const double* sigma;   // [G][N]
    const double* src;     // [G][N]
    const double* ks;      // [G][4][N]
    const double* es;      // [G][4][N]
    const double* fc;      // [G][3][N]
    const double* ff;      // [G][3][nf]
    const double* bc3;     // [G][nb][3]
    const double* fp;      // [G][nf]
};

// One half-cell relation of cell `cell` at its side s (0 L, 1 R, 2 B, 3 T),
// solved for the side's normal flux: F = u E_cell + sum_k w[k] E_face(k) + k0,
// with the four face coefficients w indexed by side.
struct Rel {
    double u, w[4], k0;
};

__device__ inline Rel side_relation(const Geo& Q, const Gen& C, int g, int cell, int s) {
    const int f = Q.cface[(size_t)s * Q.N + cell];
    const bool xs = s < 2;
    const bool high = (s == 1 || s == 3);
    const double hn = xs ? Q.hx : Q.hy, ht = xs ? Q.hy : Q.hx;
    const size_t gc = (size_t)g * 4 * Q.N + (size_t)s * Q.N + cell;
    const double a = C.ks[gc] * hn / 2.0;
    const double eta = C.es[gc];
    const double fnn = C.fc[((size_t)g * 3 + (xs ? 0 : 2)) * Q.N + cell];
    const double gnn = C.ff[((size_t)g * 3 + (xs ? 0 : 2)) * Q.nf + f];
    const int hiT = xs ? 3 : 1, loT = xs ? 2 : 0;       // transverse sides: T, B or R, L
    const int fhi = Q.cface[(size_t)hiT * Q.N + cell], flo = Q.cface[(size_t)loT * Q.N + cell];
    const double x = Q.c * hn / (2.0 * ht) / a;
    Rel r;
    r.w[0] = r.w[1] = r.w[2] = r.w[3] = 0.0;
    r.u = (high ? Q.c : -Q.c) * fnn / a;
    r.w[s] += (high ? -Q.c : Q.c) * gnn / a - (hn / 2.0) * eta / a;
    r.w[hiT] -= x * C.ff[((size_t)g * 3 + 1) * Q.nf + fhi];
    r.w[loT] += x * C.ff[((size_t)g * 3 + 1) * Q.nf + flo];
    r.k0 = (hn / 2.0) * C.fp[(size_t)g * Q.nf + f] / (Q.c_dt * a);
    return r;
}

// Cell rows: d_i, a_ik and b_i of sigma_i E_i + (F_R - F_L)/hx + (F_T - F_B)/hy = source_i
// after the half-cell relations are put in for the four fluxes.
__global__ void k_loqd_cells(Geo Q, Gen C, double* dc, double* ac, double* bcv) {
    const int g = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q.N) return;
    const size_t gi = (size_t)g * Q.N + i;
    double d = C.sigma[gi], w[4] = {0.0, 0.0, 0.0, 0.0}, rhs = C.src[gi];
    for (int s = 0; s < 4; ++s) {
        const double sg = (s == 1 || s == 3 ? 1.0 : -1.0) / (s < 2 ? Q.hx : Q.hy);
        const Rel r = side_relation(Q, C, g, i, s);
        d += sg * r.u;
        for (int k = 0; k < 4; ++k) w[k] += sg * r.w[k];
        rhs -= sg * r.k0;
    }
    dc[gi] = d;
    const size_t a0 = (size_t)g * 4 * Q.N + i;
    for (int k = 0; k < 4; ++k) ac[a0 + (size_t)k * Q.N] = w[k];
    bcv[gi] = rhs;
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
__global__ void k_loqd_faces(Geo Q, Gen C, const double* __restrict__ dc, const double* __restrict__ ac,
                             const double* __restrict__ bcv, double* val, double* dinv, double* b) {
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
    for (int side = 0; side < 2; ++side) {
        const int cell = side == 0 ? Q.lo[f] : Q.hi[f];
        if (cell < 0) continue;
        const double sg = side == 0 ? 1.0 : -1.0;
        int s = 0;
        while (Q.cface[(size_t)s * Q.N + cell] != f) ++s;   // the face's side of this cell
        const Rel r = side_relation(Q, C, g, cell, s);
        for (int k = 0; k < 4; ++k) put(row, cols, Q.cface[(size_t)k * Q.N + cell], sg * r.w[k]);
        rhs -= sg * r.k0;
        // E_cell = (b_cell - sum_k a_k E_k) / d_cell
        const double beta = sg * r.u;
        const size_t gi = (size_t)g * Q.N + cell;
        const double d = dc[gi];
        const size_t a0 = (size_t)g * 4 * Q.N + cell;
        for (int k = 0; k < 4; ++k) put(row, cols, Q.cface[(size_t)k * Q.N + cell], -beta * ac[a0 + (size_t)k * Q.N] / d);
        rhs -= beta * bcv[gi] / d;
    }
    if (Q.lo[f] < 0 || Q.hi[f] < 0) {                    // n.F = C (c E_f - Phi^-) - J^-
        const double* bb = C.bc3 + ((size_t)g * (Q.nf - Q.nint) + (f - Q.nint)) * 3;
        put(row, cols, f, -bb[0] * Q.c);
        rhs += -bb[0] * bb[1] - bb[2];
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

// A workgroup sum of two values, the same bits in every thread.  Within a
// wavefront: pairs, quads, eights and sixteens by DPP lane moves (each step
// adds two equal-order operands, so every lane of a 16-lane row ends with
// the same bits), then the four rows added in row order from their first
// lanes; then the wavefronts' partials added in wavefront order by every
// thread.  Two LDS slots alternate between calls: a call writes its slot
// only after the previous call's barrier, which no thread passes before
// every thread has read that slot in the call before, so one barrier a
// call suffices -- every thread makes the same sequence of calls.
template <int Ctrl>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, Ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), Ctrl, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]: lane ^ 1
    v += dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]: lane ^ 2
    v += dpp_move<0x141>(v);   // row_half_mirror: the other quad of the eight
    v += dpp_move<0x140>(v);   // row_mirror: the other eight of the row
    return ((read_lane(v, 0) + read_lane(v, 16)) + read_lane(v, 32)) + read_lane(v, 48);
}

struct WgRed {
    double* slot;              // [2][2][kWG / 64] in LDS
    int par;
};

__device__ inline void wg_sum2(double& a, double& b, WgRed& R) {
    constexpr int W = kWG / 64;
    a = wave_sum(a);
    b = wave_sum(b);
    double* const sa = R.slot + R.par * 2 * W;
    double* const sb = sa + W;
    R.par ^= 1;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    double ta = 0.0, tb = 0.0;
    for (int k = 0; k < W; ++k) {
        ta += sa[k];
        tb += sb[k];
    }
    a = ta;
    b = tb;
}

// One workgroup per group: Jacobi-preconditioned BiCGSTAB on the face system
// of group blockIdx.x, the same iteration as the many-block kernels above
// (restart from the current x on breakdown, true-residual check when the
// recursive residual reaches rtol, at most 3 of them).  Every scalar comes
// from a fixed-order reduction that all threads read, so the control flow
// is uniform over the workgroup.  x starts from zero, or from its
// contents with warm != 0.  report[g]: the final relative residual (as
// the many-block path reports it); report[G + g]: the iterations.
//
// R: a bound on the rows each thread owns (nf <= R kWG); this form serves
// R = 16 and 32 (systems of 4097 to 16384 faces), with its vectors in
// global memory (L2) and gathers from there; smaller systems take the
// register form below.
template <int R>
__global__ __launch_bounds__(kWG) void k_bicg_group(Geo Q, const double* __restrict__ val, const double* __restrict__ bv,
                                                     const double* __restrict__ dinv, Vecs V, int warm, double rtol,
                                                     int max_iter, double* report) {
    __shared__ double red[4 * (kWG / 64)];
    WgRed rd{red, 0};
    const int g = blockIdx.x, nf = Q.nf, tid = threadIdx.x;
    const size_t o = (size_t)g * nf;
    double *x = V.x + o, *r = V.r + o, *rh = V.rh + o, *p = V.p + o, *v = V.v + o;
    double *s = V.s + o, *t = V.t + o, *ph = V.ph + o, *sh = V.sh + o;
    const double* b = bv + o;
    const double* di = dinv + o;
    auto rows = [&](auto fn) {
#pragma unroll 1
        for (int j = 0; j < R; ++j) {
            const int f = tid + j * kWG;
            if (f < nf) fn(f);
        }
    };
    // row f of A times u (this group's vector)
    auto prod = [&](const double* u, int f) -> double {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int cidx = Q.col[(size_t)k * nf + f];
            const double a = val[((size_t)g * kSlots + k) * nf + f];
            acc += a * u[cidx];
        }
        return acc;
    };
    // make u readable by the products of every thread
    auto stage = [&](const double*) { __syncthreads(); };
    if (!warm) rows([&](int f) { x[f] = 0.0; });
    __syncthreads();
    // r = b - A x, rh = r, p = v = 0; returns (r, r) and (b, b)
    auto restart = [&](double& rr, double& bb) {
        stage(x);
        rr = 0.0;
        bb = 0.0;
        rows([&](int f) {
            const double e = b[f] - prod(x, f);
            r[f] = e;
            rh[f] = e;
            p[f] = 0.0;
            v[f] = 0.0;
            rr += e * e;
            bb += b[f] * b[f];
        });
        wg_sum2(rr, bb, rd);
    };
    double rr, bb;
    restart(rr, bb);
    const double bnorm = sqrt(bb);
    if (bnorm == 0.0) rows([&](int f) { x[f] = 0.0; });   // b = 0: x = 0
    double rho = rr, alpha = 1.0, omega = 1.0, beta = 0.0, rnorm = bnorm == 0.0 ? 0.0 : sqrt(rr);
    int it = 0, checks = 0;
    bool done = bnorm == 0.0 || rnorm <= rtol * bnorm;
    while (bnorm > 0.0) {
        if (done) {                                   // true residual
            if (checks >= 3) break;
            ++checks;
            restart(rr, bb);
            rnorm = sqrt(rr);
            rho = rr;
            alpha = omega = 1.0;
            beta = 0.0;
            if (rnorm <= rtol * bnorm) break;
            done = false;
        }
        if (it >= max_iter) break;
        ++it;
        rows([&](int f) {
            const double pv = r[f] + beta * (p[f] - omega * v[f]);
            const double q = di[f] * pv;
            p[f] = pv;
            ph[f] = q;
        });
        __syncthreads();
        double a = 0.0, c = 0.0;
        rows([&](int f) {
            const double vv = prod(ph, f);
            v[f] = vv;
            a += rh[f] * vv;
        });
        wg_sum2(a, c, rd);
        if (a == 0.0 || !std::isfinite(a)) {          // breakdown: restart from x
            restart(rr, bb);
            rho = rr;
            alpha = omega = 1.0;
            beta = 0.0;
            rnorm = sqrt(rr);
            done = rnorm <= rtol * bnorm;
            continue;
        }
        alpha = rho / a;
        rows([&](int f) {
            const double sv = r[f] - alpha * v[f];
            const double q = di[f] * sv;
            s[f] = sv;
            sh[f] = q;
        });
        __syncthreads();
        a = 0.0;
        c = 0.0;
        rows([&](int f) {
            const double tv = prod(sh, f);
            t[f] = tv;
            a += tv * s[f];
            c += tv * tv;
        });
        wg_sum2(a, c, rd);
        omega = c > 0.0 ? a / c : 0.0;
        a = 0.0;
        c = 0.0;
        rows([&](int f) {
            x[f] += alpha * ph[f] + omega * sh[f];
            const double rv = s[f] - omega * t[f];
            r[f] = rv;
            a += rh[f] * rv;
            c += rv * rv;
        });
        wg_sum2(a, c, rd);
        rnorm = sqrt(c);
        if (rnorm <= rtol * bnorm) {
            done = true;
        } else if (a == 0.0 || omega == 0.0 || !std::isfinite(a)) {
            restart(rr, bb);
            rho = rr;
            alpha = omega = 1.0;
            beta = 0.0;
            rnorm = sqrt(rr);
            done = rnorm <= rtol * bnorm;
        } else {
            beta = (a / rho) * (alpha / omega);
            rho = a;
        }
    }
    // As the many-block path: the residual of the last test -- the true one
    // after a passed check, the recursive one once the three checks are
    // spent -- and the true one when the iterations ran out.
    if (!done && bnorm > 0.0 && it >= max_iter) {
        stage(x);
        double e2 = 0.0, unused = 0.0;
        rows([&](int f) {
            const double e = b[f] - prod(x, f);
            e2 += e * e;
        });
        wg_sum2(e2, unused, rd);
        rnorm = sqrt(e2);
    }
    if (tid == 0) {
        report[g] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
        report[gridDim.x + g] = it;
    }
}

// Register form for systems of up to R <= 8 rows a thread (nf <= 4096): the
// iterate and the BiCGSTAB vectors of a thread's rows stay in registers,
// the vector a product gathers from is staged in LDS, and only the matrix
// (values and columns) is read from memory in an iteration.  The arithmetic
// and the order of every sum are those of k_bicg_group, row by row; x is
// read (warm != 0) and written in xv only at the ends.
template <int R>
__global__ __launch_bounds__(kWG) void k_bicg_reg(Geo Q, const double* __restrict__ val,
                                                   const double* __restrict__ bv, const double* __restrict__ dinv,
                                                   double* __restrict__ xv, int warm, double rtol, int max_iter,
                                                   double* report) {
    // With R <= 4 a product is unrolled over the thread's rows, all of
    // their matrix loads in flight together.  With R = 8 those loads do not
    // fit beside the vectors: the products then run row by row (no
    // unrolling) into LDS, from where each thread takes its own rows.  In
    // both, the matrix is read again (from L2) in every product.
    constexpr bool kRowLoop = R > 4;
    extern __shared__ double gsv[];                   // [nf] the gathered vector; [nf] products, r^, 1/diag (kRowLoop)
    __shared__ double red[4 * (kWG / 64)];
    WgRed rd{red, 0};
    const int g = blockIdx.x, nf = Q.nf, tid = threadIdx.x;
    const size_t o = (size_t)g * nf;
    const gptr<const double> vg = as_global(val + (size_t)g * kSlots * nf);
    const gptr<const int> cg = as_global(Q.col);
    const gptr<const double> b = as_global(bv + o);
    double x[R], r[R], p[R], v[R], s[R], t[R];
    // r^ and the inverse diagonal: registers, or (kRowLoop) LDS slots
    // [R kWG] each after the two [nf] vectors, one per (thread, row) and
    // touched by that thread only
    constexpr int RR = kRowLoop ? 1 : R;
    double rh_r[RR], di_r[RR];
    double* const rh_l = gsv + 2 * (size_t)nf;
    double* const di_l = rh_l + R * kWG;
    auto RH = [&](int j) -> double& {
        if constexpr (kRowLoop) return rh_l[tid + j * kWG];
        else return rh_r[j];
    };
    auto DI = [&](int j) -> double& {
        if constexpr (kRowLoop) return di_l[tid + j * kWG];
        else return di_r[j];
    };
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int f = tid + j * kWG;
        const bool ok = f < nf;
        DI(j) = ok ? dinv[o + f] : 0.0;
        x[j] = ok && warm ? xv[o + f] : 0.0;
        r[j] = RH(j) = p[j] = v[j] = s[j] = t[j] = 0.0;
    }
    // row f of A times the staged vector
    auto prod = [&](int f) -> double {
        int ci[kSlots];
        double av[kSlots];
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            ci[k] = cg[(size_t)k * nf + f];
            av[k] = vg[(size_t)k * nf + f];
        }
        // all of the row's loads, then all of its gathers, in flight before
        // the first use (left to itself the scheduler waits on each entry
        // in turn)
        if constexpr (kRowLoop) __builtin_amdgcn_sched_barrier(0);
        double gv[kSlots];
#pragma unroll
        for (int k = 0; k < kSlots; ++k) gv[k] = gsv[ci[k]];
        if constexpr (kRowLoop) __builtin_amdgcn_sched_barrier(0);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kSlots; ++k) acc += av[k] * gv[k];
        return acc;
    };
    // y_j = (A u)_f for this thread's rows f; out-of-range rows untouched
    auto spmv = [&](double (&y)[R]) {
        if constexpr (kRowLoop) {
            double* out = gsv + nf;
#pragma unroll 1
            for (int j = 0; j < R; ++j) {
                const int f = tid + j * kWG;
                if (f < nf) out[f] = prod(f);
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int f = tid + j * kWG;
                if (f < nf) y[j] = out[f];
            }
        } else {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int f = tid + j * kWG;
                if (f < nf) y[j] = prod(f);
            }
        }
    };
    auto stage = [&](const double (&u)[R]) {
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int f = tid + j * kWG;
            if (f < nf) gsv[f] = u[j];
        }
        __syncthreads();
    };
    // r = b - A x, rh = r, p = v = 0; returns (r, r) and (b, b)
    auto restart = [&](double& rr, double& bb) {
        stage(x);
        spmv(v);                                      // v is reset below
        rr = 0.0;
        bb = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int f = tid + j * kWG;
            if (f < nf) {
                const double bf = b[f];
                const double e = bf - v[j];
                r[j] = e;
                RH(j) = e;
                p[j] = 0.0;
                v[j] = 0.0;
                rr += e * e;
                bb += bf * bf;
            }
        }
        wg_sum2(rr, bb, rd);
    };
    double rr, bb;
    restart(rr, bb);
    const double bnorm = sqrt(bb);
    if (bnorm == 0.0)
#pragma unroll
        for (int j = 0; j < R; ++j) x[j] = 0.0;
    double rho = rr, alpha = 1.0, omega = 1.0, beta = 0.0, rnorm = bnorm == 0.0 ? 0.0 : sqrt(rr);
    int it = 0, checks = 0;
    bool done = bnorm == 0.0 || rnorm <= rtol * bnorm;
    while (bnorm > 0.0) {
        if (done) {                                   // true residual
            if (checks >= 3) break;
            ++checks;
            restart(rr, bb);
            rnorm = sqrt(rr);
            rho = rr;
            alpha = omega = 1.0;
            beta = 0.0;
            if (rnorm <= rtol * bnorm) break;
            done = false;
        }
        if (it >= max_iter) break;
        ++it;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int f = tid + j * kWG;
            p[j] = r[j] + beta * (p[j] - omega * v[j]);
            if (f < nf) gsv[f] = DI(j) * p[j];
        }
        __syncthreads();
        double a = 0.0, c = 0.0;
        spmv(v);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int f = tid + j * kWG;
            if (f < nf) a += RH(j) * v[j];
        }
        wg_sum2(a, c, rd);
        if (a == 0.0 || !std::isfinite(a)) {          // breakdown: restart from x
            restart(rr, bb);
            rho = rr;
            alpha = omega = 1.0;
            beta = 0.0;
            rnorm = sqrt(rr);
            done = rnorm <= rtol * bnorm;
            continue;
        }
        alpha = rho / a;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int f = tid + j * kWG;
            s[j] = r[j] - alpha * v[j];
            if (f < nf) gsv[f] = DI(j) * s[j];
        }
        __syncthreads();
        a = 0.0;
        c = 0.0;
        spmv(t);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int f = tid + j * kWG;
            if (f < nf) {
                a += t[j] * s[j];
                c += t[j] * t[j];
            }
        }
        wg_sum2(a, c, rd);
        omega = c > 0.0 ? a / c : 0.0;
        a = 0.0;
        c = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int f = tid + j * kWG;
            if (f < nf) {
                const double d = DI(j);
                x[j] += alpha * (d * p[j]) + omega * (d * s[j]);
                r[j] = s[j] - omega * t[j];
                a += RH(j) * r[j];
                c += r[j] * r[j];
            }
        }
        wg_sum2(a, c, rd);
        rnorm = sqrt(c);
        if (rnorm <= rtol * bnorm) {
            done = true;
        } else if (a == 0.0 || omega == 0.0 || !std::isfinite(a)) {
            restart(rr, bb);
            rho = rr;
            alpha = omega = 1.0;
            beta = 0.0;
            rnorm = sqrt(rr);
            done = rnorm <= rtol * bnorm;
        } else {
            beta = (a / rho) * (alpha / omega);
            rho = a;
        }
    }
    if (!done && bnorm > 0.0 && it >= max_iter) {
        stage(x);
        spmv(t);
        double e2 = 0.0, unused = 0.0;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int f = tid + j * kWG;
            if (f < nf) {
                const double e = b[f] - t[j];
                e2 += e * e;
            }
        }
        wg_sum2(e2, unused, rd);
        rnorm = sqrt(e2);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int f = tid + j * kWG;
        if (f < nf) xv[o + f] = x[j];
    }
    if (tid == 0) {
        report[g] = bnorm > 0.0 ? rnorm / bnorm : 0.0;
        report[gridDim.x + g] = it;
    }
}

__global__ void k_loqd_back(Geo Q, const double* __restrict__ dc, const double* __restrict__ ac,
                            const double* __restrict__ bcv, const double* __restrict__ xf, double* E_cell,
                            double* E_face) {
    const int g = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const double* X = xf + (size_t)g * Q.nf;
    if (t < Q.nf && xf != E_face) E_face[(size_t)g * Q.nf + t] = X[t];   // the solver may have written E_face
    if (t < Q.N) {
        const size_t gi = (size_t)g * Q.N + t;
        const size_t a0 = (size_t)g * 4 * Q.N + t;
        double s = bcv[gi];
        for (int k = 0; k < 4; ++k) s -= ac[a0 + (size_t)k * Q.N] * X[Q.cface[(size_t)k * Q.N + t]];
        E_cell[gi] = s / dc[gi];
    }
}

// Face fluxes from the half-cell relation of the cell below / left of the
// face (above / right on the domain's low boundaries).
__global__ void k_loqd_flux(Geo Q, Gen C, const double* __restrict__ E_cell, const double* __restrict__ E_face,
                            double* F_face) {
    const int g = blockIdx.y;
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= Q.nf) return;
    const int cell = Q.lo[f] >= 0 ? Q.lo[f] : Q.hi[f];
    int s = 0;
    while (Q.cface[(size_t)s * Q.N + cell] != f) ++s;
    const Rel r = side_relation(Q, C, g, cell, s);
    const double* Ef = E_face + (size_t)g * Q.nf;
    double F = r.u * E_cell[(size_t)g * Q.N + cell] + r.k0;
    for (int k = 0; k < 4; ++k) F += r.w[k] * Ef[Q.cface[(size_t)k * Q.N + cell]];
    F_face[(size_t)g * Q.nf + f] = F;
}

// Multigroup inputs (eq. (4)) in general form.
__device__ inline void loqd_prep_cell(const Geo& Q, int g, int i, const double* __restrict__ kappa,
                                      const double* __restrict__ planck, const double* __restrict__ E_prev,
                                      const double* __restrict__ f_cell, double* sigma, double* src, double* ks,
                                      double* es, double* fc) {
    const size_t gi = (size_t)g * Q.N + i;
    const double kap = kappa[gi];
    const double kt = kap + 1.0 / Q.c_dt;
    sigma[gi] = Q.c * kt;
    src[gi] = 4.0 * kPi * kap * planck[gi] + Q.c * E_prev[gi] / Q.c_dt;
    for (int s = 0; s < 4; ++s) {
        ks[(size_t)g * 4 * Q.N + (size_t)s * Q.N + i] = kt;
        es[(size_t)g * 4 * Q.N + (size_t)s * Q.N + i] = 0.0;
    }
    for (int q = 0; q < 3; ++q) fc[((size_t)g * 3 + q) * Q.N + i] = f_cell[((size_t)i * 4 + q) * Q.G + g];
}

__device__ inline void loqd_prep_face(const Geo& Q, int g, int f, const double* __restrict__ F_prev,
                                      const double* __restrict__ f_face, const double* __restrict__ bnd, double* ff,
                                      double* bc3, double* fp) {
    const int nb = Q.nf - Q.nint;
    for (int q = 0; q < 3; ++q)
        ff[((size_t)g * 3 + q) * Q.nf + f] = f < Q.nint ? f_face[((size_t)f * 4 + q) * Q.G + g]
                                                        : bnd[((size_t)g * nb + (f - Q.nint)) * 8 + 5 + q];
    fp[(size_t)g * Q.nf + f] = F_prev[(size_t)g * Q.nf + f];
    if (f >= Q.nint) {
        const double* bb = bnd + ((size_t)g * nb + (f - Q.nint)) * 8;
        double* o = bc3 + ((size_t)g * nb + (f - Q.nint)) * 3;
        o[0] = bb[4];
        o[1] = bb[2];
        o[2] = bb[3];
    }
}

// Both preparations in one launch: thread t takes cell t and face t.
__global__ void k_loqd_prep(Geo Q, const double* __restrict__ kappa, const double* __restrict__ planck,
                            const double* __restrict__ E_prev, const double* __restrict__ f_cell,
                            const double* __restrict__ F_prev, const double* __restrict__ f_face,
                            const double* __restrict__ bnd, double* sigma, double* src, double* ks, double* es,
                            double* fc, double* ff, double* bc3, double* fp) {
    const int g = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < Q.N) loqd_prep_cell(Q, g, t, kappa, planck, E_prev, f_cell, sigma, src, ks, es, fc);
    if (t < Q.nf) loqd_prep_face(Q, g, t, F_prev, f_face, bnd, ff, bc3, fp);
}

// Grey coefficients (eq. (5) in general form) from a multigroup solution:
// per cell the energy-weighted and Planck-weighted opacities, per cell side
// K_R from the normal face fluxes and eta, and the cell's spectrum-averaged
// tensor; fixed-order sums over the groups.
// Sum over the eight lanes of a cell in a fixed butterfly: every lane ends
// with the same total.
__device__ inline double sum8(double v) {
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 1);
    return v;
}

// Cell i's grey coefficients by its eight lanes (j = 0..7, consecutive in a
// wavefront): lane j takes groups j, j + 8, ..., the partial sums meet in
// sum8, and lane 0 writes.
__device__ inline void grey_cell(const Geo& Q, int i, int j, const double* __restrict__ kappa,
                                 const double* __restrict__ planck, const double* __restrict__ E_prev,
                                 const double* __restrict__ f_cell, const double* __restrict__ E_cell,
                                 const double* __restrict__ E_face, const double* __restrict__ F_face, double* sigma,
                                 double* src, double* ks, double* es, double* fc, double* Ep, double* kEo,
                                 double* kBo) {
    const int G = Q.G;
    double E = 0.0, kE = 0.0, sB = 0.0, kB = 0.0, sk = 0.0, ep = 0.0, t[3] = {0.0, 0.0, 0.0};
    for (int g = j; g < G; g += 8) {
        const size_t gi = (size_t)g * Q.N + i;
        const double e = E_cell[gi], k = kappa[gi], b = planck[gi];
        E += e;
        kE += k * e;
        sB += b;
        kB += k * b;
        sk += k;
        ep += E_prev[gi];
        for (int q = 0; q < 3; ++q) t[q] += f_cell[((size_t)i * 4 + q) * G + g] * e;
    }
    E = sum8(E);
    kE = sum8(kE);
    sB = sum8(sB);
    kB = sum8(kB);
    sk = sum8(sk);
    ep = sum8(ep);
    for (int q = 0; q < 3; ++q) t[q] = sum8(t[q]);
    const double mean_k = sk / G;
    double avgB = sB != 0.0 ? kB / sB : NAN;
    const double avgE = E != 0.0 ? kE / E : (std::isnan(avgB) ? mean_k : avgB);
    if (std::isnan(avgB)) avgB = avgE;
    if (j == 0) {
        sigma[i] = Q.c * (avgE + 1.0 / Q.c_dt);
        src[i] = 4.0 * kPi * avgB * sB + Q.c * ep / Q.c_dt;
        if (kEo) kEo[i] = avgE;
        if (kBo) kBo[i] = avgB;
        Ep[i] = ep;
        fc[i] = E != 0.0 ? t[0] / E : 1.0 / 3.0;
        fc[Q.N + i] = E != 0.0 ? t[1] / E : 0.0;
        fc[2 * (size_t)Q.N + i] = E != 0.0 ? t[2] / E : 1.0 / 3.0;
    }
    for (int s = 0; s < 4; ++s) {
        const int f = Q.cface[(size_t)s * Q.N + i];
        double aF = 0.0, kaF = 0.0, Ef = 0.0;
        for (int g = j; g < G; g += 8) {
            const double F = F_face[(size_t)g * Q.nf + f];
            aF += fabs(F);
            kaF += kappa[(size_t)g * Q.N + i] * fabs(F);
            Ef += E_face[(size_t)g * Q.nf + f];
        }
        aF = sum8(aF);
        kaF = sum8(kaF);
        Ef = sum8(Ef);
        const double K = aF != 0.0 ? kaF / aF : avgE;
        double num = 0.0;
        for (int g = j; g < G; g += 8) num += (kappa[(size_t)g * Q.N + i] - K) * F_face[(size_t)g * Q.nf + f];
        num = sum8(num);
        if (j == 0) {
            ks[(size_t)s * Q.N + i] = K + 1.0 / Q.c_dt;
            es[(size_t)s * Q.N + i] = Ef != 0.0 ? num / Ef : 0.0;
        }
    }
}

__device__ inline void grey_face(const Geo& Q, int f, const double* __restrict__ F_prev,
                                 const double* __restrict__ f_face, const double* __restrict__ bnd,
                                 const double* __restrict__ E_face, double* ff, double* bc3, double* fp) {
    const int G = Q.G, nb = Q.nf - Q.nint;
    double Ef = 0.0, t[3] = {0.0, 0.0, 0.0}, p = 0.0, cE = 0.0, cs = 0.0, jm = 0.0;
#pragma unroll 4
    for (int g = 0; g < G; ++g) {
        const double e = E_face[(size_t)g * Q.nf + f];
        Ef += e;
        p += F_prev[(size_t)g * Q.nf + f];
        for (int q = 0; q < 3; ++q)
            t[q] += (f < Q.nint ? f_face[((size_t)f * 4 + q) * G + g]
                                : bnd[((size_t)g * nb + (f - Q.nint)) * 8 + 5 + q]) * e;
        if (f >= Q.nint) {
            const double* bb = bnd + ((size_t)g * nb + (f - Q.nint)) * 8;
            cE += bb[4] * e;
            cs += bb[4];
            jm += bb[4] * bb[2] + bb[3];
        }
    }
    ff[f] = Ef != 0.0 ? t[0] / Ef : 1.0 / 3.0;
    ff[Q.nf + f] = Ef != 0.0 ? t[1] / Ef : 0.0;
    ff[2 * (size_t)Q.nf + f] = Ef != 0.0 ? t[2] / Ef : 1.0 / 3.0;
    fp[f] = p;
    if (f >= Q.nint) {
        double* o = bc3 + (size_t)(f - Q.nint) * 3;
        o[0] = Ef != 0.0 ? cE / Ef : cs / G;
        o[1] = 0.0;
        o[2] = jm;
    }
}

// Both in one launch: threads 8i .. 8i + 7 take cell i, thread t face t.
__global__ void k_grey_coef(Geo Q, const double* __restrict__ kappa, const double* __restrict__ planck,
                            const double* __restrict__ E_prev, const double* __restrict__ f_cell,
                            const double* __restrict__ E_cell, const double* __restrict__ E_face,
                            const double* __restrict__ F_face, const double* __restrict__ F_prev,
                            const double* __restrict__ f_face, const double* __restrict__ bnd, double* sigma,
                            double* src, double* ks, double* es, double* fc, double* Ep, double* kEo, double* kBo,
                            double* ff, double* bc3, double* fp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 8 * Q.N)                  // whole groups of eight lanes
        grey_cell(Q, t >> 3, t & 7, kappa, planck, E_prev, f_cell, E_cell, E_face, F_face, sigma, src, ks, es, fc, Ep,
                  kEo, kBo);
    if (t < Q.nf) grey_face(Q, t, F_prev, f_face, bnd, E_face, ff, bc3, fp);
}

// Grey energy balance, eq. (6) with eps = c_v T (inputs of one Newton
// iteration; arrays [G][N], one independent grey problem per group index).
struct Meb {
    const double* kE;      // <kappa>_E
    const double* kB;      // <kappa>_B
    const double* Ep;      // E^{n-1}
    const double* Tp;      // T^{n-1}
    double cv_dt;          // c_v / dt
    double a;              // a_R
};

// alpha, beta of T = alpha + beta E from the energy balance with a_R T^4
// linearised about T_k: a_R T^4 ~ A + D (T - T_k), A = a_R T_k^4,
// D = 4 a_R T_k^3.
struct MebLin {
    double A, D, alpha, beta;
};

__device__ inline MebLin meb_lin(const Geo& Q, const Meb& M, size_t gi, double Tk) {
    MebLin l;
    const double T2 = Tk * Tk;
    l.A = M.a * T2 * T2;
    l.D = 4.0 * M.a * T2 * Tk;
    const double ckB = Q.c * M.kB[gi];
    const double den = M.cv_dt + ckB * l.D;
    l.beta = Q.c * M.kE[gi] / den;
    l.alpha = (M.cv_dt * M.Tp[gi] - ckB * (l.A - l.D * Tk)) / den;
    return l;
}

// Grey balance of one Newton iteration: the emission c <kappa>_B a_R T^4
// with T = alpha + beta E moves c <kappa>_B D beta E to the left-hand side.
__global__ void k_meb_linearise(Geo Q, Meb M, const double* __restrict__ T, double* sigma, double* src) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q.N) return;
    const size_t gi = (size_t)blockIdx.y * Q.N + i;
    const double Tk = T[gi];
    const MebLin l = meb_lin(Q, M, gi, Tk);
    const double ckB = Q.c * M.kB[gi];
    sigma[gi] = Q.c * (M.kE[gi] + 1.0 / Q.c_dt) - ckB * l.D * l.beta;
    src[gi] = Q.c * M.Ep[gi] / Q.c_dt + ckB * (l.A + l.D * (l.alpha - Tk));
}

// T_{k+1} = alpha + beta E in place; per block the largest relative change
// |T_{k+1} - T_k| / |T_{k+1}| (infinity where it is not finite).
__global__ void k_meb_update(Geo Q, Meb M, double* T, const double* __restrict__ E, double* part, int nblk) {
    __shared__ double sm[kLoqdBlock];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double ch = 0.0;
    if (i < Q.N) {
        const size_t gi = (size_t)blockIdx.y * Q.N + i;
        const double Tk = T[gi];
        const MebLin l = meb_lin(Q, M, gi, Tk);
        const double Tn = l.alpha + l.beta * E[gi];
        T[gi] = Tn;
        ch = fabs(Tn - Tk) / fabs(Tn);
        if (!std::isfinite(ch)) ch = INFINITY;
    }
    sm[threadIdx.x] = ch;
    __syncthreads();
    for (int w = kLoqdBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)blockIdx.y * nblk + blockIdx.x] = sm[0];
}

}  // namespace

namespace {

void free_loqd(Loqd* q) {
    if (!q) return;
    for (void* p : q->owned) (void)hipFree(p);
    q->owned.clear();
    for (void* p : q->owned_host) (void)hipHostFree(p);
    q->owned_host.clear();
    q->magic = 0;
    delete q;
}

// pinned host allocation owned by a vector of pointers
template <typename T>
lc_status halloc(std::vector<void*>& owned, T** out, size_t n) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipHostMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
        return LC_ERR_ALLOC;
    }
    owned.push_back(p);
    *out = static_cast<T*>(p);
    return LC_OK;
}

template <typename T>
lc_status upload(Loqd* q, T** dst, const std::vector<T>& src) {
    lc_status rc = dalloc(q->owned, dst, src.size());
    if (rc) return rc;
    LC_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
    return LC_OK;
}

Geo geo(const Loqd* q, double c, double c_dt, int G) {
    return Geo{q->nx, q->ny, q->N, q->nint, q->nf, G, q->hx, q->hy, c, c_dt, q->d_cface, q->d_lo, q->d_hi, q->d_col};
}

// Assemble and solve the general-form system of every group; outputs E_cell
// [G][N], E_face [G][nf], F_face [G][nf].
// Check the queued report of the last one-workgroup solve (the caller has
// synchronised the stream since): iterations (the most of any group) and
// residuals to iters / resid, LC_ERR_UNSUPPORTED if a group missed rtol.
lc_status check_report(Loqd* q, int32_t* iters, double* resid) {
    if (!q->pending) return LC_OK;
    q->pending = false;
    int most = 0;
    double worst = 0.0;
    for (int g = 0; g < q->G; ++g) {
        const double rg = q->h_report[g];
        most = std::max(most, (int)q->h_report[q->G + g]);
        if (resid) resid[g] = rg;
        worst = std::max(worst, std::isfinite(rg) ? rg : INFINITY);
    }
    if (iters) *iters = most;
    LC_CHECK(worst <= q->pending_rtol, LC_ERR_UNSUPPORTED,
             "LOQD solve did not reach rtol %.3g: residual %.3g after %d iterations (limit %d)", q->pending_rtol,
             worst, most, q->pending_max_iter);
    return LC_OK;
}

// With defer, a one-workgroup solve only queues the copies of its report:
// the caller checks it with check_report after its next wait on the stream.
lc_status solve_general(Loqd* q, const Geo& Q, const Gen& Cg, double* E_cell, double* E_face, double* F_face,
                        double rtol, int max_iter, int32_t* iters, double* resid, hipStream_t st,
                        bool defer = false) {
    if (q->pending) {                 // a deferred report not yet read
        LC_HIP(hipStreamSynchronize(st));
        lc_status rc = check_report(q, nullptr, nullptr);
        if (rc) return rc;
    }
    const int G = Q.G, nf = q->nf, nblk = q->nblk;
    const dim3 blk(kLoqdBlock);
    const dim3 gc((q->N + kLoqdBlock - 1) / kLoqdBlock, G), gf(nblk, G);
    const dim3 gmax((std::max(q->N, nf) + kLoqdBlock - 1) / kLoqdBlock, G);
    hipLaunchKernelGGL(k_loqd_cells, gc, blk, 0, st, Q, Cg, q->d_dc, q->d_ac, q->d_bc);
    hipLaunchKernelGGL(k_loqd_faces, gf, blk, 0, st, Q, Cg, q->d_dc, q->d_ac, q->d_bc, q->d_val, q->d_dinv, q->d_b);
    LC_HIP(hipGetLastError());
    const size_t GF = (size_t)G * nf;
    Vecs V{q->d_vec, q->d_vec + GF, q->d_vec + 2 * GF, q->d_vec + 3 * GF, q->d_vec + 4 * GF, q->d_vec + 5 * GF,
           q->d_vec + 6 * GF, q->d_vec + 7 * GF, q->d_sh};
    if (q->solver != 2 && nf <= kSmallFaces) {
        const int rows_per_thread = (nf + kWG - 1) / kWG;
        // R = 8: the products and the [8 kWG] slots of r^ and 1/diag in LDS
        // too; where the device cannot give a workgroup that much, the
        // global-vector form (same arithmetic) takes these sizes
        const size_t lds = rows_per_thread > 4 ? (2 * (size_t)nf + 2 * 8 * kWG) * sizeof(double)
                                               : (size_t)nf * sizeof(double);
        const bool reg_form = rows_per_thread <= 4 || (rows_per_thread <= 8 && lds <= q->lds_max);
        // the register form starts from and writes E_face itself
        double* xf = reg_form ? E_face : V.x;
        if (q->warm && xf != E_face)
            LC_HIP(hipMemcpyAsync(V.x, E_face, GF * sizeof(double), hipMemcpyDeviceToDevice, st));
        {
            const int wv = q->warm ? 1 : 0;
            auto reg = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(G), dim3(kWG), lds, st, Q, q->d_val, q->d_b, q->d_dinv, xf, wv, rtol,
                                   max_iter, q->d_report);
            };
            auto glob = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(G), dim3(kWG), 0, st, Q, q->d_val, q->d_b, q->d_dinv, V, wv, rtol,
                                   max_iter, q->d_report);
            };
            if (rows_per_thread <= 1) reg(k_bicg_reg<1>);
            else if (rows_per_thread <= 2) reg(k_bicg_reg<2>);
            else if (rows_per_thread <= 4) reg(k_bicg_reg<4>);
            else if (reg_form) reg(k_bicg_reg<8>);
            else if (rows_per_thread <= 16) glob(k_bicg_group<16>);
            else glob(k_bicg_group<32>);
        }
        hipLaunchKernelGGL(k_loqd_back, gmax, blk, 0, st, Q, q->d_dc, q->d_ac, q->d_bc, xf, E_cell, E_face);
        hipLaunchKernelGGL(k_loqd_flux, gf, blk, 0, st, Q, Cg, E_cell, E_face, F_face);
        LC_HIP(hipGetLastError());
        LC_HIP(hipMemcpyAsync(q->h_report, q->d_report, 2 * G * sizeof(double), hipMemcpyDeviceToHost, st));
        q->pending = true;
        q->pending_rtol = rtol;
        q->pending_max_iter = max_iter;
        if (defer) return LC_OK;
        LC_HIP(hipStreamSynchronize(st));
        return check_report(q, iters, resid);
    }
    std::vector<int> flag(G, 1), hflag(G, 1);
    std::vector<double> hsc((size_t)G * kScal);
    auto set_flags = [&](const std::vector<int>& fl) -> lc_status {
        LC_HIP(hipMemcpyAsync(q->d_flag, fl.data(), G * sizeof(int), hipMemcpyHostToDevice, st));
        return LC_OK;
    };
    lc_status rc = set_flags(flag);
    if (rc) return rc;
    if (q->warm) LC_HIP(hipMemcpyAsync(V.x, E_face, GF * sizeof(double), hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_bi_init, gf, blk, 0, st, Q, q->d_val, q->d_b, V, q->d_flag, q->d_part, nblk,
                       q->warm ? 1 : 0);
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
    hipLaunchKernelGGL(k_loqd_back, gmax, blk, 0, st, Q, q->d_dc, q->d_ac, q->d_bc, V.x, E_cell, E_face);
    hipLaunchKernelGGL(k_loqd_flux, gf, blk, 0, st, Q, Cg, E_cell, E_face, F_face);
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
    if (!rc) rc = dalloc(q->owned, &q->d_sigma, GN);
    if (!rc) rc = dalloc(q->owned, &q->d_src, GN);
    if (!rc) rc = dalloc(q->owned, &q->d_ks, 4 * GN);
    if (!rc) rc = dalloc(q->owned, &q->d_es, 4 * GN);
    if (!rc) rc = dalloc(q->owned, &q->d_fc, 3 * GN);
    if (!rc) rc = dalloc(q->owned, &q->d_ff, 3 * GF);
    if (!rc) rc = dalloc(q->owned, &q->d_bc3, 3 * (size_t)G * q->nb);
    if (!rc) rc = dalloc(q->owned, &q->d_fp, GF);
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
    if (!rc) rc = dalloc(q->owned, &q->d_report, 2 * (size_t)G);
    if (!rc) rc = halloc(q->owned_host, &q->h_report, 2 * (size_t)G);
    if (!rc) rc = halloc(q->owned_host, &q->h_part, (size_t)G * q->nblk);
    if (!rc) {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) {
            set_error("hipDeviceGetAttribute(MaxSharedMemoryPerBlock) failed");
            rc = LC_ERR_HIP;
        }
        q->lds_max = (size_t)lds;
    }
    if (rc) {
        free_loqd(q);
        return rc;
    }
    q->magic = kLoqdMagic;
    *out = reinterpret_cast<lc_loqd_t>(q);
    return LC_OK;
}

lc_status lc_loqd_set_solver(lc_loqd_t h, int32_t mode) {
    Loqd* q = as_loqd(h);
    LC_CHECK(q, LC_ERR_STATE, "invalid LOQD handle");
    LC_ARG(mode >= 0 && mode <= 2, "mode must be 0, 1 or 2");
    q->solver = mode;
    return LC_OK;
}

lc_status lc_loqd_set_warm_start(lc_loqd_t h, int32_t enable) {
    Loqd* q = as_loqd(h);
    LC_CHECK(q, LC_ERR_STATE, "invalid LOQD handle");
    q->warm = enable != 0;
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
    return lc::loqd_solve(h, c, c_dt, kappa, planck, E_prev, F_prev, f_cell, f_face, bnd, E_cell, E_face, F_face, rtol,
                          max_iter, iters, resid, stream, false);
}

}  // extern "C"

namespace lc {

lc_status loqd_check_deferred(lc_loqd_t h, int32_t* iters) {
    Loqd* q = as_loqd(h);
    LC_CHECK(q, LC_ERR_STATE, "invalid LOQD handle");
    return check_report(q, iters, nullptr);
}

lc_status loqd_solve(lc_loqd_t h, double c, double c_dt, const double* kappa, const double* planck,
                     const double* E_prev, const double* F_prev, const double* f_cell, const double* f_face,
                     const double* bnd, double* E_cell, double* E_face, double* F_face, double rtol,
                     int32_t max_iter, int32_t* iters, double* resid, void* stream, bool defer) {
    Loqd* q = as_loqd(h);
    LC_CHECK(q, LC_ERR_STATE, "invalid LOQD handle");
    LC_ARG(kappa && planck && E_prev && F_prev && f_cell && bnd && E_cell && E_face && F_face,
           "inputs and outputs must not be NULL");
    LC_ARG(f_face || q->nint == 0, "f_face must not be NULL when the grid has interior faces");
    LC_ARG(std::isfinite(c) && c > 0.0 && std::isfinite(c_dt) && c_dt > 0.0, "c and c_dt must be finite and > 0");
    LC_ARG(std::isfinite(rtol) && rtol > 0.0 && rtol < 1.0, "rtol must be in (0, 1)");
    LC_ARG(max_iter >= 1, "max_iter must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Geo Q = geo(q, c, c_dt, q->G);
    const dim3 blk(kLoqdBlock);
    hipLaunchKernelGGL(k_loqd_prep, dim3((std::max(q->N, q->nf) + kLoqdBlock - 1) / kLoqdBlock, q->G), blk, 0, st, Q,
                       kappa, planck, E_prev, f_cell, F_prev, f_face, bnd, q->d_sigma, q->d_src, q->d_ks, q->d_es,
                       q->d_fc, q->d_ff, q->d_bc3, q->d_fp);
    LC_HIP(hipGetLastError());
    const Gen Cg{q->d_sigma, q->d_src, q->d_ks, q->d_es, q->d_fc, q->d_ff, q->d_bc3, q->d_fp};
    return solve_general(q, Q, Cg, E_cell, E_face, F_face, rtol, max_iter, iters, resid, st, defer);
}

}  // namespace lc

extern "C" {

lc_status lc_loqd_solve_general(lc_loqd_t h, double c, double c_dt, const double* sigma, const double* source,
                                const double* k_side, const double* eta_side, const double* F_prev,
                                const double* f_cell, const double* f_face, const double* bc, double* E_cell,
                                double* E_face, double* F_face, double rtol, int32_t max_iter, int32_t* iters,
                                double* resid, void* stream) {
    Loqd* q = as_loqd(h);
    LC_CHECK(q, LC_ERR_STATE, "invalid LOQD handle");
    LC_ARG(sigma && source && k_side && eta_side && F_prev && f_cell && f_face && bc && E_cell && E_face && F_face,
           "inputs and outputs must not be NULL");
    LC_ARG(std::isfinite(c) && c > 0.0 && std::isfinite(c_dt) && c_dt > 0.0, "c and c_dt must be finite and > 0");
    LC_ARG(std::isfinite(rtol) && rtol > 0.0 && rtol < 1.0, "rtol must be in (0, 1)");
    LC_ARG(max_iter >= 1, "max_iter must be >= 1");
    const Geo Q = geo(q, c, c_dt, q->G);
    const Gen Cg{sigma, source, k_side, eta_side, f_cell, f_face, bc, F_prev};
    return solve_general(q, Q, Cg, E_cell, E_face, F_face, rtol, max_iter, iters, resid,
                         static_cast<hipStream_t>(stream));
}

lc_status lc_loqd_grey_coefficients(lc_loqd_t h, double c, double c_dt, const double* kappa, const double* planck,
                                    const double* E_prev, const double* F_prev, const double* f_cell,
                                    const double* f_face, const double* bnd, const double* E_cell,
                                    const double* E_face, const double* F_face, double* sigma, double* source,
                                    double* k_side, double* eta_side, double* F_prev_grey, double* f_cell_grey,
                                    double* f_face_grey, double* bc_grey, double* E_prev_grey, double* kappa_E,
                                    double* kappa_B, void* stream) {
    Loqd* q = as_loqd(h);
    LC_CHECK(q, LC_ERR_STATE, "invalid LOQD handle");
    LC_ARG(kappa && planck && E_prev && F_prev && f_cell && bnd && E_cell && E_face && F_face,
           "multigroup inputs must not be NULL");
    LC_ARG(f_face || q->nint == 0, "f_face must not be NULL when the grid has interior faces");
    LC_ARG(sigma && source && k_side && eta_side && F_prev_grey && f_cell_grey && f_face_grey && bc_grey &&
               E_prev_grey,
           "outputs must not be NULL");
    LC_ARG(std::isfinite(c) && c > 0.0 && std::isfinite(c_dt) && c_dt > 0.0, "c and c_dt must be finite and > 0");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Geo Q = geo(q, c, c_dt, q->G);
    const dim3 blk(kLoqdBlock);
    hipLaunchKernelGGL(k_grey_coef, dim3((std::max(8 * q->N, q->nf) + kLoqdBlock - 1) / kLoqdBlock), blk, 0, st, Q, kappa,
                       planck, E_prev, f_cell, E_cell, E_face, F_face, F_prev, f_face, bnd, sigma, source, k_side,
                       eta_side, f_cell_grey, E_prev_grey, kappa_E, kappa_B, f_face_grey, bc_grey, F_prev_grey);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

lc_status lc_loqd_grey_meb(lc_loqd_t h, double c, double c_dt, const double* kappa_E, const double* kappa_B,
                           const double* E_prev, const double* k_side, const double* eta_side, const double* F_prev,
                           const double* f_cell, const double* f_face, const double* bc, const double* T_prev,
                           double c_v, double a_R, double* T, double* E_cell, double* E_face, double* F_face,
                           double newton_tol, int32_t max_newton, double rtol, int32_t max_iter,
                           int32_t* newton_iters, int32_t* iters, double* resid, void* stream) {
    Loqd* q = as_loqd(h);
    LC_CHECK(q, LC_ERR_STATE, "invalid LOQD handle");
    LC_ARG(kappa_E && kappa_B && E_prev && k_side && eta_side && F_prev && f_cell && f_face && bc && T_prev && T &&
               E_cell && E_face && F_face,
           "inputs and outputs must not be NULL");
    LC_ARG(std::isfinite(c) && c > 0.0 && std::isfinite(c_dt) && c_dt > 0.0, "c and c_dt must be finite and > 0");
    LC_ARG(std::isfinite(c_v) && c_v > 0.0 && std::isfinite(a_R) && a_R > 0.0, "c_v and a_R must be finite and > 0");
    LC_ARG(std::isfinite(newton_tol) && newton_tol >= 0.0, "newton_tol must be finite and >= 0");
    LC_ARG(max_newton >= 1, "max_newton must be >= 1");
    LC_ARG(std::isfinite(rtol) && rtol > 0.0 && rtol < 1.0, "rtol must be in (0, 1)");
    LC_ARG(max_iter >= 1, "max_iter must be >= 1");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int G = q->G;
    const Geo Q = geo(q, c, c_dt, G);
    const Meb M{kappa_E, kappa_B, E_prev, T_prev, c_v * c / c_dt, a_R};
    const Gen Cg{q->d_sigma, q->d_src, k_side, eta_side, f_cell, f_face, bc, F_prev};
    const int nblkc = (q->N + kLoqdBlock - 1) / kLoqdBlock;      // <= q->nblk: the partials fit d_part
    const dim3 gc(nblkc, G), blk(kLoqdBlock);
    const size_t n_part = (size_t)G * nblkc;
    int total = 0, k = 0;
    double change = INFINITY;
    std::vector<double> res(G, 0.0);
    while (k < max_newton && !(change <= newton_tol)) {
        ++k;
        hipLaunchKernelGGL(k_meb_linearise, gc, blk, 0, st, Q, M, T, q->d_sigma, q->d_src);
        LC_HIP(hipGetLastError());
        int32_t it = 0;
        // the solve's report and the update's change partials: one wait
        lc_status rc = solve_general(q, Q, Cg, E_cell, E_face, F_face, rtol, max_iter, &it, res.data(), st, true);
        if (!rc) {
            hipLaunchKernelGGL(k_meb_update, gc, blk, 0, st, Q, M, T, E_cell, q->d_part, nblkc);
            LC_HIP(hipGetLastError());
            LC_HIP(hipMemcpyAsync(q->h_part, q->d_part, n_part * sizeof(double), hipMemcpyDeviceToHost, st));
            LC_HIP(hipStreamSynchronize(st));
            rc = check_report(q, &it, res.data());
        }
        total += it;
        if (rc) {
            if (iters) *iters = total;
            if (newton_iters) *newton_iters = k;
            return rc;
        }
        change = 0.0;
        for (size_t j = 0; j < n_part; ++j) change = std::max(change, q->h_part[j]);
    }
    if (iters) *iters = total;
    if (newton_iters) *newton_iters = k;
    if (resid)
        for (int g = 0; g < G; ++g) resid[g] = res[g];
    LC_CHECK(change <= newton_tol, LC_ERR_UNSUPPORTED,
             "grey energy balance: Newton change %.3g above %.3g after %d iterations", change, newton_tol, k);
    return LC_OK;
}

}  // extern "C"
