// Characteristic grid on the GPU: characteristic offsets, segment tracing,
// cell-major segment lists C(i, m) with area weights (eq. (14)-(15)) and
// boundary exit maps F(f, m) (eq. (16)).
//
// This file is compiled with floating-point contraction off so that the
// crossing parameters are the plain IEEE results of the written expressions.
#include <climits>
#include <cmath>

#include "lc_internal.hpp"

namespace lc {
namespace {

struct PairGeo {
    double c, s, vmin, delta;
};

__device__ __forceinline__ int find_pair(const int* __restrict__ ray_off, int n_pairs, int k) {
    int lo = 0, hi = n_pairs;          // ray_off[lo] <= k < ray_off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (ray_off[mid] <= k) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ int face_of(int nx, int ny, double hx, double hy, double x, double y, bool on_x, bool far_side) {
    if (on_x) {
        int iy = clampi((int)floor(y / hy), 0, ny - 1);
        return far_side ? ny + iy : iy;
    }
    int ix = clampi((int)floor(x / hx), 0, nx - 1);
    return far_side ? 2 * ny + nx + ix : 2 * ny + ix;
}

// Walk one characteristic v = const of direction (c, s) through the grid,
// cell by cell, stepping to the nearer of the next x- and y-line crossing.
// Crossings within tol of the previous boundary point, or of the exit point,
// are merged.  Returns the number of segments; FILL writes them.
template <bool FILL>
__device__ int walk(int nx, int ny, double lx, double ly, double hx, double hy, double c, double s,
                    double v, int* face2, double* pts4, int* cell_out, double* len_out, int cap) {
    const double tol = 1e-12 * fmin(hx, hy);
    const double ux0 = (0.0 + v * s) / c, ux1 = (lx + v * s) / c;
    const double uy0 = (0.0 - v * c) / s, uy1 = (ly - v * c) / s;
    const double uxl = fmin(ux0, ux1), uxh = fmax(ux0, ux1);
    const double uyl = fmin(uy0, uy1), uyh = fmax(uy0, uy1);
    const double u_in = fmax(uxl, uyl), u_out = fmin(uxh, uyh);
    if (!(u_out - u_in > tol)) return 0;
    const bool in_on_x = uxl >= uyl;
    const bool out_on_x = uxh <= uyh;
    const double xin = u_in * c - v * s, yin = u_in * s + v * c;
    const double xout = u_out * c - v * s, yout = u_out * s + v * c;
    if (!FILL) {
        face2[0] = in_on_x ? face_of(nx, ny, hx, hy, xin, yin, true, c < 0)
                           : face_of(nx, ny, hx, hy, xin, yin, false, s < 0);
        face2[1] = out_on_x ? face_of(nx, ny, hx, hy, xout, yout, true, c > 0)
                            : face_of(nx, ny, hx, hy, xout, yout, false, s > 0);
        pts4[0] = xin; pts4[1] = yin; pts4[2] = xout; pts4[3] = yout;
    }
    int ix, iy;
    if (in_on_x) {
        ix = c > 0 ? 0 : nx - 1;
        iy = clampi((int)floor(yin / hy), 0, ny - 1);
    } else {
        iy = s > 0 ? 0 : ny - 1;
        ix = clampi((int)floor(xin / hx), 0, nx - 1);
    }
    const int sx = c > 0 ? 1 : -1, sy = s > 0 ? 1 : -1;
    double u_cur = u_in;
    int n = 0;
    for (;;) {
        const int xl = sx > 0 ? ix + 1 : ix;       // next interior x line
        const int yl = sy > 0 ? iy + 1 : iy;
        const double uxn = (xl >= 1 && xl <= nx - 1) ? ((double)xl * hx + v * s) / c : INFINITY;
        const double uyn = (yl >= 1 && yl <= ny - 1) ? ((double)yl * hy - v * c) / s : INFINITY;
        const double un = fmin(uxn, uyn);
        if (!(un < u_out - tol)) {                 // last segment ends at the exit point
            if (FILL && n < cap) {
                cell_out[n] = iy * nx + ix;
                len_out[n] = u_out - u_cur;
            }
            return n + 1;
        }
        if (un - u_cur > tol) {
            if (FILL && n < cap) {
                cell_out[n] = iy * nx + ix;
                len_out[n] = un - u_cur;
            }
            ++n;
            u_cur = un;
        }
        if (uxn - un <= tol) ix += sx;             // both when passing a vertex
        if (uyn - un <= tol) iy += sy;
    }
}

__global__ void k_uniform_offsets(const int* __restrict__ ray_off, const PairGeo* __restrict__ geo,
                                  int n_pairs, int n_rays, double* v, double* w) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_rays) return;
    int a = find_pair(ray_off, n_pairs, k);
    int kl = k - ray_off[a];
    v[k] = geo[a].vmin + ((double)kl + 0.5) * geo[a].delta;
    w[k] = geo[a].delta;
}

template <bool FILL>
__global__ void k_trace(const int* __restrict__ ray_off, const PairGeo* __restrict__ geo, int n_pairs,
                        int n_rays, int nx, int ny, double lx, double ly, double hx, double hy,
                        const double* __restrict__ v, int* count, int* face, double* pts,
                        const int* __restrict__ seg_off, int* cell, double* len) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_rays) return;
    int a = find_pair(ray_off, n_pairs, k);
    if (FILL) {
        int o = seg_off[k];
        walk<true>(nx, ny, lx, ly, hx, hy, geo[a].c, geo[a].s, v[k], nullptr, nullptr, cell + o,
                   len + o, seg_off[k + 1] - o);
    } else {
        count[k] = walk<false>(nx, ny, lx, ly, hx, hy, geo[a].c, geo[a].s, v[k], face + 2 * k,
                               pts + 4 * k, nullptr, nullptr, 0);
    }
}

// ---- exclusive scan of int32 counts: out[0..n] with out[n] = total ----------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__device__ int block_exclusive_scan(int x, int* sh) {
    int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
        int y = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    int incl = sh[t];
    __syncthreads();
    return incl - x;
}

__global__ void k_scan_tiles(const int* __restrict__ in, int* out, int* tile_sum, int64_t n) {
    __shared__ int sh[kBlock];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int vals[kScanItems];
    int sum = 0;
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = base + q;
        vals[q] = i < n ? in[i] : 0;
        sum += vals[q];
    }
    int ex = block_exclusive_scan(sum, sh);
    for (int q = 0; q < kScanItems; ++q) {
        int64_t i = base + q;
        if (i < n) out[i] = ex;
        ex += vals[q];
    }
    if (threadIdx.x == kBlock - 1) tile_sum[blockIdx.x] = ex;
}

__global__ void k_scan_tile_sums(int* tile_sum, int64_t n_tiles, int* total) {
    __shared__ int sh[kBlock];
    __shared__ int blk_total;
    int carry = 0;
    for (int64_t b = 0; b < n_tiles; b += kBlock) {
        int64_t i = b + threadIdx.x;
        int x = i < n_tiles ? tile_sum[i] : 0;
        int ex = block_exclusive_scan(x, sh);
        if (i < n_tiles) tile_sum[i] = carry + ex;
        if (threadIdx.x == kBlock - 1) blk_total = ex + x;
        __syncthreads();
        carry += blk_total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_scan_add(int* out, const int* __restrict__ tile_sum, int64_t n, const int* total) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_sum[i / kScanTile];
    if (i == n) out[n] = *total;
}

// ---- cell-major segment lists -----------------------------------------------
__global__ void k_fill_int(int* p, int64_t n, int value) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = value;
}

__global__ void k_csr_count(const int* __restrict__ ray_off, int n_pairs, int n_rays,
                            const int* __restrict__ seg_off, const int* __restrict__ cell,
                            int* cnt, int* kfirst) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_rays) return;
    int a = find_pair(ray_off, n_pairs, k);
    int kl = k - ray_off[a];
    for (int j = seg_off[k]; j < seg_off[k + 1]; ++j) {
        int key = cell[j] * n_pairs + a;
        atomicAdd(&cnt[key], 1);
        atomicMin(&kfirst[key], kl);
    }
}

// Characteristics of one direction crossing a (convex) cell form a contiguous
// run of k; the position of ray k in the cell's list is k - kfirst.
__global__ void k_csr_fill(const int* __restrict__ ray_off, int n_pairs, int n_rays,
                           const int* __restrict__ seg_off, const int* __restrict__ cell,
                           const double* __restrict__ len, const double* __restrict__ width,
                           const int* __restrict__ csr_off, const int* __restrict__ kfirst,
                           int* csr_ray, int2* csr_t, double* csr_A, int* err) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_rays) return;
    int a = find_pair(ray_off, n_pairs, k);
    int kl = k - ray_off[a];
    for (int j = seg_off[k]; j < seg_off[k + 1]; ++j) {
        int key = cell[j] * n_pairs + a;
        int pos = csr_off[key] + (kl - kfirst[key]);
        if (pos >= csr_off[key + 1]) {     // a characteristic crossed a cell twice, or a gap
            atomicOr(err, 1);
            continue;
        }
        const int sp = j - seg_off[k];
        csr_ray[pos] = k;
        csr_t[pos] = make_int2(sp, seg_off[k + 1] - seg_off[k] - 1 - sp);   // position in d = 0, 1 order
        csr_A[pos] = len[j] * width[k];
    }
}

// Normalise the areas of each (cell, pair) list into weights A / sum A and
// give every segment its sweep record: cell and length, packed so that the
// sweep reads both with one load.
__global__ void k_csr_norm(const int* __restrict__ csr_off, int64_t n_keys, const int* __restrict__ csr_ray,
                           const int2* __restrict__ csr_t, const int* __restrict__ seg_off,
                           const int* __restrict__ cell, const double* __restrict__ len, double* csr_w,
                           float* csr_w32, int2* seg32, int4* seg64, int* err) {
    int64_t key = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= n_keys) return;
    int b = csr_off[key], e = csr_off[key + 1];
    double sum = 0.0;
    for (int q = b; q < e; ++q) sum += csr_w[q];
    if (!(sum > 0.0)) {                    // a cell no characteristic of this direction crosses
        atomicOr(err, 2);
        return;
    }
    for (int q = b; q < e; ++q) {
        double w = csr_w[q] / sum;
        csr_w[q] = w;
        csr_w32[q] = (float)w;
        const int j = seg_off[csr_ray[q]] + csr_t[q].x;
        seg32[j] = make_int2(cell[j], __float_as_int((float)len[j]));
        seg64[j] = make_int4(cell[j], 0, __double2loint(len[j]), __double2hiint(len[j]));
    }
}

// ---- boundary exit maps ---------------------------------------------------------
__global__ void k_bnd_count(const int* __restrict__ ray_off, int n_pairs, int n_rays,
                            const int* __restrict__ face, int* bmin, int* bmax, int* bcnt) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_rays) return;
    int a = find_pair(ray_off, n_pairs, k);
    for (int d = 0; d < 2; ++d) {
        int fe = face[2 * k + (d == 0 ? 1 : 0)];       // the face this traversal leaves through
        int key = (fe * n_pairs + a) * 2 + d;
        atomicMin(&bmin[key], k);
        atomicMax(&bmax[key], k);
        atomicAdd(&bcnt[key], 1);
    }
}

__global__ void k_bnd_final(const int* __restrict__ ray_off, const PairGeo* __restrict__ geo,
                            int n_pairs, int nx, int ny, double lx, double ly, double hx, double hy,
                            const double* __restrict__ pts, const int* __restrict__ bmin,
                            const int* __restrict__ bmax, const int* __restrict__ bcnt, int* bmap,
                            int* err) {
    int key = blockIdx.x * blockDim.x + threadIdx.x;
    int nb = 2 * (nx + ny);
    if (key >= nb * n_pairs * 2) return;
    int d = key & 1;
    int a = (key >> 1) % n_pairs;
    int b = (key >> 1) / n_pairs;
    double nxv = 0, nyv = 0, cx = 0, cy = 0;
    if (b < ny) { nxv = -1; cx = 0; cy = ((double)b + 0.5) * hy; }
    else if (b < 2 * ny) { nxv = 1; cx = lx; cy = ((double)(b - ny) + 0.5) * hy; }
    else if (b < 2 * ny + nx) { nyv = -1; cx = ((double)(b - 2 * ny) + 0.5) * hx; cy = 0; }
    else { nyv = 1; cx = ((double)(b - 2 * ny - nx) + 0.5) * hx; cy = ly; }
    double sg = d == 0 ? 1.0 : -1.0;
    double dn = nxv * (sg * geo[a].c) + nyv * (sg * geo[a].s);
    if (!(dn > 0.0)) {                         // incoming for this traversal
        bmap[2 * key] = -1;
        bmap[2 * key + 1] = -1;
        return;
    }
    if (bcnt[key] > 0) {
        if (bmax[key] - bmin[key] + 1 != bcnt[key]) atomicOr(err, 4);
        bmap[2 * key] = bmin[key];
        bmap[2 * key + 1] = bmax[key] + 1;
        return;
    }
    // no characteristic leaves through b: take the one leaving nearest its centre
    int best = -1;
    double bd = INFINITY;
    for (int k = ray_off[a]; k < ray_off[a + 1]; ++k) {
        const double* p = pts + 4 * k + (d == 0 ? 2 : 0);
        double dist = hypot(p[0] - cx, p[1] - cy);
        if (dist < bd) { bd = dist; best = k; }
    }
    bmap[2 * key] = best;
    bmap[2 * key + 1] = best + 1;
}

// ---- the paper's construction: vertex-avoiding tubes, halved to h_moc -----------
// Projections v = -x sin(phi) + y cos(phi) of all grid vertices, padded with +inf
// to a power of two for the bitonic sort.
__global__ void k_vertex_proj(int nx, int ny, double hx, double hy, double c, double s, int64_t n_vert,
                              int64_t n_pad, double* proj) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_pad) return;
    if (idx >= n_vert) {
        proj[idx] = INFINITY;
        return;
    }
    const int i = (int)(idx / (ny + 1)), j = (int)(idx % (ny + 1));
    proj[idx] = -((double)i * hx) * s + ((double)j * hy) * c;
}

__global__ void k_bitonic_step(double* v, int64_t n, int64_t j, int64_t k) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t l = i ^ j;
    if (l <= i) return;
    const double a = v[i], b = v[l];
    const bool up = (i & k) == 0;
    if ((up && a > b) || (!up && a < b)) {
        v[i] = b;
        v[l] = a;
    }
}

// flag[i] = 1 where sorted projection i starts a new distinct value
// (differs from its predecessor by more than 1e-12 of the projected width).
__global__ void k_distinct_flags(const double* __restrict__ proj, int64_t n, int* flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double tol = 1e-12 * (proj[n - 1] - proj[0]);
    flag[i] = (i == 0 || proj[i] - proj[i - 1] > tol) ? 1 : 0;
}

__global__ void k_distinct_compact(const double* __restrict__ proj, int64_t n, const int* __restrict__ flag,
                                   const int* __restrict__ pos, double* distinct) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // the last distinct value is the maximum projection
    if (flag[i]) distinct[pos[i]] = (pos[i] == pos[n] - 1) ? proj[n - 1] : proj[i];
}

// Each gap between distinct projections is one tube, split into the least
// power of two of equal parts no wider than h_moc.
__global__ void k_tube_parts(const double* __restrict__ distinct, int64_t m, double h_moc, int* parts) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m - 1) return;
    const double width = distinct[t + 1] - distinct[t];
    int q = 1;
    while (width / q > h_moc && q < (1 << 28)) q *= 2;
    parts[t] = q;
}

__global__ void k_tube_fill(const double* __restrict__ distinct, int64_t m, const int* __restrict__ parts,
                            const int* __restrict__ roff, double* v, double* w) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m - 1) return;
    const double lo = distinct[t];
    const double width = distinct[t + 1] - lo;
    const int q = parts[t];
    const double sub = width / q;
    for (int u = 0; u < q; ++u) {
        v[roff[t] + u] = lo + ((double)u + 0.5) * sub;
        w[roff[t] + u] = sub;
    }
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ---- interior-face crossing lists F(f, m) ---------------------------------------
// The face shared by the cells of two consecutive segments, or -1 when they
// are diagonal neighbours (a passage through a vertex crosses no face).
__device__ __forceinline__ int face_of_step(int nx, int ny, int c0, int c1) {
    const int iy0 = c0 / nx, ix0 = c0 - iy0 * nx;
    const int iy1 = c1 / nx, ix1 = c1 - iy1 * nx;
    if (iy0 == iy1 && (ix1 - ix0 == 1 || ix0 - ix1 == 1)) return iy0 * (nx - 1) + min(ix0, ix1);
    if (ix0 == ix1 && (iy1 - iy0 == 1 || iy0 - iy1 == 1)) return (nx - 1) * ny + min(iy0, iy1) * nx + ix0;
    return -1;
}

__global__ void k_fcsr_count(const int* __restrict__ ray_off, int n_pairs, int n_rays,
                             const int* __restrict__ seg_off, const int* __restrict__ cell, int nx, int ny,
                             int* cnt, int* kfirst) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_rays) return;
    int a = find_pair(ray_off, n_pairs, k);
    int kl = k - ray_off[a];
    for (int j = seg_off[k] + 1; j < seg_off[k + 1]; ++j) {
        const int f = face_of_step(nx, ny, cell[j - 1], cell[j]);
        if (f < 0) continue;
        const int64_t key = (int64_t)f * n_pairs + a;
        atomicAdd(&cnt[key], 1);
        atomicMin(&kfirst[key], kl);
    }
}

// Characteristics of one direction crossing a face form a contiguous run of
// k; the position of ray k in the face's list is k - kfirst.
__global__ void k_fcsr_fill(const int* __restrict__ ray_off, int n_pairs, int n_rays,
                            const int* __restrict__ seg_off, const int* __restrict__ cell, int nx, int ny,
                            const double* __restrict__ width, const int* __restrict__ off,
                            const int* __restrict__ kfirst, int* ray, int2* t, double* w, int* err) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_rays) return;
    int a = find_pair(ray_off, n_pairs, k);
    int kl = k - ray_off[a];
    const int nk = seg_off[k + 1] - seg_off[k];
    for (int j = seg_off[k] + 1; j < seg_off[k + 1]; ++j) {
        const int f = face_of_step(nx, ny, cell[j - 1], cell[j]);
        if (f < 0) continue;
        const int64_t key = (int64_t)f * n_pairs + a;
        const int pos = off[key] + (kl - kfirst[key]);
        if (pos >= off[key + 1]) {
            atomicOr(err, 4);
            continue;
        }
        const int s = j - seg_off[k];
        ray[pos] = k;
        t[pos] = make_int2(s, nk - s);
        w[pos] = width[k];
    }
}

// Normalise each (face, pair) list's widths; a list entry left unfilled
// (a gap in the run of characteristics) is an error.
__global__ void k_fcsr_norm(const int* __restrict__ off, int64_t n_keys, const int* __restrict__ ray, double* w,
                            float* w32, int* err) {
    int64_t key = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= n_keys) return;
    const int b = off[key], e = off[key + 1];
    double sum = 0.0;
    for (int q = b; q < e; ++q) {
        if (ray[q] < 0) atomicOr(err, 8);
        sum += w[q];
    }
    for (int q = b; q < e; ++q) {
        const double v = sum > 0.0 ? w[q] / sum : 0.0;
        w[q] = v;
        w32[q] = (float)v;
    }
}


lc_status scan_counts(const int* in, int* out, int64_t n, std::vector<void*>& tmp, hipStream_t st) {
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 0) tiles = 1;
    int* tile_sum = nullptr;
    int* total = nullptr;
    lc_status rc = dalloc(tmp, &tile_sum, (size_t)tiles);
    if (rc) return rc;
    rc = dalloc(tmp, &total, 1);
    if (rc) return rc;
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kBlock), 0, st, in, out, tile_sum, n);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(kBlock), 0, st, tile_sum, tiles, total);
    hipLaunchKernelGGL(k_scan_add, dim3(nblk(n + 1)), dim3(kBlock), 0, st, out, tile_sum, n, total);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

}  // namespace

lc_status build_geometry(Rays* r, hipStream_t st) {
    std::vector<void*> tmp;
    auto cleanup = [&]() {
        for (void* p : tmp) (void)hipFree(p);
        tmp.clear();
    };
    lc_status rc = LC_OK;
#define LC_STEP(x)               \
    do {                         \
        rc = (x);                \
        if (rc) { cleanup(); return rc; } \
    } while (0)
#define LC_CHECKC(cond, code, ...)  \
    do {                            \
        if (!(cond)) {              \
            set_error(__VA_ARGS__); \
            cleanup();              \
            return (code);          \
        }                           \
    } while (0)
#define LC_HIPC(x)                                                          \
    do {                                                                    \
        hipError_t e_ = (x);                                                \
        if (e_ != hipSuccess) {                                             \
            set_error("%s failed: %s", #x, hipGetErrorString(e_));          \
            cleanup();                                                      \
            return LC_ERR_HIP;                                              \
        }                                                                   \
    } while (0)

    const int P = r->n_pairs;
    // per-pair direction and characteristic offsets
    std::vector<PairGeo> geo(P);
    r->ray_off.assign(P + 1, 0);
    for (int a = 0; a < P; ++a) {
        double c = r->cphi[a], s = r->sphi[a];
        double vs[4] = {-0.0 * s + 0.0 * c, -r->lx * s + 0.0 * c, -0.0 * s + r->ly * c,
                        -r->lx * s + r->ly * c};
        double vmin = vs[0], vmax = vs[0];
        for (double x : vs) { vmin = std::min(vmin, x); vmax = std::max(vmax, x); }
        double W = vmax - vmin;
        int64_t K = (int64_t)std::ceil(W / r->h_moc * (1.0 - 1e-12));
        if (K < 1) K = 1;
        LC_CHECK(K < (int64_t)1 << 26, LC_ERR_ARG, "too many characteristics for pair %d", a);
        geo[a] = {c, s, vmin, W / (double)K};
        r->ray_off[a + 1] = r->ray_off[a] + (int)K;
    }
    // the paper's construction: per pair, tubes between sorted vertex projections
    std::vector<double*> t_dist(P, nullptr);
    std::vector<int*> t_parts(P, nullptr), t_roff(P, nullptr);
    std::vector<int64_t> t_m(P, 0);
    if (r->mode == LC_RAYS_TUBES) {
        const int64_t n_vert = (int64_t)(r->nx + 1) * (r->ny + 1);
        int64_t n_pad = 1;
        while (n_pad < n_vert) n_pad *= 2;
        double* proj = nullptr;
        int *flag = nullptr, *pos = nullptr;
        LC_STEP(dalloc(tmp, &proj, n_pad));
        LC_STEP(dalloc(tmp, &flag, n_vert));
        LC_STEP(dalloc(tmp, &pos, n_vert + 1));
        for (int a = 0; a < P; ++a) {
            hipLaunchKernelGGL(k_vertex_proj, dim3(nblk(n_pad)), dim3(kBlock), 0, st, r->nx, r->ny, r->hx, r->hy,
                               r->cphi[a], r->sphi[a], n_vert, n_pad, proj);
            for (int64_t k = 2; k <= n_pad; k *= 2)
                for (int64_t j = k / 2; j > 0; j /= 2)
                    hipLaunchKernelGGL(k_bitonic_step, dim3(nblk(n_pad)), dim3(kBlock), 0, st, proj, n_pad, j, k);
            hipLaunchKernelGGL(k_distinct_flags, dim3(nblk(n_vert)), dim3(kBlock), 0, st, proj, n_vert, flag);
            LC_HIPC(hipGetLastError());
            LC_STEP(scan_counts(flag, pos, n_vert, tmp, st));
            int m = 0;
            LC_HIPC(hipMemcpyAsync(&m, pos + n_vert, sizeof(int), hipMemcpyDeviceToHost, st));
            LC_HIPC(hipStreamSynchronize(st));
            LC_CHECKC(m >= 2, LC_ERR_STATE, "pair %d: fewer than two distinct vertex projections", a);
            t_m[a] = m;
            LC_STEP(dalloc(tmp, &t_dist[a], m));
            LC_STEP(dalloc(tmp, &t_parts[a], m));
            LC_STEP(dalloc(tmp, &t_roff[a], m));
            hipLaunchKernelGGL(k_distinct_compact, dim3(nblk(n_vert)), dim3(kBlock), 0, st, proj, n_vert, flag,
                               pos, t_dist[a]);
            hipLaunchKernelGGL(k_tube_parts, dim3(nblk(m)), dim3(kBlock), 0, st, t_dist[a], (int64_t)m, r->h_moc,
                               t_parts[a]);
            LC_HIPC(hipGetLastError());
            LC_STEP(scan_counts(t_parts[a], t_roff[a], m - 1, tmp, st));
            int K = 0;
            LC_HIPC(hipMemcpyAsync(&K, t_roff[a] + (m - 1), sizeof(int), hipMemcpyDeviceToHost, st));
            LC_HIPC(hipStreamSynchronize(st));
            LC_CHECKC(K >= 1 && K < (1 << 26), LC_ERR_ARG, "pair %d: %d characteristics", a, K);
            r->ray_off[a + 1] = r->ray_off[a] + K;
            LC_CHECKC(r->ray_off[a + 1] < (1 << 30), LC_ERR_ARG, "too many characteristics");
        }
    }
    r->n_rays = r->ray_off[P];
    const int nr = (int)r->n_rays;
    LC_CHECKC((double)nr * (r->nx + r->ny) < 2.0e9, LC_ERR_ARG,
              "characteristic grid too large for 32-bit segment indices (%d characteristics)", nr);
    PairGeo* d_geo = nullptr;
    int* d_count = nullptr;
    int* d_err = nullptr;
    LC_STEP(dalloc(tmp, &d_geo, P));
    LC_STEP(dalloc(tmp, &d_count, nr));
    LC_STEP(dalloc(tmp, &d_err, 1));
    LC_STEP(dalloc(r->owned, &r->d_ray_off, P + 1));
    LC_STEP(dalloc(r->owned, &r->d_v, nr));
    LC_STEP(dalloc(r->owned, &r->d_width, nr));
    LC_STEP(dalloc(r->owned, &r->d_face, 2 * (size_t)nr));
    LC_STEP(dalloc(r->owned, &r->d_pts, 4 * (size_t)nr));
    LC_STEP(dalloc(r->owned, &r->d_seg_off, (size_t)nr + 1));
    LC_HIPC(hipMemcpyAsync(d_geo, geo.data(), P * sizeof(PairGeo), hipMemcpyHostToDevice, st));
    LC_HIPC(hipMemcpyAsync(r->d_ray_off, r->ray_off.data(), (P + 1) * sizeof(int),
                           hipMemcpyHostToDevice, st));
    LC_HIPC(hipMemsetAsync(d_err, 0, sizeof(int), st));
    if (r->mode == LC_RAYS_TUBES) {
        for (int a = 0; a < P; ++a)
            hipLaunchKernelGGL(k_tube_fill, dim3(nblk(t_m[a])), dim3(kBlock), 0, st, t_dist[a], t_m[a], t_parts[a],
                               t_roff[a], r->d_v + r->ray_off[a], r->d_width + r->ray_off[a]);
    } else {
        hipLaunchKernelGGL(k_uniform_offsets, dim3(nblk(nr)), dim3(kBlock), 0, st, r->d_ray_off, d_geo, P,
                           nr, r->d_v, r->d_width);
    }
    hipLaunchKernelGGL(k_trace<false>, dim3(nblk(nr)), dim3(kBlock), 0, st, r->d_ray_off, d_geo, P, nr,
                       r->nx, r->ny, r->lx, r->ly, r->hx, r->hy, r->d_v, d_count, r->d_face, r->d_pts,
                       nullptr, nullptr, nullptr);
    LC_HIPC(hipGetLastError());
    LC_STEP(scan_counts(d_count, r->d_seg_off, nr, tmp, st));
    int total = 0;
    LC_HIPC(hipMemcpyAsync(&total, r->d_seg_off + nr, sizeof(int), hipMemcpyDeviceToHost, st));
    LC_HIPC(hipStreamSynchronize(st));
    {
        std::vector<int> so(nr + 1);
        LC_HIPC(hipMemcpy(so.data(), r->d_seg_off, (nr + 1) * sizeof(int), hipMemcpyDeviceToHost));
        int mx = 0;
        for (int k = 0; k < nr; ++k) {
            int c = so[k + 1] - so[k];
            mx = std::max(mx, c);
            if (c == 0) {
                set_error("characteristic %d misses the domain", k);
                cleanup();
                return LC_ERR_STATE;
            }
        }
        r->max_seg = mx;
        r->seg_off = so;
    }
    r->n_seg = total;
    const int64_t ns = total;
    LC_STEP(dalloc(r->owned, &r->d_cell, ns));
    LC_STEP(dalloc(r->owned, &r->d_len, ns));
    hipLaunchKernelGGL(k_trace<true>, dim3(nblk(nr)), dim3(kBlock), 0, st, r->d_ray_off, d_geo, P, nr,
                       r->nx, r->ny, r->lx, r->ly, r->hx, r->hy, r->d_v, nullptr, nullptr, nullptr,
                       r->d_seg_off, r->d_cell, r->d_len);
    LC_HIPC(hipGetLastError());

    // C(i, m): cell-major lists per (cell, pair)
    const int64_t n_keys = (int64_t)r->cells * P;
    int* d_cnt = nullptr;
    int* d_kfirst = nullptr;
    LC_STEP(dalloc(tmp, &d_cnt, n_keys));
    LC_STEP(dalloc(tmp, &d_kfirst, n_keys));
    LC_STEP(dalloc(r->owned, &r->d_csr_off, n_keys + 1));
    LC_STEP(dalloc(r->owned, &r->d_csr_ray, ns));
    LC_STEP(dalloc(r->owned, &r->d_csr_t, ns));
    LC_STEP(dalloc(r->owned, &r->d_csr_w, ns));
    LC_STEP(dalloc(r->owned, &r->d_csr_w32, ns));
    hipLaunchKernelGGL(k_fill_int, dim3(nblk(n_keys)), dim3(kBlock), 0, st, d_cnt, n_keys, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(nblk(n_keys)), dim3(kBlock), 0, st, d_kfirst, n_keys, INT_MAX);
    hipLaunchKernelGGL(k_csr_count, dim3(nblk(nr)), dim3(kBlock), 0, st, r->d_ray_off, P, nr,
                       r->d_seg_off, r->d_cell, d_cnt, d_kfirst);
    LC_HIPC(hipGetLastError());
    LC_STEP(scan_counts(d_cnt, r->d_csr_off, n_keys, tmp, st));
    hipLaunchKernelGGL(k_csr_fill, dim3(nblk(nr)), dim3(kBlock), 0, st, r->d_ray_off, P, nr,
                       r->d_seg_off, r->d_cell, r->d_len, r->d_width, r->d_csr_off, d_kfirst,
                       r->d_csr_ray, r->d_csr_t, r->d_csr_w, d_err);
    LC_STEP(dalloc(r->owned, &r->d_seg32, ns));
    LC_STEP(dalloc(r->owned, &r->d_seg64, ns));
    hipLaunchKernelGGL(k_csr_norm, dim3(nblk(n_keys)), dim3(kBlock), 0, st, r->d_csr_off, n_keys,
                       r->d_csr_ray, r->d_csr_t, r->d_seg_off, r->d_cell, r->d_len, r->d_csr_w,
                       r->d_csr_w32, r->d_seg32, r->d_seg64, d_err);
    LC_HIPC(hipGetLastError());

    // F(f, m) on the boundary: rays leaving through each face, per traversal
    const int64_t n_bkeys = (int64_t)r->nb * P * 2;
    int *d_bmin = nullptr, *d_bmax = nullptr, *d_bcnt = nullptr;
    LC_STEP(dalloc(tmp, &d_bmin, n_bkeys));
    LC_STEP(dalloc(tmp, &d_bmax, n_bkeys));
    LC_STEP(dalloc(tmp, &d_bcnt, n_bkeys));
    LC_STEP(dalloc(r->owned, &r->d_bmap, 2 * n_bkeys));
    hipLaunchKernelGGL(k_fill_int, dim3(nblk(n_bkeys)), dim3(kBlock), 0, st, d_bmin, n_bkeys, INT_MAX);
    hipLaunchKernelGGL(k_fill_int, dim3(nblk(n_bkeys)), dim3(kBlock), 0, st, d_bmax, n_bkeys, -1);
    hipLaunchKernelGGL(k_fill_int, dim3(nblk(n_bkeys)), dim3(kBlock), 0, st, d_bcnt, n_bkeys, 0);
    hipLaunchKernelGGL(k_bnd_count, dim3(nblk(nr)), dim3(kBlock), 0, st, r->d_ray_off, P, nr,
                       r->d_face, d_bmin, d_bmax, d_bcnt);
    hipLaunchKernelGGL(k_bnd_final, dim3(nblk(n_bkeys)), dim3(kBlock), 0, st, r->d_ray_off, d_geo, P,
                       r->nx, r->ny, r->lx, r->ly, r->hx, r->hy, r->d_pts, d_bmin, d_bmax, d_bcnt,
                       r->d_bmap, d_err);
    LC_HIPC(hipGetLastError());
    int err = 0;
    LC_HIPC(hipMemcpyAsync(&err, d_err, sizeof(int), hipMemcpyDeviceToHost, st));
    LC_HIPC(hipStreamSynchronize(st));
    cleanup();
    if (err & 2) {
        set_error("characteristic spacing %g too coarse: some cell is crossed by no characteristic "
                  "of some direction", r->h_moc);
        return LC_ERR_ARG;
    }
    if (err) {
        set_error("inconsistent characteristic grid (flags %d)", err);
        return LC_ERR_STATE;
    }
    return LC_OK;
#undef LC_STEP
#undef LC_HIPC
#undef LC_CHECKC
}

lc_status build_face_lists(Rays* r, hipStream_t st) {
    std::vector<void*> tmp;
    auto cleanup = [&]() {
        for (void* p : tmp) (void)hipFree(p);
        tmp.clear();
    };
    lc_status rc = LC_OK;
#define LC_STEP(x)               \
    do {                         \
        rc = (x);                \
        if (rc) { cleanup(); return rc; } \
    } while (0)
#define LC_HIPC(x)                                                          \
    do {                                                                    \
        hipError_t e_ = (x);                                                \
        if (e_ != hipSuccess) {                                             \
            set_error("%s failed: %s", #x, hipGetErrorString(e_));          \
            cleanup();                                                      \
            return LC_ERR_HIP;                                              \
        }                                                                   \
    } while (0)
    const int P = r->n_pairs;
    const int nr = (int)r->n_rays;
    const int64_t n_keys = std::max<int64_t>(n_interior_faces(r) * P, 1);
    int *d_cnt = nullptr, *d_kfirst = nullptr, *d_err = nullptr, *d_off = nullptr;
    LC_STEP(dalloc(tmp, &d_cnt, n_keys));
    LC_STEP(dalloc(tmp, &d_kfirst, n_keys));
    LC_STEP(dalloc(tmp, &d_err, 1));
    LC_STEP(dalloc(tmp, &d_off, n_keys + 1));
    hipLaunchKernelGGL(k_fill_int, dim3(nblk(n_keys)), dim3(kBlock), 0, st, d_cnt, n_keys, 0);
    hipLaunchKernelGGL(k_fill_int, dim3(nblk(n_keys)), dim3(kBlock), 0, st, d_kfirst, n_keys, INT_MAX);
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(kBlock), 0, st, d_err, 1, 0);
    hipLaunchKernelGGL(k_fcsr_count, dim3(nblk(nr)), dim3(kBlock), 0, st, r->d_ray_off, P, nr, r->d_seg_off,
                       r->d_cell, r->nx, r->ny, d_cnt, d_kfirst);
    LC_HIPC(hipGetLastError());
    LC_STEP(scan_counts(d_cnt, d_off, n_keys, tmp, st));
    int total = 0;
    LC_HIPC(hipMemcpyAsync(&total, d_off + n_keys, sizeof(int), hipMemcpyDeviceToHost, st));
    LC_HIPC(hipStreamSynchronize(st));
    const int64_t ne = std::max(total, 1);
    std::vector<void*> fresh;
    auto drop = [&]() {
        for (void* p : fresh) (void)hipFree(p);
        fresh.clear();
    };
    int* off = nullptr;
    int* ray = nullptr;
    int2* tt = nullptr;
    double* w = nullptr;
    float* w32 = nullptr;
    rc = dalloc(fresh, &off, n_keys + 1);
    if (rc == LC_OK) rc = dalloc(fresh, &ray, ne);
    if (rc == LC_OK) rc = dalloc(fresh, &tt, ne);
    if (rc == LC_OK) rc = dalloc(fresh, &w, ne);
    if (rc == LC_OK) rc = dalloc(fresh, &w32, ne);
    if (rc) {
        drop();
        cleanup();
        return rc;
    }
    auto fail = [&](lc_status code) {
        drop();
        cleanup();
        return code;
    };
    if (hipMemcpyAsync(off, d_off, (n_keys + 1) * sizeof(int), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(LC_ERR_HIP);
    hipLaunchKernelGGL(k_fill_int, dim3(nblk(ne)), dim3(kBlock), 0, st, ray, ne, -1);
    hipLaunchKernelGGL(k_fcsr_fill, dim3(nblk(nr)), dim3(kBlock), 0, st, r->d_ray_off, P, nr, r->d_seg_off,
                       r->d_cell, r->nx, r->ny, r->d_width, off, d_kfirst, ray, tt, w, d_err);
    hipLaunchKernelGGL(k_fcsr_norm, dim3(nblk(n_keys)), dim3(kBlock), 0, st, off, n_keys, ray, w, w32, d_err);
    if (hipGetLastError() != hipSuccess) {
        set_error("face list kernels failed to launch");
        return fail(LC_ERR_HIP);
    }
    int err = 0;
    if (hipMemcpyAsync(&err, d_err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        set_error("face list build failed");
        return fail(LC_ERR_HIP);
    }
    if (err) {
        set_error("interior-face crossings do not form contiguous runs (flags %d)", err);
        return fail(LC_ERR_STATE);
    }
    for (void* p : fresh) r->owned.push_back(p);
    fresh.clear();
    r->n_fent = total;
    r->d_fcsr_off = off;
    r->d_fcsr_ray = ray;
    r->d_fcsr_t = tt;
    r->d_fcsr_w = w;
    r->d_fcsr_w32 = w32;
    cleanup();
    return LC_OK;
#undef LC_STEP
#undef LC_HIPC
}

}  // namespace lc
