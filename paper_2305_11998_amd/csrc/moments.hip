// Angular moments of the swept state, eq. (7), (14)-(16), and boundary
// factors.  Each lane owns one (cell, group) -- or (boundary face, group) --
// and gathers its segments in a fixed order (the cell-major lists built with
// the characteristic grid), so the sums are deterministic and need no atomics.
// The float32 form accumulates with compensated (Kahan) sums and divides in
// float64.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "lc_internal.hpp"

namespace lc {
namespace {

struct MomArgs {
    const int* csr_off;       // [cells * n_pairs + 1] cell-major lists C(i, m)
    const unsigned* ent_off;  // [n_seg][4] per entry: {lane record in the first bundle for d0, the same for
                              // d1, offset of the second bundle's records, bits of the float32 weight};
                              // with multi: {first bundle, step d0, step d1, lane of group 0}
    const unsigned* bun_rec;  // [n_bun] first lane record of each bundle (multi only)
    unsigned half_rec;        // lane records of one traversal half
    int multi;                // G > 64: a characteristic's groups may span three or more bundles
    const void* csr_w;        // area weights A / sum A, double or float (float32 without multi: unused)
    const double* dirw;       // [n_pairs][2][P][kDirW]
    const void* state;        // values
    const int* e;             // per-group exponents of the state (float32 only)
    int nx, ny, G, P, n_pairs;
    int tw, th, tiles_x;      // tile of tw x th cells; tiles in row-major order
    int wpt;                  // wavefronts per tile (tw * th * G lanes)
    int64_t n_tiles;
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

constexpr int kMomWaves = 4;   // wavefronts per block of the moment kernels
constexpr int kXcdRun = 64;    // consecutive blocks per XCD in the batched moment launch
constexpr int kTileWaves = kMomWaves * kXcdRun;   // wavefronts of a tile at most: one XCD run

// Hardware hands workgroups to the 8 XCDs round-robin; give each XCD a
// contiguous range of tiles so that neighbouring tiles share an L2.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t hw, int64_t n) {
    const int64_t q = n >> 3, r = n & 7;
    const int64_t x = hw & 7, i = hw >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Lane records of one C(i, m) entry as seen by lane g.  A lane record is the
// P values of one lane at one step, so element offset = record * P; bundle
// bases and step rows hold whole multiples of 64 records, so the lane of the
// ray's group 0 is the first record mod 64.  The groups past the first
// bundle's end sit at a fixed offset in the next bundle, the same for both
// traversals.  In float32 the entry's weight travels in the same 16-byte
// record, so an entry costs one load besides its state values.  A slot past
// the end of its list reads entry 0 (which always exists) and gets weight 0,
// so every load is unconditional and stays inside the arrays.
template <typename T> struct Slot {
    unsigned r0, r1;   // this lane's record in the two traversals
    T w;
};

// With G > 64 (`multi`) an entry holds its first bundle and steps instead,
// and each lane reads the first record of its own bundle from bun_rec.
template <typename T>
__device__ __forceinline__ Slot<T> load_slot(gptr<const unsigned> eo, gptr<const T> cw, int e, bool ok, int g,
                                             const MomArgs& A) {
    Slot<T> s;
    const int ee = ok ? e : 0;
    using U4 = unsigned __attribute__((ext_vector_type(4)));
    const U4 q = *(gptr<const U4>)(eo + (size_t)ee * 4);
    T w;
    if (sizeof(T) == 4 && !A.multi) w = (T)__uint_as_float(q.w);
    else w = cw[ee];
    s.w = ok ? w : (T)0;
    if (A.multi) {
        const unsigned f = q.w + (unsigned)g;        // lane within the bundles from the first
        const unsigned base = as_global(A.bun_rec)[q.x + (f >> 6)];
        s.r0 = base + q.y * kWave + (f & (kWave - 1));
        s.r1 = A.half_rec + base + q.z * kWave + (f & (kWave - 1));
    } else {
        const int lane0 = (int)(q.x & (kWave - 1));  // lane of the ray's group 0
        const unsigned sh = g < kWave - lane0 ? 0u : q.z;
        s.r0 = q.x + sh + (unsigned)g;
        s.r1 = q.y + sh + (unsigned)g;
    }
    return s;
}

// The P values of one entry for one traversal (contiguous, [lane][p]); with
// P == PM one vector load (a power of two) or pairs (an even count).
template <typename T, int PM>
__device__ __forceinline__ void load_entry(gptr<const T> st, size_t o, int P, T (&x)[PM]) {
    constexpr bool kVecOk = PM >= 2 && (PM & (PM - 1)) == 0;
    constexpr bool kPairsOk = !kVecOk && PM % 2 == 0;    // 6 values: three pairs
    if (kVecOk && P == PM) {
        using V = T __attribute__((ext_vector_type(PM)));
        const V v = *(gptr<const V>)(st + o);
#pragma unroll
        for (int p = 0; p < PM; ++p) x[p] = v[p];
    } else if (kPairsOk && P == PM) {
        using V2 = T __attribute__((ext_vector_type(2)));
#pragma unroll
        for (int h = 0; h < PM / 2; ++h) {
            const V2 v = *(gptr<const V2>)(st + o + 2 * h);
            x[2 * h] = v.x;
            x[2 * h + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int p = 0; p < PM; ++p) x[p] = p < P ? st[o + p] : (T)0;
    }
}

// Cell and group of lane tid of a tile of tw x th cells (false for the
// lanes past the tile's cells or the grid's edge).
__device__ __forceinline__ bool tile_lane(const MomArgs& A, int64_t tile, int tid, int& cell, int& g) {
    const int cl = tid / A.G;
    g = tid - cl * A.G;
    if (cl >= A.tw * A.th) return false;
    const int cx = (int)(tile % A.tiles_x) * A.tw + cl % A.tw;
    const int cy = (int)(tile / A.tiles_x) * A.th + cl / A.tw;
    if (cx >= A.nx || cy >= A.ny) return false;
    cell = cy * A.nx + cx;
    return true;
}

// One pair's contribution to the seven angular moments from the
// direction-averaged intensities I_{i,m} of both traversals.
template <typename T, int PM>
__device__ __forceinline__ void pair_moments(const MomArgs& A, int a, const T (&Iim)[2][PM], T (&part)[7]) {
    const int P = A.P;
#pragma unroll
    for (int c = 0; c < 7; ++c) part[c] = (T)0;
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int p = 0; p < PM; ++p) {
            if (p >= P) continue;
            const gptr<const double> dw = as_global(A.dirw + (((size_t)a * 2 + d) * P + p) * kDirW);
#pragma unroll
            for (int c = 0; c < 7; ++c) part[c] += (T)dw[c] * Iim[d][p];
        }
}

// E, F and the Eddington tensor of lane (cell, g) from its seven sums.
template <typename T>
__device__ __forceinline__ void moments_store(const MomArgs& A, int cell, int g, const Acc<T> (&acc)[7]) {
    const int G = A.G;
    double sc = 1.0;
    if (sizeof(T) == 4) sc = ldexp(1.0, as_global(A.e)[g]);
    const double Phi = acc[0].value() * sc;
    const size_t o = (size_t)cell * G + g;
    if (A.E) as_global_w(A.E)[o] = Phi * A.inv_c;
    if (A.F) {
        const gptr<double> F = as_global_w(A.F);
        F[((size_t)cell * 2 + 0) * G + g] = acc[1].value() * sc;
        F[((size_t)cell * 2 + 1) * G + g] = acc[2].value() * sc;
    }
    if (A.f) {
        const gptr<double> f = as_global_w(A.f);
        const bool z = Phi == 0.0;
        const double inv = z ? 0.0 : 1.0 / Phi;
        f[((size_t)cell * 4 + 0) * G + g] = z ? 1.0 / 3 : acc[3].value() * sc * inv;
        f[((size_t)cell * 4 + 1) * G + g] = z ? 0.0 : acc[4].value() * sc * inv;
        f[((size_t)cell * 4 + 2) * G + g] = z ? 1.0 / 3 : acc[5].value() * sc * inv;
        f[((size_t)cell * 4 + 3) * G + g] = z ? 1.0 / 3 : acc[6].value() * sc * inv;
    }
}

// Lane (cell, g) of a tile of tw x th cells.  For each azimuth
// pair the lane gathers the segment averages of the characteristics crossing
// its cell (the C(i, m) list, in (k, s) order) with the area weights, giving
// I_{i,m} for both traversals and every polar angle, then adds that pair's
// contribution to the seven angular moments (compensated float32 or plain
// float64 sums, fixed order).  A cache line of the state holds neighbouring
// characteristics at the same step, which cross neighbouring cells, so the
// wavefronts of a tile -- run together on one XCD -- share the lines they
// fetch.  The outputs are cell-major, so a wavefront's 64 (cell, g) lanes
// store contiguous doubles.
//
// The loads are pipelined over pairs: while the state values of pair a are
// in flight, the entry offsets of pair a+1 and the list end of pair a+2 are
// fetched, so a pair costs about one memory round trip.  The first K entries
// of a list go through the pipeline; longer lists finish in a plain loop.
// The sums run in list order whatever K is.  PM bounds the polar count.
template <typename T, int PM, int K>
__device__ __forceinline__ void moments_tile(const MomArgs& A, int64_t tile, int tid) {
    const int P = A.P;
    int cell, g;
    if (!tile_lane(A, tile, tid, cell, g)) return;
    const int np = A.n_pairs;
    const gptr<const T> st = as_global(static_cast<const T*>(A.state));
    const gptr<const T> cw = as_global(static_cast<const T*>(A.csr_w));
    const gptr<const unsigned> eo = as_global(A.ent_off);
    const gptr<const int> co = as_global(A.csr_off + (size_t)cell * np);
    Acc<T> acc[7];
    // list bounds: pair a is [b0, b1), pair a+1 is [b1, b2)
    int b0 = co[0], b1 = co[1];
    int b2 = co[min(2, np)];
    Slot<T> cur[K];
#pragma unroll
    for (int u = 0; u < K; ++u) cur[u] = load_slot(eo, cw, b0 + u, b0 + u < b1, g, A);
    for (int a = 0; a < np; ++a) {
        T x[K][2][PM];
#pragma unroll
        for (int u = 0; u < K; ++u) {
            load_entry<T, PM>(st, (size_t)cur[u].r0 * P, P, x[u][0]);
            load_entry<T, PM>(st, (size_t)cur[u].r1 * P, P, x[u][1]);
        }
        const bool more = a + 1 < np;
        Slot<T> nxt[K];
#pragma unroll
        for (int u = 0; u < K; ++u) nxt[u] = load_slot(eo, cw, b1 + u, more && b1 + u < b2, g, A);
        const int b3 = co[min(a + 3, np)];
        T Iim[2][PM];
#pragma unroll
        for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int p = 0; p < PM; ++p) Iim[d][p] = (T)0;
#pragma unroll
        for (int u = 0; u < K; ++u)
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
                for (int p = 0; p < PM; ++p) Iim[d][p] += cur[u].w * x[u][d][p];
        for (int e = b0 + K; e < b1; ++e) {
            const Slot<T> t = load_slot(eo, cw, e, true, g, A);
            T y[2][PM];
            load_entry<T, PM>(st, (size_t)t.r0 * P, P, y[0]);
            load_entry<T, PM>(st, (size_t)t.r1 * P, P, y[1]);
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
                for (int p = 0; p < PM; ++p) Iim[d][p] += t.w * y[d][p];
        }
        T part[7];
        pair_moments<T, PM>(A, a, Iim, part);
#pragma unroll
        for (int c = 0; c < 7; ++c) acc[c].add(part[c]);
#pragma unroll
        for (int u = 0; u < K; ++u) cur[u] = nxt[u];
        b0 = b1;
        b1 = b2;
        b2 = b3;
    }
    moments_store<T>(A, cell, g, acc);
}

// Split form, for plans whose (cell, g) lanes are too few to fill the device
// while each list is long (fine characteristic grids on coarse material
// grids): one lane per (pair, cell, g) sums that pair's list -- U entries'
// loads in flight at a time, added in list order -- and stores the pair's
// seven partial sums; a second kernel adds them in pair order.  The terms
// and their order are those of moments_tile (a padding entry adds w = 0), so
// both forms give the same bits.
template <typename T, int PM>
__device__ __forceinline__ void pair_list(const MomArgs& A, int cell, int g, int a, T (&Iim)[2][PM]) {
    constexpr int U = PM <= 2 ? 8 : 4;
    const int P = A.P;
    const gptr<const T> st = as_global(static_cast<const T*>(A.state));
    const gptr<const T> cw = as_global(static_cast<const T*>(A.csr_w));
    const gptr<const unsigned> eo = as_global(A.ent_off);
    const gptr<const int> co = as_global(A.csr_off + (size_t)cell * A.n_pairs + a);
    const int b0 = co[0], b1 = co[1];
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int p = 0; p < PM; ++p) Iim[d][p] = (T)0;
    for (int e = b0; e < b1; e += U) {
        Slot<T> s[U];
#pragma unroll
        for (int u = 0; u < U; ++u) s[u] = load_slot(eo, cw, e + u, e + u < b1, g, A);
        T x[U][2][PM];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            load_entry<T, PM>(st, (size_t)s[u].r0 * P, P, x[u][0]);
            load_entry<T, PM>(st, (size_t)s[u].r1 * P, P, x[u][1]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
                for (int p = 0; p < PM; ++p) Iim[d][p] += s[u].w * x[u][d][p];
    }
}

// Partial sums [pair][7][lane] over the tile lanes (n_tiles * wpt * 64 of
// them); work items (pair, wavefront of a tile), pair-major, so each XCD
// streams the state of a few pairs.
template <typename T, int PM>
__global__ __launch_bounds__(kMomWaves * kWave) void k_moments_pairs(MomArgs A, T* __restrict__ part) {
    const int64_t waves = A.n_tiles * A.wpt;
    const int64_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t wi = lb * kMomWaves + (threadIdx.x >> 6);
    if (wi >= waves * A.n_pairs) return;
    const int a = (int)(wi / waves);
    const int64_t wv = wi - (int64_t)a * waves;
    const int64_t tile = wv / A.wpt;
    const int tid = (int)(wv - tile * A.wpt) * kWave + (threadIdx.x & (kWave - 1));
    int cell, g;
    if (!tile_lane(A, tile, tid, cell, g)) return;
    T Iim[2][PM];
    pair_list<T, PM>(A, cell, g, a, Iim);
    T pt[7];
    pair_moments<T, PM>(A, a, Iim, pt);
    const int64_t n_lanes = waves * kWave;
    const gptr<T> o = as_global_w(part) + (size_t)a * 7 * n_lanes + wv * kWave + (threadIdx.x & (kWave - 1));
#pragma unroll
    for (int c = 0; c < 7; ++c) o[(size_t)c * n_lanes] = pt[c];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_moments_combine(MomArgs A, const T* __restrict__ part) {
    const int64_t n_lanes = A.n_tiles * A.wpt * kWave;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n_lanes) return;
    const int64_t tile = t / ((int64_t)A.wpt * kWave);
    int cell, g;
    if (!tile_lane(A, tile, (int)(t - tile * A.wpt * kWave), cell, g)) return;
    Acc<T> acc[7];
    const gptr<const T> p = as_global(part) + t;
    for (int a = 0; a < A.n_pairs; ++a)
#pragma unroll
        for (int c = 0; c < 7; ++c) acc[c].add(p[((size_t)a * 7 + c) * n_lanes]);
    moments_store<T>(A, cell, g, acc);
}

// Work unit: one wavefront of a tile, i.e. 64 consecutive (cell, g) lanes of
// the tile's cell-major lane order.  Wavefronts need no barrier, so
// occupancy follows from registers alone.  Blocks of kMomWaves wavefronts
// are remapped so that each XCD takes a contiguous run of tiles.
template <typename T, int PM, int K>
__global__ __launch_bounds__(kMomWaves * kWave) void k_cell_moments(MomArgs A) {
    const int64_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int64_t wi = lb * kMomWaves + (threadIdx.x >> 6);
    if (wi >= A.n_tiles * A.wpt) return;
    const int64_t tile = wi / A.wpt;
    const int w = (int)(wi - tile * A.wpt);
    moments_tile<T, PM, K>(A, tile, w * kWave + (threadIdx.x & (kWave - 1)));
}

// Batched form: one launch over the wavefront items of every problem
// ({problem, wavefront of a tile}, problems in decreasing cost).  Blocks are
// remapped in groups of 8 * kXcdRun: within a group, XCD x takes kXcdRun
// consecutive blocks, so neighbouring tiles share one L2 while all XCDs move
// through the item list together and finish together.
template <typename T, int PM, int K>
__global__ __launch_bounds__(kMomWaves * kWave) void k_cell_moments_batch(const MomArgs* __restrict__ probs,
                                                                         const int2* __restrict__ items,
                                                                         int64_t n_items) {
    const int64_t hw = blockIdx.x;
    const int64_t grp = hw / (8 * kXcdRun);
    const int64_t in = hw - grp * (8 * kXcdRun);
    const int64_t lb = grp * (8 * kXcdRun) + (in & 7) * kXcdRun + (in >> 3);
    const int64_t gi = lb * kMomWaves + (threadIdx.x >> 6);
    if (gi >= n_items) return;
    const int pr = __builtin_amdgcn_readfirstlane(items[gi].x);
    const int lw = __builtin_amdgcn_readfirstlane(items[gi].y);
    const MomArgs& A = probs[pr];
    const int tile = lw / A.wpt;
    const int w = lw - tile * A.wpt;
    moments_tile<T, PM, K>(A, tile, w * kWave + (threadIdx.x & (kWave - 1)));
}

// Offsets of every C(i, m) entry into the bundle-major state of a plan
// ([t][lane][p] per bundle): lanes g < 64 - lane0 lie in the bundle of the
// ray's group 0, the rest in the next bundle, whose records for the same
// step sit 64 (L - 1) records further on (L the first bundle's length) in
// either traversal.  The entry's float32 weight rides along.
__global__ void k_entry_offsets(const int* __restrict__ csr_off, const int* __restrict__ csr_ray,
                                const int2* __restrict__ csr_t, const int* __restrict__ ray_off,
                                const int* __restrict__ bun_off, const int64_t* __restrict__ bun_base,
                                const float* __restrict__ w32, int64_t n_keys, int n_pairs, int G, int P,
                                int64_t half, unsigned* out) {
    const int64_t key = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= n_keys) return;
    const int a = (int)(key % n_pairs);
    for (int e = csr_off[key]; e < csr_off[key + 1]; ++e) {
        const int k = csr_ray[e];
        const int2 t = csr_t[e];
        const int f0 = (k - ray_off[a]) * G;
        const int B0 = bun_off[a] + f0 / kWave;
        const int lane0 = f0 & (kWave - 1);
        unsigned* o = out + (size_t)e * 4;
        if (G > kWave) {                            // groups may span three or more bundles
            o[0] = (unsigned)B0;
            o[1] = (unsigned)t.x;
            o[2] = (unsigned)t.y;
            o[3] = (unsigned)lane0;
            continue;
        }
        // lane records: bases and halves are whole multiples of 64 * P elements
        const int64_t b0 = bun_base[B0] / P, hr = half / P;
        o[0] = (unsigned)(b0 + (int64_t)t.x * kWave + lane0);
        o[1] = (unsigned)(hr + b0 + (int64_t)t.y * kWave + lane0);
        // group g >= 64 - lane0 sits at record b1 + t * 64 + (g - (64 - lane0))
        // = (first-bundle record of g) + (b1 - b0) - 64, in both traversals
        o[2] = lane0 + G > kWave ? (unsigned)(bun_base[B0 + 1] / P - b0 - kWave) : 0u;
        o[3] = __float_as_uint(w32[e]);
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
    int64_t blk_off;        // first block of this problem in a batched launch
};

// Boundary factors per (face b, group g): the outgoing intensity of a
// direction is the width-weighted mean exit intensity of the characteristics
// leaving through b; incoming directions take I_in.  One pass over the exit
// characteristics of each (pair, traversal) accumulates every polar angle.
struct BndSums {
    double Pp = 0, Jp = 0, Pm = 0, Jm = 0, S = 0, Sxx = 0, Sxy = 0, Syy = 0, wo = 0, wodn = 0;
};

// Width-weighted sums of the exit intensities of characteristics [k0, k1)
// leaving through the face in traversal d, every polar angle, two
// characteristics' loads in flight.
__device__ __forceinline__ void bnd_exit_sums(const BndArgs& A, int g, int d, int k0, int k1,
                                              double (&acc)[kMaxPol], double& wsum) {
    const int P = A.P;
    const int G = A.G;
    const gptr<const double> width = as_global(A.width);
    const gptr<const double> I_exit = as_global(A.I_exit);
    wsum = 0.0;
#pragma unroll
    for (int p = 0; p < kMaxPol; ++p) acc[p] = 0.0;
    for (int k = k0; k < k1; k += 2) {
        const bool two = k + 1 < k1;
        const double w0 = width[k];
        const double w1 = two ? width[k + 1] : 0.0;
        const gptr<const double> ie0 = I_exit + (size_t)(2 * k + d) * P * G + g;
        const gptr<const double> ie1 = ie0 + (size_t)2 * P * G;
        double x0[kMaxPol], x1[kMaxPol];
#pragma unroll
        for (int p = 0; p < kMaxPol; ++p) {
            x0[p] = p < P ? ie0[(size_t)p * G] : 0.0;
            x1[p] = p < P && two ? ie1[(size_t)p * G] : 0.0;
        }
        wsum += w0;
#pragma unroll
        for (int p = 0; p < kMaxPol; ++p)
            if (p < P) acc[p] += w0 * x0[p];
        if (two) {
            wsum += w1;
#pragma unroll
            for (int p = 0; p < kMaxPol; ++p)
                if (p < P) acc[p] += w1 * x1[p];
        }
    }
}

// Adds the directions of one (pair, traversal) to the face's sums: outgoing
// ones (the face has exit characteristics) from the exit means, incoming ones
// from I_in.
__device__ __forceinline__ void bnd_add(const BndArgs& A, int b, int g, int a, int d, bool out,
                                        const double (&acc)[kMaxPol], double wsum, BndSums& s) {
    const int P = A.P;
    const int G = A.G;
    const int M = A.n_az * P;
    double nxv = 0, nyv = 0;
    if (b < A.ny) nxv = -1;
    else if (b < 2 * A.ny) nxv = 1;
    else if (b < 2 * A.ny + A.nx) nyv = -1;
    else nyv = 1;
    const gptr<const double> I_in = as_global(A.I_in);
#pragma unroll
    for (int p = 0; p < kMaxPol; ++p) {
        if (p >= P) continue;
        const gptr<const double> dw = as_global(A.dirw + ((size_t)(a * 2 + d) * P + p) * kDirW);
        const double om = dw[0];
        const double odn = dw[7] * nxv + dw[8] * nyv;
        double I;
        if (out) {
            I = acc[p] / wsum;
            s.Pp += om * I;
            s.Jp += om * odn * I;
            s.wo += om;
            s.wodn += om * odn;
        } else {
            const int m = (a + d * (A.n_az >> 1)) * P + p;
            I = I_in[((size_t)b * M + m) * G + g];
            s.Pm += om * I;
            s.Jm += om * fabs(odn) * I;
        }
        s.S += om * I;
        s.Sxx += dw[3] * I;
        s.Sxy += dw[4] * I;
        s.Syy += dw[5] * I;
    }
}

__device__ __forceinline__ void bnd_store(const BndArgs& A, int b, int g, const BndSums& s) {
    const gptr<double> out = as_global_w(A.bnd + ((size_t)g * A.nb + b) * 8);
    out[0] = s.Pp;
    out[1] = s.Jp;
    out[2] = s.Pm;
    out[3] = s.Jm;
    out[4] = s.Pp > 0.0 ? s.Jp / s.Pp : s.wodn / s.wo;
    const bool z = s.S == 0.0;
    out[5] = z ? 1.0 / 3 : s.Sxx / s.S;
    out[6] = z ? 0.0 : s.Sxy / s.S;
    out[7] = z ? 1.0 / 3 : s.Syy / s.S;
}

using I2 = int __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void boundary_lane(const BndArgs& A, int lane) {
    const int G = A.G;
    if (lane >= A.nb * G) return;
    const int b = lane / G;
    const int g = lane - b * G;
    BndSums s;
    // exit ranges of face b, one int2 per (pair, traversal); the next one is
    // loaded while the current one is summed
    const int nad = 2 * A.n_pairs;
    const gptr<const I2> bmv = (gptr<const I2>)as_global(A.bmap + (size_t)b * nad * 2);
    I2 nxt = bmv[0];
    for (int ad = 0; ad < nad; ++ad) {
        const int k0 = nxt.x, k1 = nxt.y;
        if (ad + 1 < nad) nxt = bmv[ad + 1];
        double wsum = 0.0;
        double acc[kMaxPol];
#pragma unroll
        for (int p = 0; p < kMaxPol; ++p) acc[p] = 0.0;
        if (k0 >= 0) bnd_exit_sums(A, g, ad & 1, k0, k1, acc, wsum);
        bnd_add(A, b, g, ad >> 1, ad & 1, k0 >= 0, acc, wsum, s);
    }
    bnd_store(A, b, g, s);
}

// Split form of the boundary factors (few (face, g) lanes, many exit
// characteristics per face): one lane per ((pair, traversal), face, g) stores
// the exit sums {wsum, acc[p]} as [ad][1 + P][lane]; the combine kernel adds
// the directions in (pair, traversal) order exactly as boundary_lane does.
__global__ __launch_bounds__(kBlock) void k_boundary_parts(BndArgs A, double* __restrict__ part) {
    const int64_t nl = (int64_t)A.nb * A.G;
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int nad = 2 * A.n_pairs;
    if (t >= nl * nad) return;
    const int ad = (int)(t / nl);
    const int lane = (int)(t - ad * nl);
    const int b = lane / A.G;
    const int g = lane - b * A.G;
    const I2 r = *(gptr<const I2>)as_global(A.bmap + ((size_t)b * nad + ad) * 2);
    if (r.x < 0) return;
    double wsum, acc[kMaxPol];
    bnd_exit_sums(A, g, ad & 1, r.x, r.y, acc, wsum);
    const gptr<double> o = as_global_w(part) + (size_t)ad * (1 + A.P) * nl + lane;
    o[0] = wsum;
#pragma unroll
    for (int p = 0; p < kMaxPol; ++p)
        if (p < A.P) o[(size_t)(1 + p) * nl] = acc[p];
}

__global__ __launch_bounds__(kBlock) void k_boundary_combine(BndArgs A, const double* __restrict__ part) {
    const int64_t nl = (int64_t)A.nb * A.G;
    const int lane = (int)((int64_t)blockIdx.x * kBlock + threadIdx.x);
    if (lane >= nl) return;
    const int b = lane / A.G;
    const int g = lane - b * A.G;
    const int nad = 2 * A.n_pairs;
    const gptr<const I2> bmv = (gptr<const I2>)as_global(A.bmap + (size_t)b * nad * 2);
    BndSums s;
    for (int ad = 0; ad < nad; ++ad) {
        const bool out = bmv[ad].x >= 0;
        double wsum = 0.0, acc[kMaxPol];
        const gptr<const double> q = as_global(part) + (size_t)ad * (1 + A.P) * nl + lane;
#pragma unroll
        for (int p = 0; p < kMaxPol; ++p) acc[p] = out && p < A.P ? q[(size_t)(1 + p) * nl] : 0.0;
        if (out) wsum = q[0];
        bnd_add(A, b, g, ad >> 1, ad & 1, out, acc, wsum, s);
    }
    bnd_store(A, b, g, s);
}

__global__ __launch_bounds__(kBlock) void k_boundary(BndArgs A) {
    boundary_lane(A, blockIdx.x * blockDim.x + threadIdx.x);
}

// Batched form: each problem owns a contiguous range of blocks (blk_off), so
// a block finds its problem with a block-uniform search.
__global__ __launch_bounds__(kBlock) void k_boundary_batch(const BndArgs* __restrict__ P, int n) {
    const int64_t blk = blockIdx.x;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (P[mid].blk_off <= blk) lo = mid; else hi = mid;
    }
    boundary_lane(P[lo], (int)((blk - P[lo].blk_off) * kBlock + threadIdx.x));
}

template <typename T, int P>
void launch_cell_moments_e(int ent, const MomArgs& A, hipStream_t st) {
    const int64_t waves = A.n_tiles * A.wpt;
    dim3 grid((unsigned)((waves + kMomWaves - 1) / kMomWaves)), block(kMomWaves * kWave);
    switch (ent) {
        case 1: hipLaunchKernelGGL((k_cell_moments<T, P, 1>), grid, block, 0, st, A); break;
        case 2: hipLaunchKernelGGL((k_cell_moments<T, P, 2>), grid, block, 0, st, A); break;
        case 4: hipLaunchKernelGGL((k_cell_moments<T, P, 4>), grid, block, 0, st, A); break;
        default: hipLaunchKernelGGL((k_cell_moments<T, P, 3>), grid, block, 0, st, A); break;
    }
}

template <typename T>
lc_status launch_cell_moments_p(int P, int ent, const MomArgs& A, hipStream_t st) {
    switch (P) {
        case 1: launch_cell_moments_e<T, 1>(ent, A, st); break;
        case 2: launch_cell_moments_e<T, 2>(ent, A, st); break;
        case 3: launch_cell_moments_e<T, 3>(ent, A, st); break;
        case 4: launch_cell_moments_e<T, 4>(ent, A, st); break;
        case 5: launch_cell_moments_e<T, 5>(ent, A, st); break;
        case 6: launch_cell_moments_e<T, 6>(ent, A, st); break;
        case 7: launch_cell_moments_e<T, 7>(ent, A, st); break;
        case 8: launch_cell_moments_e<T, 8>(ent, A, st); break;
        default:
            set_error("n_pol = %d not supported (1..8)", P);
            return LC_ERR_UNSUPPORTED;
    }
    LC_HIP(hipGetLastError());
    return LC_OK;
}

template <typename T, int PM>
void launch_split_e(const MomArgs& A, void* part, hipStream_t st) {
    const int64_t waves = A.n_tiles * A.wpt * A.n_pairs;
    hipLaunchKernelGGL((k_moments_pairs<T, PM>), dim3((unsigned)((waves + kMomWaves - 1) / kMomWaves)),
                       dim3(kMomWaves * kWave), 0, st, A, static_cast<T*>(part));
    const int64_t lanes = A.n_tiles * A.wpt * kWave;
    hipLaunchKernelGGL((k_moments_combine<T>), dim3((unsigned)((lanes + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                       A, static_cast<const T*>(part));
}

template <typename T>
lc_status launch_split_p(int P, const MomArgs& A, void* part, hipStream_t st) {
    switch (P) {
        case 1: launch_split_e<T, 1>(A, part, st); break;
        case 2: launch_split_e<T, 2>(A, part, st); break;
        case 3: launch_split_e<T, 3>(A, part, st); break;
        case 4: launch_split_e<T, 4>(A, part, st); break;
        case 5: launch_split_e<T, 5>(A, part, st); break;
        case 6: launch_split_e<T, 6>(A, part, st); break;
        case 7: launch_split_e<T, 7>(A, part, st); break;
        case 8: launch_split_e<T, 8>(A, part, st); break;
        default:
            set_error("n_pol = %d not supported (1..8)", P);
            return LC_ERR_UNSUPPORTED;
    }
    LC_HIP(hipGetLastError());
    return LC_OK;
}

// Bytes of the split gather's partial sums for a grid of n_tiles x wpt
// wavefronts: [pair][7][lane].
size_t split_part_bytes(int64_t n_tiles, int wpt, int n_pairs, size_t el) {
    return (size_t)n_pairs * 7 * (size_t)n_tiles * wpt * kWave * el;
}

// The cell-moment gather of one grid (cells or a family of interior faces),
// whole or split over pairs as the plan says.
lc_status launch_gather(Plan* pl, const MomArgs& A, hipStream_t st) {
    const bool f32 = pl->prec == LC_F32;
    const int P = pl->rays->n_pol;
    if (pl->mom_split & 1) {
        const size_t need = split_part_bytes(A.n_tiles, A.wpt, A.n_pairs, f32 ? 4 : 8);
        LC_CHECK(need <= pl->mom_part_bytes, LC_ERR_STATE, "split gather: %zu bytes of partial sums needed, %zu held",
                 need, pl->mom_part_bytes);
        return f32 ? launch_split_p<float>(P, A, pl->d_mom_part, st) : launch_split_p<double>(P, A, pl->d_mom_part, st);
    }
    return f32 ? launch_cell_moments_p<float>(P, pl->moments_entries, A, st)
               : launch_cell_moments_p<double>(P, pl->moments_entries, A, st);
}

// Tiles of an interior-face grid of fnx x fny faces: as for cells.
void face_tiles(int G, int fnx, int fny, MomArgs& A) {
    const int cells_max = std::max(1, kTileWaves * kWave / G);
    A.tw = std::max(1, std::min({16, cells_max, fnx}));
    A.th = std::max(1, std::min({16, cells_max / A.tw, fny}));
    A.tiles_x = (fnx + A.tw - 1) / A.tw;
    A.n_tiles = (int64_t)A.tiles_x * ((fny + A.th - 1) / A.th);
    A.wpt = (A.tw * A.th * G + kWave - 1) / kWave;
}

constexpr int64_t kSplitMaxWaves = 2048;   // tile wavefronts (two per SIMD) below which a gather may split
constexpr double kSplitMinList = 8.0;      // and its lists must hold this many entries on average
constexpr int64_t kSplitFewLanes = 16384;  // boundary lanes (under one wavefront per CU): split whatever the lists

}  // namespace

lc_status plan_set_moment_split(Plan* pl, int mode) {
    Rays* r = pl->rays;
    int want = 0;
    if (mode < 0) {
        const int64_t waves = moment_tiles(pl) * moment_tile_waves(pl);
        const double per_list = (double)r->n_seg / std::max(1.0, (double)r->cells * r->n_pairs);
        if (r->n_pairs > 1 && waves < kSplitMaxWaves && per_list >= kSplitMinList) want |= 1;
        const int64_t lanes = (int64_t)r->nb * pl->G;
        const double per_face = (double)r->n_rays / std::max(1.0, (double)r->nb * r->n_pairs);
        if (lanes < kSplitFewLanes || (lanes < kSplitMaxWaves * kWave && per_face >= kSplitMinList)) want |= 2;
    } else if (mode > 0) {
        want = 3;
    }
    const size_t el = pl->prec == LC_F32 ? 4 : 8;
    size_t bytes = 0;
    if (want & 1) {
        bytes = split_part_bytes(moment_tiles(pl), moment_tile_waves(pl), r->n_pairs, el);
        for (int part = 0; part < 2; ++part) {
            const int fnx = part == 0 ? r->nx - 1 : r->nx;
            const int fny = part == 0 ? r->ny : r->ny - 1;
            if (fnx < 1 || fny < 1) continue;
            MomArgs A{};
            face_tiles(pl->G, fnx, fny, A);
            bytes = std::max(bytes, split_part_bytes(A.n_tiles, A.wpt, r->n_pairs, el));
        }
    }
    if (want & 2) bytes = std::max(bytes, (size_t)2 * r->n_pairs * (1 + r->n_pol) * (size_t)r->nb * pl->G * 8);
    if (bytes > pl->mom_part_bytes) {
        LC_HIP(hipDeviceSynchronize());   // no gather in flight still uses the old buffer
        if (pl->d_mom_part) (void)hipFree(pl->d_mom_part);
        pl->d_mom_part = nullptr;
        pl->mom_part_bytes = 0;
        pl->mom_split = 0;
        hipError_t e = lc_malloc(&pl->d_mom_part, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            pl->d_mom_part = nullptr;
            set_error("allocation of the split gathers' partial sums (%zu bytes) failed: %s", bytes,
                      hipGetErrorString(e));
            return LC_ERR_ALLOC;
        }
        pl->mom_part_bytes = bytes;
    }
    pl->mom_split = want;
    return LC_OK;
}

lc_status plan_init_moments(Plan* pl) {
    Rays* r = pl->rays;
    LC_CHECK(2 * pl->half_elems / r->n_pol < (1LL << 32), LC_ERR_UNSUPPORTED,
             "state too large for the 32-bit moment gather offsets (2^32 lane records)");
    const int64_t n_keys = (int64_t)r->cells * r->n_pairs;
    {
        std::vector<unsigned> rec(std::max<size_t>((size_t)pl->n_bun, 1), 0u);
        for (int64_t B = 0; B < pl->n_bun; ++B) rec[B] = (unsigned)(pl->bun_base_h[B] / r->n_pol);
        hipError_t e = lc_malloc(reinterpret_cast<void**>(&pl->d_bun_rec), rec.size() * sizeof(unsigned));
        if (e == hipSuccess) e = hipMemcpy(pl->d_bun_rec, rec.data(), rec.size() * sizeof(unsigned), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("allocation of the bundle record table failed: %s", hipGetErrorString(e));
            return LC_ERR_ALLOC;
        }
    }
    hipError_t e = lc_malloc(reinterpret_cast<void**>(&pl->d_ent_off),
                             std::max<size_t>((size_t)r->n_seg, 1) * 4 * sizeof(unsigned));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc of the moment offsets failed: %s", hipGetErrorString(e));
        return LC_ERR_ALLOC;
    }
    hipLaunchKernelGGL(k_entry_offsets, dim3((unsigned)((n_keys + kBlock - 1) / kBlock)), dim3(kBlock), 0, 0,
                       r->d_csr_off, r->d_csr_ray, r->d_csr_t, r->d_ray_off, pl->d_bun_off, pl->d_bun_base,
                       r->d_csr_w32, n_keys, r->n_pairs, pl->G, r->n_pol, pl->half_elems, pl->d_ent_off);
    LC_HIP(hipGetLastError());
    LC_HIP(hipDeviceSynchronize());
    // tile: up to 16 x 16 cells, as many as fit in kTileWaves wavefronts
    // (narrower for large G); neighbouring cells are crossed by the same
    // characteristics, so the waves of a tile read overlapping state lines
    const int cells_max = std::max(1, kTileWaves * kWave / pl->G);
    pl->tile_w = std::max(1, std::min({16, cells_max, r->nx}));
    pl->tile_h = std::max(1, std::min({16, cells_max / pl->tile_w, r->ny}));
    return plan_set_moment_split(pl, -1);
}

// Interior-face crossing lists of a plan: the geometry's lists (built once
// per characteristic grid) and their state lane records for this plan.
lc_status plan_enable_faces(Plan* pl, hipStream_t st) {
    Rays* r = pl->rays;
    if (!r->d_fcsr_off) {
        lc_status rc = build_face_lists(r, st);
        if (rc) return rc;
    }
    if (pl->d_fent_off) return LC_OK;
    const int64_t n_keys = n_interior_faces(r) * r->n_pairs;
    hipError_t e = lc_malloc(reinterpret_cast<void**>(&pl->d_fent_off),
                             std::max<size_t>((size_t)r->n_fent, 1) * 4 * sizeof(unsigned));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        pl->d_fent_off = nullptr;
        set_error("hipMalloc of the face offsets failed: %s", hipGetErrorString(e));
        return LC_ERR_ALLOC;
    }
    if (n_keys > 0) {
        hipLaunchKernelGGL(k_entry_offsets, dim3((unsigned)((n_keys + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           r->d_fcsr_off, r->d_fcsr_ray, r->d_fcsr_t, r->d_ray_off, pl->d_bun_off, pl->d_bun_base,
                           r->d_fcsr_w32, n_keys, r->n_pairs, pl->G, r->n_pol, pl->half_elems, pl->d_fent_off);
        LC_HIP(hipGetLastError());
    }
    LC_HIP(hipStreamSynchronize(st));
    return LC_OK;
}

// Face averages of eq. (16) on the interior faces: the cell-moment gather run
// over the face crossing lists, on the stored upwind-face intensities.  The
// x-faces ((nx-1) x ny) and the y-faces (nx x (ny-1)) are two grids of their
// own.
lc_status launch_face_moments(Plan* pl, const void* point, const void* state, double c, double* E, double* F,
                              double* f, hipStream_t st) {
    Rays* r = pl->rays;
    LC_CHECK(pl->d_fent_off, LC_ERR_STATE, "interior faces are not enabled on this plan (lc_plan_enable_faces)");
    const bool f32 = pl->prec == LC_F32;
    const int G = pl->G;
    for (int part = 0; part < 2; ++part) {
        const int fnx = part == 0 ? r->nx - 1 : r->nx;
        const int fny = part == 0 ? r->ny : r->ny - 1;
        if (fnx < 1 || fny < 1) continue;
        const int64_t face0 = part == 0 ? 0 : (int64_t)(r->nx - 1) * r->ny;
        MomArgs A{};
        A.csr_off = r->d_fcsr_off + face0 * r->n_pairs;
        A.ent_off = pl->d_fent_off;
        A.bun_rec = pl->d_bun_rec;
        A.half_rec = (unsigned)(pl->half_elems / r->n_pol);
        A.multi = G > kWave ? 1 : 0;
        A.csr_w = f32 ? static_cast<const void*>(r->d_fcsr_w32) : static_cast<const void*>(r->d_fcsr_w);
        A.dirw = r->d_dirw;
        A.state = state_values(pl, point);
        A.e = static_cast<const int*>(state);        // the scale of the values the sweep stored
        A.nx = fnx;
        A.ny = fny;
        A.P = r->n_pol;
        face_tiles(G, fnx, fny, A);
        A.G = G;
        A.n_pairs = r->n_pairs;
        A.inv_c = 1.0 / c;
        A.E = E ? E + face0 * G : nullptr;
        A.F = F ? F + face0 * 2 * G : nullptr;
        A.f = f ? f + face0 * 4 * G : nullptr;
        lc_status rc = launch_gather(pl, A, st);
        if (rc) return rc;
    }
    return LC_OK;
}

// Argument records of a plan's cell gather and boundary factors.
static MomArgs cell_moment_args(Plan* pl, const void* state, double c, double* E, double* F, double* f) {
    Rays* r = pl->rays;
    const bool f32 = pl->prec == LC_F32;
    MomArgs A{};
    A.csr_off = r->d_csr_off;
    A.ent_off = pl->d_ent_off;
    A.bun_rec = pl->d_bun_rec;
    A.half_rec = (unsigned)(pl->half_elems / r->n_pol);
    A.multi = pl->G > kWave ? 1 : 0;
    A.csr_w = f32 ? static_cast<const void*>(r->d_csr_w32) : static_cast<const void*>(r->d_csr_w);
    A.dirw = r->d_dirw;
    A.state = state_values(pl, state);
    A.e = static_cast<const int*>(state);
    A.nx = r->nx;
    A.ny = r->ny;
    A.P = r->n_pol;
    A.tw = pl->tile_w;
    A.th = pl->tile_h;
    A.tiles_x = (r->nx + pl->tile_w - 1) / pl->tile_w;
    A.n_tiles = moment_tiles(pl);
    A.wpt = moment_tile_waves(pl);
    A.G = pl->G;
    A.n_pairs = r->n_pairs;
    A.inv_c = 1.0 / c;
    A.E = E;
    A.F = F;
    A.f = f;
    return A;
}

static BndArgs boundary_args(Plan* pl, const double* I_exit, const double* I_in, double* bnd) {
    Rays* r = pl->rays;
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
    return B;
}

lc_status launch_moments(Plan* pl, const void* state, const double* I_exit, const double* I_in,
                         double c, double* E, double* F, double* f, double* bnd, hipStream_t st) {
    Rays* r = pl->rays;
    if (E || F || f) {
        const MomArgs A = cell_moment_args(pl, state, c, E, F, f);
        lc_status rc = prof_begin(pl, pl->ev_mom, st);
        if (rc) return rc;
        rc = launch_gather(pl, A, st);
        if (rc) return rc;
        rc = prof_end(pl, pl->ev_mom, st);
        if (rc) return rc;
    }
    if (bnd) {
        const BndArgs B = boundary_args(pl, I_exit, I_in, bnd);
        const int lanes = r->nb * pl->G;
        if (pl->mom_split & 2) {
            const int64_t parts = (int64_t)lanes * 2 * r->n_pairs;
            LC_CHECK(parts * (1 + r->n_pol) * 8 <= (int64_t)pl->mom_part_bytes, LC_ERR_STATE,
                     "split boundary factors: partial-sum buffer too small");
            hipLaunchKernelGGL(k_boundary_parts, dim3((unsigned)((parts + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                               B, static_cast<double*>(pl->d_mom_part));
            hipLaunchKernelGGL(k_boundary_combine, dim3((lanes + kBlock - 1) / kBlock), dim3(kBlock), 0, st, B,
                               static_cast<const double*>(pl->d_mom_part));
        } else {
            hipLaunchKernelGGL(k_boundary, dim3((lanes + kBlock - 1) / kBlock), dim3(kBlock), 0, st, B);
        }
        LC_HIP(hipGetLastError());
    }
    return LC_OK;
}

namespace {

template <typename T, int PM, int K>
lc_status launch_moments_batch_e(const void* args, const int2* items, int64_t n_items, hipStream_t st) {
    const int64_t blocks = (n_items + kMomWaves - 1) / kMomWaves;
    const int64_t grid = (blocks + 8 * kXcdRun - 1) / (8 * kXcdRun) * (8 * kXcdRun);
    hipLaunchKernelGGL((k_cell_moments_batch<T, PM, K>), dim3((unsigned)grid), dim3(kMomWaves * kWave), 0, st,
                       static_cast<const MomArgs*>(args), items, n_items);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

template <typename T, int PM>
lc_status launch_moments_batch_p(int ent, const void* args, const int2* items, int64_t n_items, hipStream_t st) {
    switch (ent) {
        case 1: return launch_moments_batch_e<T, PM, 1>(args, items, n_items, st);
        case 2: return launch_moments_batch_e<T, PM, 2>(args, items, n_items, st);
        case 4: return launch_moments_batch_e<T, PM, 4>(args, items, n_items, st);
        default: return launch_moments_batch_e<T, PM, 3>(args, items, n_items, st);
    }
}

}  // namespace

size_t mom_args_bytes() { return sizeof(MomArgs); }
size_t bnd_args_bytes() { return sizeof(BndArgs); }

// Host copies of the moment and boundary records of one problem of a batch;
// the moments read `state`.
void make_moment_args(Plan* pl, const void* state, const double* I_exit, const double* I_in, double c,
                      double* E, double* F, double* f, double* bnd, int64_t bnd_blk_off, void* mom_out,
                      void* bnd_out) {
    const MomArgs A = cell_moment_args(pl, state, c, E, F, f);
    std::memcpy(mom_out, &A, sizeof(A));
    BndArgs B = boundary_args(pl, I_exit, I_in, bnd);
    B.blk_off = bnd_blk_off;
    std::memcpy(bnd_out, &B, sizeof(B));
}

int64_t moment_tiles(const Plan* pl) {
    const Rays* r = pl->rays;
    return (int64_t)((r->nx + pl->tile_w - 1) / pl->tile_w) * ((r->ny + pl->tile_h - 1) / pl->tile_h);
}

int moment_tile_waves(const Plan* pl) { return (pl->tile_w * pl->tile_h * pl->G + kWave - 1) / kWave; }

lc_status launch_moments_batch(int prec, int pm, int ent, const void* args, const int2* items, int64_t n_items,
                               hipStream_t st) {
    const bool f32 = prec == LC_F32;
    switch (pm) {
        case 1: return f32 ? launch_moments_batch_p<float, 1>(ent, args, items, n_items, st)
                           : launch_moments_batch_p<double, 1>(ent, args, items, n_items, st);
        case 2: return f32 ? launch_moments_batch_p<float, 2>(ent, args, items, n_items, st)
                           : launch_moments_batch_p<double, 2>(ent, args, items, n_items, st);
        case 4: return f32 ? launch_moments_batch_p<float, 4>(ent, args, items, n_items, st)
                           : launch_moments_batch_p<double, 4>(ent, args, items, n_items, st);
        case 8: return f32 ? launch_moments_batch_p<float, 8>(ent, args, items, n_items, st)
                           : launch_moments_batch_p<double, 8>(ent, args, items, n_items, st);
    }
    set_error("batched moments: polar bound %d not supported", pm);
    return LC_ERR_UNSUPPORTED;
}

lc_status launch_boundary_batch(const void* args, int n, int64_t blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_boundary_batch, dim3((unsigned)blocks), dim3(kBlock), 0, st,
                       static_cast<const BndArgs*>(args), n);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

}  // namespace lc
