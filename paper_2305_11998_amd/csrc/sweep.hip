// The transport sweep, eq. (10)-(13), on gfx950.
//
// Work decomposition: the lanes (characteristic k, group g) of an azimuth
// pair, g fastest, are cut into bundles of 64 -- one wavefront per bundle and
// traversal.  Each lane walks its characteristic segment by segment, carrying
// the intensity of every polar angle p in registers; per segment it reads the
// segment's packed {cell, length} record (one load), one cell-coefficient
// record (coalesced over g) and the stored I_bar^{n-1} of every p, and writes
// I_bar^n.  The state is laid out bundle-major, step-minor, so
// every wavefront streams its own contiguous, aligned 64-lane runs.  Polar
// angles with equal sin(zeta) (the +mu/-mu pairs of a symmetric set) share
// the exponential and the weight alpha.  Blocks are remapped so that each
// XCD's L2 serves a contiguous band of characteristics.  A split form cuts
// each traversal into chunks whose affine transfer maps are composed by a
// scan (for problems with too few lanes to fill the device).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "lc_internal.hpp"

namespace lc {
namespace {

struct SweepArgs {
    const int* bun_off;      // [n_pairs + 1] first bundle of each pair
    const int* bun_len;      // [n_bun] steps of each bundle
    const int64_t* bun_base; // [n_bun] element offset of each bundle within a traversal half
    int n_pairs;
    int64_t n_bun;
    int64_t half;            // elements of one traversal half of the state
    int64_t n_blocks;
    const int* ray_off;
    const int* seg_off;
    const int* face;
    const void* seg;         // [n_seg] {cell, length}: int2 (float32 bits) or int4 (cell, 0, float64 words)
    const void* coef;        // Coef<T> [cells][G]
    const void* prev;        // state values
    void* next;
    void* point;             // values entering each segment, state layout, or null
    const double* I_in;      // [nb][M][G]
    double* I_exit;          // [n_rays][2][P][G] or null
    int P;                   // polar angles
    int sym;                 // polar set mirror-symmetric
    const int* e_prev;       // per-group exponent of the old state (float32 only)
    const int* e_new;        // per-group exponent of the new state (float32 only)
    double inv_cdt;          // 1 / (c dt)
    int G, n_az, M;
    double inv_sinz[kMaxPol];
};

// Split sweep (chunks of a traversal): the transfer records, the first
// record of each wavefront (d * n_bun + B) and the chunk length in steps.
struct SplitArgs {
    void* carry;             // [record][slot][lane] of {A, B} pairs (T)
    const int64_t* cbase;    // [2 n_bun + 1]
    int len;
};

// Hardware hands workgroups to the 8 XCDs round-robin; give each XCD a
// contiguous range of logical blocks (a band of neighbouring characteristics)
// so the cell coefficients they share stay in that XCD's L2.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t hw, int64_t n) {
    const int64_t q = n >> 3, r = n & 7;
    const int64_t x = hw & 7, i = hw >> 3;
    return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ int find_pair(gptr<const int> off, int n, int64_t v) {
    int lo = 0, hi = n;                // off[lo] <= v < off[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= v) lo = mid; else hi = mid;
    }
    return lo;
}

// Blocks of a sweep launch resident on one CU at most (two wavefronts per
// SIMD), enforced by the LDS each block reserves: more resident wavefronts
// were measured to make the sweep slower (the caches serve fewer streams
// better).
constexpr int kSweepBlocksPerCU = 2;
constexpr int kPointUnroll = 4;       // chunk length of the sweep that also stores upwind intensities

template <typename T> struct Att { T E, D, al, be; };

// This file is compiled without floating-point contraction: every fused
// multiply-add is written out, so each instantiation (polar bound, chunk
// length, branch-free or not, single or batched) rounds identically and the
// results do not depend on the launch tuning.
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }

// e^{-tau}, 1 - e^{-tau} and alpha of eq. (13) in float32: series below the
// thresholds where the closed forms cancel, convex forms everywhere.
__device__ __forceinline__ Att<float> attenuate(float tau) {
    const float E = __expf(-tau);
    float p = fma_(-tau, 1.f / 5040.f, 1.f / 720.f);          // (1 - e^{-tau}) / tau, Horner in -tau
    p = fma_(-tau, p, 1.f / 120.f);
    p = fma_(-tau, p, 1.f / 24.f);
    p = fma_(-tau, p, 1.f / 6.f);
    p = fma_(-tau, p, 0.5f);
    p = fma_(-tau, p, 1.f);
    const float D = tau < 0.25f ? tau * p : 1.f - E;
    const float t2 = tau * tau;
    float q = fma_(-t2, 1.f / 47900160.f, 1.f / 1209600.f);  // alpha = 1/2 - tau/12 + tau^3/720 - ...
    q = fma_(-t2, q, 1.f / 30240.f);
    q = fma_(-t2, q, 1.f / 720.f);
    q = fma_(-t2, q, 1.f / 12.f);
    const float as = fma_(-tau, q, 0.5f);
    const float ac = fma_(-tau, E, D) * __builtin_amdgcn_rcpf(tau * D);
    const float al = tau < 1.f ? as : ac;
    return {E, D, al, 1.f - al};
}

// Same in float64 (series below tau = 0.1).
__device__ __forceinline__ Att<double> attenuate(double tau) {
    const double E = exp(-tau);
    double p = fma_(-tau, 1.0 / 3628800, 1.0 / 362880);
    p = fma_(-tau, p, 1.0 / 40320);
    p = fma_(-tau, p, 1.0 / 5040);
    p = fma_(-tau, p, 1.0 / 720);
    p = fma_(-tau, p, 1.0 / 120);
    p = fma_(-tau, p, 1.0 / 24);
    p = fma_(-tau, p, 1.0 / 6);
    p = fma_(-tau, p, 1.0 / 2);
    p = fma_(-tau, p, 1.0);
    const bool small = tau < 0.1;
    const double D = small ? tau * p : 1.0 - E;
    const double t2 = tau * tau;
    double q = fma_(-t2, 1.0 / 1209600, 1.0 / 30240);
    q = fma_(-t2, q, 1.0 / 720);
    q = fma_(-t2, q, 1.0 / 12);
    const double as = fma_(-tau, q, 0.5);
    double al;
    if (small) al = as;
    else al = fma_(-tau, E, D) / (tau * D);
    return {E, D, al, 1.0 - al};
}

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// Two-component records (int2, float2/double2, Coef<T>) loaded as native
// clang vectors: the HIP class types cannot be copied out of address space 1.
template <typename E> using vec2 = E __attribute__((ext_vector_type(2)));
template <typename E> using vec4 = E __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int2 ld2(gptr<const int2> p) {
    const vec2<int> v = *(gptr<const vec2<int>>)p;
    return make_int2(v.x, v.y);
}
__device__ __forceinline__ float2 ld2(gptr<const float2> p) {
    const vec2<float> v = *(gptr<const vec2<float>>)p;
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ double2 ld2(gptr<const double2> p) {
    const vec2<double> v = *(gptr<const vec2<double>>)p;
    return make_double2(v.x, v.y);
}
template <typename T> __device__ __forceinline__ Coef<T> ld2(gptr<const Coef<T>> p) {
    const vec2<T> v = *(gptr<const vec2<T>>)p;
    Coef<T> c;
    c.kt = v.x;
    c.a = v.y;
    return c;
}

// Element-wise state accesses (a polar count that is not a power of two):
// a lane's P values share cache lines with its neighbours', so they go
// through the caches -- non-temporal element accesses fetched the same lines
// once per polar slot (measured 2.7x slower at 512^2 with 6 polar angles).
template <typename T>
__device__ __forceinline__ T ldg_elem(gptr<const T> p) { return *p; }
template <typename T>
__device__ __forceinline__ void stg_elem(gptr<T> p, T v) { *p = v; }

// One wavefront per (traversal d, bundle B) of a problem.  Lane (k, g) walks
// its characteristic; step t reads the P stored values of the lane at
// [t][lane][p] of the bundle (contiguous per lane, 64 * P contiguous values
// per step) and writes the new ones at the same place.  Loads run one chunk of U steps ahead of the
// arithmetic: the geometry two chunks ahead, the cell coefficients (which
// depend on it) and the stored values one chunk ahead.  Each chunk's loads
// are issued together, so a wavefront asks for U consecutive rows of its
// bundle at once.
//
// Polar angles sit in PM register slots (PM >= P): lower slot i holds polar
// p = i, upper slot i holds p = P - 1 - i, so that with a mirror-symmetric
// polar set (mu_p = -mu_{P-1-p}, equal sin(zeta)) an upper slot reuses the
// exponential and alpha of the lower slot with the same index.
//
// FULL: P == PM and the polar set is mirror-symmetric, known at compile
// time, so a step has no per-slot branches (used for power-of-two P, whose
// batched launches share the polar bound P).  A FULL wavefront also stores
// every row of its bundle: the rows past the end of a lane's characteristic
// are that lane's padding, which nothing reads.
//
// POINT: also store the intensity entering each segment (the value at its
// upwind face) into A.point, in the state layout.
//
// SPLIT (a traversal cut into chunks of A.split_len steps, chunk c of the
// wavefront's traversal): the recurrence of eq. (12) maps the intensity
// entering a chunk affinely onto the one leaving it, I -> A I + B, A the
// product of the chunk's attenuation factors.  SPLIT == 1 computes that map
// of chunk c (for c = 0 from the true boundary intensity, so A = 0 and B is
// the exact exit of the chunk) into transfer record c of the wavefront, and
// stores no state; SPLIT == 2 sweeps chunk c from the intensity the scan of
// the records left in record c - 1 (chunk 0 from the boundary) and stores
// its rows, and the exit intensities at the last chunk.
template <typename T, int PM, int U, bool FULL, bool POINT = false, int SPLIT = 0>
__device__ __forceinline__ void sweep_wave(const SweepArgs& A, int64_t w, int lane, int chunk = 0,
                                           const SplitArgs& S = SplitArgs{}) {
    constexpr int NL = (PM + 1) / 2, NU = PM / 2, NS = NL + NU;
    const int d = w >= A.n_bun ? 1 : 0;
    const int64_t B = w - (d ? A.n_bun : 0);
    const gptr<const int> bun_off = as_global(A.bun_off);
    const gptr<const int> ray_off = as_global(A.ray_off);
    const gptr<const int> seg_off = as_global(A.seg_off);
    const int a = find_pair(bun_off, A.n_pairs, B);
    const int G = A.G;
    const int P = A.P;
    const int r0 = ray_off[a];
    const int Ka = ray_off[a + 1] - r0;
    const int f = (int)(B - bun_off[a]) * kWave + lane;
    int kl = f / G;
    const int g = f - kl * G;
    const bool active = kl < Ka;
    if (!active) kl = Ka - 1;                  // keep addresses valid; nothing is stored
    const int k = r0 + kl;
    const int s0 = seg_off[k];
    const int nk = seg_off[k + 1] - s0;
    const int n = active ? nk : 0;
    const int L = as_global(A.bun_len)[B];
    // steps [tb, te) of the traversal (all of it unless split)
    const int tb = SPLIT ? chunk * S.len : 0;
    const int te = SPLIT ? min(tb + S.len, L) : L;
    const int az = a + d * (A.n_az >> 1);
    const gptr<const Coef<T>> coef = as_global(static_cast<const Coef<T>*>(A.coef));
    const size_t boff = (size_t)d * A.half + (size_t)as_global(A.bun_base)[B] + (size_t)lane * P;
    const gptr<const T> xin = as_global(static_cast<const T*>(A.prev) + boff);
    const gptr<T> xout = as_global_w(static_cast<T*>(A.next) + boff);
    // optional: the intensity entering each segment (its upwind-face value)
    const gptr<T> pout = as_global_w(static_cast<T*>(POINT ? A.point : A.next) + boff);
    const size_t SP = (size_t)P * kWave;       // elements per step of a bundle ([lane][p])
    // a lane's P values of one step are contiguous: with P == PM (a power of
    // two) they move as one vector load or store
    constexpr bool kVecOk = PM >= 2 && (PM & (PM - 1)) == 0;
    const bool vec = kVecOk && (FULL || P == PM);
    // an even polar count that is not a power of two (6): pairs of values,
    // through the caches (the pairs of neighbouring lanes share lines)
    constexpr bool kPairsOk = !kVecOk && PM % 2 == 0;
    const bool pairs = kPairsOk && (FULL || P == PM);
    using V2 = T __attribute__((ext_vector_type(2)));
    using V = T __attribute__((ext_vector_type(PM)));

    int pol[NS];
    bool val[NS];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
        pol[i] = i;
        val[i] = FULL || i < (P + 1) / 2;
    }
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        pol[NL + i] = P - 1 - i;
        val[NL + i] = FULL || i < P / 2;
    }
    const bool sym = FULL || A.sym;

    double sc_in = 1.0, sc_out = 1.0, cb = A.inv_cdt;
    if (sizeof(T) == 4) {
        const int e = as_global(A.e_new)[g];
        sc_in = ldexp(1.0, -e);
        sc_out = ldexp(1.0, e);
        cb = ldexp(A.inv_cdt, as_global(A.e_prev)[g] - e);   // old-state scale folded into 1/(c dt)
    }
    const T cbt = (T)cb;
    T isz[NS];
    T I[NS];
    const int face_in = as_global(A.face)[2 * k + d];
    const gptr<const double> I_in = as_global(A.I_in);
#pragma unroll
    for (int r = 0; r < NS; ++r) {
        isz[r] = val[r] ? (T)A.inv_sinz[pol[r]] : (T)1;
        I[r] = val[r] ? (T)(I_in[((size_t)face_in * A.M + (size_t)az * P + pol[r]) * G + g] * sc_in) : (T)0;
    }
    // split: transfer records of this wavefront, [slot][lane] pairs each
    using T2v = T __attribute__((ext_vector_type(2)));
    const gptr<T2v> rec = as_global_w(static_cast<T2v*>(S.carry)) +
                          (SPLIT ? (size_t)as_global(S.cbase)[w] * NS * kWave + lane : 0);
    T Am[NS];                                      // SPLIT == 1: product of the attenuation factors
#pragma unroll
    for (int r = 0; r < NS; ++r) Am[r] = (T)1;
    if (SPLIT && chunk > 0) {
#pragma unroll
        for (int r = 0; r < NS; ++r) {
            if (SPLIT == 1) I[r] = (T)0;
            else I[r] = val[r] ? rec[((size_t)(chunk - 1) * NS + r) * kWave].y : (T)0;
        }
    }
    // segment index of step t (clamped into the characteristic)
    auto seg = [&](int t) -> int {
        const int tt = t < nk ? t : nk - 1;
        return d == 0 ? s0 + tt : s0 + nk - 1 - tt;
    };
    auto srow = [&](int t) -> gptr<const T> { return xin + (size_t)(t < L ? t : L - 1) * SP; };
    // the stored values of one step into the polar slots
    auto load_row = [&](gptr<const T> r, T (&x)[NS]) {
        if (vec) {
            const V v = __builtin_nontemporal_load((gptr<const V>)r);
#pragma unroll
            for (int i = 0; i < NL; ++i) x[i] = v[i];
#pragma unroll
            for (int i = 0; i < NU; ++i) x[NL + i] = v[PM - 1 - i];
        } else if (pairs) {
            T y[PM];
#pragma unroll
            for (int h = 0; h < PM / 2; ++h) {
                const V2 v = *(gptr<const V2>)(r + 2 * h);
                y[2 * h] = v.x;
                y[2 * h + 1] = v.y;
            }
#pragma unroll
            for (int i = 0; i < NL; ++i) x[i] = y[i];
#pragma unroll
            for (int i = 0; i < NU; ++i) x[NL + i] = y[PM - 1 - i];
        } else {
#pragma unroll
            for (int q = 0; q < NS; ++q) x[q] = val[q] ? ldg_elem(r + pol[q]) : (T)0;
        }
    };

    // the values of one step from the polar slots
    auto store_row = [&](gptr<T> o, const T (&x)[NS]) {
        if (vec) {
            V v;
#pragma unroll
            for (int i = 0; i < NL; ++i) v[i] = x[i];
#pragma unroll
            for (int i = 0; i < NU; ++i) v[PM - 1 - i] = x[NL + i];
            __builtin_nontemporal_store(v, (gptr<V>)o);
        } else if (pairs) {
            T y[PM];
#pragma unroll
            for (int i = 0; i < NL; ++i) y[i] = x[i];
#pragma unroll
            for (int i = 0; i < NU; ++i) y[PM - 1 - i] = x[NL + i];
#pragma unroll
            for (int h = 0; h < PM / 2; ++h) {
                V2 v;
                v.x = y[2 * h];
                v.y = y[2 * h + 1];
                *(gptr<V2>)(o + 2 * h) = v;
            }
        } else {
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (val[q]) stg_elem(o + pol[q], x[q]);
        }
    };

    // a segment's cell index and length arrive in one load
    const gptr<const int> gseg = as_global(static_cast<const int*>(A.seg));
    auto seg_rec = [&](int j, int& cell, T& len) {
        if constexpr (sizeof(T) == 4) {
            const vec2<int> v = *(gptr<const vec2<int>>)(gseg + 2 * (size_t)j);
            cell = v.x;
            len = __int_as_float(v.y);
        } else {
            const vec4<int> v = *(gptr<const vec4<int>>)(gseg + 4 * (size_t)j);
            cell = v.x;
            len = __hiloint2double(v.w, v.z);
        }
    };
    int cell1[U];
    T len0[U], len1[U];
    Coef<T> c0[U];
    T x0[U][NS];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j0 = seg(tb + u), j1 = seg(tb + U + u);
        int cell0;
        seg_rec(j0, cell0, len0[u]);
        c0[u] = ld2(coef + ((size_t)cell0 * G + g));
        seg_rec(j1, cell1[u], len1[u]);
        load_row(srow(tb + u), x0[u]);
    }
    for (int t0 = tb; t0 < te; t0 += U) {
        Coef<T> c1[U];
        T x1[U][NS];
        int cell2[U];
        T len2[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c1[u] = ld2(coef + ((size_t)cell1[u] * G + g));
            load_row(srow(t0 + U + u), x1[u]);
            const int j2 = seg(t0 + 2 * U + u);
            seg_rec(j2, cell2[u], len2[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int t = t0 + u;
            const bool live = t < n;
            const T ktl = c0[u].kt * len0[u];
            const T b = cbt * recip(c0[u].kt);                      // 1/(c dt kappa_t)
            Att<T> at[NS];
#pragma unroll
            for (int i = 0; i < NL; ++i)
                if (val[i]) at[i] = attenuate(ktl * isz[i]);
#pragma unroll
            for (int i = 0; i < NU; ++i)
                if (val[NL + i]) at[NL + i] = sym ? at[i] : attenuate(ktl * isz[NL + i]);
            T ob[NS], ib[NS];
#pragma unroll
            for (int q = 0; q < NS; ++q) {
                ob[q] = (T)0;
                ib[q] = I[q];
                if (!val[q]) continue;
                const T S = fma_(b, x0[u][q], c0[u].a);               // Q / kappa_t
                const T Io = fma_(at[q].E, I[q], at[q].D * S);        // eq. (12)
                ob[q] = fma_(at[q].al, I[q], at[q].be * Io);          // segment average
                I[q] = live ? Io : I[q];
                if (SPLIT == 1) Am[q] = live ? Am[q] * at[q].E : Am[q];
            }
            if (SPLIT != 1 && (FULL ? t < te : live)) {
                store_row(xout + (size_t)t * SP, ob);
                if (POINT) store_row(pout + (size_t)t * SP, ib);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c0[u] = c1[u];
            len0[u] = len1[u];
            cell1[u] = cell2[u];
            len1[u] = len2[u];
#pragma unroll
            for (int q = 0; q < NS; ++q) x0[u][q] = x1[u][q];
        }
    }
    if (SPLIT == 1) {
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            T2v v;
            v.x = chunk > 0 ? Am[q] : (T)0;
            v.y = I[q];
            rec[((size_t)chunk * NS + q) * kWave] = v;
        }
        return;
    }
    if (A.I_exit && active && te == L) {
        const gptr<double> I_exit = as_global_w(A.I_exit);
#pragma unroll
        for (int q = 0; q < NS; ++q)
            if (val[q]) I_exit[((size_t)(2 * k + d) * P + pol[q]) * G + g] = (double)I[q] * sc_out;
    }
}

template <typename T, int PM, int U, bool FULL, bool POINT>
__global__ __launch_bounds__(kBlock) void k_sweep(SweepArgs A) {
    const int64_t lb = xcd_logical_block(blockIdx.x, A.n_blocks);
    const int64_t w = lb * (kBlock / kWave) + (threadIdx.x / kWave);
    if (w >= 2 * A.n_bun) return;
    sweep_wave<T, PM, U, FULL, POINT>(A, w, threadIdx.x & (kWave - 1));
}

// Batched form: a persistent grid whose wavefronts take work items
// (problem, wavefront of that problem) from eight queues, one per XCD --
// block b is assumed to run on XCD b mod 8, the hardware's round-robin order.
// Queue x holds a contiguous range of the item list (problems in decreasing
// cost, the two traversals of a bundle side by side) of about one eighth of
// the summed bundle lengths, so the characteristics crossing a cell are swept
// on one XCD and share its L2 copy of the cell coefficients.  A wavefront
// whose queue is empty moves on to the next one and stops after finding all
// eight empty; counters only grow, so every wavefront exits.  FULL holds for
// every problem of the launch.
template <typename T, int PM, int U, bool FULL>
__global__ __launch_bounds__(kBlock) void k_sweep_batch(const SweepArgs* __restrict__ probs,
                                                        const int2* __restrict__ items,
                                                        const int64_t* __restrict__ qb, int* counters) {
    const int lane = threadIdx.x & (kWave - 1);
    int q = blockIdx.x & 7;
    for (int empty = 0; empty < 8;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(&counters[q], 1);
        it = __builtin_amdgcn_readfirstlane(__shfl(it, 0));
        const int64_t gi = qb[q] + it;
        if (gi >= qb[q + 1]) {
            ++empty;
            q = (q + 1) & 7;
            continue;
        }
        const int pr = __builtin_amdgcn_readfirstlane(items[gi].x);
        const int w = __builtin_amdgcn_readfirstlane(items[gi].y);
        sweep_wave<T, PM, U, FULL>(probs[pr], w, lane);
    }
}

// Split sweep: one wavefront per item {wavefront of the plain sweep, chunk},
// in either mode; blocks remapped per XCD as in the plain sweep.
template <typename T, int PM, int MODE>
__global__ __launch_bounds__(kBlock) void k_sweep_split(SweepArgs A, SplitArgs S, const int2* __restrict__ items,
                                                        int64_t n_items, int64_t n_blocks) {
    const int64_t lb = xcd_logical_block(blockIdx.x, n_blocks);
    const int64_t i = lb * (kBlock / kWave) + (threadIdx.x / kWave);
    if (i >= n_items) return;
    const int2 it = ld2(as_global(items) + i);
    const int w = __builtin_amdgcn_readfirstlane(it.x);
    const int c = __builtin_amdgcn_readfirstlane(it.y);
    sweep_wave<T, PM, kSplitUnroll, false, false, MODE>(A, w, threadIdx.x & (kWave - 1), c, S);
}

// Sequential composition of the transfer records of each wavefront: one
// thread per (wavefront, slot, lane) walks the records of its chunks in
// order, I <- A I + B from I = 0, and leaves in record c the intensity
// entering chunk c + 1 (record 0 holds the exact exit of chunk 0, A = 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_split_scan(T* carry, const int64_t* __restrict__ cbase, int per,
                                                       int64_t n_threads) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n_threads) return;
    const int64_t w = e / per, o = e - w * per;
    const gptr<const int64_t> cb = as_global(cbase);
    const int64_t r0 = cb[w], r1 = cb[w + 1];
    using T2v = T __attribute__((ext_vector_type(2)));
    const gptr<T2v> rec = as_global_w(reinterpret_cast<T2v*>(carry));
    // records are read kScanBatch at a time (independent loads in flight
    // together), then composed in order
    constexpr int kScanBatch = 8;
    T I = (T)0;
    for (int64_t r = r0; r < r1; r += kScanBatch) {
        T2v v[kScanBatch];
#pragma unroll
        for (int j = 0; j < kScanBatch; ++j)
            if (r + j < r1) v[j] = rec[(r + j) * per + o];
#pragma unroll
        for (int j = 0; j < kScanBatch; ++j)
            if (r + j < r1) {
                I = fma_(v[j].x, I, v[j].y);
                v[j].y = I;
                rec[(r + j) * per + o] = v[j];
            }
    }
}

__global__ void k_zero_counter(int* c, int n) {
    if ((int)threadIdx.x < n) c[threadIdx.x] = 0;
}

// One sweep launch: a single problem (args1, blocks) or a batch (args,
// items, qb, counters, grid), or, with grid_out, the query of the batch's
// persistent grid.  lds is the dynamic LDS each block reserves to cap the
// blocks resident on a CU.
struct SweepCall {
    int unroll = 8;
    bool full = false;
    bool point = false;       // single problems: store the upwind intensities too
    size_t lds = 0;
    hipStream_t st = nullptr;
    const SweepArgs* args1 = nullptr;
    unsigned blocks = 0;
    const void* args = nullptr;
    const int2* items = nullptr;
    const int64_t* qb = nullptr;
    int* counters = nullptr;
    int grid = 0;
    int* grid_out = nullptr;
};

template <bool BATCH, typename T, int PM, int U, bool FULL, bool POINT = false>
lc_status sweep_call(const SweepCall& c) {
    if constexpr (!BATCH) {
        hipLaunchKernelGGL((k_sweep<T, PM, U, FULL, POINT>), dim3(c.blocks), dim3(kBlock), c.lds, c.st, *c.args1);
    } else if (c.grid_out) {
        // as many blocks as the device keeps resident, a multiple of 8 so
        // that every XCD gets the same count
        int dev = 0, cus = 0, per_cu = 0;
        LC_HIP(hipGetDevice(&dev));
        LC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        LC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_sweep_batch<T, PM, U, FULL>), kBlock, c.lds));
        *c.grid_out = std::max(8, cus * std::max(per_cu, 1) / 8 * 8);
        return LC_OK;
    } else {
        hipLaunchKernelGGL((k_sweep_batch<T, PM, U, FULL>), dim3(c.grid), dim3(kBlock), c.lds, c.st,
                           static_cast<const SweepArgs*>(c.args), c.items, c.qb, c.counters);
    }
    LC_HIP(hipGetLastError());
    return LC_OK;
}

template <bool BATCH, typename T, int PM, bool FULL>
lc_status sweep_call_u(const SweepCall& c) {
    // the upwind-intensity form has one chunk length (results do not depend on it)
    if constexpr (!BATCH)
        if (c.point) return sweep_call<BATCH, T, PM, kPointUnroll, FULL, true>(c);
    switch (c.unroll) {
        case 1: return sweep_call<BATCH, T, PM, 1, FULL>(c);
        case 2: return sweep_call<BATCH, T, PM, 2, FULL>(c);
        case 4: return sweep_call<BATCH, T, PM, 4, FULL>(c);
        case 16:
            // 16-step chunks fit the registers of two wavefronts per SIMD in
            // float32 with up to four polar angles only
            if constexpr (sizeof(T) == 4 && PM <= kMaxPolUnroll16) return sweep_call<BATCH, T, PM, 16, FULL>(c);
            set_error("sweep_unroll 16 needs float32 and n_pol <= %d", kMaxPolUnroll16);
            return LC_ERR_UNSUPPORTED;
        default: return sweep_call<BATCH, T, PM, 8, FULL>(c);
    }
}

template <bool BATCH, typename T, int PM>
lc_status sweep_call_f(const SweepCall& c) {
    return c.full ? sweep_call_u<BATCH, T, PM, true>(c) : sweep_call_u<BATCH, T, PM, false>(c);
}

// Single problems: PM = n_pol exactly.
template <typename T>
lc_status sweep_call_single(int n_pol, const SweepCall& c) {
    switch (n_pol) {
        case 1: return sweep_call_f<false, T, 1>(c);
        case 2: return sweep_call_f<false, T, 2>(c);
        case 3: return sweep_call_f<false, T, 3>(c);
        case 4: return sweep_call_f<false, T, 4>(c);
        case 5: return sweep_call_f<false, T, 5>(c);
        case 6: return sweep_call_f<false, T, 6>(c);
        case 7: return sweep_call_f<false, T, 7>(c);
        case 8: return sweep_call_f<false, T, 8>(c);
    }
    set_error("n_pol = %d not supported (1..8)", n_pol);
    return LC_ERR_UNSUPPORTED;
}

// Batches: PM = the polar bound of a group of problems, a power of two.
lc_status sweep_call_batch(int prec, int pm, const SweepCall& c) {
    const bool f32 = prec == LC_F32;
    switch (pm) {
        case 1: return f32 ? sweep_call_f<true, float, 1>(c) : sweep_call_f<true, double, 1>(c);
        case 2: return f32 ? sweep_call_f<true, float, 2>(c) : sweep_call_f<true, double, 2>(c);
        case 4: return f32 ? sweep_call_f<true, float, 4>(c) : sweep_call_f<true, double, 4>(c);
        case 8: return f32 ? sweep_call_f<true, float, 8>(c) : sweep_call_f<true, double, 8>(c);
    }
    set_error("batched sweep: polar bound %d not supported", pm);
    return LC_ERR_UNSUPPORTED;
}

// Split sweep of a single problem (PM = n_pol): mode 1 over the transfer
// items, the scan, mode 2 over the sweep items.  Its problems are the ones
// with too few lanes to fill the device, whose time is the latency of a
// chunk's steps: the blocks reserve no LDS, so as many wavefronts stay
// resident as the registers allow.
template <typename T, int PM>
lc_status split_call(const Plan* pl, const SweepArgs& A, hipStream_t st) {
    const int64_t per = (int64_t)PM * kWave;
    SplitArgs S;
    S.carry = pl->d_carry;
    S.cbase = pl->d_cbase;
    S.len = pl->split_len;
    const int64_t n1 = pl->n_split1, n2 = pl->n_split_items - pl->n_split1;
    const int wpb = kBlock / kWave;
    if (n1 > 0) {
        const int64_t nb = (n1 + wpb - 1) / wpb;
        hipLaunchKernelGGL((k_sweep_split<T, PM, 1>), dim3((unsigned)nb), dim3(kBlock), 0, st, A, S,
                           pl->d_split_items, n1, nb);
        LC_HIP(hipGetLastError());
        const int64_t nt = 2 * pl->n_bun * per;
        hipLaunchKernelGGL(k_split_scan<T>, dim3((unsigned)((nt + kBlock - 1) / kBlock)), dim3(kBlock), 0, st,
                           static_cast<T*>(pl->d_carry), pl->d_cbase, (int)per, nt);
        LC_HIP(hipGetLastError());
    }
    if (n2 == 0) return LC_OK;
    const int64_t nb = (n2 + wpb - 1) / wpb;
    hipLaunchKernelGGL((k_sweep_split<T, PM, 2>), dim3((unsigned)nb), dim3(kBlock), 0, st, A, S,
                       pl->d_split_items + n1, n2, nb);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

template <typename T>
lc_status split_call_p(const Plan* pl, const SweepArgs& A, hipStream_t st) {
    switch (pl->rays->n_pol) {
        case 1: return split_call<T, 1>(pl, A, st);
        case 2: return split_call<T, 2>(pl, A, st);
        case 3: return split_call<T, 3>(pl, A, st);
        case 4: return split_call<T, 4>(pl, A, st);
        case 5: return split_call<T, 5>(pl, A, st);
        case 6: return split_call<T, 6>(pl, A, st);
        case 7: return split_call<T, 7>(pl, A, st);
        case 8: return split_call<T, 8>(pl, A, st);
    }
    set_error("n_pol = %d not supported (1..8)", pl->rays->n_pol);
    return LC_ERR_UNSUPPORTED;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

size_t sweep_args_bytes() { return sizeof(SweepArgs); }

// Host copies of the sweep records of one problem of a batch (one per step parity).
void make_batch_args(Plan* pl, double c_dt, void* state_a, void* state_b, const double* I_in, double* I_exit,
                     void* sweep_out2) {
    Rays* r = pl->rays;
    const bool f32 = pl->prec == LC_F32;
    for (int parity = 0; parity < 2; ++parity) {
        void* prev = parity ? state_b : state_a;
        void* next = parity ? state_a : state_b;
        SweepArgs A{};
        A.bun_off = pl->d_bun_off;
        A.bun_len = pl->d_bun_len;
        A.bun_base = pl->d_bun_base;
        A.n_pairs = r->n_pairs;
        A.n_bun = pl->n_bun;
        A.half = pl->half_elems;
        A.n_blocks = pl->sweep_blocks;
        A.ray_off = r->d_ray_off;
        A.seg_off = r->d_seg_off;
        A.face = r->d_face;
        A.seg = f32 ? static_cast<const void*>(r->d_seg32) : static_cast<const void*>(r->d_seg64);
        A.coef = pl->d_coef;
        A.prev = state_values(pl, prev);
        A.next = state_values(pl, next);
        A.I_in = I_in;
        A.I_exit = I_exit;
        A.P = r->n_pol;
        A.sym = r->sym ? 1 : 0;
        A.e_prev = static_cast<const int*>(prev);
        A.e_new = static_cast<const int*>(next);
        A.inv_cdt = 1.0 / c_dt;
        A.G = pl->G;
        A.n_az = r->n_az;
        A.M = r->n_az * r->n_pol;
        for (int p = 0; p < r->n_pol; ++p) A.inv_sinz[p] = r->inv_sinz[p];
        std::memcpy(static_cast<char*>(sweep_out2) + parity * sizeof(SweepArgs), &A, sizeof(A));
    }
}

lc_status launch_zero_counters(int* c, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, st, c, n);
    LC_HIP(hipGetLastError());
    return LC_OK;
}

lc_status sweep_lds_bytes(size_t* lds) {
    *lds = 0;
    int dev = 0, per_cu = 0;
    LC_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess ||
        per_cu <= 0)
        return LC_OK;                 // no cap
    *lds = (size_t)per_cu / (kSweepBlocksPerCU + 1) + 1;
    return LC_OK;
}

lc_status sweep_batch_grid(int prec, int pm, int unroll, bool full, size_t lds, int* grid) {
    SweepCall c;
    c.unroll = unroll;
    c.full = full;
    c.lds = lds;
    c.grid_out = grid;
    return sweep_call_batch(prec, pm, c);
}

lc_status launch_sweep_batch(int prec, int pm, int unroll, bool full, size_t lds, int grid, const void* args,
                             const int2* items, const int64_t* qb, int* counters, hipStream_t st) {
    SweepCall c;
    c.unroll = unroll;
    c.full = full;
    c.lds = lds;
    c.st = st;
    c.args = args;
    c.items = items;
    c.qb = qb;
    c.counters = counters;
    c.grid = grid;
    return sweep_call_batch(prec, pm, c);
}

lc_status plan_init_sweep(Plan* pl) {
    Rays* r = pl->rays;
    const int G = pl->G, P = r->n_pol;
    pl->bun_off.assign(r->n_pairs + 1, 0);
    pl->bun_len_h.clear();
    pl->bun_base_h.clear();
    int64_t base = 0;
    for (int a = 0; a < r->n_pairs; ++a) {
        const int r0 = r->ray_off[a], Ka = r->ray_off[a + 1] - r0;
        const int64_t lanes = (int64_t)Ka * G;
        const int64_t nb = (lanes + kWave - 1) / kWave;
        for (int64_t b = 0; b < nb; ++b) {
            const int64_t f0 = b * kWave, f1 = std::min(lanes, f0 + kWave) - 1;
            int L = 0;
            for (int64_t kl = f0 / G; kl <= f1 / G; ++kl)
                L = std::max(L, r->seg_off[r0 + kl + 1] - r->seg_off[r0 + kl]);
            pl->bun_len_h.push_back(L);
            pl->bun_base_h.push_back(base);
            base += (int64_t)L * P * kWave;
        }
        LC_CHECK((int64_t)pl->bun_len_h.size() < INT32_MAX, LC_ERR_UNSUPPORTED, "too many bundles");
        pl->bun_off[a + 1] = (int)pl->bun_len_h.size();
    }
    pl->n_bun = (int64_t)pl->bun_len_h.size();
    pl->half_elems = base;
    const int64_t waves = 2 * pl->n_bun;
    pl->sweep_blocks = (waves + kBlock / kWave - 1) / (kBlock / kWave);
    LC_CHECK(pl->sweep_blocks < INT32_MAX, LC_ERR_UNSUPPORTED, "sweep grid too large");
    return sweep_lds_bytes(&pl->sweep_lds);
}

void plan_free_split(Plan* pl) {
    for (void* q : {static_cast<void*>(pl->d_split_items), static_cast<void*>(pl->d_cbase), pl->d_carry})
        if (q) (void)hipFree(q);
    pl->d_split_items = nullptr;
    pl->d_cbase = nullptr;
    pl->d_carry = nullptr;
    pl->n_split1 = pl->n_split_items = 0;
    pl->split_len = 0;
}

lc_status plan_set_split(Plan* pl, int len) {
    plan_free_split(pl);
    if (len == 0) return LC_OK;
    const int64_t nw = 2 * pl->n_bun;
    std::vector<int64_t> cbase(nw + 1, 0);
    std::vector<int2> items1, items2;
    for (int64_t w = 0; w < nw; ++w) {
        const int L = pl->bun_len_h[w % pl->n_bun];
        const int nc = std::max(1, (L + len - 1) / len);
        for (int c = 0; c + 1 < nc; ++c) items1.push_back(make_int2((int)w, c));
        for (int c = 0; c < nc; ++c) items2.push_back(make_int2((int)w, c));
        cbase[w + 1] = cbase[w] + (nc - 1);
    }
    const int64_t wpb = kBlock / kWave;
    LC_CHECK(((int64_t)items2.size() + wpb - 1) / wpb < INT32_MAX, LC_ERR_UNSUPPORTED, "split sweep grid too large");
    LC_CHECK((nw * pl->rays->n_pol * kWave + kBlock - 1) / kBlock < INT32_MAX, LC_ERR_UNSUPPORTED,
             "split sweep scan grid too large");
    const size_t elem = pl->prec == LC_F32 ? sizeof(float) : sizeof(double);
    const size_t carry = (size_t)std::max<int64_t>(cbase[nw], 1) * pl->rays->n_pol * kWave * 2 * elem;
    std::vector<int2> items(items1);
    items.insert(items.end(), items2.begin(), items2.end());
    lc_status rc = LC_OK;
    auto put = [&](void** dst, const void* src, size_t bytes) {
        if (rc != LC_OK) return;
        if (lc_malloc(dst, bytes) != hipSuccess) {
            (void)hipGetLastError();
            *dst = nullptr;
            set_error("hipMalloc of %zu bytes for the split sweep failed", bytes);
            rc = LC_ERR_ALLOC;
            return;
        }
        if (src && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
            set_error("copy of the split sweep items failed");
            rc = LC_ERR_HIP;
        }
    };
    put(reinterpret_cast<void**>(&pl->d_split_items), items.data(), items.size() * sizeof(int2));
    put(reinterpret_cast<void**>(&pl->d_cbase), cbase.data(), cbase.size() * sizeof(int64_t));
    put(&pl->d_carry, nullptr, carry);
    if (rc != LC_OK) {
        plan_free_split(pl);
        return rc;
    }
    pl->n_split1 = (int64_t)items1.size();
    pl->n_split_items = (int64_t)items.size();
    pl->split_len = len;
    return LC_OK;
}

lc_status launch_sweep(Plan* pl, const double* kappa, const double* planck, double c_dt,
                       const void* state_prev, void* state_new, const double* I_in, double* I_exit,
                       hipStream_t st, void* point, const SweepScratch* ws) {
    Rays* r = pl->rays;
    const int G = pl->G;
    const bool f32 = pl->prec == LC_F32;
    const int* e_prev = static_cast<const int*>(state_prev);   // header: per-group exponents
    int* e_new = static_cast<int*>(state_new);
    void* coef = ws ? ws->coef : pl->d_coef;
    unsigned long long* gmax = ws ? ws->gmax : pl->d_gmax;
    lc_status rc = launch_prologue(pl, kappa, planck, c_dt, state_prev, state_new, I_in, st, coef, gmax);
    if (rc) return rc;
    SweepArgs A{};
    A.bun_off = pl->d_bun_off;
    A.bun_len = pl->d_bun_len;
    A.bun_base = pl->d_bun_base;
    A.n_pairs = r->n_pairs;
    A.n_bun = pl->n_bun;
    A.half = pl->half_elems;
    A.n_blocks = pl->sweep_blocks;
    A.ray_off = r->d_ray_off;
    A.seg_off = r->d_seg_off;
    A.face = r->d_face;
    A.seg = f32 ? static_cast<const void*>(r->d_seg32) : static_cast<const void*>(r->d_seg64);
    A.coef = coef;
    A.prev = state_values(pl, state_prev);
    A.next = state_values(pl, state_new);
    A.point = point ? state_values(pl, point) : nullptr;

    A.I_in = I_in;
    A.I_exit = I_exit;
    A.e_prev = e_prev;
    A.e_new = e_new;
    A.inv_cdt = 1.0 / c_dt;
    A.G = G;
    A.n_az = r->n_az;
    A.M = r->n_az * r->n_pol;
    A.P = r->n_pol;
    A.sym = r->sym ? 1 : 0;
    for (int p = 0; p < r->n_pol; ++p) A.inv_sinz[p] = r->inv_sinz[p];
    if (!ws) {
        rc = prof_begin(pl, pl->ev_sweep, st);
        if (rc) return rc;
    }
    if (pl->split_len > 0 && !point && !ws) {
        rc = f32 ? split_call_p<float>(pl, A, st) : split_call_p<double>(pl, A, st);
        if (rc) return rc;
        return prof_end(pl, pl->ev_sweep, st);
    }
    SweepCall c;
    c.unroll = pl->sweep_unroll;
    c.full = sweep_full(r);
    c.point = point != nullptr;
    c.lds = pl->sweep_lds;
    c.st = st;
    c.args1 = &A;
    c.blocks = (unsigned)pl->sweep_blocks;
    rc = f32 ? sweep_call_single<float>(r->n_pol, c) : sweep_call_single<double>(r->n_pol, c);
    if (rc) return rc;
    return ws ? LC_OK : prof_end(pl, pl->ev_sweep, st);
}

}  // namespace lc
