// Batched form: many independent problems advanced together.  Problems are
// grouped by polar bound and sweep form; per step and group there is one
// persistent sweep
// kernel whose wavefronts pull (problem, bundle traversal) items from eight
// per-XCD queues and one cell-moment launch over the (problem, tile
// wavefront) items; the coefficient prologue and the boundary factors are one
// launch over all problems.  Items are ordered by problem cost, largest
// first, so the small problems fill the tail.  The step sequence is captured
// in a HIP graph per step count and replayed.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <numeric>

#include "lc_internal.hpp"

namespace lc {
namespace {

// Problems of one polar bound (the power of two >= their polar count) and
// one sweep form: their sweep and moment kernels are compiled for that bound,
// so a class of two-angle problems does not carry the registers of a
// four-angle one, and each member runs the sweep code of its single-problem
// run.
struct PolarClass {
    int pm = 1;
    int unroll = 2, ent = 3;            // launch tuning of the class's lowest-index member
    bool full = false;                  // members run the FULL sweep (sweep_full)
    size_t sweep_lds = 0;               // LDS reserved per sweep block
    int sweep_grid = 0;                 // resident blocks of the persistent sweep on this device
    int2* d_sweep_items = nullptr;      // {problem, bundle traversal}
    int64_t* d_sweep_qb = nullptr;      // [9] bounds of the eight per-XCD sweep queues
    int2* d_mom_items = nullptr;        // {problem, wavefront of a tile}
    int64_t n_mom_items = 0;
};

struct Batch {
    uint32_t magic = 0;
    int n = 0, prec = 0;
    double c = 0.0;
    std::vector<lc_problem_t> probs;
    std::vector<Plan*> plans;
    std::vector<char> h_mom;            // host copy of the moment records [2][n]
    void* d_sweep_args = nullptr;       // [2][n] sweep records (parity of the step)
    void* d_coef_args = nullptr;        // [n]
    void* d_mom_args = nullptr;         // [2][n]
    void* d_bnd_args = nullptr;         // [n]
    std::vector<PolarClass> cls;
    int* d_counters = nullptr;          // [8 * classes] counters of the sweep queues
    unsigned long long* d_gmax = nullptr;   // [2][n_gmax] per-group maxima of |B|, then of |I_in|, of every problem
    int64_t n_gmax = 0, max_blocks = 0, coef_blocks = 0, bnd_blocks = 0;
    int max_G = 1;
    std::vector<GraphEntry> graphs;
    hipStream_t capture = nullptr;
    hipStream_t side = nullptr;         // captured side branch (boundary factors, next prologue)
    hipStream_t side_mom = nullptr;     // captured branch of the moments
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_mom[2] = {nullptr, nullptr};   // end of the moments of steps of either parity
    bool profile = false;               // eager steps with events around each phase
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[3];   // prologue, sweep, moments
};

void clear_events(Batch* b) {
    for (auto& v : b->ev) {
        for (auto& e : v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        v.clear();
    }
}

lc_status ev_begin(Batch* b, int k, hipStream_t st) {
    if (!b->profile) return LC_OK;
    hipEvent_t x = nullptr, y = nullptr;
    LC_HIP(hipEventCreate(&x));
    hipError_t e = hipEventCreate(&y);
    if (e != hipSuccess) {
        (void)hipEventDestroy(x);
        set_error("hipEventCreate failed: %s", hipGetErrorString(e));
        return LC_ERR_HIP;
    }
    b->ev[k].push_back({x, y});
    LC_HIP(hipEventRecord(x, st));
    return LC_OK;
}

lc_status ev_end(Batch* b, int k, hipStream_t st) {
    if (!b->profile) return LC_OK;
    LC_HIP(hipEventRecord(b->ev[k].back().second, st));
    return LC_OK;
}

// Enqueue n_steps time steps of every problem on st.  Running the polar
// groups on streams of their own was measured slower: their kernels contend
// for the same caches and bandwidth rather than filling each other's tails.
//
// Eager (profiling): one phase after the other, with the phase timers.
//
// Captured graph: the sweeps stay on the main branch; after the sweep of step
// t two branches fork from it:
//   - the boundary factors of step t (they need only the exit intensities)
//     and the prologue of step t + 1 (queue counters, source maxima,
//     coefficient table, and the scale in the header of the state buffer
//     that step t + 1 writes), joined before the sweep of step t + 1;
//   - the moments of step t, which read the state of step t -- the sweep of
//     step t + 1 only reads it too, so the two run side by side.
// The sweep of step t + 2 and the prologue of step t + 2 write the buffer
// (values and header) the moments of step t read, so both wait for them;
// the moments of consecutive steps keep their order on their branch (they
// write the same outputs).
lc_status enqueue_steps(Batch* b, int n_steps, hipStream_t st) {
    const size_t sb = sweep_args_bytes(), mb = mom_args_bytes();
    const bool branch = !b->profile;
    auto prologue = [&](int t, hipStream_t s) {
        lc_status rc = launch_zero_counters(b->d_counters, 8 * (int)b->cls.size(), s);
        if (rc == LC_OK) rc = ev_begin(b, 0, s);
        if (rc == LC_OK)
            rc = launch_prologue_batch(b->prec, b->d_coef_args, b->n, b->max_blocks, b->coef_blocks, b->max_G,
                                       b->d_gmax, b->n_gmax, t, s);
        if (rc == LC_OK) rc = ev_end(b, 0, s);
        return rc;
    };
    auto moments = [&](int t, hipStream_t s) {
        lc_status rc = ev_begin(b, 2, s);
        for (size_t c = 0; c < b->cls.size() && rc == LC_OK; ++c)
            rc = launch_moments_batch(b->prec, b->cls[c].pm, b->cls[c].ent,
                                      static_cast<char*>(b->d_mom_args) + (t & 1) * b->n * mb,
                                      b->cls[c].d_mom_items, b->cls[c].n_mom_items, s);
        if (rc == LC_OK) rc = ev_end(b, 2, s);
        return rc;
    };
    auto wait = [&](hipStream_t s, hipEvent_t e) {
        return hipStreamWaitEvent(s, e, 0) == hipSuccess ? LC_OK : LC_ERR_HIP;
    };
    auto record = [&](hipEvent_t e, hipStream_t s) {
        return hipEventRecord(e, s) == hipSuccess ? LC_OK : LC_ERR_HIP;
    };
    lc_status rc = LC_OK;
    for (int t = 0; t < n_steps && rc == LC_OK; ++t) {
        const int parity = t & 1;
        if (t == 0 || !branch) rc = prologue(t, st);  // later steps: on the previous step's branch
        if (rc == LC_OK && branch && t >= 2) rc = wait(st, b->ev_mom[parity]);   // moments of step t - 2
        if (rc == LC_OK) rc = ev_begin(b, 1, st);
        for (size_t c = 0; c < b->cls.size() && rc == LC_OK; ++c)
            rc = launch_sweep_batch(b->prec, b->cls[c].pm, b->cls[c].unroll, b->cls[c].full, b->cls[c].sweep_lds,
                                    b->cls[c].sweep_grid, static_cast<char*>(b->d_sweep_args) + parity * b->n * sb,
                                    b->cls[c].d_sweep_items, b->cls[c].d_sweep_qb, b->d_counters + 8 * c, st);
        if (rc == LC_OK) rc = ev_end(b, 1, st);
        if (!branch) {
            if (rc == LC_OK) rc = moments(t, st);
            if (rc == LC_OK && b->bnd_blocks > 0) rc = launch_boundary_batch(b->d_bnd_args, b->n, b->bnd_blocks, st);
            continue;
        }
        const bool side = b->bnd_blocks > 0 || t + 1 < n_steps;
        if (rc == LC_OK) rc = record(b->ev_fork, st);
        if (rc == LC_OK && side) {
            rc = wait(b->side, b->ev_fork);
            if (rc == LC_OK && b->bnd_blocks > 0) rc = launch_boundary_batch(b->d_bnd_args, b->n, b->bnd_blocks, b->side);
            if (rc == LC_OK && t + 1 < n_steps && t >= 1) rc = wait(b->side, b->ev_mom[parity ^ 1]);   // step t - 1
            if (rc == LC_OK && t + 1 < n_steps) rc = prologue(t + 1, b->side);
            if (rc == LC_OK) rc = record(b->ev_join, b->side);
        }
        if (rc == LC_OK) rc = wait(b->side_mom, b->ev_fork);
        if (rc == LC_OK) rc = moments(t, b->side_mom);
        if (rc == LC_OK) rc = record(b->ev_mom[parity], b->side_mom);
        if (rc == LC_OK && side) rc = wait(st, b->ev_join);
    }
    if (rc == LC_OK && branch && n_steps > 0) rc = wait(st, b->ev_mom[(n_steps - 1) & 1]);   // join the moments
    return rc;
}

Batch* as_batch(lc_batch_t b) {
    Batch* p = reinterpret_cast<Batch*>(b);
    return (p && p->magic == kBatchMagic) ? p : nullptr;
}

void free_batch(Batch* b) {
    if (!b) return;
    clear_events(b);
    for (auto& g : b->graphs)
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (b->capture) (void)hipStreamDestroy(b->capture);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->side_mom) (void)hipStreamDestroy(b->side_mom);
    for (hipEvent_t e : b->ev_mom)
        if (e) (void)hipEventDestroy(e);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    for (void* p : {b->d_sweep_args, b->d_coef_args, b->d_mom_args, b->d_bnd_args,
                    static_cast<void*>(b->d_counters), static_cast<void*>(b->d_gmax)})
        if (p) (void)hipFree(p);
    for (auto& c : b->cls)
        for (void* p : {static_cast<void*>(c.d_sweep_items), static_cast<void*>(c.d_sweep_qb),
                        static_cast<void*>(c.d_mom_items)})
            if (p) (void)hipFree(p);
    b->magic = 0;
    delete b;
}

lc_status upload(void** dst, const void* src, size_t bytes) {
    hipError_t e = lc_malloc(dst, std::max<size_t>(bytes, 1));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return LC_ERR_ALLOC;
    }
    LC_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
    return LC_OK;
}

// Moment records for the current speed of light.
lc_status build_moment_args(Batch* b, double c) {
    const size_t mb = mom_args_bytes(), bb = bnd_args_bytes();
    b->h_mom.assign(2 * b->n * mb, 0);
    std::vector<char> hb(b->n * bb);
    int64_t blk_off = 0;
    for (int q = 0; q < b->n; ++q) {
        const lc_problem_t& P = b->probs[q];
        Plan* pl = b->plans[q];
        for (int parity = 0; parity < 2; ++parity) {
            const void* st = parity ? P.state_a : P.state_b;      // the state the step writes
            std::vector<char> tmp(bb);
            make_moment_args(pl, st, P.I_exit, P.I_in, c, P.E, P.F, P.f, P.bnd, blk_off,
                             b->h_mom.data() + (parity * b->n + q) * mb, tmp.data());
            if (parity == 0) std::memcpy(hb.data() + q * bb, tmp.data(), bb);
        }
        if (P.bnd) blk_off += ((int64_t)pl->rays->nb * pl->G + kBlock - 1) / kBlock;
    }
    b->bnd_blocks = blk_off;
    if (!b->d_mom_args) {
        lc_status rc = upload(&b->d_mom_args, b->h_mom.data(), b->h_mom.size());
        if (rc) return rc;
        rc = upload(&b->d_bnd_args, hb.data(), hb.size());
        if (rc) return rc;
    } else {
        // a step launched earlier (on any stream) may still read the records
        LC_HIP(hipDeviceSynchronize());
        LC_HIP(hipMemcpy(b->d_mom_args, b->h_mom.data(), b->h_mom.size(), hipMemcpyHostToDevice));
        LC_HIP(hipMemcpy(b->d_bnd_args, hb.data(), hb.size(), hipMemcpyHostToDevice));
    }
    b->c = c;
    return LC_OK;
}

}  // namespace
}  // namespace lc

using namespace lc;

extern "C" {

lc_status lc_batch_create(int32_t n_problems, const lc_problem_t* problems, lc_batch_t* out) {
    LC_ARG(out, "out is NULL");
    *out = nullptr;
    LC_ARG(n_problems >= 1 && problems, "need at least one problem");
    int prec = -1;
    for (int q = 0; q < n_problems; ++q) {
        const lc_problem_t& P = problems[q];
        Plan* pl = as_plan(P.plan);
        LC_CHECK(pl, LC_ERR_STATE, "problem %d: invalid plan handle", q);
        LC_ARG(P.kappa && P.planck && P.state_a && P.state_b && P.I_in && P.I_exit,
               "problem %d: kappa, planck, states, I_in and I_exit are required", q);
        LC_ARG(P.state_a != P.state_b, "problem %d: state_a and state_b must be distinct", q);
        LC_ARG(std::isfinite(P.c_dt) && P.c_dt > 0.0, "problem %d: c_dt must be finite and > 0", q);
        LC_ARG(P.material_stride >= 0, "problem %d: material_stride must be >= 0", q);
        if (prec < 0) prec = pl->prec;
        LC_ARG(pl->prec == prec, "all problems of a batch must use one precision");
    }
    Batch* b = new (std::nothrow) Batch();
    LC_CHECK(b, LC_ERR_ALLOC, "host allocation failed");
    b->magic = kBatchMagic;
    b->n = n_problems;
    b->prec = prec;
    b->probs.assign(problems, problems + n_problems);
    for (int q = 0; q < n_problems; ++q) b->plans.push_back(as_plan(problems[q].plan));
    lc_status rc = LC_OK;
    // argument records
    const size_t sb = sweep_args_bytes(), cb = coef_args_bytes();
    std::vector<char> hs(2 * n_problems * sb), hc(n_problems * cb);
    for (int q = 0; q < n_problems; ++q) {
        b->n_gmax += b->plans[q]->G;
        b->max_G = std::max(b->max_G, b->plans[q]->G);
    }
    {
        hipError_t e =
            lc_malloc(reinterpret_cast<void**>(&b->d_gmax), 2 * (size_t)b->n_gmax * sizeof(unsigned long long));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of the batch maxima failed: %s", hipGetErrorString(e));
            free_batch(b);
            return LC_ERR_ALLOC;
        }
    }
    int64_t g_off = 0;
    for (int q = 0; q < n_problems; ++q) {
        const lc_problem_t& P = problems[q];
        Plan* pl = b->plans[q];
        std::vector<char> two(2 * sb);
        make_batch_args(pl, P.c_dt, P.state_a, P.state_b, P.I_in, P.I_exit, two.data());
        std::memcpy(hs.data() + q * sb, two.data(), sb);
        std::memcpy(hs.data() + (n_problems + q) * sb, two.data() + sb, sb);
        int64_t nmb = 0, ncb = 0;
        make_coef_args(pl, P.c_dt, P.kappa, P.planck, P.material_stride, P.state_a, P.state_b, P.I_in, b->d_gmax,
                       b->d_gmax + b->n_gmax, b->max_blocks, b->coef_blocks, g_off, hc.data() + q * cb, &nmb, &ncb);
        b->max_blocks += nmb;
        b->coef_blocks += ncb;
        g_off += pl->G;
    }
    if (b->max_blocks >= INT32_MAX || b->coef_blocks >= INT32_MAX) {
        set_error("batched prologue grid too large");
        free_batch(b);
        return LC_ERR_UNSUPPORTED;
    }
    // work items per polar class, problems in decreasing cost
    std::vector<int> order(n_problems);
    std::iota(order.begin(), order.end(), 0);
    auto cost = [&](int q) { return (double)b->plans[q]->half_elems; };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
    auto pm_of = [&](int q) {
        int pm = 1;
        while (pm < b->plans[q]->rays->n_pol) pm *= 2;
        return pm;
    };
    if (rc == LC_OK) rc = upload(&b->d_sweep_args, hs.data(), hs.size());
    if (rc == LC_OK) rc = upload(&b->d_coef_args, hc.data(), hc.size());
    // one class per polar bound and sweep form, so that every member runs
    // the sweep code of its single-problem run (bit-identical results)
    for (int key = 0; key < 2 * 4 && rc == LC_OK; ++key) {
        const int pm = 1 << (key >> 1);
        const bool full = (key & 1) == 0;
        auto member = [&](int q) { return pm_of(q) == pm && sweep_full(b->plans[q]->rays) == full; };
        std::vector<int2> si, mi;
        std::vector<double> scost;      // summed steps of the sweep items, for the queue split
        for (int q : order) {
            if (!member(q)) continue;
            const Plan* pl = b->plans[q];
            for (int64_t B = 0; B < pl->n_bun; ++B)
                for (int d = 0; d < 2; ++d) {
                    si.push_back(make_int2(q, (int)(d * pl->n_bun + B)));
                    scost.push_back((double)pl->bun_len_h[B] * pl->rays->n_pol);
                }
            const int64_t mw = moment_tiles(pl) * moment_tile_waves(pl);
            if (mw >= INT32_MAX) {
                rc = LC_ERR_UNSUPPORTED;
                set_error("batched moments: too many work items in problem %d", q);
            }
            for (int64_t w = 0; w < mw && rc == LC_OK; ++w) mi.push_back(make_int2(q, (int)w));
        }
        if (si.empty() || rc != LC_OK) continue;
        if ((int64_t)mi.size() / 4 >= INT32_MAX / 2) {
            rc = LC_ERR_UNSUPPORTED;
            set_error("batched moments: grid too large");
            break;
        }
        int64_t sqb[9];
        double tot = 0.0;
        for (double c : scost) tot += c;
        double acc = 0.0;
        int x = 1;
        sqb[0] = 0;
        for (int64_t i = 0; i < (int64_t)scost.size() && x < 8; ++i) {
            acc += scost[i];
            while (x < 8 && acc >= tot * x / 8.0) sqb[x++] = i + 1;
        }
        while (x < 9) sqb[x++] = (int64_t)scost.size();
        PolarClass c;
        c.pm = pm;
        c.full = full;
        for (int q = 0; q < n_problems; ++q)
            if (member(q)) {
                c.unroll = b->plans[q]->sweep_unroll;
                c.ent = b->plans[q]->moments_entries;
                break;
            }
        c.n_mom_items = (int64_t)mi.size();
        rc = sweep_lds_bytes(&c.sweep_lds);
        if (rc == LC_OK) rc = sweep_batch_grid(b->prec, pm, c.unroll, c.full, c.sweep_lds, &c.sweep_grid);
        if (rc != LC_OK) break;
        b->cls.push_back(c);
        PolarClass& cc = b->cls.back();
        rc = upload(reinterpret_cast<void**>(&cc.d_sweep_items), si.data(), si.size() * sizeof(int2));
        if (rc == LC_OK) rc = upload(reinterpret_cast<void**>(&cc.d_sweep_qb), sqb, sizeof(sqb));
        if (rc == LC_OK) rc = upload(reinterpret_cast<void**>(&cc.d_mom_items), mi.data(), mi.size() * sizeof(int2));
    }
    if (rc == LC_OK) {
        const std::vector<int> zero(8 * b->cls.size(), 0);
        rc = upload(reinterpret_cast<void**>(&b->d_counters), zero.data(), zero.size() * sizeof(int));
    }
    if (rc == LC_OK) rc = build_moment_args(b, 1.0);
    if (rc == LC_OK) {
        hipError_t e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side_mom, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_mom[0], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_mom[1], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
        if (e != hipSuccess) {
            set_error("hipStreamCreate failed: %s", hipGetErrorString(e));
            rc = LC_ERR_HIP;
        }
    }
    if (rc != LC_OK) {
        free_batch(b);
        return rc;
    }
    *out = reinterpret_cast<lc_batch_t>(b);
    return LC_OK;
}

lc_status lc_batch_step(lc_batch_t batch, int32_t n_steps, double c, void* stream) {
    Batch* b = as_batch(batch);
    LC_CHECK(b, LC_ERR_STATE, "invalid batch handle");
    LC_ARG(n_steps >= 1, "n_steps must be >= 1");
    LC_ARG(std::isfinite(c) && c > 0.0, "c must be finite and > 0");
    for (int q = 0; q < b->n; ++q) LC_CHECK(as_plan(b->probs[q].plan), LC_ERR_STATE, "problem %d: plan freed", q);
    if (c != b->c) {
        lc_status rc = build_moment_args(b, c);
        if (rc) return rc;
        for (auto& g : b->graphs)
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
        b->graphs.clear();
    }
    if (b->profile) return enqueue_steps(b, n_steps, static_cast<hipStream_t>(stream));
    hipGraphExec_t exec = nullptr;
    for (auto& g : b->graphs)
        if (g.key.size() == 1 && g.key[0] == (uintptr_t)n_steps) exec = g.exec;
    if (!exec) {
        LC_HIP(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        lc_status rc = enqueue_steps(b, n_steps, b->capture);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(b->capture, &graph);
        if (rc != LC_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        LC_CHECK(e == hipSuccess && graph, LC_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        LC_CHECK(e == hipSuccess, LC_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
        b->graphs.push_back({{(uintptr_t)n_steps}, exec});
    }
    LC_HIP(hipGraphLaunch(exec, static_cast<hipStream_t>(stream)));
    return LC_OK;
}

lc_status lc_batch_profile(lc_batch_t batch, int32_t enable) {
    Batch* b = as_batch(batch);
    LC_CHECK(b, LC_ERR_STATE, "invalid batch handle");
    b->profile = enable != 0;
    return LC_OK;
}

lc_status lc_batch_profile_read(lc_batch_t batch, double* out) {
    Batch* b = as_batch(batch);
    LC_CHECK(b, LC_ERR_STATE, "invalid batch handle");
    LC_ARG(out, "out is NULL");
    for (int k = 0; k < 3; ++k) {
        double ms_tot = 0.0;
        for (auto& e : b->ev[k]) {
            LC_HIP(hipEventSynchronize(e.second));
            float ms = 0.f;
            LC_HIP(hipEventElapsedTime(&ms, e.first, e.second));
            ms_tot += ms;
        }
        out[2 * k] = ms_tot;
        out[2 * k + 1] = (double)b->ev[k].size();
    }
    clear_events(b);
    return LC_OK;
}

lc_status lc_batch_free(lc_batch_t batch) {
    if (!batch) return LC_OK;
    Batch* b = as_batch(batch);
    LC_CHECK(b, LC_ERR_STATE, "invalid batch handle");
    free_batch(b);
    return LC_OK;
}

}  // extern "C"
