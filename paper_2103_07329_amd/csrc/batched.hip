// batched.hip -- many independent systems of uneven size n_s and column
// count m_s solved together: the AMG-preconditioned CG iterations of every
// system are captured into one HIP graph (one branch per system, on its own
// stream), and that graph -- several iterations deep -- is launched again
// and again until every system has converged.  Systems that have converged
// keep their branch, whose kernels then exit at once (every kernel reads
// its system's count of active columns first).  Between launches the host
// reads each system's column state; the true-residual check and the rare
// restart run eagerly on the system's stream.
//
// This extends the paper's multi-RHS solve (many right-hand sides of one
// matrix, Sections 2.2 and 3.2) to many matrices at once: small systems,
// whose coarse levels are latency-bound, overlap with the large ones.
#include <chrono>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "solver.hpp"

struct xamg_batch {};   // opaque ABI tag; the real object is xamg::Batch

namespace xamg {

// One captured graph: `iters` CG iterations of every system.
struct Captured {
    int iters = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uintptr_t> key;   // B, X, m, buffers and launch shapes baked in
    void reset()
    {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        key.clear();
    }
};

struct Batch : xamg_batch {
    std::vector<Handle*> hs;
    int iters_per_launch = 4;     // iterations of the follow-up graph
    bool predict = true;          // first launch: the iterations the last solve needed
    int last_iters = 0;           // largest iteration count of the last solve
    hipStream_t s0 = nullptr;
    std::vector<hipStream_t> ss;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> joins;
    Captured main, step;

    ~Batch()
    {
        main.reset();
        step.reset();
        if (fork) hipEventDestroy(fork);
        for (hipEvent_t e : joins) hipEventDestroy(e);
        for (hipStream_t s : ss) hipStreamDestroy(s);
        if (s0) hipStreamDestroy(s0);
    }
};

namespace {

int padded(int m)
{
    int mp = 1;
    while (mp < m) mp <<= 1;
    return mp;
}

template <class F>
int with_m(int mp, F&& f)
{
    switch (mp) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 8: return f(std::integral_constant<int, 8>{});
    case 16: return f(std::integral_constant<int, 16>{});
    case 32: return f(std::integral_constant<int, 32>{});
    default: return XAMG_EINVAL;
    }
}

void chk(hipError_t e, const char* what)
{
    if (e != hipSuccess) {
        set_error("HIP error %d (%s) in %s", int(e), hipGetErrorString(e), what);
        throw DevFail{XAMG_EHIP};
    }
}

}  // namespace

int solve_batched(Batch& b, const double* const* B, double* const* X, const int32_t* m, double tol,
                  xamg_stats_t* const* stats)
{
    const int ns = int(b.hs.size());
    std::vector<int> mp(ns);
    std::vector<const double*> Bs(ns);
    std::vector<double*> Xs(ns);
    std::vector<hipStream_t> saved(ns);
    std::vector<int> saved_timer(ns);
    for (int s = 0; s < ns; ++s) {
        Handle& h = *b.hs[s];
        saved[s] = h.stream;
        saved_timer[s] = h.timer_kind;
        h.stream = b.ss[s];
        h.timer_kind = 0;
    }
    struct Restore {
        Batch& b;
        std::vector<hipStream_t>& saved;
        std::vector<int>& timer;
        ~Restore()
        {
            for (size_t s = 0; s < b.hs.size(); ++s) {
                b.hs[s]->stream = saved[s];
                b.hs[s]->timer_kind = timer[s];
            }
        }
    } restore{b, saved, saved_timer};

    // per system: buffers and tuning, then (timed) padding and the start of CG
    for (int s = 0; s < ns; ++s) {
        Handle& h = *b.hs[s];
        mp[s] = padded(m[s]);
        ensure_work(h, mp[s], false);
        if (h.autotune)
            with_m(mp[s], [&](auto mc) {
                autotune<decltype(mc)::value>(h);
                return 0;
            });
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (int s = 0; s < ns; ++s) {
        Handle& h = *b.hs[s];
        Bs[s] = B[s];
        Xs[s] = X[s];
        const int n = h.lev[0].n;
        if (mp[s] != m[s]) {
            if (!h.w.bpad) {
                h.w.bpad = h.alloc<double>(size_t(n) * h.w.mcap);
                h.w.xpad = h.alloc<double>(size_t(n) * h.w.mcap);
            }
            hipLaunchKernelGGL((dev::copy_cols_kernel<double, double>), dim3(2048), dim3(256), 0,
                               h.stream, B[s], m[s], h.w.bpad, mp[s], n, m[s]);
            hipLaunchKernelGGL((dev::copy_cols_kernel<double, double>), dim3(2048), dim3(256), 0,
                               h.stream, X[s], m[s], h.w.xpad, mp[s], n, m[s]);
            Bs[s] = h.w.bpad;
            Xs[s] = h.w.xpad;
        }
        with_m(mp[s], [&](auto mc) {
            pcg_start<decltype(mc)::value>(h, Bs[s], Xs[s], tol);
            return 0;
        });
    }
    bool bad = false;
    for (int s = 0; s < ns; ++s) {
        poll_state(*b.hs[s]);
        bad |= b.hs[s]->st_host->nrestart < 0;
    }
    if (bad) {
        set_error("B contains NaN or Inf");
        return XAMG_EINVAL;
    }

    // capture (or reuse) a graph of K iterations of every system
    std::vector<uintptr_t> key;
    for (int s = 0; s < ns; ++s) {
        key.push_back(reinterpret_cast<uintptr_t>(Bs[s]));
        key.push_back(reinterpret_cast<uintptr_t>(Xs[s]));
        key.push_back(uintptr_t(mp[s]));
        // work buffers and launch shapes baked into the graph
        key.push_back(reinterpret_cast<uintptr_t>(b.hs[s]->w.r));
        key.push_back(reinterpret_cast<uintptr_t>(b.hs[s]->part));
        key.push_back(uintptr_t(b.hs[s]->tune_epoch));
    }
    auto capture = [&](Captured& g, int iters) {
        if (g.exec && g.key == key && g.iters == iters) return;
        g.reset();
        chk(hipStreamBeginCapture(b.s0, hipStreamCaptureModeThreadLocal), "begin capture");
        chk(hipEventRecord(b.fork, b.s0), "fork");
        for (int s = 0; s < ns; ++s) {
            Handle& h = *b.hs[s];
            chk(hipStreamWaitEvent(b.ss[s], b.fork, 0), "fork wait");
            for (int k = 0; k < iters; ++k)
                with_m(mp[s], [&](auto mc) {
                    pcg_iteration<decltype(mc)::value>(h, Xs[s]);
                    return 0;
                });
            chk(hipEventRecord(b.joins[s], b.ss[s]), "join");
            chk(hipStreamWaitEvent(b.s0, b.joins[s], 0), "join wait");
        }
        chk(hipStreamEndCapture(b.s0, &g.graph), "end capture");
        chk(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0), "instantiate");
        g.key = key;
        g.iters = iters;
    };

    std::vector<char> finished(ns, 0);
    std::vector<int> launched(ns, 0);
    int remaining = ns;
    // true-residual checks of every system whose columns have all stopped:
    // enqueued on the systems' streams, one wait, then restarts (rare)
    auto check_done = [&](bool after_launch) {
        std::vector<int> chk_s;
        for (int s = 0; s < ns; ++s) {
            if (finished[s]) continue;
            Handle& h = *b.hs[s];
            const bool capped = after_launch && launched[s] >= h.opt.max_iters;
            if (h.st_host->nactive == 0 || capped) {
                with_m(mp[s], [&](auto mc) {
                    pcg_true_enqueue<decltype(mc)::value>(h, Bs[s], Xs[s], capped ? 0 : 1);
                    return 0;
                });
                chk_s.push_back(s);
            }
        }
        for (int s : chk_s) chk(hipStreamSynchronize(b.hs[s]->stream), "check sync");
        for (int s : chk_s) {
            Handle& h = *b.hs[s];
            const bool capped = after_launch && launched[s] >= h.opt.max_iters;
            const int nr = with_m(mp[s], [&](auto mc) {
                return pcg_true_finish<decltype(mc)::value>(h);
            });
            if (nr == 0 || capped) {
                finished[s] = 1;
                --remaining;
            } else {
                chk(hipStreamSynchronize(h.stream), "restart sync");
            }
        }
    };
    // systems with nothing to do (all columns zero or already converged)
    check_done(false);
    // the first launch runs as many iterations as the last solve needed (one
    // graph launch and one poll in the common case); further launches run
    // iters_per_launch iterations each
    bool first = true;
    while (remaining > 0) {
        Captured* g = &b.step;
        if (first && b.predict && b.last_iters > b.iters_per_launch) {
            capture(b.main, b.last_iters);
            g = &b.main;
        } else {
            capture(b.step, b.iters_per_launch);
        }
        first = false;
        chk(hipGraphLaunch(g->exec, b.s0), "graph launch");
        // after the graph: the 16 polled bytes of every running system, all
        // copied on the batch stream, then one wait
        for (int s = 0; s < ns; ++s)
            if (!finished[s])
                chk(hipMemcpyAsync(b.hs[s]->st_host, b.hs[s]->st, 16, hipMemcpyDeviceToHost, b.s0),
                    "poll copy");
        chk(hipStreamSynchronize(b.s0), "graph sync");
        for (int s = 0; s < ns; ++s)
            if (!finished[s]) launched[s] += g->iters;
        check_done(true);
    }

    int rc = XAMG_OK, maxit = 0;
    for (int s = 0; s < ns; ++s) {
        Handle& h = *b.hs[s];
        const int n = h.lev[0].n;
        if (mp[s] != m[s])
            hipLaunchKernelGGL((dev::copy_cols_kernel<double, double>), dim3(2048), dim3(256), 0,
                               h.stream, h.w.xpad, mp[s], X[s], m[s], n, m[s]);
    }
    for (int s = 0; s < ns; ++s) b.hs[s]->check(hipStreamSynchronize(b.hs[s]->stream), "batched sync");
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (int s = 0; s < ns; ++s) {
        Handle& h = *b.hs[s];
        const dev::ColState& st = *h.st_host;
        for (int j = 0; j < m[s]; ++j) {
            const bool conv = st.conv[j] && !(st.true_relres[j] > st.tol);
            if (stats && stats[s]) {
                stats[s][j].iters = st.iters[j];
                stats[s][j].converged = conv ? 1 : 0;
                stats[s][j].relres = st.relres[j];
                stats[s][j].true_relres = st.true_relres[j];
                stats[s][j].restarts = st.nrst[j];
                stats[s][j].reserved = 0;
                stats[s][j].ms = ms;
            }
            if (st.failed[j]) rc = XAMG_EBREAKDOWN;
            else if (!conv && rc == XAMG_OK) rc = XAMG_NOT_CONVERGED;
            maxit = std::max(maxit, int(st.iters[j]));
        }
    }
    b.last_iters = maxit;
    return rc;
}

}  // namespace xamg

using xamg::Batch;
using xamg::Handle;

extern "C" {

int xamg_batch_create(xamg_handle_t* const* handles, int32_t nsys, int32_t iters_per_launch,
                      xamg_batch_t** out)
{
    xamg::clear_error();
    if (!handles || !out || nsys < 1) return xamg::fail(XAMG_EINVAL, "bad arguments");
    *out = nullptr;
    if (iters_per_launch < 0 || iters_per_launch > 64)
        return xamg::fail(XAMG_EINVAL, "iters_per_launch must be 0..64");
    for (int s = 0; s < nsys; ++s) {
        if (!handles[s]) return xamg::fail(XAMG_EINVAL, "null handle");
        for (int t = 0; t < s; ++t)
            if (handles[t] == handles[s]) return xamg::fail(XAMG_EINVAL, "handle repeated");
        if (static_cast<Handle*>(handles[s])->opt.method != XAMG_CG)
            return xamg::fail(XAMG_EINVAL, "batched solves use CG handles");
    }
    Batch* b = new (std::nothrow) Batch;
    if (!b) return xamg::fail(XAMG_ENOMEM, "host allocation");
    try {
        b->iters_per_launch = iters_per_launch ? iters_per_launch : 4;
        for (int s = 0; s < nsys; ++s) b->hs.push_back(static_cast<Handle*>(handles[s]));
        xamg::chk(hipStreamCreateWithFlags(&b->s0, hipStreamNonBlocking), "stream");
        b->ss.resize(nsys, nullptr);
        b->joins.resize(nsys, nullptr);
        for (int s = 0; s < nsys; ++s) {
            xamg::chk(hipStreamCreateWithFlags(&b->ss[s], hipStreamNonBlocking), "stream");
            xamg::chk(hipEventCreateWithFlags(&b->joins[s], hipEventDisableTiming), "event");
        }
        xamg::chk(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming), "event");
    } catch (const xamg::DevFail& f) {
        delete b;
        return f.code;
    }
    *out = static_cast<xamg_batch_t*>(b);
    return XAMG_OK;
}

int xamg_solve_batched(xamg_batch_t* bb, const double* const* B, double* const* X,
                       const int32_t* m, double tol, xamg_stats_t* const* stats)
{
    xamg::clear_error();
    Batch* b = static_cast<Batch*>(bb);
    if (!b || !B || !X || !m) return xamg::fail(XAMG_EINVAL, "null argument");
    if (!(tol > 0.0) || !std::isfinite(tol)) return xamg::fail(XAMG_EINVAL, "tol must be positive");
    for (size_t s = 0; s < b->hs.size(); ++s) {
        if (!B[s] || !X[s]) return xamg::fail(XAMG_EINVAL, "null B or X");
        if (m[s] < 1 || m[s] > XAMG_MAX_M) return xamg::fail(XAMG_EINVAL, "m must be in 1..32");
        if ((reinterpret_cast<uintptr_t>(B[s]) & 15u) || (reinterpret_cast<uintptr_t>(X[s]) & 15u))
            return xamg::fail(XAMG_EINVAL, "B and X must be 16-byte aligned");
    }
    try {
        return xamg::solve_batched(*b, B, X, m, tol, stats);
    } catch (const xamg::DevFail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        return xamg::fail(XAMG_ENOMEM, "host allocation");
    }
}

int xamg_batch_destroy(xamg_batch_t* bb)
{
    Batch* b = static_cast<Batch*>(bb);
    if (!b) return XAMG_OK;
    hipStreamSynchronize(b->s0);
    for (hipStream_t s : b->ss) hipStreamSynchronize(s);
    delete b;
    return XAMG_OK;
}

}  // extern "C"
