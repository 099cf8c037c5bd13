// pa_fused.cpp -- many population-annealing runs per kernel launch (the
// pa_fused_* calls of include/pa.h).
//
// Runs of one record mode (unsigned graphs, or signed graphs with sign-bit
// entries) and one graph-size class form a group that shares one launch
// shape of the node-per-lane sweep kernel. Step k of the whole group is one sweep launch over a work
// list of {run, tile} entries and one epilogue launch with a workgroup per
// run, so small runs that would leave most compute units idle alone fill the
// device together, and the per-step launch count no longer grows with the
// number of runs. Groups run on their own streams, forked from and joined
// back to the caller's stream; the K-step loop is captured once into a HIP
// graph and replayed. A measuring autotuner picks each group's replicas per
// workgroup and threads. Every run gives exactly the results of the same run
// alone (the launch shape never changes results), and afterwards its solver
// answers the result calls as after pa_run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "pa.h"
#include "pa_device.h"
#include "pa_host.h"

using namespace pa_host;

struct pa_fused {
    struct Run {
        pa_solver *s = nullptr;
        pa_schedule sch{};                // copy; beta and order point into the vectors below
        std::vector<double> beta;
        std::vector<int32_t> order;
        int32_t R = 0;
        uint64_t seed = 0;
        uint32_t inst = 0;
        size_t off = 0, bytes = 0;        // the run's region of the workspace
        double cost = 0;                  // work per tile, for the dispatch order
    };
    struct Group {
        int bsg = 0;                      // 0 unsigned records, 2 sign bits
        std::vector<int> members;         // run indices, most work per tile first
        std::vector<Shape> candidates;
        Shape shape;
        double probe_ns_per_attempt = 0;  // measured for the chosen shape (0: not tuned)
        int max_R = 0, steps = 0, blocks = 0, lds = 0;
        size_t args_off = 0, work_off = 0, work_cap = 0;
        hipStream_t stream = nullptr;
        hipEvent_t done = nullptr;
    };
    std::vector<Run> runs;
    std::vector<Group> groups;
    size_t total = 0;
    int max_lds = 160 * 1024;
    unsigned char *stage = nullptr;       // pinned: run arguments and work lists
    size_t stage_cap = 0, stage_used = 0;
    hipEvent_t fork = nullptr;
    // The step loop as a HIP graph, valid for one workspace address and shapes.
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    unsigned char *graph_ws = nullptr;
    uint64_t graph_sig = 0;
    int use_graph = 1;
};

// The work list of a multi-run sweep launch: the tiles of the runs (run q
// has nblk[q] tiles of W replicas), taken in 64-replica words (64/W tiles
// that share spin words), the words dealt round-robin over the 8 XCDs in run
// order, so that tiles sharing a word meet in one L2 and every XCD gets a
// like mix. Empty slots are {-1, 0}.
std::vector<int2> pa_host::multi_work_list(const std::vector<int> &nblk, int W)
{
    const int per = 64 / W;
    std::vector<int2> words;                      // {run, first tile}
    for (int q = 0; q < (int)nblk.size(); ++q)
        for (int t = 0; t < nblk[q]; t += per) words.push_back(int2{q, t});
    const int nw = (int)words.size();
    const int rows = (nw + 7) / 8;
    std::vector<int2> w((size_t)rows * 8 * per, int2{-1, 0});
    for (int b = 0; b < (int)w.size(); ++b) {
        const int x = b & 7, slot = b >> 3;
        const int wi = x + 8 * (slot / per), t = slot % per;
        if (wi >= nw) continue;
        const int q = words[wi].x;
        const int tile = words[wi].y + t;
        if (tile < nblk[q]) w[b] = int2{q, tile};
    }
    return w;
}

// After its last step is enqueued on `hs`: the solver holds the finished
// run, as after pa_run (the population of step k is written to X1 for even
// k, so the last step's output is X(K & 1)).
void pa_host::finish_run(pa_solver *s, hipStream_t hs)
{
    pa_solver::RunCtx &c = s->rc;
    const int K = s->plan.K;
    const bool odd = (K & 1) != 0;
    c.Xc = odd ? s->plan.L.X1 : s->plan.L.X0;
    c.Xn = odd ? s->plan.L.X0 : s->plan.L.X1;
    c.Ec = odd ? s->plan.L.E1 : s->plan.L.E0;
    c.En = odd ? s->plan.L.E0 : s->plan.L.E1;
    c.parents_pending = false;
    c.next_step = K;
    c.valid = true;
    s->final_x = c.Xc;
    s->final_E = c.Ec;
    s->stream = hs;
    s->has_run = true;
}

int pa_host::device_max_lds()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
        return v;
    (void)hipGetLastError();
    return 160 * 1024;
}

namespace {

// Tile widths the autotuner tries, each with 64, 128, 256 and 512 threads.
constexpr int kTileCand[] = {4, 8, 16};

bool direct_fits(const pa_solver *s, int W)
{
    return pa::kBytesRecBase + (size_t)(s->n + 1) * W <= 0xFFFF;
}

// Plan a run with a shape without tables (sizes only).
pa_status plan_size(pa_fused::Run &r, const Shape &sh, size_t *bytes)
{
    Plan p;
    const pa_status st = build_plan(r.s, &r.sch, r.R, p, false, &sh);
    if (st == PA_OK) *bytes = p.L.total;
    return st;
}

uint64_t shapes_sig(const pa_fused *f)
{
    uint64_t h = 1469598103934665603ull;
    for (const auto &g : f->groups) {
        const uint64_t v = (uint64_t)g.shape.W | (uint64_t)g.shape.threads << 8 | (uint64_t)g.shape.direct << 24;
        h = (h ^ v) * 1099511628211ull;
    }
    return h;
}

void drop_graph(pa_fused *f)
{
    if (f->exec) (void)hipGraphExecDestroy(f->exec);
    if (f->graph) (void)hipGraphDestroy(f->graph);
    f->exec = nullptr;
    f->graph = nullptr;
    f->graph_ws = nullptr;
}

std::vector<int2> work_list(const pa_fused *f, const pa_fused::Group &g)
{
    std::vector<int> nblk;
    for (int i : g.members) nblk.push_back((f->runs[i].R + g.shape.W - 1) / g.shape.W);
    return multi_work_list(nblk, g.shape.W);
}

// Work-list length and sweep LDS of a group's current shape.
void shape_facts(const pa_fused *f, pa_fused::Group &g)
{
    g.blocks = (int)work_list(f, g).size();
    g.lds = 0;
    for (int i : g.members)
        g.lds = std::max(g.lds, pa::sweep_bytes_lds(g.shape.W, 0, f->runs[i].s->n, f->runs[i].s->dmax));
}

// Prepare every run of the groups in `which` (all if empty) for the group
// shapes: tables and inputs uploaded, initial population and its best, and
// the group's run arguments and work list uploaded. Enqueued on `hs`.
pa_status prepare(pa_fused *f, unsigned char *ws, hipStream_t hs, const std::vector<int> &which)
{
    // The last copy from the pinned buffer (an earlier prepare) ran on this
    // stream: wait for it before the buffer is rewritten.
    HIP_TRY(hipStreamSynchronize(hs));
    std::vector<pa::MultiRun> mr;
    f->stage_used = 0;
    struct Up {
        size_t dst, src, bytes;
    };
    std::vector<Up> ups;
    std::vector<unsigned char> host;
    for (int gi = 0; gi < (int)f->groups.size(); ++gi) {
        if (!which.empty() && std::find(which.begin(), which.end(), gi) == which.end()) continue;
        pa_fused::Group &g = f->groups[gi];
        mr.assign(g.members.size(), pa::MultiRun{});
        g.max_R = 0;
        g.steps = 0;
        g.lds = 0;
        for (int q = 0; q < (int)g.members.size(); ++q) {
            pa_fused::Run &r = f->runs[g.members[q]];
            pa_status st = start_run(r.s, &r.sch, r.R, r.seed, r.inst, ws + r.off, r.bytes, hs, true, true,
                                     &g.shape);
            if (st != PA_OK) return st;
            const Plan &P = r.s->plan;
            pa::MultiRun &m = mr[q];
            m.sweep = r.s->rc.sa;
            m.epi = r.s->rc.ea;
            m.X0 = reinterpret_cast<uint64_t *>(ws + r.off + P.L.X0);
            m.X1 = reinterpret_cast<uint64_t *>(ws + r.off + P.L.X1);
            m.E0 = reinterpret_cast<int *>(ws + r.off + P.L.E0);
            m.E1 = reinterpret_cast<int *>(ws + r.off + P.L.E1);
            m.steps = P.K;
            m.nblk = P.nblk;
            g.max_R = std::max(g.max_R, r.R);
            g.steps = std::max(g.steps, P.K);
            g.lds = std::max(g.lds, pa::sweep_bytes_lds(g.shape.W, 0, r.s->n, r.s->dmax));
        }
        const std::vector<int2> w = work_list(f, g);
        if (w.size() > g.work_cap) return fail(PA_EINVAL, "internal: work list exceeds its reservation");
        g.blocks = (int)w.size();
        size_t at = host.size();
        host.resize(at + sizeof(pa::MultiRun) * mr.size());
        std::memcpy(host.data() + at, mr.data(), sizeof(pa::MultiRun) * mr.size());
        ups.push_back({g.args_off, at, sizeof(pa::MultiRun) * mr.size()});
        at = host.size();
        host.resize(at + sizeof(int2) * w.size());
        std::memcpy(host.data() + at, w.data(), sizeof(int2) * w.size());
        ups.push_back({g.work_off, at, sizeof(int2) * w.size()});
    }
    if (host.empty()) return PA_OK;
    if (f->stage_cap < host.size()) {
        if (f->stage) HIP_TRY(hipHostFree(f->stage));
        f->stage = nullptr;
        f->stage_cap = 0;
        HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&f->stage), host.size(), hipHostMallocDefault));
        f->stage_cap = host.size();
    }
    std::memcpy(f->stage, host.data(), host.size());
    for (const Up &u : ups)
        HIP_TRY(hipMemcpyAsync(ws + u.dst, f->stage + u.src, u.bytes, hipMemcpyHostToDevice, hs));
    return PA_OK;
}

pa_status enqueue_group_steps(pa_fused *f, pa_fused::Group &g, unsigned char *ws, int k0, int k1,
                              hipStream_t hs)
{
    const pa::MultiRun *args = reinterpret_cast<const pa::MultiRun *>(ws + g.args_off);
    const int2 *work = reinterpret_cast<const int2 *>(ws + g.work_off);
    for (int k = k0; k < k1 && k < g.steps; ++k) {
        LAUNCH_TRY(pa::launch_sweep_multi(g.shape.W, g.bsg, g.shape.direct != 0, g.shape.threads, g.blocks,
                                          g.lds, args, work, k, hs));
        LAUNCH_TRY(pa::launch_epilogue_multi((int)g.members.size(), g.max_R, args, k, hs));
    }
    return PA_OK;
}

// The step loop of every group, each on its own stream, forked from and
// joined back to `hs`.
pa_status enqueue_all_steps(pa_fused *f, unsigned char *ws, hipStream_t hs)
{
    HIP_TRY(hipEventRecord(f->fork, hs));
    for (auto &g : f->groups) {
        HIP_TRY(hipStreamWaitEvent(g.stream, f->fork, 0));
        pa_status st = enqueue_group_steps(f, g, ws, 0, g.steps, g.stream);
        if (st != PA_OK) return st;
        HIP_TRY(hipEventRecord(g.done, g.stream));
        HIP_TRY(hipStreamWaitEvent(hs, g.done, 0));
    }
    return PA_OK;
}

// After the step loop: each solver holds its finished run, as after pa_run.
void finish_runs(pa_fused *f, hipStream_t hs)
{
    for (auto &r : f->runs) finish_run(r.s, hs);
}

}  // namespace

extern "C" pa_status pa_fused_create(pa_fused **out, const pa_fused_entry *runs, int32_t count)
{
    g_error[0] = 0;
    if (!out || !runs || count < 1) return fail(PA_EINVAL, "pa_fused_create: null array or count < 1");
    *out = nullptr;
    pa_fused *f = new (std::nothrow) pa_fused;
    if (!f) return fail(PA_ERANGE, "pa_fused_create: out of host memory");
    std::vector<const pa_solver *> seen;
    f->max_lds = device_max_lds();
    auto bail = [&](pa_status st) {
        delete f;
        return st;
    };
    for (int i = 0; i < count; ++i) {
        const pa_fused_entry &in = runs[i];
        pa_status st = check_schedule(in.solver, in.schedule, in.R);
        if (st != PA_OK) {
            char msg[400];
            std::snprintf(msg, sizeof msg, "%s", pa_last_error());
            return bail(fail(st, "pa_fused_create: run %d: %s", i, msg));
        }
        if (in.instance > 65535) return bail(fail(PA_ERANGE, "pa_fused_create: run %d: instance > 65535", i));
        if (in.schedule->nl_period != 0 || in.schedule->beta_adapt != 0)
            return bail(fail(PA_EINVAL, "pa_fused_create: run %d: runs sharing launches take no non-local "
                                        "moves and no adaptive steps (use pa_run_batch)", i));
        seen.push_back(in.solver);
        pa_fused::Run r;
        r.s = in.solver;
        r.sch = *in.schedule;
        r.beta.assign(in.schedule->beta, in.schedule->beta + in.schedule->n_steps);
        r.sch.beta = r.beta.data();
        if (in.schedule->order) {
            r.order.assign(in.schedule->order, in.schedule->order + in.solver->n);
            r.sch.order = r.order.data();
        }
        r.R = in.R;
        r.seed = in.seed;
        r.inst = in.instance;
        r.cost = (double)in.solver->n * (1.0 + (double)in.solver->nnz / in.solver->n) * in.schedule->sweeps_per_step;
        f->runs.push_back(std::move(r));
    }
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
        return bail(fail(PA_EINVAL, "pa_fused_create: a solver appears in two runs"));

    // Threads per workgroup of each run for the untuned shape: the smallest
    // of 64, 128, 256, 512 that needs no more rounds (one barrier each) per
    // sweep than 512; a round covers one dependency level, and graphs of a
    // few thousand nodes have levels of 50 to 300 nodes.
    std::vector<int> threads(count, 512);
    for (int i = 0; i < count; ++i) {
        pa_fused::Run &r = f->runs[i];
        Shape probe;
        probe.W = 4;
        probe.threads = 512;
        probe.bsg = r.s->has_neg ? 2 : 0;
        probe.direct = 0;
        Plan p;
        pa_status st = build_plan(r.s, &r.sch, r.R, p, false, &probe);
        if (st != PA_OK) {
            char msg[400];
            std::snprintf(msg, sizeof msg, "%s", pa_last_error());
            return bail(fail(st, "pa_fused_create: run %d: %s", i, msg));
        }
        auto rounds_at = [&](int T) {
            long long n = 0;
            for (int l = 0; l < p.n_levels; ++l) n += (p.level_off[l + 1] - p.level_off[l] + T - 1) / T;
            return n;
        };
        const long long r512 = rounds_at(512);
        for (int T : {256, 128, 64})
            if (rounds_at(T) <= r512) threads[i] = T;
    }
    // Groups by record mode and graph size (the spin records of a tile take
    // n * W bytes of LDS, which with the threads sets how many workgroups
    // share a compute unit); members ordered by work per tile, largest first.
    auto size_class = [](int n) { return n < 1500 ? 0 : n < 3000 ? 1 : n < 5000 ? 2 : 3; };
    for (int bsg : {0, 2})
        for (int sc = 3; sc >= 0; --sc) {
        pa_fused::Group g;
        g.bsg = bsg;
        int T0 = 64;
        for (int i = 0; i < count; ++i)
            if ((f->runs[i].s->has_neg ? 2 : 0) == bsg && size_class(f->runs[i].s->n) == sc) {
                g.members.push_back(i);
                T0 = std::max(T0, threads[i]);
            }
        if (g.members.empty()) continue;
        std::stable_sort(g.members.begin(), g.members.end(),
                         [&](int a, int b) { return f->runs[a].cost > f->runs[b].cost; });
        for (int W : kTileCand)
            for (int T : {64, 128, 256, 512}) {
                Shape sh;
                sh.W = W;
                sh.threads = T;
                sh.bsg = bsg;
                sh.direct = 1;
                bool ok = true;
                for (int i : g.members) {
                    const pa_solver *s = f->runs[i].s;
                    if (pa::sweep_bytes_lds(W, 0, s->n, s->dmax) > f->max_lds) ok = false;
                    if (!direct_fits(s, W)) sh.direct = 0;
                }
                if (ok) g.candidates.push_back(sh);
            }
        if (g.candidates.empty())
            return bail(fail(PA_ERANGE, "pa_fused_create: a graph does not fit LDS at any shared shape"));
        // Untuned shape: 8 replicas per workgroup and the group's thread count
        // when they fit, else the first fit.
        g.shape = g.candidates[0];
        for (const Shape &c : g.candidates)
            if (c.W == 8 && c.threads == T0) g.shape = c;
        f->groups.push_back(std::move(g));
    }

    // Workspace: each run's region sized for its largest candidate plan, then
    // per group the run arguments and the longest work list of any candidate.
    size_t o = 0;
    for (auto &g : f->groups) {
        for (int i : g.members) {
            pa_fused::Run &r = f->runs[i];
            size_t need = 0;
            for (const Shape &c : g.candidates) {
                size_t b = 0;
                pa_status st = plan_size(r, c, &b);
                if (st != PA_OK) {
                    char msg[400];
                    std::snprintf(msg, sizeof msg, "%s", pa_last_error());
                    return bail(fail(st, "pa_fused_create: run %d: %s", i, msg));
                }
                need = std::max(need, b);
            }
            r.off = o;
            r.bytes = need;
            o = align_up(o + need);
        }
    }
    for (auto &g : f->groups) {
        g.args_off = o;
        o = align_up(o + sizeof(pa::MultiRun) * g.members.size());
        size_t cap = 0;
        for (const Shape &c : g.candidates) {
            pa_fused::Group t = g;
            t.shape = c;
            cap = std::max(cap, work_list(f, t).size());
        }
        g.work_cap = cap;
        g.work_off = o;
        o = align_up(o + sizeof(int2) * cap);
        shape_facts(f, g);
    }
    f->total = o;
    *out = f;
    return PA_OK;
}

extern "C" pa_status pa_fused_destroy(pa_fused *f)
{
    if (!f) return PA_OK;
    for (auto &g : f->groups) {
        if (g.stream) {
            (void)hipStreamSynchronize(g.stream);
            (void)hipStreamDestroy(g.stream);
        }
        if (g.done) (void)hipEventDestroy(g.done);
    }
    drop_graph(f);
    if (f->cap) (void)hipStreamDestroy(f->cap);
    if (f->fork) (void)hipEventDestroy(f->fork);
    if (f->stage) (void)hipHostFree(f->stage);
    delete f;
    return PA_OK;
}

extern "C" pa_status pa_fused_workspace_bytes(const pa_fused *f, size_t *bytes)
{
    if (!f || !bytes) return fail(PA_EINVAL, "pa_fused_workspace_bytes: null argument");
    *bytes = f->total;
    return PA_OK;
}

static pa_status check_ws(pa_fused *f, void *workspace, size_t bytes)
{
    if (!f) return fail(PA_EINVAL, "null batch");
    if (!workspace) return fail(PA_EWORKSPACE, "workspace is null");
    if (((uintptr_t)workspace) % kAlign) return fail(PA_EWORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < f->total) return fail(PA_EWORKSPACE, "workspace of %zu bytes < %zu needed", bytes, f->total);
    return PA_OK;
}

// Streams and events of the batch (created on first use, default priority).
static pa_status ensure_streams(pa_fused *f)
{
    if (!f->fork) HIP_TRY(hipEventCreateWithFlags(&f->fork, hipEventDisableTiming));
    if (!f->cap) HIP_TRY(hipStreamCreateWithFlags(&f->cap, hipStreamNonBlocking));
    for (auto &g : f->groups) {
        if (!g.stream) HIP_TRY(hipStreamCreateWithFlags(&g.stream, hipStreamNonBlocking));
        if (!g.done) HIP_TRY(hipEventCreateWithFlags(&g.done, hipEventDisableTiming));
    }
    return PA_OK;
}

extern "C" pa_status pa_fused_tune(pa_fused *f, void *workspace, size_t workspace_bytes, void *stream,
                                   int32_t probe_steps)
{
    g_error[0] = 0;
    pa_status st = check_ws(f, workspace, workspace_bytes);
    if (st != PA_OK) return st;
    if (probe_steps < 1 || probe_steps > 64) return fail(PA_EINVAL, "probe_steps must be in [1, 64]");
    st = ensure_streams(f);
    if (st != PA_OK) return st;
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    pa_status result = PA_OK;
    for (int gi = 0; gi < (int)f->groups.size() && result == PA_OK; ++gi) {
        pa_fused::Group &g = f->groups[gi];
        double attempts = 0;
        int steps = probe_steps;
        for (int i : g.members) steps = std::min(steps, f->runs[i].sch.n_steps);
        for (int i : g.members) {
            const pa_fused::Run &r = f->runs[i];
            attempts += (double)r.R * r.s->n * r.sch.sweeps_per_step * steps;
        }
        double best = -1;
        Shape pick = g.shape;
        for (const Shape &c : g.candidates) {
            g.shape = c;
            double ms_best = -1;
            // Two probes per shape; the first also absorbs one-time costs.
            for (int rep = 0; rep < 2 && result == PA_OK; ++rep) {
                result = prepare(f, ws, hs, {gi});
                if (result != PA_OK) break;
                if (hipEventRecord(e0, hs) != hipSuccess) { result = hip_fail(hipGetLastError(), "hipEventRecord"); break; }
                result = enqueue_group_steps(f, g, ws, 0, steps, hs);
                if (result != PA_OK) break;
                if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                    result = hip_fail(hipGetLastError(), "probe timing");
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (rep == 1) ms_best = ms;
            }
            if (result != PA_OK) break;
            const double ns = ms_best * 1e6 / attempts;
            if (best < 0 || ns < best) {
                best = ns;
                pick = c;
            }
        }
        g.shape = pick;
        g.probe_ns_per_attempt = best;
        shape_facts(f, g);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // The probes leave the runs part-way: they are no valid results.
    for (auto &r : f->runs) {
        r.s->has_run = false;
        r.s->rc.valid = false;
    }
    drop_graph(f);
    return result;
}

extern "C" pa_status pa_fused_run(pa_fused *f, void *workspace, size_t workspace_bytes, void *stream)
{
    g_error[0] = 0;
    pa_status st = check_ws(f, workspace, workspace_bytes);
    if (st != PA_OK) return st;
    st = ensure_streams(f);
    if (st != PA_OK) return st;
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    st = prepare(f, ws, hs, {});
    if (st != PA_OK) return st;
    if (!f->use_graph) {
        st = enqueue_all_steps(f, ws, hs);
        if (st != PA_OK) return st;
        finish_runs(f, hs);
        return PA_OK;
    }
    const uint64_t sig = shapes_sig(f);
    if (!f->exec || f->graph_ws != ws || f->graph_sig != sig) {
        drop_graph(f);
        HIP_TRY(hipStreamBeginCapture(f->cap, hipStreamCaptureModeRelaxed));
        st = enqueue_all_steps(f, ws, f->cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(f->cap, &g);
        if (st != PA_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        f->graph = g;
        HIP_TRY(hipGraphInstantiate(&f->exec, f->graph, nullptr, nullptr, 0));
        f->graph_ws = ws;
        f->graph_sig = sig;
    }
    HIP_TRY(hipGraphLaunch(f->exec, hs));
    finish_runs(f, hs);
    return PA_OK;
}

extern "C" pa_status pa_fused_set_graph(pa_fused *f, int32_t on)
{
    if (!f || (on != 0 && on != 1)) return fail(PA_EINVAL, "pa_fused_set_graph: null batch or flag not 0/1");
    f->use_graph = on;
    return PA_OK;
}

extern "C" pa_status pa_fused_info(const pa_fused *f, int64_t *out, int32_t max_groups, int32_t *groups)
{
    if (!f || !groups) return fail(PA_EINVAL, "pa_fused_info: null argument");
    *groups = (int32_t)f->groups.size();
    if (!out) return PA_OK;
    for (int gi = 0; gi < (int)f->groups.size() && gi < max_groups; ++gi) {
        const pa_fused::Group &g = f->groups[gi];
        int64_t *o = out + 8 * (size_t)gi;
        o[0] = g.bsg;
        o[1] = (int64_t)g.members.size();
        o[2] = g.shape.W;
        o[3] = g.shape.threads;
        o[4] = g.shape.direct;
        o[5] = g.blocks;
        o[6] = g.lds;
        o[7] = (int64_t)(g.probe_ns_per_attempt * 1e6);   // femtoseconds per attempt, 0 untuned
    }
    return PA_OK;
}
