// pa_pool.cpp -- a resident pool of population-annealing runs advanced
// together, one step per iteration (the pa_pool_* calls of include/pa.h).
//
// The pool owns a caller-provided device region (the HBM budget of the runs
// in flight). Submitted runs wait in arrival order and are admitted, without
// overtaking, as their state fits the free memory. Admitted runs with one
// launch shape (record mode, tile width, entry form, threads, LDS occupancy
// class) form a lane: a stream of its own on which each iteration advances
// every run of the lane by one temperature step -- one sweep launch over the
// work list of all their replica tiles and one epilogue launch with a
// workgroup per run, each run at its own step. Lanes progress independently,
// so runs of small graphs are not held to the pace of large ones, and they
// share the device. A run's memory returns to the pool when the caller
// releases it after reading its results, so runs join and leave between
// iterations (continuous batching) while their populations stay resident on
// the device. Every run gives exactly the results of pa_run with the same
// arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "pa.h"
#include "pa_device.h"
#include "pa_host.h"

using namespace pa_host;

namespace {

constexpr int kLanes = 16;               // lanes at most (each a stream)
constexpr int kLaneMaxRuns = 128;        // runs per lane at most
constexpr int kLaneMaxWork = 1 << 15;    // work-list entries per lane iteration at most
constexpr int kSlots = 2;                // argument tables per lane (membership versions in flight)

size_t slot_bytes()
{
    return align_up(sizeof(pa::MultiRun) * kLaneMaxRuns) + align_up(sizeof(int2) * kLaneMaxWork);
}

size_t lane_bytes() { return kSlots * slot_bytes(); }

struct Key {
    int bsg = 0, W = 8, direct = 1, threads = 256, cls = 1;
    bool operator==(const Key &o) const
    {
        return bsg == o.bsg && W == o.W && direct == o.direct && threads == o.threads && cls == o.cls;
    }
};

}  // namespace

struct pa_pool {
    struct Job {
        pa_solver *s = nullptr;
        pa_schedule sch{};
        std::vector<double> beta;
        std::vector<int32_t> order;
        int32_t R = 0;
        uint64_t seed = 0;
        uint32_t inst = 0;
        Shape shape;
        Key key;
        int lds = 0;
        size_t need = 0, off = 0;
        int lane = -1, k_off = 0, K = 0;
        int state = 0;                 // 0 waiting, 1 stepping, 2 last step enqueued, 3 done, 4 reported
        hipEvent_t done = nullptr;
    };
    struct Lane {
        bool used = false;
        Key key;
        hipStream_t st = nullptr;
        int iter = 0;                  // launch index of the next iteration
        bool dirty = true;
        bool wait_setup = false;       // new runs' setup (on the pool's stream) precedes the next step
        int slot = 0;
        unsigned char *host[kSlots] = {};
        hipEvent_t slot_ev[kSlots] = {};
        bool slot_pending[kSlots] = {};
        hipEvent_t call_ev[2] = {};    // end of the lane's last two advance batches
        bool call_pending[2] = {};
        int call = 0;
        std::vector<int64_t> runs;     // stepping runs, in admission order
        int blocks = 0, lds = 0, max_R = 0;
        size_t args = 0, work = 0;     // current argument tables (offsets in the pool)
    };
    unsigned char *ws = nullptr;
    size_t bytes = 0;
    size_t heap_off = 0;               // runs' memory: [heap_off, bytes)
    std::map<size_t, size_t> free_;    // offset -> length, coalesced
    std::map<int64_t, Job> jobs;
    std::deque<int64_t> waiting;
    int64_t next_ticket = 1;
    int max_lds = 160 * 1024;
    hipStream_t stream = nullptr;
    bool have_stream = false;
    hipEvent_t setup_ev = nullptr;
    size_t in_use = 0;
    long long iterations = 0;          // lane iterations enqueued so far
    Lane lanes[kLanes];
};

namespace {

bool take_region(pa_pool *p, size_t need, size_t *off)
{
    for (auto it = p->free_.begin(); it != p->free_.end(); ++it) {
        if (it->second < need) continue;
        *off = it->first;
        const size_t rest = it->second - need;
        const size_t at = it->first + need;
        p->free_.erase(it);
        if (rest) p->free_[at] = rest;
        p->in_use += need;
        return true;
    }
    return false;
}

void give_region(pa_pool *p, size_t off, size_t len)
{
    p->in_use -= len;
    auto it = p->free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != p->free_.end() && it->first + it->second == nx->first) {
        it->second += nx->second;
        p->free_.erase(nx);
    }
    if (it != p->free_.begin()) {
        auto pv = std::prev(it);
        if (pv->first + pv->second == it->first) {
            pv->second += it->second;
            p->free_.erase(it);
        }
    }
}

// Check the events of runs whose last step was enqueued.
void collect(pa_pool *p)
{
    for (auto &kv : p->jobs) {
        pa_pool::Job &j = kv.second;
        if (j.state == 2 && j.done && hipEventQuery(j.done) == hipSuccess) j.state = 3;
    }
    (void)hipGetLastError();   // a pending event's "not ready" is no error of a later call
}

}  // namespace

extern "C" pa_status pa_pool_create(pa_pool **out, void *workspace, size_t workspace_bytes)
{
    g_error[0] = 0;
    if (!out) return fail(PA_EINVAL, "pa_pool_create: null output");
    *out = nullptr;
    if (!workspace) return fail(PA_EWORKSPACE, "pa_pool_create: workspace is null");
    if (((uintptr_t)workspace) % kAlign) return fail(PA_EWORKSPACE, "pool workspace must be 256-byte aligned");
    const size_t fixed = kLanes * lane_bytes();
    if (workspace_bytes <= fixed)
        return fail(PA_EWORKSPACE, "pool workspace of %zu bytes leaves nothing beyond its %zu bytes of tables",
                    workspace_bytes, fixed);
    pa_pool *p = new (std::nothrow) pa_pool;
    if (!p) return fail(PA_ERANGE, "pa_pool_create: out of host memory");
    p->ws = static_cast<unsigned char *>(workspace);
    p->bytes = workspace_bytes;
    p->heap_off = fixed;
    p->free_[fixed] = (workspace_bytes - fixed) / kAlign * kAlign;
    p->max_lds = device_max_lds();
    *out = p;
    return PA_OK;
}

extern "C" pa_status pa_pool_destroy(pa_pool *p)
{
    if (!p) return PA_OK;
    if (p->have_stream) (void)hipStreamSynchronize(p->stream);
    for (auto &L : p->lanes) {
        if (L.st) {
            (void)hipStreamSynchronize(L.st);
            (void)hipStreamDestroy(L.st);
        }
        for (int q = 0; q < kSlots; ++q) {
            if (L.slot_ev[q]) (void)hipEventDestroy(L.slot_ev[q]);
            if (L.host[q]) (void)hipHostFree(L.host[q]);
        }
        for (auto &e : L.call_ev)
            if (e) (void)hipEventDestroy(e);
    }
    for (auto &kv : p->jobs)
        if (kv.second.done) (void)hipEventDestroy(kv.second.done);
    if (p->setup_ev) (void)hipEventDestroy(p->setup_ev);
    delete p;
    return PA_OK;
}

extern "C" pa_status pa_pool_submit(pa_pool *p, const pa_fused_entry *run, int64_t *ticket)
{
    g_error[0] = 0;
    if (!p || !run || !ticket) return fail(PA_EINVAL, "pa_pool_submit: null argument");
    pa_status st = check_schedule(run->solver, run->schedule, run->R);
    if (st != PA_OK) return st;
    if (run->instance > 65535) return fail(PA_ERANGE, "instance=%u outside [0, 65535]", run->instance);
    if (run->schedule->nl_period != 0 || run->schedule->beta_adapt != 0)
        return fail(PA_EINVAL, "pooled runs take no non-local moves and no adaptive steps (use pa_run)");
    for (auto &kv : p->jobs)
        if (kv.second.s == run->solver)
            return fail(PA_EINVAL, "the solver already has a run in the pool (release it first)");
    pa_pool::Job j;
    j.s = run->solver;
    j.sch = *run->schedule;
    j.beta.assign(run->schedule->beta, run->schedule->beta + run->schedule->n_steps);
    j.sch.beta = j.beta.data();
    if (run->schedule->order) {
        j.order.assign(run->schedule->order, run->schedule->order + run->solver->n);
        j.sch.order = j.order.data();
    }
    j.R = run->R;
    j.seed = run->seed;
    j.inst = run->instance;
    j.K = run->schedule->n_steps;
    // Shape: 8 replicas per workgroup where a tile's records fit LDS, else 4;
    // sign-bit entries for graphs with -1 weights; LDS offsets as entries
    // where they fit 16 bits; threads: the smallest of 64, 128, 256, 512 whose
    // rounds per sweep (one per dependency-level chunk) are no more than
    // with 512.
    const pa_solver *s = run->solver;
    j.shape.bsg = s->has_neg ? 2 : 0;
    j.shape.W = pa::sweep_bytes_lds(8, 0, s->n, s->dmax) <= p->max_lds ? 8 : 4;
    j.shape.threads = 512;
    j.shape.direct = pa::kBytesRecBase + (size_t)(s->n + 1) * j.shape.W <= 0xFFFF;
    Plan plan;
    st = build_plan(j.s, &j.sch, j.R, plan, false, &j.shape);
    if (st != PA_OK) return st;
    {
        auto rounds_at = [&](int T) {
            long long n = 0;
            for (int l = 0; l < plan.n_levels; ++l) n += (plan.level_off[l + 1] - plan.level_off[l] + T - 1) / T;
            return n;
        };
        const long long r512 = rounds_at(512);
        for (int T : {256, 128, 64})
            if (rounds_at(T) <= r512) j.shape.threads = T;
        if (j.shape.threads != 512) {
            plan = Plan();
            st = build_plan(j.s, &j.sch, j.R, plan, false, &j.shape);
            if (st != PA_OK) return st;
        }
    }
    j.lds = pa::sweep_bytes_lds(j.shape.W, 0, s->n, s->dmax);
    j.key.bsg = j.shape.bsg;
    j.key.W = j.shape.W;
    j.key.direct = j.shape.direct;
    j.key.threads = j.shape.threads;
    j.key.cls = std::min(8, p->max_lds / std::max(j.lds, 1));
    j.need = align_up(plan.L.total);
    if (j.need > p->bytes - p->heap_off)
        return fail(PA_EWORKSPACE, "run needs %zu bytes, more than the pool's %zu", j.need,
                    p->bytes - p->heap_off);
    if ((j.R + 63) / 64 * (64 / j.shape.W) + 64 * 8 > kLaneMaxWork)
        return fail(PA_ERANGE, "run of %d replicas exceeds a lane's work list", j.R);
    const int64_t t = p->next_ticket++;
    p->jobs.emplace(t, std::move(j));
    p->waiting.push_back(t);
    *ticket = t;
    return PA_OK;
}

extern "C" pa_status pa_pool_cancel(pa_pool *p, int64_t ticket)
{
    g_error[0] = 0;
    if (!p) return fail(PA_EINVAL, "null pool");
    auto it = std::find(p->waiting.begin(), p->waiting.end(), ticket);
    if (it == p->waiting.end()) return fail(PA_ESTATE, "ticket %lld is not waiting", (long long)ticket);
    p->waiting.erase(it);
    p->jobs.erase(ticket);
    return PA_OK;
}

namespace {

int lane_work(const pa_pool *p, const pa_pool::Lane &L)
{
    int w = 0;
    for (int64_t t : L.runs) {
        const pa_pool::Job &j = p->jobs.at(t);
        w += (j.R + 63) / 64 * (64 / j.shape.W);
    }
    return w;
}

// Admit waiting runs in arrival order, without overtaking, while their
// memory fits and their lane (an existing lane of their shape, else a free
// one) has room; set them up on the pool's stream `hs`.
pa_status admit(pa_pool *p, hipStream_t hs)
{
    bool any = false;
    while (!p->waiting.empty()) {
        pa_pool::Job &j = p->jobs.at(p->waiting.front());
        int li = -1;
        for (int q = 0; q < kLanes && li < 0; ++q)
            if (p->lanes[q].used && p->lanes[q].key == j.key) li = q;
        for (int q = 0; q < kLanes && li < 0; ++q)
            if (!p->lanes[q].used) li = q;
        if (li < 0) break;
        pa_pool::Lane &L = p->lanes[li];
        const int tiles = (j.R + 63) / 64 * (64 / j.shape.W);
        if ((int)L.runs.size() >= kLaneMaxRuns || lane_work(p, L) + tiles + 64 * 8 > kLaneMaxWork) break;
        size_t off = 0;
        if (!take_region(p, j.need, &off)) break;
        pa_status st = start_run(j.s, &j.sch, j.R, j.seed, j.inst, p->ws + off, j.need, hs, true, true, &j.shape);
        if (st != PA_OK) {
            give_region(p, off, j.need);
            return st;
        }
        if (!L.used) {
            L.used = true;
            L.key = j.key;
        }
        j.off = off;
        j.lane = li;
        j.k_off = L.iter;
        j.state = 1;
        L.runs.push_back(p->waiting.front());
        L.dirty = true;
        L.wait_setup = true;
        p->waiting.pop_front();
        any = true;
    }
    if (any) {
        if (!p->setup_ev) HIP_TRY(hipEventCreateWithFlags(&p->setup_ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(p->setup_ev, hs));
    }
    return PA_OK;
}

// The lane's argument tables for its current runs, uploaded on its stream
// into its next slot (after the iterations that last read that slot).
pa_status rebuild(pa_pool *p, int li)
{
    pa_pool::Lane &L = p->lanes[li];
    L.slot = (L.slot + 1) % kSlots;
    const int q = L.slot;
    if (!L.slot_ev[q]) HIP_TRY(hipEventCreateWithFlags(&L.slot_ev[q], hipEventDisableTiming));
    if (!L.host[q]) HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&L.host[q]), slot_bytes(), hipHostMallocDefault));
    if (L.slot_pending[q]) {
        HIP_TRY(hipEventSynchronize(L.slot_ev[q]));
        L.slot_pending[q] = false;
    }
    std::vector<pa::MultiRun> mr;
    std::vector<int> nblk;
    int lds = 0, max_R = 0;
    for (int64_t t : L.runs) {
        const pa_pool::Job &j = p->jobs.at(t);
        const pa_solver *s = j.s;
        const Plan &P = s->plan;
        pa::MultiRun m{};
        m.sweep = s->rc.sa;
        m.epi = s->rc.ea;
        m.X0 = reinterpret_cast<uint64_t *>(p->ws + j.off + P.L.X0);
        m.X1 = reinterpret_cast<uint64_t *>(p->ws + j.off + P.L.X1);
        m.E0 = reinterpret_cast<int *>(p->ws + j.off + P.L.E0);
        m.E1 = reinterpret_cast<int *>(p->ws + j.off + P.L.E1);
        m.steps = P.K;
        m.nblk = P.nblk;
        m.k_off = j.k_off;
        mr.push_back(m);
        nblk.push_back(P.nblk);
        lds = std::max(lds, j.lds);
        max_R = std::max(max_R, j.R);
    }
    const std::vector<int2> w = multi_work_list(nblk, L.key.W);
    const size_t ab = align_up(sizeof(pa::MultiRun) * mr.size());
    if (mr.size() > (size_t)kLaneMaxRuns || w.size() > (size_t)kLaneMaxWork)
        return fail(PA_ERANGE, "internal: lane tables overflow");
    std::memcpy(L.host[q], mr.data(), sizeof(pa::MultiRun) * mr.size());
    std::memcpy(L.host[q] + ab, w.data(), sizeof(int2) * w.size());
    const size_t base = (size_t)li * lane_bytes() + (size_t)q * slot_bytes();
    HIP_TRY(hipMemcpyAsync(p->ws + base, L.host[q], ab + sizeof(int2) * w.size(), hipMemcpyHostToDevice, L.st));
    L.args = base;
    L.work = base + ab;
    L.blocks = (int)w.size();
    L.lds = lds;
    L.max_R = max_R;
    L.dirty = false;
    return PA_OK;
}

// One iteration of lane li on its stream: every run of the lane one step.
pa_status iterate(pa_pool *p, int li)
{
    pa_pool::Lane &L = p->lanes[li];
    const pa::MultiRun *args = reinterpret_cast<const pa::MultiRun *>(p->ws + L.args);
    const int2 *work = reinterpret_cast<const int2 *>(p->ws + L.work);
    LAUNCH_TRY(pa::launch_sweep_multi(L.key.W, L.key.bsg, L.key.direct != 0, L.key.threads, L.blocks, L.lds, args,
                                      work, L.iter, L.st));
    LAUNCH_TRY(pa::launch_epilogue_multi((int)L.runs.size(), L.max_R, args, L.iter, L.st));
    HIP_TRY(hipEventRecord(L.slot_ev[L.slot], L.st));
    L.slot_pending[L.slot] = true;
    // Runs whose last step this was leave the lane once it is done.
    std::vector<int64_t> keep;
    for (int64_t t : L.runs) {
        pa_pool::Job &j = p->jobs.at(t);
        if (L.iter - j.k_off == j.K - 1) {
            if (!j.done) HIP_TRY(hipEventCreateWithFlags(&j.done, hipEventDisableTiming));
            HIP_TRY(hipEventRecord(j.done, L.st));
            finish_run(j.s, L.st);
            j.state = 2;
            L.dirty = true;
        } else {
            keep.push_back(t);
        }
    }
    L.runs.swap(keep);
    ++L.iter;
    ++p->iterations;
    return PA_OK;
}

}  // namespace

extern "C" pa_status pa_pool_advance(pa_pool *p, void *stream, int32_t iterations, int32_t *done)
{
    g_error[0] = 0;
    if (!p || !done) return fail(PA_EINVAL, "pa_pool_advance: null argument");
    if (iterations < 1 || iterations > 1024) return fail(PA_EINVAL, "iterations must be in [1, 1024]");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (p->have_stream && hs != p->stream)
        return fail(PA_EINVAL, "a pool advances on one stream (the first advance's)");
    p->stream = hs;
    p->have_stream = true;
    *done = 0;
    collect(p);
    pa_status st = admit(p, hs);
    if (st != PA_OK) return st;
    for (int li = 0; li < kLanes; ++li) {
        pa_pool::Lane &L = p->lanes[li];
        if (!L.used) continue;
        if (L.runs.empty()) {
            // An empty lane is free for another shape once its work is done.
            bool busy = false;
            for (int c = 0; c < 2; ++c)
                if (L.call_pending[c] && hipEventQuery(L.call_ev[c]) != hipSuccess) busy = true;
            (void)hipGetLastError();
            if (!busy) {
                L.used = false;
                L.dirty = true;
                for (auto &b : L.call_pending) b = false;
            }
            continue;
        }
        if (!L.st) HIP_TRY(hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking));
        // At most two batches in flight per lane; a lane still busy is
        // skipped (the caller advances again), so slow lanes never hold up
        // fast ones.
        const int c = L.call;
        if (L.call_pending[c]) {
            const hipError_t e = hipEventQuery(L.call_ev[c]);
            if (e == hipErrorNotReady) {
                (void)hipGetLastError();
                continue;
            }
            if (e != hipSuccess) return hip_fail(e, "hipEventQuery(lane)");
            L.call_pending[c] = false;
        }
        if (L.wait_setup) {
            HIP_TRY(hipStreamWaitEvent(L.st, p->setup_ev, 0));
            L.wait_setup = false;
        }
        int n = 0;
        for (; n < iterations && !L.runs.empty(); ++n) {
            if (L.dirty) {
                st = rebuild(p, li);
                if (st != PA_OK) return st;
            }
            st = iterate(p, li);
            if (st != PA_OK) return st;
        }
        if (n) {
            if (!L.call_ev[c]) HIP_TRY(hipEventCreateWithFlags(&L.call_ev[c], hipEventDisableTiming));
            HIP_TRY(hipEventRecord(L.call_ev[c], L.st));
            L.call_pending[c] = true;
            L.call ^= 1;
            *done += n;
        }
    }
    return PA_OK;
}

extern "C" pa_status pa_pool_poll(pa_pool *p, int64_t *tickets, int32_t cap, int32_t *count)
{
    g_error[0] = 0;
    if (!p || !count || (cap > 0 && !tickets)) return fail(PA_EINVAL, "pa_pool_poll: null argument");
    collect(p);
    int32_t n = 0;
    for (auto &kv : p->jobs)
        if (kv.second.state == 3 && n < cap) {
            tickets[n++] = kv.first;
            kv.second.state = 4;           // reported
        }
    *count = n;
    return PA_OK;
}

extern "C" pa_status pa_pool_release(pa_pool *p, int64_t ticket)
{
    g_error[0] = 0;
    if (!p) return fail(PA_EINVAL, "null pool");
    auto it = p->jobs.find(ticket);
    if (it == p->jobs.end()) return fail(PA_EINVAL, "unknown ticket %lld", (long long)ticket);
    pa_pool::Job &j = it->second;
    if (j.state < 2) return fail(PA_ESTATE, "ticket %lld has not finished", (long long)ticket);
    if (j.done) {
        HIP_TRY(hipEventSynchronize(j.done));
        (void)hipEventDestroy(j.done);
    }
    give_region(p, j.off, j.need);
    // Its memory will be reused: the solver no longer holds results.
    j.s->has_run = false;
    j.s->rc.valid = false;
    p->jobs.erase(it);
    return PA_OK;
}

extern "C" pa_status pa_pool_info(const pa_pool *p, int64_t out[6])
{
    if (!p || !out) return fail(PA_EINVAL, "pa_pool_info: null argument");
    int64_t w = 0, r = 0, f = 0;
    for (auto &kv : p->jobs) {
        w += kv.second.state == 0;
        r += kv.second.state == 1;
        f += kv.second.state >= 2;
    }
    out[0] = w;
    out[1] = r;
    out[2] = f;
    out[3] = (int64_t)p->in_use;
    out[4] = (int64_t)(p->bytes - p->heap_off);
    out[5] = p->iterations;
    return PA_OK;
}
