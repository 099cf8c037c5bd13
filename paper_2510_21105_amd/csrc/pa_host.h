// pa_host.h -- host-side internals shared by the files that implement the C
// ABI of include/pa.h: the validated graph (pa_solver), a run's plan and
// workspace layout, and the steps that prepare and enqueue runs. pa_api.cpp
// implements single runs, pa_fused.cpp many runs per kernel launch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "pa.h"
#include "pa_device.h"

namespace pa_host {

// Text of the last error on this thread (pa_last_error).
extern thread_local char g_error[512];

// Record the error text (thread-local, read by pa_last_error) and return st.
pa_status fail(pa_status st, const char *fmt, ...);
pa_status hip_fail(hipError_t e, const char *what);

#define HIP_TRY(call)                                                    \
    do {                                                                 \
        hipError_t _e = (call);                                          \
        if (_e != hipSuccess) return pa_host::hip_fail(_e, #call);       \
    } while (0)

#define LAUNCH_TRY(call)                                                 \
    do {                                                                 \
        if ((call) != 0) return pa_host::fail(PA_EDEVICE, "%s", pa::last_hip_error()); \
    } while (0)

constexpr int kMaxN = 32767;   // node ids and LDS word indices fit 16 bits
constexpr int kMaxDegree = 4096;
constexpr int kMaxBytesDegree = 127;   // byte counters of kernel 1 (2u must fit a byte)
constexpr int kMaxR = 32768;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t b, size_t a = kAlign) { return (b + a - 1) / a * a; }

struct Layout {
    // Host inputs, uploaded together: [0, inputs_end).
    size_t row_ptr, col, npos, edges, qtab, sched, level_off, blocks, stream, thr, wtab, wtab_off,
        wtab_len, inputs_end;
    size_t vout;
    size_t X0, X1, E0, E1, cand, snap, counters, as_state, best, best_x, stats, parent;
    size_t counts, xinit, total;
};

struct Plan {
    int K = 0, S = 0, R = 0, G = 0, Rp = 0, W = 0, threads = 0, nblk = 0, nw32 = 0;
    int lmax1 = 1, n_levels = 0, record = 0;
    int kind = 2, sgn = 0, block_bytes = 0, qpad = 0, n_rounds = 0, flush_every = 1;
    int direct = 0;   // kernel 1: block entries are LDS byte offsets (else record indices)
    int prio_mode = 0;  // kernel 1: issue-priority turns (SweepArgs::prio_mode)
    int bsg = 0;      // kernel 1 records: 0 unsigned, 1 complemented copies, 2 sign bits in entries
    std::vector<int> sched, level_off;
    std::vector<uint32_t> blocks;   // [n][block_bytes / 4] + 128 B
    std::vector<int> stream;        // kernel 2: [waves][qpad][2]
    std::vector<int> rounds;        // kernel 1: [n_rounds][4]
    std::vector<uint64_t> thr, wtab;
    std::vector<uint32_t> thr32;   // kernel 1: [K][lmax1][dmax + 1] = T[1..dmax], saturation flag
    std::vector<uint64_t> qtab;    // single-replica cluster moves: [K][lmax1] bond thresholds
    std::vector<int> wtab_off, wtab_len;
    Layout L{};
};

// A launch shape imposed on kernel 1 (multi-run launches share one shape):
// replicas per workgroup, threads, record mode (0 unsigned, 2 sign bits) and
// block-entry form (1 LDS byte offsets, 0 record indices).
struct Shape {
    int W = 8, threads = 512, bsg = 0, direct = 1;
};

pa_status check_schedule(const pa_solver *s, const pa_schedule *sch, int R);
pa_status build_plan(pa_solver *s, const pa_schedule *sch, int R, Plan &p, bool tables,
                     const Shape *force = nullptr);
uint64_t run_key(const pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed, uint32_t instance);
pa_status start_run(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed, uint32_t instance,
                    void *workspace, size_t workspace_bytes, void *stream, bool fresh, bool pinned = true,
                    const Shape *force = nullptr);

// Work list {run, tile} of a multi-run sweep launch (pa_fused.cpp).
std::vector<int2> multi_work_list(const std::vector<int> &nblk, int W);
// Mark a run whose last step has been enqueued on `hs` as finished.
void finish_run(pa_solver *s, hipStream_t hs);
// The largest dynamic LDS of a workgroup on the current device.
int device_max_lds();

}  // namespace pa_host

struct pa_solver {
    int n = 0;
    long long nnz = 0;
    int dmax = 0;
    long long w_tot = 0;
    int has_neg = 0;
    std::vector<int> row_ptr, col, npos;
    std::vector<uint32_t> edges;   // each edge once (i < j): i | j << 15 | negative << 30
    // last run
    bool has_run = false;
    pa_host::Plan plan;
    unsigned char *ws = nullptr;
    hipStream_t stream = nullptr;
    size_t final_x = 0, final_E = 0;
    int device = 0;
    // State carried from one pa_run_steps call to the next.
    struct RunCtx {
        bool valid = false;
        uint64_t key = 0;               // run_key of the run in the workspace
        int next_step = 0;              // first step not run yet
        bool parents_pending = false;   // kernel 1: the next population is Xc read through the parents
        size_t Xc = 0, Xn = 0, Ec = 0, En = 0;
        uint32_t seed_lo = 0, seed_hi = 0, instance = 0;
        int nl_period = 0, nl_kind = 0;
        int adapt = 0;                  // adaptive steps: the run may end before step K
        pa::GraphDev gd{};
        pa::SweepArgs sa{};
        pa::EpiArgs ea{};
    } rc;
    // Pinned host copy of a run's inputs in workspace layout, uploaded with one
    // copy; the event marks the end of the last upload from it.
    unsigned char *stage = nullptr;
    size_t stage_cap = 0;
    hipEvent_t stage_ev = nullptr;
    bool stage_pending = false;
    // Pageable host copy of the inputs for runs that allocate no pinned or
    // device memory (pa_run_static).
    std::vector<unsigned char> stage_host;
    // timing: 0 off, else the sweep launches of every timing-th step are timed
    int timing = 0, timing_run = 0;
    // fault injection: the next run stops before enqueuing this step (-1: off)
    int fault_step = -1;
    std::vector<hipEvent_t> ev;
    int ev_first = 0, ev_used = 0;
};

