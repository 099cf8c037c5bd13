// pa_device.h -- argument blocks shared by the host driver (pa_api.cpp) and
// the gfx950 kernels (pa_kernels.hip). Plain structs passed by value.
//
// Device data layout (all inside the caller's workspace):
//   X[g][i]   uint64: bit b is the spin of replica 64g+b at node i (1 = +1).
//             Group-major, so the 64-replica group g is n contiguous words.
//   E[r]      int32 Ising energy sum_{i<j} w_ij x_i x_j of replica r.
//   CSR       row_ptr[n+1], col[nnz] with each row's +1-weight neighbours
//             first, npos[i] = their count.
//   sched     nodes grouped by dependency level of the sweep order: nodes in
//             one level are pairwise non-adjacent, and every node comes after
//             all its earlier-ordered neighbours' levels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pa.h"

namespace pa {

constexpr int kStatFields = PA_STAT_FIELDS;
constexpr int kMaxJump = 64;     // largest grid jump of an adaptive step
constexpr int kMaxThreads = 1024;
// Kernel 1 LDS: the 256-entry u32 threshold table (indexed by a move byte),
// then the byte records.
constexpr int kBytesRecBase = 1024;
// Size of the static device workspace of pa_run_static.
constexpr size_t kStaticScratchBytes = PA_STATIC_SCRATCH_BYTES;

struct GraphDev {
    int n;
    int dmax;
    const int *row_ptr;
    const int *col;
    const int *npos;
    const uint32_t *edges;      // [ne] each edge once, i < j: i | j << 15 | negative << 30
    int ne;
};

struct SweepArgs {
    int n;
    int dmax;
    int R;            // real replicas
    int S;            // sweeps in this step
    int k;            // step index (Philox counter)
    int K;            // grid points; as_state[3] >= K marks a finished run
    int adapt;        // adaptive steps: the grid point is as_state[3], else k
    int lmax1;        // number of noise levels
    int n_levels;
    uint32_t seed_lo, seed_hi, inst;
    const int *sched;           // [n] nodes in level order
    const int *level_off;       // [n_levels + 1]
    const uint4 *blocks;        // [n][block_u4] adjacency block per schedule slot (+128 B pad)
    int block_u4;
    const int2 *stream;         // [waves][qpad] {first slot, max degree} per pass
    int qpad;
    const int4 *rounds;         // [n_rounds] {first slot, level end, last round of level, 0}
    int n_rounds;
    int flush_every;            // rounds between widenings of the byte energy accumulators
    int direct;                 // kernel 1: block entries are LDS byte offsets
    int prio_mode;              // kernel 1: 1 = issue-priority turns of the two workgroups
                                // sharing a compute unit (8-replica tiles), else 0
    const uint64_t *thr;        // kernel 2: [K][lmax1][dmax+1] T[m] (T[0] unused), by grid point
    const uint32_t *thr32;      // kernel 1: [K][lmax1][dmax+1] T[1..dmax], all-accept flag
    const int *as_state;        // [0] level, [3] grid point of this step
    uint64_t *X;                // [G][n] population written by the sweep (kernel 2: in place)
    int *E;                     // [Rp]
    const uint64_t *Xin;        // kernel 1: population before resampling, read through parent
    const int *Ein;             // kernel 1: its energies
    const int *parent;          // kernel 1: [R] resampling parent of each slot, null = identity
    const int *best_E;          // global best so far
    unsigned long long *cand;   // [nblk] (E+2^31)<<32 | s<<15 | r, or ~0
    uint32_t *snap;             // [nblk][nw32]
    unsigned long long *counters; // [0] uphill attempts, [1] uphill accepts
    int nw32;
};

struct EpiArgs {
    int R, n, nw32, nblk, W, k, K, S;
    int do_cand, do_pop, do_rest;
    int pop_step, pop_sweep;    // best record when the population check wins
    int as_enable, as_stall, as_lmax, as_frozen_inv;
    int adapt, adapt_jump, adapt_num, adapt_den;   // adaptive steps (jump <= kMaxJump)
    int *as_state;              // [0] level, [1] stall, [2] improved this step, [3] grid point
    const unsigned long long *cand;
    const uint32_t *snap;
    int *best;                  // [0] E, [1] step, [2] sweep, [3] replica, [4] valid
    uint32_t *best_x;           // [nw32]
    unsigned long long *counters;
    const int *E;
    const uint64_t *X;
    long long *stats;           // [K][kStatFields]
    const uint64_t *wtab;       // weight tables
    const int *wtab_off;        // fixed steps: [K] table of the step from grid point g
                                // (g < K-1); adaptive: [jumps] table of jump j at j - 1
    const int *wtab_len;
    uint32_t seed_lo, seed_hi, inst;
    int *parent;                // [R] parent replica of each new slot
    int *counts_rec;            // [K][R] or null
};

// One run of a multi-run launch (several runs' steps in one sweep launch and
// one epilogue launch): its sweep and epilogue arguments without the per-step
// fields (step, population buffers, resampling parents), which the kernels
// derive from the step index.
struct MultiRun {
    SweepArgs sweep;
    EpiArgs epi;                // epi.parent: the resampling parents the next sweep reads
    uint64_t *X0, *X1;          // population ping-pong; the initial population is in X0
    int *E0, *E1;
    int steps;                  // K: steps at or past it do nothing
    int nblk;                   // sweep tiles of this run
    int k_off;                  // launch index of the run's step 0
};

struct GatherArgs {
    int n, R, G;
    const int *parent;
    const uint64_t *Xin;
    uint64_t *Xout;
    const int *Ein;
    int *Eout;
};

struct IcmArgs {
    GraphDev g;
    int R, G, k, K, nw32;
    int adapt;                  // adaptive steps: grid point as_state[3], else k
    int kind;                   // 0: pairs (p, p + R/2); 1: single-replica Wolff update
    int lmax1;                  // noise levels per step in qtab
    uint32_t seed_lo, seed_hi, inst;
    uint64_t *X;
    int *E;
    uint32_t *vout;             // [R/2 or R][nw32] cluster bitmap of each pair or replica
    const uint64_t *qtab;       // kind 1: [K][lmax1] bond thresholds floor(2^32 (1 - e^{-2 beta'}))
    const int *as_state;        // kind 1: [0] = the noise level of the step's sweeps
};

struct InitArgs {
    GraphDev g;
    int R, G;
    uint32_t seed_lo, seed_hi, inst;
    uint64_t *X;
    int *E;
};

// Host-side launchers (defined in pa_kernels.hip).
int launch_init(const InitArgs &a, void *stream);
int launch_energy(const InitArgs &a, void *stream);
int sweep_lds_bytes(int W, int sgn, int n, int dmax, int threads);
int launch_sweep(int W, int sgn, int threads, int nblk, const SweepArgs &a, void *stream);
int sweep_bytes_lds(int W, int sgn, int n, int dmax);
int launch_sweep_bytes(int W, int sgn, int threads, int nblk, const SweepArgs &a, void *stream);
int launch_epilogue(const EpiArgs &a, void *stream);
// Multi-run launches: `blocks` workgroups over the work list {run, tile}
// (sgn 0 unsigned records, 2 sign bits; `lds` the largest run's sweep LDS),
// and one epilogue workgroup per run (max_R: the largest population).
int launch_sweep_multi(int W, int sgn, bool direct, int threads, int blocks, int lds, const MultiRun *runs,
                       const int2 *work, int k, void *stream);
int launch_epilogue_multi(int runs_count, int max_R, const MultiRun *runs, int k, void *stream);
int launch_gather(const GatherArgs &a, void *stream);
int launch_icm(const IcmArgs &a, void *stream);
int icm_lds_bytes(int n, int nw32);
int launch_fill_u64(unsigned long long *p, unsigned long long v, long long count, void *stream);
const char *last_hip_error();
// Device address of the static workspace on the current device (taken once
// per device with hipGetSymbolAddress); 0 on success, else -1 with the error
// in last_hip_error().
int static_scratch(void **ptr);

}  // namespace pa
