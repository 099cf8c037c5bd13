// pa_api.cpp -- host side of the C ABI declared in include/pa.h.
//
// Validates the graph (paper section 1: undirected graph, binary weights),
// builds the device-friendly CSR, the dependency-level schedule of the sweep
// order, and the fixed-point tables of the Metropolis thresholds and
// resampling weights (FP64 exp on the host, then floor(2^32 * value)), lays
// out the caller's workspace and enqueues the step loop on the caller's
// stream. Device work is in pa_kernels.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <thread>
#include <new>
#include <vector>

#include "pa.h"
#include "pa_device.h"
#include "pa_host.h"

namespace pa_host {

thread_local char g_error[512] = "";

pa_status fail(pa_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_error, sizeof g_error, fmt, ap);
    va_end(ap);
    return st;
}

pa_status hip_fail(hipError_t e, const char *what)
{
    return fail(PA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace pa_host

using namespace pa_host;

extern "C" const char *pa_last_error(void) { return g_error; }

// --------------------------------------------------------------- create ----

extern "C" pa_status pa_create(pa_solver **out, int32_t n, const int32_t *row_ptr,
                               const int32_t *col, const int8_t *w)
{
    g_error[0] = 0;
    if (!out || !row_ptr || (!col && row_ptr && n > 0 && row_ptr[n] > 0) || (!w && col))
        return fail(PA_EINVAL, "pa_create: null pointer argument");
    *out = nullptr;
    if (n < 2 || n > kMaxN) return fail(PA_ERANGE, "pa_create: n=%d outside [2, %d]", n, kMaxN);
    if (row_ptr[0] != 0) return fail(PA_EINVAL, "pa_create: row_ptr[0] must be 0");
    for (int i = 0; i < n; ++i)
        if (row_ptr[i + 1] < row_ptr[i]) return fail(PA_EINVAL, "pa_create: row_ptr decreases at %d", i);
    const long long nnz = row_ptr[n];
    std::vector<std::vector<std::pair<int, int>>> rows(n);
    int dmax = 0;
    for (int i = 0; i < n; ++i) {
        const int d = row_ptr[i + 1] - row_ptr[i];
        if (d > kMaxDegree) return fail(PA_ERANGE, "pa_create: degree %d of node %d > %d", d, i, kMaxDegree);
        dmax = std::max(dmax, d);
        rows[i].reserve(d);
        for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int j = col[e];
            if (j < 0 || j >= n) return fail(PA_EINVAL, "pa_create: column %d out of range in row %d", j, i);
            if (j == i) return fail(PA_EINVAL, "pa_create: self loop at node %d", i);
            if (w[e] != 1 && w[e] != -1)
                return fail(PA_EINVAL, "pa_create: weight %d of edge (%d,%d) is not +-1", (int)w[e], i, j);
            rows[i].push_back({j, (int)w[e]});
        }
        std::sort(rows[i].begin(), rows[i].end());
        for (size_t q = 1; q < rows[i].size(); ++q)
            if (rows[i][q].first == rows[i][q - 1].first)
                return fail(PA_EINVAL, "pa_create: repeated neighbour %d in row %d", rows[i][q].first, i);
    }
    long long wsum = 0;
    for (int i = 0; i < n; ++i)
        for (auto &jw : rows[i]) {
            auto &rj = rows[jw.first];
            auto it = std::lower_bound(rj.begin(), rj.end(), std::make_pair(i, -2));
            if (it == rj.end() || it->first != i || it->second != jw.second)
                return fail(PA_EINVAL, "pa_create: edge (%d,%d) has no symmetric partner", i, jw.first);
            wsum += jw.second;
        }
    pa_solver *s = new (std::nothrow) pa_solver;
    if (!s) return fail(PA_ERANGE, "pa_create: out of host memory");
    s->n = n;
    s->nnz = nnz;
    s->dmax = dmax;
    s->w_tot = wsum / 2;
    s->row_ptr.resize(n + 1);
    s->col.resize(nnz);
    s->npos.resize(n);
    long long e = 0;
    for (int i = 0; i < n; ++i) {
        s->row_ptr[i] = (int)e;
        int np = 0;
        for (auto &jw : rows[i])
            if (jw.second > 0) { s->col[e++] = jw.first; ++np; }
        for (auto &jw : rows[i])
            if (jw.second < 0) { s->col[e++] = jw.first; s->has_neg = 1; }
        s->npos[i] = np;
    }
    s->row_ptr[n] = (int)e;
    s->edges.reserve(nnz / 2);
    for (int i = 0; i < n; ++i)
        for (auto &jw : rows[i])
            if (jw.first > i)
                s->edges.push_back((uint32_t)i | ((uint32_t)jw.first << 15) | (jw.second < 0 ? 1u << 30 : 0u));
    {
        // Fixed pseudo-random order (xorshift64 Fisher-Yates): concurrent
        // unions in the cluster move then rarely meet the same root.
        uint64_t z = 0x9E3779B97F4A7C15ull;
        for (size_t q = s->edges.size(); q > 1; --q) {
            z ^= z << 13;
            z ^= z >> 7;
            z ^= z << 17;
            std::swap(s->edges[q - 1], s->edges[z % q]);
        }
    }
    *out = s;
    return PA_OK;
}

extern "C" pa_status pa_destroy(pa_solver *s)
{
    if (!s) return PA_OK;
    if (s->has_run && s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->stage_pending) (void)hipEventSynchronize(s->stage_ev);
    if (s->stage_ev) (void)hipEventDestroy(s->stage_ev);
    if (s->stage) (void)hipHostFree(s->stage);
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    delete s;
    return PA_OK;
}

extern "C" pa_status pa_graph_info(const pa_solver *s, int64_t out[4])
{
    if (!s || !out) return fail(PA_EINVAL, "pa_graph_info: null argument");
    out[0] = s->n;
    out[1] = s->nnz;
    out[2] = s->w_tot;
    out[3] = s->dmax;
    return PA_OK;
}

// ----------------------------------------------------------------- plan ----

// Adaptive steps reweight a jump of j grid points by beta[j] - beta[0], which
// is the jump's own increase beta[g + j] - beta[g] only on an evenly spaced
// grid. Returns the index of the first spacing beta[k + 1] - beta[k] that
// differs from the mean spacing by more than 1e-9 of it plus 8 ulps of the
// largest |beta| (the rounding of a linear grid in FP64), or -1 if none does.
static int uneven_grid(const double *beta, int K)
{
    if (K < 3) return -1;
    const double h = (beta[K - 1] - beta[0]) / (double)(K - 1);
    const double big = std::max(std::fabs(beta[0]), std::fabs(beta[K - 1]));
    const double tol = 1e-9 * std::fabs(h) + 8.0 * std::ldexp(big, -52);
    for (int k = 0; k + 1 < K; ++k)
        if (std::fabs((beta[k + 1] - beta[k]) - h) > tol) return k;
    return -1;
}

pa_status pa_host::check_schedule(const pa_solver *s, const pa_schedule *sch, int R)
{
    if (!s || !sch) return fail(PA_EINVAL, "null solver or schedule");
    if (sch->n_steps < 1) return fail(PA_EINVAL, "n_steps must be >= 1");
    if (!sch->beta) return fail(PA_EINVAL, "beta is null");
    if (sch->sweeps_per_step < 1 || sch->sweeps_per_step > 65535)
        return fail(PA_ERANGE, "sweeps_per_step=%d outside [1, 65535]", sch->sweeps_per_step);
    for (int k = 0; k < sch->n_steps; ++k) {
        const double b = sch->beta[k];
        if (!std::isfinite(b) || b < 0.0) return fail(PA_EINVAL, "beta[%d] is not finite and >= 0", k);
        if (k > 0 && b < sch->beta[k - 1]) return fail(PA_EINVAL, "beta decreases at step %d", k);
    }
    if (sch->as_enable != 0 && sch->as_enable != 1) return fail(PA_EINVAL, "as_enable must be 0 or 1");
    if (sch->as_enable) {
        if (sch->as_stall_steps < 1) return fail(PA_EINVAL, "as_stall_steps must be >= 1");
        if (sch->as_max_level < 0 || sch->as_max_level > 15)
            return fail(PA_ERANGE, "as_max_level outside [0, 15]");
        if (sch->as_frozen_inv < 1) return fail(PA_EINVAL, "as_frozen_inv must be >= 1");
        if (!(sch->as_gamma > 0.0 && sch->as_gamma <= 1.0)) return fail(PA_EINVAL, "as_gamma outside (0, 1]");
    }
    if (sch->nl_period < 0) return fail(PA_EINVAL, "nl_period must be >= 0");
    if (sch->field_bits != 0 && sch->field_bits != 8 && sch->field_bits != 16)
        return fail(PA_EINVAL, "field_bits=%d is not 0, 8 or 16", sch->field_bits);
    if (sch->field_bits == 8 && s->dmax > 127)
        return fail(PA_ERANGE, "a local field reaches the maximum degree %d, beyond 8-bit fields", s->dmax);
    if (R < 1 || R > kMaxR) return fail(PA_ERANGE, "R=%d outside [1, %d]", R, kMaxR);
    if (sch->nl_kind != 0 && sch->nl_kind != 1) return fail(PA_EINVAL, "nl_kind must be 0 or 1");
    if (sch->beta_adapt != 0 && sch->beta_adapt != 1) return fail(PA_EINVAL, "beta_adapt must be 0 or 1");
    if (sch->beta_adapt) {
        if (sch->adapt_jump < 1 || sch->adapt_jump > pa::kMaxJump)
            return fail(PA_EINVAL, "adapt_jump must be in [1, %d]", pa::kMaxJump);
        if (sch->adapt_den < 1 || sch->adapt_den > 65536 || sch->adapt_num < 0 || sch->adapt_num > sch->adapt_den)
            return fail(PA_EINVAL, "adaptive target needs 0 <= adapt_num <= adapt_den <= 65536, den >= 1");
        const int bad = uneven_grid(sch->beta, sch->n_steps);
        if (bad >= 0)
            return fail(PA_EINVAL, "adaptive steps need an evenly spaced beta grid (spacing %d differs)", bad);
    }
    if (sch->nl_period > 0 && sch->nl_kind == 0 && (R & 1))
        return fail(PA_EINVAL, "pair cluster moves pair replicas: R must be even");
    if (sch->tile_replicas != 0 && sch->tile_replicas != 4 && sch->tile_replicas != 8 &&
        sch->tile_replicas != 16 && sch->tile_replicas != 32 && sch->tile_replicas != 64)
        return fail(PA_EINVAL, "tile_replicas must be 0, 4, 8, 16, 32 or 64");
    if (sch->record < 0 || sch->record > 3) return fail(PA_EINVAL, "record must be in [0, 3]");
    if (sch->wg_threads != 0 && (sch->wg_threads < 64 || sch->wg_threads > 1024 || sch->wg_threads % 64))
        return fail(PA_EINVAL, "wg_threads must be 0 or a multiple of 64 in [64, 1024]");
    if (sch->order) {
        std::vector<char> seen(s->n, 0);
        for (int t = 0; t < s->n; ++t) {
            const int i = sch->order[t];
            if (i < 0 || i >= s->n || seen[i]) return fail(PA_EINVAL, "order is not a permutation (position %d)", t);
            seen[i] = 1;
        }
    }
    return PA_OK;
}

// Dependency levels of the sweep order: level(i) = 1 + max level of the
// neighbours visited before i (0 if none). Nodes of one level are pairwise
// non-adjacent, and visiting levels in increasing order reproduces the
// sequential sweep exactly, since each attempt only reads its neighbours.
static void build_levels(const pa_solver *s, const int32_t *order, Plan &p)
{
    const int n = s->n;
    std::vector<int> pos(n), lvl(n, 0);
    for (int t = 0; t < n; ++t) pos[order ? order[t] : t] = t;
    int nl = 0;
    for (int t = 0; t < n; ++t) {
        const int i = order ? order[t] : t;
        int l = 0;
        for (int e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
            const int j = s->col[e];
            if (pos[j] < t) l = std::max(l, lvl[j] + 1);
        }
        lvl[i] = l;
        nl = std::max(nl, l + 1);
    }
    p.n_levels = nl;
    p.level_off.assign(nl + 1, 0);
    for (int i = 0; i < n; ++i) p.level_off[lvl[i] + 1]++;
    for (int l = 0; l < nl; ++l) p.level_off[l + 1] += p.level_off[l];
    std::vector<int> fill(p.level_off.begin(), p.level_off.end() - 1);
    p.sched.assign(n, 0);
    for (int t = 0; t < n; ++t) {
        const int i = order ? order[t] : t;
        p.sched[fill[lvl[i]]++] = i;
    }
    // Within a level the visiting order is free; grouping equal degrees
    // keeps the slots of one pass (which loop to their largest degree) even.
    auto deg = [&](int i) { return s->row_ptr[i + 1] - s->row_ptr[i]; };
    for (int l = 0; l < nl; ++l)
        std::stable_sort(p.sched.begin() + p.level_off[l], p.sched.begin() + p.level_off[l + 1],
                         [&](int x, int y) { return deg(x) > deg(y); });
}

// Adjacency blocks in schedule order, one fixed-size block per slot:
// u32 {LDS byte offset of the node's spin word, degree, node, 0}, then the LDS
// byte offsets of the neighbours' words, padded with the zero word to a
// multiple of 4 entries. A neighbour joined by a negative weight points at
// the complemented copy of its spin word (word n + j), so every entry counts
// "w_ij x_j = +1" by a plain bit read. Each wave's pass stream lists
// {first slot, largest degree among the pass's slots}.
// direct: 1 or 0 imposes the entry form of kernel 1's blocks, -1 takes
// offsets whenever they fit 16 bits.
static void build_blocks(const pa_solver *s, Plan &p, int direct)
{
    const int n = s->n;
    if (p.kind == 1) {
        // Kernel 1: u16 {node, degree, neighbour record indices...}, padded
        // with the zero record's index to 8m - 2 entries (a multiple of 16
        // bytes with the header, at least the degree rounded up to 4).
        // Negative edges name the complemented record n + j (record mode 1)
        // or carry a sign bit, bit 0 of a byte offset or bit 15 of an index
        // (record mode 2). Record indices
        // count from the start of LDS (the threshold table occupies the first
        // rb records). Blocks n .. n + threads - 1 are all-padding blocks:
        // a lane reads the block of slot (first slot of its round + lane),
        // which may lie past the last node.
        const int rb = pa::kBytesRecBase / p.W;     // records start after the threshold table
        const int zrec = p.bsg == 1 ? 2 * n : n;    // index of the zero record
        // Entries are LDS byte offsets when every record's offset fits in 16
        // bits (one instruction to decode), else record indices.
        p.direct = direct >= 0 ? direct : pa::kBytesRecBase + zrec * p.W <= 0xFFFF;
        auto enc = [&](int rec) {
            return (uint16_t)(p.direct ? pa::kBytesRecBase + rec * p.W : rec + rb);
        };
        const uint16_t zi = enc(zrec);
        const int need = 4 * ((std::max(s->dmax, 1) + 3) / 4);
        int capk = 6;
        while (capk < need) capk += 8;
        p.block_bytes = 2 * (2 + capk);
        const int bw16 = p.block_bytes / 2;
        std::vector<uint16_t> b16((size_t)(n + p.threads) * bw16 + 32, zi);
        for (int t = 0; t < n; ++t) {
            const int i = p.sched[t];
            uint16_t *b = &b16[(size_t)t * bw16];
            const int e0 = s->row_ptr[i], e1 = s->row_ptr[i + 1];
            b[0] = (uint16_t)i;
            b[1] = (uint16_t)(e1 - e0);
            for (int e = e0; e < e1; ++e) {
                const int j = s->col[e];
                const bool neg = e >= e0 + s->npos[i];
                if (p.bsg == 2)
                    b[2 + (e - e0)] = (uint16_t)(enc(j) | (neg ? (p.direct ? 1u : 0x8000u) : 0u));
                else
                    b[2 + (e - e0)] = enc(neg ? n + j : j);
            }
        }
        for (int t = n; t < n + p.threads; ++t) {
            b16[(size_t)t * bw16] = 0;
            b16[(size_t)t * bw16 + 1] = 0;
        }
        p.blocks.assign((b16.size() + 1) / 2, 0u);
        std::memcpy(p.blocks.data(), b16.data(), b16.size() * sizeof(uint16_t));
        // Rounds: a level is cut into chunks of one node per thread.
        p.rounds.clear();
        for (int l = 0; l < p.n_levels; ++l) {
            const int beg = p.level_off[l], end = p.level_off[l + 1];
            for (int f = beg; f < end; f += p.threads) {
                p.rounds.push_back(f);
                p.rounds.push_back(end);
                p.rounds.push_back(f + p.threads >= end ? 1 : 0);
                p.rounds.push_back(0);
            }
        }
        p.n_rounds = (int)p.rounds.size() / 4;
        // A byte accumulator gains at most d_max per round; the kernel runs
        // rounds in pairs, so the count is even (d_max <= 127 keeps it >= 2).
        p.flush_every = std::max(2, (255 / std::max(s->dmax, 1)) & ~1);
        return;
    }
    const int cap = 4 * ((std::max(s->dmax, 1) + 3) / 4);
    p.block_bytes = 16 + 4 * cap;
    const int bw = p.block_bytes / 4;
    const int NS = 64 / p.W, NW = p.threads / 64;
    const int sh = p.W == 16 ? 1 : (p.W == 32 ? 2 : 3);
    const uint32_t zero = (uint32_t)(p.sgn ? 2 * n : n) << sh;
    p.blocks.assign((size_t)n * bw + 32, zero);
    for (int t = 0; t < n; ++t) {
        const int i = p.sched[t];
        uint32_t *b = &p.blocks[(size_t)t * bw];
        const int e0 = s->row_ptr[i], e1 = s->row_ptr[i + 1];
        b[0] = (uint32_t)i << sh;
        b[1] = (uint32_t)(e1 - e0);
        b[2] = (uint32_t)i;
        b[3] = 0;
        for (int e = e0; e < e1; ++e) {
            const int j = s->col[e];
            const bool neg = e >= e0 + s->npos[i];
            b[4 + (e - e0)] = (uint32_t)(neg ? n + j : j) << sh;
        }
    }
    std::vector<std::vector<int>> st(NW);
    for (int l = 0; l < p.n_levels; ++l) {
        const int beg = p.level_off[l], end = p.level_off[l + 1], Lsz = end - beg;
        for (int w = 0; w < NW; ++w) {
            const int npass = Lsz > w * NS ? (Lsz - w * NS + NW * NS - 1) / (NW * NS) : 0;
            for (int q = 0; q < npass; ++q) {
                const int base = beg + w * NS + q * NW * NS;
                int md = 0;
                for (int t = base; t < base + NS && t < end; ++t) {
                    const int i = p.sched[t];
                    md = std::max(md, s->row_ptr[i + 1] - s->row_ptr[i]);
                }
                st[w].push_back(base);
                st[w].push_back(md);
            }
        }
    }
    size_t qmax = 0;
    for (auto &v : st) qmax = std::max(qmax, v.size() / 2);
    p.qpad = (int)qmax + 4;
    p.stream.assign((size_t)NW * p.qpad * 2, 0);
    for (int w = 0; w < NW; ++w)
        for (int q = 0; q < p.qpad; ++q) {
            const bool have = (size_t)q < st[w].size() / 2;
            p.stream[((size_t)w * p.qpad + q) * 2] = have ? st[w][2 * q] : -1;
            p.stream[((size_t)w * p.qpad + q) * 2 + 1] = have ? st[w][2 * q + 1] : 0;
        }
}

// floor(2^32 * exp(-(beta * 2m))): the acceptance threshold of an uphill
// flip raising E by 2m at inverse temperature beta.
static uint64_t threshold_fixed(double beta, int m)
{
    const double x = std::exp(-(beta * (double)(2 * m)));
    return (uint64_t)std::floor(std::ldexp(x, 32));
}

// floor(2^32 (1 - exp(-2 beta))): activation of a satisfied unit bond in the
// single-replica cluster update (1 - exp as -expm1 in FP64).
static uint64_t bond_fixed(double beta)
{
    const double q = -std::expm1(-2.0 * beta);
    return (uint64_t)std::floor(std::ldexp(q, 32));
}

// floor(2^32 * exp(-(dbeta * n))): Boltzmann reweighting factor of a replica
// n above the population minimum when beta grows by dbeta.
static uint64_t weight_fixed(double dbeta, long long n)
{
    const double x = std::exp(-(dbeta * (double)n));
    return (uint64_t)std::floor(std::ldexp(x, 32));
}

// Calls fn(k0, k1) over [0, K) in contiguous chunks, on up to 8 host threads
// when the work (entries) is large enough to pay for them.
static void parallel_rows(int K, long long work, const std::function<void(int, int)> &fn)
{
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = (int)std::min<long long>({8, (long long)hw, K, work / 20000 + 1});
    if (nt <= 1) {
        fn(0, K);
        return;
    }
    std::vector<std::thread> pool;
    const int per = (K + nt - 1) / nt;
    for (int t = 1; t < nt; ++t) {
        const int k0 = t * per, k1 = std::min(K, k0 + per);
        if (k0 < k1) pool.emplace_back(fn, k0, k1);
    }
    fn(0, std::min(K, per));
    for (auto &th : pool) th.join();
}

pa_status pa_host::build_plan(pa_solver *s, const pa_schedule *sch, int R, Plan &p, bool tables,
                              const Shape *force)
{
    const int n = s->n;
    p.K = sch->n_steps;
    p.S = sch->sweeps_per_step;
    p.R = R;
    p.G = (R + 63) / 64;
    p.Rp = p.G * 64;
    p.nw32 = (n + 31) / 32;
    p.record = sch->record;
    p.lmax1 = sch->as_enable ? sch->as_max_level + 1 : 1;

    int dev = 0, cus = 256, max_lds = 65536;
    if (hipGetDevice(&dev) == hipSuccess) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            max_lds = v;
    } else {
        (void)hipGetLastError();
        max_lds = 160 * 1024;
    }
    p.threads = sch->wg_threads ? sch->wg_threads : pa::kMaxThreads;
    p.sgn = s->has_neg;
    const int req = sch->sweep_kernel, tile = sch->tile_replicas;
    if (req < 0 || req > 2) return fail(PA_EINVAL, "sweep_kernel must be 0, 1 or 2");
    // The cluster move keeps n union-find parents and three n-bit bitmaps in LDS
    // (plus 2.2 KB of fixed scratch).
    if (sch->nl_period > 0 && pa::icm_lds_bytes(n, p.nw32) + 4096 > max_lds)
        return fail(PA_ERANGE, "cluster moves on %d nodes exceed the LDS of a workgroup", n);
    // Kernel 1 on a signed graph reads complemented copies of the records for
    // negative edges (no per-neighbour work), or marks them with a sign bit in
    // the block entry (one XOR per neighbour, half the LDS). Measured on
    // MI355X: sign bits pay on low-degree graphs whose workgroups (8 replicas
    // each) would otherwise queue for LDS -- at least two full waves of them
    // beyond what fits with copies (100 x 100 torus, R 16,384: 0.83 -> 0.66 ms
    // per step); with fewer workgroups the XOR only costs (+2 to +8 % on small
    // tori). Sign bits take bit 15 of a record index, so indices stay below 2^15.
    p.bsg = p.sgn ? 1 : 0;
    if (p.sgn && s->dmax <= 8 && n + pa::kBytesRecBase / 4 <= 0x7FFF) {
        const long long per_cu = max_lds / pa::sweep_bytes_lds(8, 1, n, s->dmax);
        if (per_cu == 0 || (R + 7) / 8 >= 2LL * cus * per_cu) p.bsg = 2;
    }
    // Large signed graphs (above about 20,000 nodes) whose complemented
    // records do not fit a workgroup's LDS even at 4 replicas take sign bits,
    // which halve the records, rather than the word kernel (which holds 2n
    // words of a signed graph and n sweep-order entries).
    if (p.bsg == 1 && n + pa::kBytesRecBase / 4 <= 0x7FFF &&
        pa::sweep_bytes_lds(4, 1, n, s->dmax) > max_lds && pa::sweep_bytes_lds(4, 0, n, s->dmax) <= max_lds)
        p.bsg = 2;
    const int comp = p.bsg == 1 ? 1 : 0;
    auto bytes_fit = [&](int W) { return pa::sweep_bytes_lds(W, comp, n, s->dmax) <= max_lds; };
    auto words_fit = [&](int W) { return pa::sweep_lds_bytes(W, p.sgn, n, s->dmax, p.threads) <= max_lds; };
    int W = 0;
    // Kernel 1 compares draws with 32-bit thresholds. A row whose threshold
    // is exactly 2^32 for some but not all uphill moves (beta * gamma^l nonzero
    // but below about 6e-17, where exp rounds to 1) needs kernel 2.
    bool partial_sat = false;
    if (s->dmax >= 1)
        for (int k = 0; k < p.K && !partial_sat; ++k) {
            double g = 1.0;
            for (int l = 0; l < p.lmax1; ++l) {
                const double b = sch->beta[k] * g;
                if (threshold_fixed(b, 1) == (1ull << 32) && threshold_fixed(b, s->dmax) != (1ull << 32))
                    partial_sat = true;
                g = g * sch->as_gamma;
            }
        }
    if (req == 1 && partial_sat)
        return fail(PA_ERANGE, "sweep kernel 1 cannot take an inverse temperature whose "
                               "acceptance rounds to 1 for some uphill moves only");
    // Record indices (complements and the zero record included, offset by the
    // threshold table) are u16.
    const bool idx_fit = p.bsg == 2 ? n + pa::kBytesRecBase / 4 <= 0x7FFF
                                    : (p.sgn ? 2 * n : n) + pa::kBytesRecBase / 4 <= 0xFFFF;
    bool bytes_ok = s->dmax <= kMaxBytesDegree && (tile == 0 || tile <= 16) && !partial_sat && idx_fit;
    if (req == 1 && !bytes_ok)
        return fail(PA_EINVAL, "sweep kernel 1 needs max degree <= %d and tile 4, 8 or 16", kMaxBytesDegree);
    if (force) {
        // A shape imposed by a multi-run launch: kernel 1 with the given tile,
        // threads, record mode and entry form, or an error.
        if (s->dmax > kMaxBytesDegree || partial_sat)
            return fail(PA_EINVAL, "runs sharing a launch need max degree <= %d and no partly saturated "
                                   "threshold row", kMaxBytesDegree);
        if (force->W != 4 && force->W != 8 && force->W != 16)
            return fail(PA_EINVAL, "shared launch tile %d is not 4, 8 or 16", force->W);
        if (force->threads < 64 || force->threads > 1024 || force->threads % 64)
            return fail(PA_EINVAL, "shared launch threads %d", force->threads);
        if ((force->bsg != 0 && force->bsg != 2) || (force->bsg == 0 && p.sgn) ||
            (force->bsg == 2 && n + pa::kBytesRecBase / 4 > 0x7FFF))
            return fail(PA_EINVAL, "shared launch record mode %d does not suit this graph", force->bsg);
        p.bsg = force->bsg;
        if (pa::sweep_bytes_lds(force->W, 0, n, s->dmax) > max_lds)
            return fail(PA_ERANGE, "graph of %d nodes does not fit LDS with %d replicas per workgroup", n,
                        force->W);
        if (force->direct && pa::kBytesRecBase + (size_t)(n + 1) * force->W > 0xFFFF)
            return fail(PA_ERANGE, "graph of %d nodes too large for offset entries at tile %d", n, force->W);
        p.kind = 1;
        p.W = force->W;
        p.threads = force->threads;
        p.nblk = (R + p.W - 1) / p.W;
        build_levels(s, sch->order, p);
        build_blocks(s, p, force->direct);
    } else if (req != 2 && bytes_ok) {
        W = tile;
        // A requested tile takes the thread count of the automatic plan for
        // that tile: 512 (refined by the level rule below) when two
        // workgroups fit a CU, else 1,024.
        if (W != 0 && sch->wg_threads == 0)
            p.threads = 2 * pa::sweep_bytes_lds(W, comp, n, s->dmax) <= max_lds ? 512 : 1024;
        if (W == 0 && s->dmax <= 8 && bytes_fit(8)) {
            // Measured on MI355X: on low-degree graphs (tori) a round's work per
            // node is small and 8-replica tiles spread the per-node cost over
            // the most replicas, even with fewer workgroups than CUs. 512
            // threads, or 256 when two workgroups fit a CU and there are fewer
            // than four workgroups per CU in all; 1,024 when only one fits a CU
            // (tori of about 15,000 nodes and more: 11-13 % faster than 512).
            W = 8;
            if (sch->wg_threads == 0) {
                const bool two = 2 * pa::sweep_bytes_lds(8, comp, n, s->dmax) <= max_lds;
                p.threads = !two ? 1024 : ((R + 7) / 8 < 4 * cus ? 256 : 512);
            }
        }
        if (W == 0) {
            // Measured on MI355X: two resident workgroups of 512 threads per CU
            // hide the per-level latency best. Take the widest tile whose LDS
            // allows two per CU and that still gives two workgroups per CU;
            // else the narrowest tile that fits (most workgroups).
            for (int w = 16; w >= 4 && W == 0; w >>= 1)
                if (2 * pa::sweep_bytes_lds(w, comp, n, s->dmax) <= max_lds && (R + w - 1) / w >= 2 * cus)
                    W = w;
            for (int w = 4; w <= 16 && W == 0; w <<= 1)
                if (bytes_fit(w)) W = w;
            if (W == 0) W = 4;
            if (sch->wg_threads == 0)
                p.threads = 2 * pa::sweep_bytes_lds(W, comp, n, s->dmax) <= max_lds ? 512 : 1024;
        }
        if (!bytes_fit(W)) {
            if (req == 1)
                return fail(PA_ERANGE, "graph of %d nodes does not fit LDS with %d replicas per workgroup", n, W);
            W = 0;
        } else {
            p.kind = 1;
        }
    }
    if (!force && W == 0) {
        if (req == 2 && tile != 0 && tile < 16) return fail(PA_EINVAL, "sweep kernel 2 takes tile 16, 32 or 64");
        p.kind = 2;
        W = tile >= 16 ? tile : 0;
        if (W == 0) {
            W = 64;
            while (W > 16 && ((R + W - 1) / W < cus || !words_fit(W))) W >>= 1;
        }
        if (!words_fit(W))
            return fail(PA_ERANGE, "graph of %d nodes does not fit LDS with %d replicas per workgroup", n, W);
    }
    if (!force) {
    p.W = W;
    p.nblk = (R + W - 1) / W;

    build_levels(s, sch->order, p);
    if (p.kind == 1 && sch->wg_threads == 0 && p.threads == 512) {
        // Measured on MI355X: a sweep's time follows its number of rounds
        // (one barrier each), and at equal rounds fewer waves per workgroup
        // idle less. Take the smallest multiple of 64 in [256, 512] that
        // needs no more rounds than 512 threads (C2-shaped graph: 448
        // threads, 32 rounds, 2 % faster than 320 threads with 35).
        auto rounds_at = [&](int T) {
            long long r = 0;
            for (int l = 0; l < p.n_levels; ++l) r += (p.level_off[l + 1] - p.level_off[l] + T - 1) / T;
            return r;
        };
        const long long r512 = rounds_at(512);
        for (int T = 256; T < 512; T += 64)
            if (rounds_at(T) <= r512) {
                p.threads = T;
                break;
            }
    }
    build_blocks(s, p, -1);
    if (p.kind == 1) {
        // Two workgroups sharing a compute unit: the issue arbiter breaks
        // ties by age, so the one dispatched first would finish far earlier
        // and leave the other alone on the unit for the launch's tail.
        // Measured on MI355X with the G63-shaped run (8-replica tiles, two
        // per CU, all resident at once): the second one's waves ahead in 6 of
        // every 10 sweeps even them out (durations 709k / 915k cycles ->
        // 840k / 850k), the launch 7 % shorter. Launches of several
        // generations of workgroups (the 100 x 100 torus) were 2 % slower
        // with the slots alternating, so they keep the plain kernel.
        const int lds = pa::sweep_bytes_lds(p.W, p.bsg == 1 ? 1 : 0, n, s->dmax);
        const int waves = (p.threads + 63) / 64;
        const int per_cu = std::min(max_lds / std::max(lds, 1), 16 / std::max(waves, 1));
        const long long slots = (long long)cus * per_cu;
        if (p.W == 8 && per_cu == 2 && p.nblk > slots / 2 && p.nblk <= slots) p.prio_mode = 1;
    }
    }

    // Weight-table sizes (needed for the workspace size even without tables).
    const long long span = s->nnz;  // E_r - E_min <= sum |w_ij| over both directions
    // Fixed steps: the table of step k (beta_{k+1} - beta_k). Adaptive steps:
    // the table of jump j at index j - 1 (beta_j - beta_0).
    const int n_tab = sch->beta_adapt ? std::min(sch->adapt_jump, p.K - 1) : p.K - 1;
    p.wtab_off.assign(std::max(p.K, 1), 0);
    p.wtab_len.assign(std::max(p.K, 1), 0);
    std::map<uint64_t, std::pair<int, int>> seen;
    struct Tab {
        double db;
        long long off, len;
    };
    std::vector<Tab> distinct;
    long long total = 0;
    for (int k = 0; k < n_tab; ++k) {
        const double db = sch->beta_adapt ? sch->beta[k + 1] - sch->beta[0] : sch->beta[k + 1] - sch->beta[k];
        uint64_t key;
        std::memcpy(&key, &db, sizeof key);
        auto it = seen.find(key);
        if (it == seen.end()) {
            // The table runs to its first zero entry (at most span + 1
            // entries); the weights fall with n, so the first zero is found
            // by bisection and only the entries kept are evaluated.
            long long len = span + 1;
            if (weight_fixed(db, span) == 0) {
                long long lo = 0, hi = span;          // weight(lo) != 0 or lo = 0; weight(hi) == 0
                if (weight_fixed(db, 0) == 0) hi = 0;
                while (hi - lo > 1) {
                    const long long mid = lo + (hi - lo) / 2;
                    (weight_fixed(db, mid) != 0 ? lo : hi) = mid;
                }
                len = hi;
            }
            if (tables) distinct.push_back({db, total, len});
            it = seen.emplace(key, std::make_pair((int)total, (int)len)).first;
            total += len;
        }
        p.wtab_off[k] = it->second.first;
        p.wtab_len[k] = it->second.second;
    }
    if (tables && !distinct.empty()) {
        // The distinct tables' entries, filled by table on host threads.
        p.wtab.assign((size_t)total, 0);
        parallel_rows((int)distinct.size(), total, [&](int t0, int t1) {
            for (int t = t0; t < t1; ++t)
                for (long long q = 0; q < distinct[t].len; ++q)
                    p.wtab[(size_t)(distinct[t].off + q)] = weight_fixed(distinct[t].db, q);
        });
    }
    if (total == 0) {
        total = 1;
        if (tables) p.wtab.push_back(0);
    }
    if (tables && sch->nl_period > 0 && sch->nl_kind == 1) {
        p.qtab.assign((size_t)p.K * p.lmax1, 0);
        for (int k = 0; k < p.K; ++k) {
            double g = 1.0;
            for (int l = 0; l < p.lmax1; ++l) {
                p.qtab[(size_t)k * p.lmax1 + l] = bond_fixed(sch->beta[k] * g);
                g = g * sch->as_gamma;
            }
        }
    }
    if (tables) {
        // Threshold rows, one per (step, noise level); rows are independent,
        // so large tables are filled by several host threads.
        const int D = s->dmax + 1;
        if (p.kind == 1) p.thr32.assign((size_t)p.K * p.lmax1 * D, 0);
        else p.thr.assign((size_t)p.K * p.lmax1 * D, 0);
        auto fill = [&](int k0, int k1) {
            for (int k = k0; k < k1; ++k) {
                double g = 1.0;
                for (int l = 0; l < p.lmax1; ++l) {
                    const double b = sch->beta[k] * g;
                    if (p.kind == 1) {
                        uint32_t *row = &p.thr32[((size_t)k * p.lmax1 + l) * D];
                        for (int m = 1; m < D; ++m)
                            row[m - 1] = (uint32_t)std::min<uint64_t>(threshold_fixed(b, m), 0xFFFFFFFFull);
                        // Every uphill move accepted (exp rounds to 1 up to the max degree).
                        row[D - 1] = s->dmax >= 1 && threshold_fixed(b, s->dmax) == (1ull << 32) ? 1u : 0u;
                    } else {
                        uint64_t *row = &p.thr[((size_t)k * p.lmax1 + l) * D];
                        row[0] = 0;
                        for (int m = 1; m < D; ++m) row[m] = threshold_fixed(b, m);
                    }
                    g = g * sch->as_gamma;
                }
            }
        };
        parallel_rows(p.K, (long long)p.K * p.lmax1 * D, fill);
    }

    Layout &L = p.L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + std::max<size_t>(bytes, 1));
        return at;
    };
    L.row_ptr = take(sizeof(int) * (n + 1));
    L.col = take(sizeof(int) * s->nnz);
    L.npos = take(sizeof(int) * n);
    L.edges = take(sizeof(uint32_t) * s->edges.size());
    L.qtab = sch->nl_period > 0 && sch->nl_kind == 1 ? take(sizeof(uint64_t) * (size_t)p.K * p.lmax1) : 0;
    L.sched = take(sizeof(int) * n);
    L.level_off = take(sizeof(int) * (p.n_levels + 1));
    L.blocks = take(sizeof(uint32_t) * p.blocks.size());
    L.stream = take(sizeof(int) * (p.kind == 1 ? p.rounds.size() : p.stream.size()));
    L.thr = take(sizeof(uint64_t) * (size_t)p.K * p.lmax1 * (s->dmax + 1));
    L.wtab = take(sizeof(uint64_t) * (size_t)total);
    L.wtab_off = take(sizeof(int) * p.K);
    L.wtab_len = take(sizeof(int) * p.K);
    L.inputs_end = o;
    L.vout = sch->nl_period > 0
                 ? take(sizeof(uint32_t) * (size_t)(sch->nl_kind == 1 ? R : R / 2) * p.nw32)
                 : 0;
    L.X0 = take(sizeof(uint64_t) * (size_t)p.G * n);
    L.X1 = take(sizeof(uint64_t) * (size_t)p.G * n);
    L.E0 = take(sizeof(int) * p.Rp);
    L.E1 = take(sizeof(int) * p.Rp);
    L.cand = take(sizeof(uint64_t) * p.nblk);
    L.snap = take(sizeof(uint32_t) * (size_t)p.nblk * p.nw32);
    L.counters = take(sizeof(uint64_t) * 2);
    L.as_state = take(sizeof(int) * 4);
    L.best = take(sizeof(int) * 8);
    L.best_x = take(sizeof(uint32_t) * p.nw32);
    L.stats = take(sizeof(long long) * (size_t)p.K * pa::kStatFields);
    L.parent = take(sizeof(int) * p.Rp);
    L.counts = (p.record & 1) ? take(sizeof(int) * (size_t)p.K * R) : 0;
    L.xinit = (p.record & 2) ? take(sizeof(uint64_t) * (size_t)p.G * n) : 0;
    L.total = o;
    return PA_OK;
}

extern "C" pa_status pa_workspace_bytes(const pa_solver *s, const pa_schedule *sch, int32_t R,
                                        size_t *bytes)
{
    g_error[0] = 0;
    if (!bytes) return fail(PA_EINVAL, "pa_workspace_bytes: null output");
    pa_status st = check_schedule(s, sch, R);
    if (st != PA_OK) return st;
    Plan p;
    st = build_plan(const_cast<pa_solver *>(s), sch, R, p, false);
    if (st != PA_OK) return st;
    *bytes = p.L.total;
    return PA_OK;
}

// ------------------------------------------------------------------ run ----

// Hash (FNV-1a, 64 bit) of everything a run's results depend on: the graph,
// the schedule without its launch-shape fields, R, seed and instance.
static uint64_t fnv(uint64_t h, const void *p, size_t n)
{
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t q = 0; q < n; ++q) h = (h ^ b[q]) * 0x100000001B3ull;
    return h;
}

uint64_t pa_host::run_key(const pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                          uint32_t instance)
{
    uint64_t h = 0xCBF29CE484222325ull;
    h = fnv(h, &s->n, sizeof s->n);
    h = fnv(h, s->row_ptr.data(), sizeof(int) * s->row_ptr.size());
    h = fnv(h, s->col.data(), sizeof(int) * s->col.size());
    h = fnv(h, s->npos.data(), sizeof(int) * s->npos.size());
    const int32_t ints[] = {sch->n_steps, sch->sweeps_per_step, sch->as_enable, sch->as_stall_steps,
                            sch->as_max_level, sch->as_frozen_inv, sch->nl_period, sch->nl_kind,
                            sch->record, R, (int32_t)instance, sch->beta_adapt,
                            sch->beta_adapt ? sch->adapt_jump : 0, sch->beta_adapt ? sch->adapt_num : 0,
                            sch->beta_adapt ? sch->adapt_den : 0};
    h = fnv(h, ints, sizeof ints);
    h = fnv(h, &sch->as_gamma, sizeof sch->as_gamma);
    h = fnv(h, &seed, sizeof seed);
    h = fnv(h, sch->beta, sizeof(double) * (size_t)sch->n_steps);
    if (sch->order) h = fnv(h, sch->order, sizeof(int32_t) * (size_t)s->n);
    return h;
}

// Plan the run, upload the graph and tables into the workspace and set up the
// launch arguments. A fresh run also clears the state, draws the initial
// population and takes its best; a restored one leaves the state to the caller.
// `pinned`: the host inputs go through the solver's pinned staging buffer
// (allocated on first use); otherwise from a pageable host buffer, so that no
// pinned or device memory is allocated.
pa_status pa_host::start_run(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                             uint32_t instance, void *workspace, size_t workspace_bytes, void *stream,
                             bool fresh, bool pinned, const Shape *force)
{
    g_error[0] = 0;
    pa_status st = check_schedule(s, sch, R);
    if (st != PA_OK) return st;
    if (instance > 65535) return fail(PA_ERANGE, "instance=%u outside [0, 65535]", instance);
    if (!workspace) return fail(PA_EWORKSPACE, "workspace is null");
    if (((uintptr_t)workspace) % kAlign) return fail(PA_EWORKSPACE, "workspace must be 256-byte aligned");
    // The previous run may still be using its workspace (perhaps this one, from
    // another stream).
    if (s->has_run && s->stream) HIP_TRY(hipStreamSynchronize(s->stream));
    s->has_run = false;
    s->rc.valid = false;          // until this run's state is complete in the workspace
    Plan p;
    st = build_plan(s, sch, R, p, true, force);
    if (st != PA_OK) return st;
    if (workspace_bytes < p.L.total)
        return fail(PA_EWORKSPACE, "workspace of %zu bytes < %zu needed", workspace_bytes, p.L.total);

    s->plan = std::move(p);
    Plan &P = s->plan;
    const Layout &L = P.L;
    unsigned char *ws = static_cast<unsigned char *>(workspace);
    hipStream_t hs = static_cast<hipStream_t>(stream);
    s->ws = ws;
    s->stream = hs;
    HIP_TRY(hipGetDevice(&s->device));
    const int n = s->n;

    // All host inputs go to the device in one copy, through the pinned
    // staging buffer or a pageable one.
    unsigned char *stage = nullptr;
    if (pinned) {
        if (s->stage_pending) {
            HIP_TRY(hipEventSynchronize(s->stage_ev));
            s->stage_pending = false;
        }
        if (s->stage_cap < L.inputs_end) {
            if (s->stage) HIP_TRY(hipHostFree(s->stage));
            s->stage = nullptr;
            s->stage_cap = 0;
            HIP_TRY(hipHostMalloc(reinterpret_cast<void **>(&s->stage), L.inputs_end, hipHostMallocDefault));
            std::memset(s->stage, 0, L.inputs_end);
            s->stage_cap = L.inputs_end;
        }
        if (!s->stage_ev) HIP_TRY(hipEventCreateWithFlags(&s->stage_ev, hipEventDisableTiming));
        stage = s->stage;
    } else {
        s->stage_host.assign(L.inputs_end, 0);
        stage = s->stage_host.data();
    }
    auto put = [&](size_t off, const void *src, size_t bytes) {
        if (bytes) std::memcpy(stage + off, src, bytes);
    };
    put(L.row_ptr, s->row_ptr.data(), sizeof(int) * (n + 1));
    put(L.col, s->col.data(), sizeof(int) * s->nnz);
    put(L.npos, s->npos.data(), sizeof(int) * n);
    put(L.edges, s->edges.data(), sizeof(uint32_t) * s->edges.size());
    put(L.sched, P.sched.data(), sizeof(int) * n);
    put(L.level_off, P.level_off.data(), sizeof(int) * (P.n_levels + 1));
    put(L.blocks, P.blocks.data(), sizeof(uint32_t) * P.blocks.size());
    if (P.kind == 1)
        put(L.stream, P.rounds.data(), sizeof(int) * P.rounds.size());
    else
        put(L.stream, P.stream.data(), sizeof(int) * P.stream.size());
    put(L.qtab, P.qtab.data(), sizeof(uint64_t) * P.qtab.size());
    if (P.kind == 1)
        put(L.thr, P.thr32.data(), sizeof(uint32_t) * P.thr32.size());
    else
        put(L.thr, P.thr.data(), sizeof(uint64_t) * P.thr.size());
    put(L.wtab, P.wtab.data(), sizeof(uint64_t) * P.wtab.size());
    put(L.wtab_off, P.wtab_off.data(), sizeof(int) * P.K);
    put(L.wtab_len, P.wtab_len.data(), sizeof(int) * P.K);
    HIP_TRY(hipMemcpyAsync(ws, stage, L.inputs_end, hipMemcpyHostToDevice, hs));
    if (pinned) {
        HIP_TRY(hipEventRecord(s->stage_ev, hs));
        s->stage_pending = true;
    }

    auto U64 = [&](size_t off) { return reinterpret_cast<unsigned long long *>(ws + off); };
    if (fresh) {
        LAUNCH_TRY(pa::launch_fill_u64(U64(L.counters), 0ull, 2, hs));
        LAUNCH_TRY(pa::launch_fill_u64(U64(L.as_state), 0ull, 2, hs));
        LAUNCH_TRY(pa::launch_fill_u64(U64(L.best), 0ull, 4, hs));
        LAUNCH_TRY(pa::launch_fill_u64(U64(L.stats), 0ull, (long long)P.K * pa::kStatFields, hs));
        if (P.record & 1)
            LAUNCH_TRY(pa::launch_fill_u64(U64(L.counts), 0ull, ((long long)P.K * R + 1) / 2, hs));
    }

    pa::GraphDev gd;
    gd.n = n;
    gd.dmax = s->dmax;
    gd.row_ptr = reinterpret_cast<const int *>(ws + L.row_ptr);
    gd.col = reinterpret_cast<const int *>(ws + L.col);
    gd.npos = reinterpret_cast<const int *>(ws + L.npos);
    gd.edges = reinterpret_cast<const uint32_t *>(ws + L.edges);
    gd.ne = (int)s->edges.size();
    const uint32_t seed_lo = (uint32_t)seed, seed_hi = (uint32_t)(seed >> 32);

    size_t Xc = L.X0, Xn = L.X1, Ec = L.E0, En = L.E1;
    pa::InitArgs ia;
    ia.g = gd;
    ia.R = R;
    ia.G = P.G;
    ia.seed_lo = seed_lo;
    ia.seed_hi = seed_hi;
    ia.inst = instance;
    ia.X = reinterpret_cast<uint64_t *>(ws + Xc);
    ia.E = reinterpret_cast<int *>(ws + Ec);
    if (fresh) {
        LAUNCH_TRY(pa::launch_init(ia, hs));
        LAUNCH_TRY(pa::launch_energy(ia, hs));
        if (P.record & 2)
            HIP_TRY(hipMemcpyAsync(ws + L.xinit, ws + Xc, sizeof(uint64_t) * (size_t)P.G * n,
                                   hipMemcpyDeviceToDevice, hs));
    }

    pa::EpiArgs ea{};
    ea.R = R;
    ea.n = n;
    ea.nw32 = P.nw32;
    ea.nblk = P.nblk;
    ea.W = P.W;
    ea.K = P.K;
    ea.S = P.S;
    ea.as_enable = sch->as_enable;
    ea.as_stall = sch->as_stall_steps;
    ea.as_lmax = sch->as_enable ? sch->as_max_level : 0;
    ea.as_frozen_inv = sch->as_frozen_inv;
    ea.adapt = sch->beta_adapt;
    ea.adapt_jump = sch->adapt_jump;
    ea.adapt_num = sch->adapt_num;
    ea.adapt_den = sch->adapt_den;
    ea.as_state = reinterpret_cast<int *>(ws + L.as_state);
    ea.cand = U64(L.cand);
    ea.snap = reinterpret_cast<const uint32_t *>(ws + L.snap);
    ea.best = reinterpret_cast<int *>(ws + L.best);
    ea.best_x = reinterpret_cast<uint32_t *>(ws + L.best_x);
    ea.counters = U64(L.counters);
    ea.stats = reinterpret_cast<long long *>(ws + L.stats);
    ea.wtab = reinterpret_cast<const uint64_t *>(ws + L.wtab);
    ea.wtab_off = reinterpret_cast<const int *>(ws + L.wtab_off);
    ea.wtab_len = reinterpret_cast<const int *>(ws + L.wtab_len);
    ea.seed_lo = seed_lo;
    ea.seed_hi = seed_hi;
    ea.inst = instance;
    ea.parent = reinterpret_cast<int *>(ws + L.parent);
    ea.counts_rec = (P.record & 1) ? reinterpret_cast<int *>(ws + L.counts) : nullptr;

    // Best of the initial population.
    if (fresh) {
        pa::EpiArgs e0 = ea;
        e0.k = 0;
        e0.do_pop = 1;
        e0.pop_step = -1;
        e0.pop_sweep = -1;
        e0.E = reinterpret_cast<const int *>(ws + Ec);
        e0.X = reinterpret_cast<const uint64_t *>(ws + Xc);
        LAUNCH_TRY(pa::launch_epilogue(e0, hs));
    }

    pa::SweepArgs sa;
    sa.n = n;
    sa.dmax = s->dmax;
    sa.blocks = reinterpret_cast<const uint4 *>(ws + L.blocks);
    sa.block_u4 = P.block_bytes / 16;
    sa.stream = reinterpret_cast<const int2 *>(ws + L.stream);
    sa.qpad = P.qpad;
    sa.rounds = reinterpret_cast<const int4 *>(ws + L.stream);
    sa.n_rounds = P.n_rounds;
    sa.flush_every = P.flush_every;
    sa.direct = P.direct;
    sa.prio_mode = P.prio_mode;
    sa.R = R;
    sa.S = P.S;
    sa.lmax1 = P.lmax1;
    sa.n_levels = P.n_levels;
    sa.K = P.K;
    sa.adapt = sch->beta_adapt;
    sa.seed_lo = seed_lo;
    sa.seed_hi = seed_hi;
    sa.inst = instance;
    sa.sched = reinterpret_cast<const int *>(ws + L.sched);
    sa.level_off = reinterpret_cast<const int *>(ws + L.level_off);
    sa.thr = reinterpret_cast<const uint64_t *>(ws + L.thr);
    sa.thr32 = reinterpret_cast<const uint32_t *>(ws + L.thr);
    sa.as_state = reinterpret_cast<const int *>(ws + L.as_state);
    sa.best_E = reinterpret_cast<const int *>(ws + L.best);
    sa.cand = U64(L.cand);
    sa.snap = reinterpret_cast<uint32_t *>(ws + L.snap);
    sa.counters = U64(L.counters);
    sa.nw32 = P.nw32;
    sa.Xin = nullptr;
    sa.Ein = nullptr;
    sa.parent = nullptr;

    if (s->timing && pinned) {
        const size_t need = 2 * (size_t)P.K;
        while (s->ev.size() < need) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            s->ev.push_back(e);
        }
    }
    s->ev_first = 0;
    s->ev_used = 0;
    s->timing_run = pinned ? s->timing : 0;

    pa_solver::RunCtx &c = s->rc;
    c.valid = fresh;              // a restored run becomes valid once its state is loaded
    c.key = run_key(s, sch, R, seed, instance);
    c.next_step = 0;
    c.parents_pending = false;
    c.Xc = Xc; c.Xn = Xn; c.Ec = Ec; c.En = En;
    c.seed_lo = seed_lo; c.seed_hi = seed_hi; c.instance = instance;
    c.nl_period = sch->nl_period;
    c.nl_kind = sch->nl_kind;
    c.adapt = sch->beta_adapt;
    c.gd = gd;
    c.sa = sa;
    c.ea = ea;
    s->final_x = Xc;
    s->final_E = Ec;
    return PA_OK;
}

// Steps [k0, k1) of the run prepared by start_run (and any steps before k0).
static pa_status run_range(pa_solver *s, int k0, int k1)
{
    Plan &P = s->plan;
    const Layout &L = P.L;
    pa_solver::RunCtx &c = s->rc;
    unsigned char *ws = s->ws;
    hipStream_t hs = s->stream;
    const int n = s->n, R = P.R;
    const uint32_t seed_lo = c.seed_lo, seed_hi = c.seed_hi, instance = c.instance;
    const pa::GraphDev gd = c.gd;
    const pa::EpiArgs ea = c.ea;
    pa::SweepArgs sa = c.sa;
    size_t Xc = c.Xc, Xn = c.Xn, Ec = c.Ec, En = c.En;
    if (s->ev_used < k0) s->ev_first = k0;     // steps before k0 ran in another call or process
    c.valid = false;                           // until every step of the range is enqueued

    int stop = k1;
    if (s->fault_step >= k0 && s->fault_step < k1) stop = s->fault_step;
    for (int k = k0; k < stop; ++k) {
        if (c.adapt && k > 0 && (k - k0) % 64 == 0) {
            // Adaptive steps end at the last grid point, usually well before
            // step K: look every 64 steps and enqueue no more once it is done
            // (the remaining steps would do nothing).
            int g = 0;
            HIP_TRY(hipMemcpyAsync(&g, ws + L.as_state + 3 * sizeof(int), sizeof g, hipMemcpyDeviceToHost, hs));
            HIP_TRY(hipStreamSynchronize(hs));
            if (g >= P.K) break;
        }
        sa.k = k;
        // (the stride fixed when the run started, which sized the events)
        const bool timed = s->timing_run && k % s->timing_run == 0;
        if (timed) HIP_TRY(hipEventRecord(s->ev[2 * k], hs));
        if (P.kind == 1) {
            // Kernel 1 reads the previous population through the resampling
            // parents and writes the other buffer (no separate gather).
            sa.Xin = reinterpret_cast<const uint64_t *>(ws + Xc);
            sa.Ein = reinterpret_cast<const int *>(ws + Ec);
            sa.X = reinterpret_cast<uint64_t *>(ws + Xn);
            sa.E = reinterpret_cast<int *>(ws + En);
            sa.parent = c.parents_pending ? reinterpret_cast<const int *>(ws + L.parent) : nullptr;
            LAUNCH_TRY(pa::launch_sweep_bytes(P.W, P.bsg, P.threads, P.nblk, sa, hs));
            std::swap(Xc, Xn);
            std::swap(Ec, En);
            c.parents_pending = false;
        } else {
            sa.X = reinterpret_cast<uint64_t *>(ws + Xc);
            sa.E = reinterpret_cast<int *>(ws + Ec);
            LAUNCH_TRY(pa::launch_sweep(P.W, P.sgn, P.threads, P.nblk, sa, hs));
        }
        if (timed) HIP_TRY(hipEventRecord(s->ev[2 * k + 1], hs));
        if (s->timing_run) s->ev_used = k + 1;
        pa::EpiArgs e = ea;
        e.k = k;
        e.E = reinterpret_cast<const int *>(ws + Ec);
        e.X = reinterpret_cast<const uint64_t *>(ws + Xc);
        const bool nl = c.nl_period > 0 && (k + 1) % c.nl_period == 0;
        if (nl) {
            pa::EpiArgs e1 = e;
            e1.do_cand = 1;
            LAUNCH_TRY(pa::launch_epilogue(e1, hs));
            pa::IcmArgs ic;
            ic.g = gd;
            ic.R = R;
            ic.G = P.G;
            ic.k = k;
            ic.K = P.K;
            ic.adapt = c.adapt;
            ic.nw32 = P.nw32;
            ic.seed_lo = seed_lo;
            ic.seed_hi = seed_hi;
            ic.inst = instance;
            ic.X = reinterpret_cast<uint64_t *>(ws + Xc);
            ic.E = reinterpret_cast<int *>(ws + Ec);
            ic.vout = reinterpret_cast<uint32_t *>(ws + L.vout);
            ic.kind = c.nl_kind;
            ic.lmax1 = P.lmax1;
            ic.qtab = reinterpret_cast<const uint64_t *>(ws + L.qtab);
            ic.as_state = reinterpret_cast<const int *>(ws + L.as_state);
            LAUNCH_TRY(pa::launch_icm(ic, hs));
            e.do_pop = 1;
            e.pop_step = k;
            e.pop_sweep = P.S;
            e.do_rest = 1;
        } else {
            e.do_cand = 1;
            e.do_rest = 1;
        }
        LAUNCH_TRY(pa::launch_epilogue(e, hs));
        if (P.kind == 1 && k + 1 < P.K) c.parents_pending = true;
        if (P.kind == 2 && k + 1 < P.K) {
            pa::GatherArgs ga;
            ga.n = n;
            ga.R = R;
            ga.G = P.G;
            ga.parent = reinterpret_cast<const int *>(ws + L.parent);
            ga.Xin = reinterpret_cast<const uint64_t *>(ws + Xc);
            ga.Xout = reinterpret_cast<uint64_t *>(ws + Xn);
            ga.Ein = reinterpret_cast<const int *>(ws + Ec);
            ga.Eout = reinterpret_cast<int *>(ws + En);
            LAUNCH_TRY(pa::launch_gather(ga, hs));
            std::swap(Xc, Xn);
            std::swap(Ec, En);
        }
    }
    c.Xc = Xc; c.Xn = Xn; c.Ec = Ec; c.En = En;
    c.next_step = stop;
    c.valid = true;
    s->final_x = Xc;
    s->final_E = Ec;
    s->has_run = true;
    if (stop < k1) {
        // Injected fault: the steps before it are enqueued and the run can
        // continue from it.
        s->fault_step = -1;
        HIP_TRY(hipStreamSynchronize(hs));
        return fail(PA_EABORTED, "run stopped before step %d by pa_set_fault_step", stop);
    }
    return PA_OK;
}

extern "C" pa_status pa_set_fault_step(pa_solver *s, int32_t k)
{
    g_error[0] = 0;
    if (!s) return fail(PA_EINVAL, "null solver");
    if (k < -1) return fail(PA_EINVAL, "fault step %d < -1", k);
    s->fault_step = k;
    return PA_OK;
}

extern "C" pa_status pa_run_steps(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                                  uint32_t instance, int32_t k_begin, int32_t k_end, void *workspace,
                                  size_t workspace_bytes, void *stream)
{
    g_error[0] = 0;
    if (!s) return fail(PA_EINVAL, "null solver");
    pa_status st = check_schedule(s, sch, R);
    if (st != PA_OK) return st;
    if (instance > 65535) return fail(PA_ERANGE, "instance=%u outside [0, 65535]", instance);
    if (k_begin < 0 || k_end < k_begin || k_end > sch->n_steps)
        return fail(PA_EINVAL, "steps [%d, %d) outside the schedule's [0, %d]", k_begin, k_end, sch->n_steps);
    if (k_begin == 0) {
        st = start_run(s, sch, R, seed, instance, workspace, workspace_bytes, stream, true);
        if (st != PA_OK) return st;
    } else {
        const pa_solver::RunCtx &c = s->rc;
        if (!c.valid || c.key != run_key(s, sch, R, seed, instance))
            return fail(PA_ESTATE, "no run of this schedule, R, seed and instance to continue");
        if (c.next_step != k_begin)
            return fail(PA_ESTATE, "the run in the workspace continues at step %d, not %d", c.next_step, k_begin);
        if (workspace != s->ws) return fail(PA_EWORKSPACE, "a run continues in its own workspace");
        if (stream != (void *)s->stream) {
            // The previous steps were enqueued on another stream: order after them.
            HIP_TRY(hipStreamSynchronize(s->stream));
            s->stream = static_cast<hipStream_t>(stream);
        }
    }
    return run_range(s, k_begin, k_end);
}

extern "C" pa_status pa_run(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                            uint32_t instance, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!sch) {
        g_error[0] = 0;
        return fail(PA_EINVAL, "null schedule");
    }
    return pa_run_steps(s, sch, R, seed, instance, 0, sch->n_steps, workspace, workspace_bytes, stream);
}

extern "C" pa_status pa_run_static(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                                   uint32_t instance, void *stream)
{
    g_error[0] = 0;
    pa_status st = check_schedule(s, sch, R);
    if (st != PA_OK) return st;
    if (instance > 65535) return fail(PA_ERANGE, "instance=%u outside [0, 65535]", instance);
    Plan p;
    st = build_plan(s, sch, R, p, false);
    if (st != PA_OK) return st;
    if (p.L.total > pa::kStaticScratchBytes)
        return fail(PA_EWORKSPACE, "run needs %zu workspace bytes, more than the %zu of the static "
                                   "workspace: use pa_run with a workspace", p.L.total,
                    (size_t)pa::kStaticScratchBytes);
    void *ws = nullptr;
    if (pa::static_scratch(&ws) != 0) return fail(PA_EDEVICE, "%s", pa::last_hip_error());
    st = start_run(s, sch, R, seed, instance, ws, pa::kStaticScratchBytes, stream, true, false);
    if (st != PA_OK) return st;
    return run_range(s, 0, sch->n_steps);
}

// -------------------------------------------------------------- results ----

static pa_status fetch(pa_solver *s, void *dst, size_t off, size_t bytes)
{
    if (!s || !s->has_run) return fail(PA_ESTATE, "no completed pa_run on this solver");
    HIP_TRY(hipSetDevice(s->device));
    HIP_TRY(hipMemcpyAsync(dst, s->ws + off, bytes, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return PA_OK;
}

extern "C" pa_status pa_best_info(pa_solver *s, int64_t out[4])
{
    if (!out) return fail(PA_EINVAL, "null output");
    int b[8];
    pa_status st = fetch(s, b, s ? s->plan.L.best : 0, sizeof b);
    if (st != PA_OK) return st;
    for (int q = 0; q < 4; ++q) out[q] = b[q];
    return PA_OK;
}

extern "C" pa_status pa_build_tables(const pa_schedule *sch, int32_t d_max, int32_t e_span,
                                     void *out, size_t *bytes)
{
    g_error[0] = 0;
    if (!sch || !bytes || !sch->beta) return fail(PA_EINVAL, "pa_build_tables: null argument");
    if (sch->n_steps < 1) return fail(PA_EINVAL, "pa_build_tables: n_steps must be >= 1");
    if (d_max < 0 || e_span < 0) return fail(PA_EINVAL, "pa_build_tables: negative size");
    if (d_max > kMaxDegree || e_span > (1 << 26))
        return fail(PA_ERANGE, "pa_build_tables: d_max or e_span too large");
    for (int k = 0; k < sch->n_steps; ++k) {
        const double b = sch->beta[k];
        if (!std::isfinite(b) || b < 0 || (k > 0 && b < sch->beta[k - 1]))
            return fail(PA_EINVAL, "pa_build_tables: beta must be finite, >= 0 and non-decreasing");
    }
    if (sch->as_enable && (sch->as_max_level < 0 || sch->as_max_level > 15 || !(sch->as_gamma > 0) ||
                           sch->as_gamma > 1))
        return fail(PA_EINVAL, "pa_build_tables: noise levels need 0 <= as_max_level <= 15, 0 < gamma <= 1");
    if (sch->beta_adapt && uneven_grid(sch->beta, sch->n_steps) >= 0)
        return fail(PA_EINVAL, "pa_build_tables: adaptive steps need an evenly spaced beta grid");
    const int K = sch->n_steps, Lv = sch->as_enable ? sch->as_max_level + 1 : 1, D = d_max + 1;
    const int n_tab = sch->beta_adapt ? std::min(std::max(sch->adapt_jump, 1), K - 1) : K - 1;
    const size_t n_thr = (size_t)K * Lv * D, n_w = (size_t)n_tab * (size_t)(e_span + 1);
    const size_t need = 8 * (n_thr + n_w);
    if (!out) {
        *bytes = need;
        return PA_OK;
    }
    if (*bytes < need) return fail(PA_ERANGE, "pa_build_tables: %zu bytes < %zu needed", *bytes, need);
    *bytes = need;
    uint64_t *o = static_cast<uint64_t *>(out);
    for (int k = 0; k < K; ++k) {
        double g = 1.0;
        for (int l = 0; l < Lv; ++l) {
            const double b = sch->beta[k] * g;
            uint64_t *row = o + ((size_t)k * Lv + l) * D;
            row[0] = 1ull << 32;
            for (int m = 1; m < D; ++m) row[m] = threshold_fixed(b, m);
            g = g * sch->as_gamma;
        }
    }
    uint64_t *wt = o + n_thr;
    for (int k = 0; k < n_tab; ++k) {
        const double db = sch->beta_adapt ? sch->beta[k + 1] - sch->beta[0] : sch->beta[k + 1] - sch->beta[k];
        for (int m = 0; m <= e_span; ++m) wt[(size_t)k * (e_span + 1) + m] = weight_fixed(db, m);
    }
    return PA_OK;
}

extern "C" pa_status pa_run_batch(const pa_batch_run *runs, int32_t count, void *const *streams,
                                  int32_t n_streams)
{
    g_error[0] = 0;
    if (!runs || !streams || count < 1 || n_streams < 1)
        return fail(PA_EINVAL, "pa_run_batch: null array, count < 1 or n_streams < 1");
    std::vector<const pa_solver *> seen;
    seen.reserve(count);
    for (int i = 0; i < count; ++i) {
        if (!runs[i].solver) return fail(PA_EINVAL, "pa_run_batch: run %d has no solver", i);
        seen.push_back(runs[i].solver);
    }
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
        return fail(PA_EINVAL, "pa_run_batch: a solver appears in two runs");
    auto failed = [&](int i, pa_status st) {
        char msg[sizeof g_error];
        std::snprintf(msg, sizeof msg, "%s", g_error);
        return fail(st, "pa_run_batch: run %d: %s", i, msg);
    };
    bool adaptive = false;
    for (int i = 0; i < count; ++i) adaptive |= runs[i].schedule && runs[i].schedule->beta_adapt;
    if (!adaptive) {
        for (int i = 0; i < count; ++i) {
            const pa_batch_run &r = runs[i];
            const pa_status st = pa_run(r.solver, r.schedule, r.R, r.seed, r.instance, r.workspace,
                                        r.workspace_bytes, streams[i % n_streams]);
            if (st != PA_OK) return failed(i, st);
        }
        return PA_OK;
    }
    // An adaptive run's host looks at its grid point every 64 steps and waits
    // for the device there. Every run is started first, then the steps go in
    // chunks of 64, one chunk of each run in turn, so that while the host
    // waits on one run the chunks of the others are already queued.
    int kmax = 0;
    for (int i = 0; i < count; ++i) {
        const pa_batch_run &r = runs[i];
        const pa_status st = pa_run_steps(r.solver, r.schedule, r.R, r.seed, r.instance, 0, 0, r.workspace,
                                          r.workspace_bytes, streams[i % n_streams]);
        if (st != PA_OK) return failed(i, st);
        kmax = std::max(kmax, r.schedule->n_steps);
    }
    constexpr int kChunk = 64;
    for (int k0 = 0; k0 < kmax; k0 += kChunk)
        for (int i = 0; i < count; ++i) {
            const pa_batch_run &r = runs[i];
            const int K = r.schedule->n_steps;
            if (k0 >= K) continue;
            const pa_status st = pa_run_steps(r.solver, r.schedule, r.R, r.seed, r.instance, k0,
                                              std::min(k0 + kChunk, K), r.workspace, r.workspace_bytes,
                                              streams[i % n_streams]);
            if (st != PA_OK) return failed(i, st);
        }
    return PA_OK;
}

extern "C" pa_status pa_best_cut(pa_solver *s, int64_t *cut, int32_t *energy)
{
    int64_t info[4];
    pa_status st = pa_best_info(s, info);
    if (st != PA_OK) return st;
    if (cut) *cut = (s->w_tot - info[0]) / 2;
    if (energy) *energy = (int32_t)info[0];
    return PA_OK;
}

extern "C" pa_status pa_best_config(pa_solver *s, int8_t *x)
{
    if (!x) return fail(PA_EINVAL, "null output");
    if (!s || !s->has_run) return fail(PA_ESTATE, "no completed pa_run on this solver");
    std::vector<uint32_t> bits(s->plan.nw32);
    pa_status st = fetch(s, bits.data(), s->plan.L.best_x, sizeof(uint32_t) * bits.size());
    if (st != PA_OK) return st;
    for (int i = 0; i < s->n; ++i) x[i] = ((bits[i >> 5] >> (i & 31)) & 1u) ? 1 : -1;
    return PA_OK;
}

extern "C" pa_status pa_best_config_hex(pa_solver *s, char *buf, size_t len)
{
    if (!buf) return fail(PA_EINVAL, "null output");
    if (!s || !s->has_run) return fail(PA_ESTATE, "no completed pa_run on this solver");
    const size_t digits = ((size_t)s->n + 3) / 4;
    if (len < digits + 1) return fail(PA_ERANGE, "hex buffer of %zu bytes < %zu needed", len, digits + 1);
    std::vector<int8_t> x(s->n);
    pa_status st = pa_best_config(s, x.data());
    if (st != PA_OK) return st;
    static const char hexd[] = "0123456789abcdef";
    for (size_t p = 0; p < digits; ++p) {
        int v = 0;
        for (int q = 0; q < 4; ++q) {
            const size_t i = 4 * p + q;
            v = (v << 1) | ((i < (size_t)s->n && x[i] > 0) ? 1 : 0);
        }
        buf[p] = hexd[v];
    }
    buf[digits] = 0;
    return PA_OK;
}

static void unpack_population(const std::vector<uint64_t> &X, int n, int R, int8_t *x)
{
    for (int r = 0; r < R; ++r) {
        const uint64_t *Xg = &X[(size_t)(r >> 6) * n];
        const int b = r & 63;
        int8_t *xr = x + (size_t)r * n;
        for (int i = 0; i < n; ++i) xr[i] = ((Xg[i] >> b) & 1ull) ? 1 : -1;
    }
}

extern "C" pa_status pa_get_population(pa_solver *s, int8_t *x, int16_t *h, int32_t *E)
{
    if (!s || !s->has_run) return fail(PA_ESTATE, "no completed pa_run on this solver");
    const Plan &P = s->plan;
    const int n = s->n;
    // After a range that stopped before the last step, kernel 1 still holds
    // the population of the next step as the current buffer read through the
    // resampling parents: apply them here.
    std::vector<int> parent;
    if (s->rc.parents_pending) {
        parent.resize(P.R);
        pa_status st = fetch(s, parent.data(), P.L.parent, sizeof(int) * P.R);
        if (st != PA_OK) return st;
    }
    if (x || h) {
        std::vector<uint64_t> X((size_t)P.G * n);
        pa_status st = fetch(s, X.data(), s->final_x, sizeof(uint64_t) * X.size());
        if (st != PA_OK) return st;
        std::vector<int8_t> own;
        int8_t *xs = x;
        if (!xs) {
            own.resize((size_t)P.R * n);
            xs = own.data();
        }
        if (parent.empty()) {
            unpack_population(X, n, P.R, xs);
        } else {
            std::vector<int8_t> all((size_t)P.R * n);
            unpack_population(X, n, P.R, all.data());
            for (int r = 0; r < P.R; ++r)
                std::memcpy(xs + (size_t)r * n, all.data() + (size_t)parent[r] * n, (size_t)n);
        }
        if (h) {
            // The device keeps no fields: h_i = sum_j w_ij x_j from the spins
            // (the positive neighbours of a row come first).
            parallel_rows(P.R, (long long)P.R * s->nnz, [&](int r0, int r1) {
                for (int r = r0; r < r1; ++r) {
                    const int8_t *xr = xs + (size_t)r * n;
                    int16_t *hr = h + (size_t)r * n;
                    for (int i = 0; i < n; ++i) {
                        const int e0 = s->row_ptr[i], e1 = s->row_ptr[i + 1], em = e0 + s->npos[i];
                        int acc = 0;
                        for (int e = e0; e < em; ++e) acc += xr[s->col[e]];
                        for (int e = em; e < e1; ++e) acc -= xr[s->col[e]];
                        hr[i] = (int16_t)acc;
                    }
                }
            });
        }
    }
    if (E) {
        std::vector<int> Eall(P.R);
        pa_status st = fetch(s, Eall.data(), s->final_E, sizeof(int) * P.R);
        if (st != PA_OK) return st;
        for (int r = 0; r < P.R; ++r) E[r] = Eall[parent.empty() ? r : parent[r]];
    }
    return PA_OK;
}

extern "C" pa_status pa_get_initial_population(pa_solver *s, int8_t *x)
{
    if (!x) return fail(PA_EINVAL, "null output");
    if (!s || !s->has_run) return fail(PA_ESTATE, "no completed pa_run on this solver");
    const Plan &P = s->plan;
    if (!(P.record & 2)) return fail(PA_ESTATE, "run did not record the initial population (record bit 1)");
    std::vector<uint64_t> X((size_t)P.G * s->n);
    pa_status st = fetch(s, X.data(), P.L.xinit, sizeof(uint64_t) * X.size());
    if (st != PA_OK) return st;
    unpack_population(X, s->n, P.R, x);
    return PA_OK;
}

extern "C" pa_status pa_get_step_stats(pa_solver *s, int64_t *out)
{
    if (!out) return fail(PA_EINVAL, "null output");
    if (!s || !s->has_run) return fail(PA_ESTATE, "no completed pa_run on this solver");
    return fetch(s, out, s->plan.L.stats, sizeof(long long) * (size_t)s->plan.K * pa::kStatFields);
}

extern "C" pa_status pa_get_counts(pa_solver *s, int32_t *out)
{
    if (!out) return fail(PA_EINVAL, "null output");
    if (!s || !s->has_run) return fail(PA_ESTATE, "no completed pa_run on this solver");
    if (!(s->plan.record & 1)) return fail(PA_ESTATE, "run did not record copy counts (record bit 0)");
    return fetch(s, out, s->plan.L.counts, sizeof(int) * (size_t)s->plan.K * s->plan.R);
}

extern "C" pa_status pa_get_launch_info(pa_solver *s, int64_t out[8])
{
    if (!out) return fail(PA_EINVAL, "null output");
    if (!s || !s->has_run) return fail(PA_ESTATE, "no completed pa_run on this solver");
    const Plan &P = s->plan;
    out[0] = P.kind;
    out[1] = P.W;
    out[2] = P.threads;
    out[3] = P.nblk;
    out[4] = P.kind == 1 ? pa::sweep_bytes_lds(P.W, P.bsg == 1 ? 1 : 0, s->n, s->dmax)
                         : pa::sweep_lds_bytes(P.W, P.sgn, s->n, s->dmax, P.threads);
    out[5] = P.n_levels;
    out[6] = P.kind == 1 ? P.n_rounds : P.qpad - 4;
    out[7] = P.K;
    return PA_OK;
}

// ------------------------------------------------------------ checkpoint ----

namespace {
struct CkptHeader {
    char magic[8];
    uint64_t key;
    uint64_t bytes;
    int32_t n, R, K, G, nw32, next_step, record, version;
};
constexpr char kCkptMagic[8] = {'P', 'A', 'C', 'K', 'P', 'T', '0', '1'};

// Device regions of the state between steps, in blob order.
struct CkptPart {
    size_t off, bytes;
};

std::vector<CkptPart> ckpt_parts(const pa_solver *s)
{
    const Plan &P = s->plan;
    const Layout &L = P.L;
    std::vector<CkptPart> v;
    v.push_back({s->rc.Xc, sizeof(uint64_t) * (size_t)P.G * s->n});
    v.push_back({s->rc.Ec, sizeof(int) * (size_t)P.R});
    v.push_back({L.as_state, sizeof(int) * 4});
    v.push_back({L.best, sizeof(int) * 8});
    v.push_back({L.counters, sizeof(uint64_t) * 2});
    v.push_back({L.best_x, sizeof(uint32_t) * (size_t)P.nw32});
    v.push_back({L.stats, sizeof(long long) * (size_t)P.K * pa::kStatFields});
    if (P.record & 1) v.push_back({L.counts, sizeof(int) * (size_t)P.K * P.R});
    if (P.record & 2) v.push_back({L.xinit, sizeof(uint64_t) * (size_t)P.G * s->n});
    return v;
}

size_t ckpt_bytes(const std::vector<CkptPart> &parts)
{
    size_t b = sizeof(CkptHeader);
    for (const CkptPart &q : parts) b += (q.bytes + 7) & ~size_t(7);
    return b;
}
}  // namespace

extern "C" pa_status pa_checkpoint_bytes(const pa_solver *s, size_t *bytes)
{
    g_error[0] = 0;
    if (!s || !bytes) return fail(PA_EINVAL, "pa_checkpoint_bytes: null argument");
    if (!s->rc.valid || !s->has_run) return fail(PA_ESTATE, "no run on this solver to checkpoint");
    *bytes = ckpt_bytes(ckpt_parts(s));
    return PA_OK;
}

extern "C" pa_status pa_checkpoint_save(pa_solver *s, void *out, size_t bytes)
{
    g_error[0] = 0;
    if (!s || !out) return fail(PA_EINVAL, "pa_checkpoint_save: null argument");
    if (!s->rc.valid || !s->has_run) return fail(PA_ESTATE, "no run on this solver to checkpoint");
    pa_solver::RunCtx &c = s->rc;
    const Plan &P = s->plan;
    if (bytes < ckpt_bytes(ckpt_parts(s)))
        return fail(PA_EINVAL, "checkpoint buffer of %zu bytes < %zu", bytes, ckpt_bytes(ckpt_parts(s)));
    HIP_TRY(hipSetDevice(s->device));
    if (c.parents_pending) {
        // Store the population itself: copy it through the parent list into
        // the other buffer, which becomes the current one.
        pa::GatherArgs ga;
        ga.n = s->n;
        ga.R = P.R;
        ga.G = P.G;
        ga.parent = reinterpret_cast<const int *>(s->ws + P.L.parent);
        ga.Xin = reinterpret_cast<const uint64_t *>(s->ws + c.Xc);
        ga.Xout = reinterpret_cast<uint64_t *>(s->ws + c.Xn);
        ga.Ein = reinterpret_cast<const int *>(s->ws + c.Ec);
        ga.Eout = reinterpret_cast<int *>(s->ws + c.En);
        LAUNCH_TRY(pa::launch_gather(ga, s->stream));
        std::swap(c.Xc, c.Xn);
        std::swap(c.Ec, c.En);
        c.parents_pending = false;
        s->final_x = c.Xc;
        s->final_E = c.Ec;
    }
    const std::vector<CkptPart> parts = ckpt_parts(s);
    unsigned char *o = static_cast<unsigned char *>(out);
    CkptHeader h;
    std::memcpy(h.magic, kCkptMagic, 8);
    h.key = c.key;
    h.bytes = ckpt_bytes(parts);
    h.n = s->n;
    h.R = P.R;
    h.K = P.K;
    h.G = P.G;
    h.nw32 = P.nw32;
    h.next_step = c.next_step;
    h.record = P.record;
    h.version = 1;
    std::memcpy(o, &h, sizeof h);
    size_t at = sizeof h;
    for (const CkptPart &q : parts) {
        HIP_TRY(hipMemcpyAsync(o + at, s->ws + q.off, q.bytes, hipMemcpyDeviceToHost, s->stream));
        at += (q.bytes + 7) & ~size_t(7);
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return PA_OK;
}

extern "C" pa_status pa_checkpoint_load(pa_solver *s, const pa_schedule *sch, int32_t R, uint64_t seed,
                                        uint32_t instance, const void *in, size_t bytes, void *workspace,
                                        size_t workspace_bytes, void *stream)
{
    g_error[0] = 0;
    if (!s || !sch || !in) return fail(PA_EINVAL, "pa_checkpoint_load: null argument");
    pa_status st = check_schedule(s, sch, R);
    if (st != PA_OK) return st;
    if (instance > 65535) return fail(PA_ERANGE, "instance=%u outside [0, 65535]", instance);
    CkptHeader h;
    if (bytes < sizeof h) return fail(PA_EINVAL, "checkpoint of %zu bytes is too short", bytes);
    std::memcpy(&h, in, sizeof h);
    if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 1)
        return fail(PA_EINVAL, "not a checkpoint of this library");
    if (h.bytes > bytes) return fail(PA_EINVAL, "checkpoint truncated: %zu of %llu bytes", bytes,
                                     (unsigned long long)h.bytes);
    if (h.key != run_key(s, sch, R, seed, instance) || h.n != s->n || h.R != R || h.K != sch->n_steps ||
        h.record != sch->record)
        return fail(PA_EINVAL, "checkpoint belongs to another graph, schedule, population, seed or instance");
    if (h.next_step < 0 || h.next_step > h.K) return fail(PA_EINVAL, "checkpoint step %d outside the schedule", h.next_step);
    st = start_run(s, sch, R, seed, instance, workspace, workspace_bytes, stream, false);
    if (st != PA_OK) return st;
    const std::vector<CkptPart> parts = ckpt_parts(s);
    if (ckpt_bytes(parts) != h.bytes || h.G != s->plan.G || h.nw32 != s->plan.nw32)
        return fail(PA_EINVAL, "checkpoint layout does not match this run");
    const unsigned char *p = static_cast<const unsigned char *>(in);
    size_t at = sizeof h;
    for (const CkptPart &q : parts) {
        HIP_TRY(hipMemcpyAsync(s->ws + q.off, p + at, q.bytes, hipMemcpyHostToDevice, s->stream));
        at += (q.bytes + 7) & ~size_t(7);
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->rc.valid = true;
    s->rc.next_step = h.next_step;
    s->rc.parents_pending = false;
    s->ev_first = s->ev_used = h.next_step;
    s->has_run = true;
    return PA_OK;
}

extern "C" pa_status pa_set_timing(pa_solver *s, int32_t on)
{
    if (!s) return fail(PA_EINVAL, "null solver");
    if (on < 0) return fail(PA_EINVAL, "timing stride must be >= 0");
    s->timing = on;
    return PA_OK;
}

extern "C" pa_status pa_get_sweep_time(pa_solver *s, double *ms, int64_t *launches)
{
    if (!s || !s->has_run) return fail(PA_ESTATE, "no completed pa_run on this solver");
    const int stride = s->timing_run;
    if (!stride) return fail(PA_ESTATE, "timing mode was off during the run");
    HIP_TRY(hipStreamSynchronize(s->stream));
    double tot = 0.0;
    int64_t count = 0;
    for (int k = s->ev_first; k < s->ev_used; ++k) {
        if (k % stride) continue;
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, s->ev[2 * k], s->ev[2 * k + 1]));
        tot += t;
        ++count;
    }
    if (ms) *ms = tot;
    if (launches) *launches = count;
    return PA_OK;
}
