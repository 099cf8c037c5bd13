// pa_kernels.hip -- gfx950 kernels of the population-annealing Max-Cut engine.
//
// Paper: arXiv 2510.21105. Objective eq. (1) (section 1), Ising mapping with
// J_ij = -w_ij (section 2), population annealing with adaptive stochasticity
// and non-local moves (abstract, section 3). Everything here is integer: the
// FP64 Metropolis thresholds and resampling weights arrive as fixed-point
// tables built on the host.
//
// Design (MI355X): the population lives bit-packed in HBM, 64 replicas per
// 64-bit word per node. A sweep kernel workgroup owns W replicas for a whole
// temperature step: it loads their spins into LDS, runs all S sweeps there and
// writes them back once, so the sweeps never touch HBM. Local fields are
// recomputed from the neighbours' spins (one LDS read per neighbour, no stored
// field array). The workgroup's lanes cover the nodes of one dependency level
// of the sweep order at a time (those nodes are pairwise non-adjacent), with a
// barrier between levels -- the same result as the sequential sweep.
//
//   sweep_bytes_kernel (kernel 1, default): one lane = one node for all W = 4,
//     8 or 16 replicas, spins as byte records, bytewise neighbour counts.
//   sweep_kernel (kernel 2): one lane = one replica, W = 16, 32 or 64 replicas
//     as bit words; for degrees above 127 and as an independent check.
//   epilogue_kernel: best tracking, noise level, the adaptive step's jump,
//     reweighting and systematic resampling of a step (one workgroup).
//   icm_kernel / icm_apply_kernel: the cluster move on replica pairs;
//     wolff_kernel (+ icm_apply_kernel): the single-replica cluster update.
//   gather_kernel: resampling copies for kernel 2 (kernel 1 reads through the
//     parent list itself).
#include <hip/hip_runtime.h>

#include <mutex>

#include "pa_device.h"

namespace pa {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 products with multipliers 0xD2511F53 / 0xCD9E8D57 and a Weyl key
// schedule 0x9E3779B9 / 0xBB67AE85. Each product is one 64-bit multiply (a
// single v_mad_u64_u32 gives both halves) and the two XORs of an output word
// are one 3-input bit operation (0x96 = a ^ b ^ c).
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        c = U4{(uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.y, k0, 0x96),
               (uint32_t)p1,
               (uint32_t)__builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w, k1, 0x96),
               (uint32_t)p0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Word (r & 3) of Philox(key = seed, ctr = (i, s | tag << 16, k, (r >> 2) | inst << 16)).
__device__ __forceinline__ uint32_t draw(uint32_t seed_lo, uint32_t seed_hi, uint32_t inst,
                                         uint32_t tag, uint32_t s, uint32_t k, uint32_t i,
                                         uint32_t r)
{
    const U4 o = philox10(U4{i, s | (tag << 16), k, (r >> 2) | (inst << 16)}, seed_lo, seed_hi);
    const uint32_t q = r & 3u;
    return q == 0 ? o.x : (q == 1 ? o.y : (q == 2 ? o.z : o.w));
}

// ---------------------------------------------------------------------------
// Small wave / block reductions (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long wave_sum_ll(long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_xor(v, o, 64);
        v = t < v ? t : v;
    }
    return v;
}

// Block-wide reductions for blockDim.x a multiple of 64 (<= 1024). `red`
// is >= 16 entries of shared scratch. Every thread gets the result.
__device__ unsigned long long block_min_u64(unsigned long long v, unsigned long long *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_min_u64(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    unsigned long long r = red[0];
    for (int w = 1; w < nw; ++w) r = red[w] < r ? red[w] : r;
    __syncthreads();
    return r;
}

__device__ long long block_sum_ll(long long v, long long *red)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum_ll(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    long long r = 0;
    for (int w = 0; w < nw; ++w) r += red[w];
    __syncthreads();
    return r;
}

__host__ __device__ constexpr size_t align16(size_t b) { return (b + 15) & ~size_t(15); }

// ---------------------------------------------------------------------------
// Initial population: x_i^r = +1 iff bit 0 of draw(1, 0, 0, i, r).
// One wave per (group, node chunk); the ballot of the 64 lanes is the word.
// ---------------------------------------------------------------------------
constexpr int kInitNodesPerWave = 16;

__global__ __launch_bounds__(256) void init_kernel(InitArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = blockIdx.y;
    const int r = g * 64 + lane;
    const int i0 = (blockIdx.x * 4 + wave) * kInitNodesPerWave;
    for (int t = 0; t < kInitNodesPerWave; ++t) {
        const int i = i0 + t;
        if (i >= a.g.n) break;
        const int bit = r < a.R ? (int)(draw(a.seed_lo, a.seed_hi, a.inst, 1, 0, 0, (uint32_t)i,
                                             (uint32_t)r) & 1u)
                                : 0;
        const unsigned long long mask = __ballot(bit);
        if (lane == 0) a.X[(size_t)g * a.g.n + i] = mask;
    }
}

// E_r = sum_{i<j} w_ij x_i x_j from the bit-packed population (E zeroed first).
__global__ __launch_bounds__(256) void energy_kernel(InitArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = blockIdx.y;
    const int r = g * 64 + lane;
    const int n = a.g.n;
    const uint64_t *Xg = a.X + (size_t)g * n;
    const int i0 = (blockIdx.x * 4 + wave) * kInitNodesPerWave;
    int acc = 0;
    for (int t = 0; t < kInitNodesPerWave; ++t) {
        const int i = i0 + t;
        if (i >= n) break;
        const int bi = (int)((Xg[i] >> lane) & 1ull);
        const int e0 = a.g.row_ptr[i], e1 = a.g.row_ptr[i + 1], em = e0 + a.g.npos[i];
        for (int e = e0; e < e1; ++e) {
            const int j = a.g.col[e];
            if (j <= i) continue;
            const int bj = (int)((Xg[j] >> lane) & 1ull);
            const int neg = e >= em;
            acc += 1 - 2 * (bi ^ bj ^ neg);
        }
    }
    if (r < a.R && acc != 0) atomicAdd(&a.E[r], acc);
}

// ---------------------------------------------------------------------------
// Sweep kernel: all S sweeps of one step for W replicas per workgroup.
//
// LDS (dynamic, starting at LDS address 0 -- the kernel declares no static
// LDS, so the host can hand out raw LDS byte offsets) holds one W-bit spin
// word per node, for graphs with negative weights a complemented copy (so a
// negative edge reads "w_ij x_j = +1" directly), one always-zero word that
// padded adjacency entries point to, the step's threshold row, the
// level-ordered node list and a per-wave buffer of Philox draws.
//
// The host lays the adjacency out as one fixed-size block per schedule slot:
// u32 {LDS byte offset of the node's word, degree, node id, 0} followed by
// the LDS byte offsets of the neighbours' words, padded with the zero word.
// Every wave gets its stream of passes (first slot, largest degree among the
// pass's 64/W slots); a pass keeps its block in registers, loaded one pass
// ahead, so a neighbour costs one LDS read, one bit extract and half an add.
//
// Draws: one Philox call gives the draws of 4 consecutive replicas at one
// node, so every fourth pass each of the 64 lanes computes one call for the
// wave's next 4 passes and parks the 4 words in LDS; a pass then reads one
// word per lane.
// ---------------------------------------------------------------------------
struct SweepLds {
    size_t xs, thr, part, eblk, misc, sched, draws, total;
};

__host__ __device__ inline SweepLds sweep_lds_layout(int W, int sgn, int n, int dmax, int nwaves)
{
    SweepLds L;
    const size_t words = (size_t)(sgn ? 2 * n : n) + 1;
    L.xs = 0;
    L.thr = align16(words * (size_t)(W / 8));
    L.part = L.thr + align16((size_t)(dmax + 1) * 8);
    L.eblk = L.part + (size_t)kMaxThreads * 4;
    L.misc = L.eblk + 64 * 4;
    L.sched = L.misc + 16 * 8;
    L.draws = L.sched + align16((size_t)n * 2);
    L.total = L.draws + (size_t)nwaves * 256 * 4;
    return L;
}

int sweep_lds_bytes(int W, int sgn, int n, int dmax, int threads)
{
    return (int)sweep_lds_layout(W, sgn, n, dmax, threads / 64).total;
}

typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// Spin words in LDS, addressed by byte offset. For W = 64 a lane reads the
// 32-bit half that holds its replica (lanes 32..63: offset + 4).
template <int W>
__device__ __forceinline__ uint32_t lds_word(uint32_t off)
{
    if constexpr (W == 16) return *(lds_u16 *)(uintptr_t)off;
    else return *(lds_u32 *)(uintptr_t)off;
}

template <int W>
__device__ __forceinline__ void lds_put(uint32_t off, uint32_t v)
{
    if constexpr (W == 16) *(lds_u16 *)(uintptr_t)off = (uint16_t)v;
    else *(lds_u32 *)(uintptr_t)off = v;
}

template <int W>
__device__ __forceinline__ uint64_t field_of(uint64_t v, int sub)
{
    if constexpr (W == 64) return v;
    else return (v >> (W * sub)) & ((1ull << W) - 1ull);
}

constexpr int kRegCols = 28;   // neighbour entries held in registers (128-byte block head)

template <int W, bool SIGNED>
__global__ __launch_bounds__(1024) void sweep_kernel(SweepArgs a, const int2 *__restrict__ stream_all,
                                                    const int *__restrict__ level_off,
                                                    const uint4 *__restrict__ blocks)
{
    // A finished run (adaptive steps past the last grid point): nothing to do.
    const int gk = a.adapt ? a.as_state[3] : a.k;
    if (gk >= a.K) return;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NS = 64 / W;      // node slots per wave
    constexpr int GPS = W / 4;      // Philox calls per slot
    constexpr int SH = W == 16 ? 1 : (W == 32 ? 2 : 3);
    const int n = a.n;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = blockDim.x >> 6;
    const int blk = blockIdx.x;
    const int r0 = blk * W;
    const int grp = r0 >> 6;
    const int sub = (r0 & 63) / W;
    const int slot_w = lane / W;
    const int rl = lane % W;
    const int bitpos = rl & 31;
    const uint32_t half4 = W == 64 ? 4u * (uint32_t)(rl >> 5) : 0u;
    const int r = r0 + rl;
    const int real = r < a.R ? 1 : 0;

    const SweepLds L = sweep_lds_layout(W, SIGNED ? 1 : 0, n, a.dmax, nwaves);
    uint64_t *T = reinterpret_cast<uint64_t *>(smem + L.thr);
    int *part = reinterpret_cast<int *>(smem + L.part);
    int *Eblk = reinterpret_cast<int *>(smem + L.eblk);
    long long *misc = reinterpret_cast<long long *>(smem + L.misc);
    uint16_t *sched16 = reinterpret_cast<uint16_t *>(smem + L.sched);
    uint32_t *dbuf = reinterpret_cast<uint32_t *>(smem + L.draws) + wave * 256;
    const uint32_t comp = (uint32_t)n << SH;  // byte distance to the complemented copy

    uint64_t *Xg = a.X + (size_t)grp * n;
    for (int i = tid; i < n; i += blockDim.x) {
        const uint64_t v = field_of<W>(Xg[i], sub);
        const uint32_t off = (uint32_t)i << SH;
        if constexpr (W == 64) {
            lds_put<W>(off, (uint32_t)v);
            lds_put<W>(off + 4, (uint32_t)(v >> 32));
            if constexpr (SIGNED) {
                lds_put<W>(comp + off, ~(uint32_t)v);
                lds_put<W>(comp + off + 4, ~(uint32_t)(v >> 32));
            }
        } else {
            lds_put<W>(off, (uint32_t)v);
            if constexpr (SIGNED) lds_put<W>(comp + off, ~(uint32_t)v);
        }
        sched16[i] = (uint16_t)a.sched[i];
    }
    if (tid == 0) {
        const uint32_t zoff = (uint32_t)(SIGNED ? 2 * n : n) << SH;
        lds_put<W>(zoff, 0u);
        if constexpr (W == 64) lds_put<W>(zoff + 4, 0u);
    }
    const int level = a.as_state[0];
    const uint64_t *trow = a.thr + ((size_t)gk * a.lmax1 + level) * (size_t)(a.dmax + 1);
    for (int m = tid; m <= a.dmax; m += blockDim.x) T[m] = m == 0 ? (1ull << 32) : trow[m];
    if (tid < W) Eblk[tid] = (r0 + tid < a.R) ? a.E[r0 + tid] : 0;
    if (tid == 0) {
        misc[0] = a.best_E[0];
        misc[1] = -1;  // no candidate (reads back as ~0ull)
        misc[12] = 0;  // uphill attempts and accepts of this workgroup
        misc[13] = 0;
    }
    __syncthreads();

    const uint32_t k = (uint32_t)a.k;
    // Read-only tables come in as separate restrict arguments so that their
    // uniform reads become scalar loads, which do not wait on the vector
    // prefetch of the adjacency blocks.
    const int2 *stream = stream_all + (size_t)wave * a.qpad;
    const int bu4 = a.block_u4;
    const uint32_t rgrp = ((uint32_t)(r0 >> 2) + (uint32_t)((lane & 15) % GPS)) | (a.inst << 16);
    const int fill_slot = (lane & 15) / GPS;
    const int fill_pass = lane >> 4;

    int dE = 0;
    unsigned int att = 0, acc = 0;
    for (int s = 0; s < a.S; ++s) {
        int q = 0;
        int2 se = stream[0];
        uint4 h, c0, c1, c2, c3, c4, c5, c6;
        {
            // a wave without passes in this sweep still loads (and ignores) slot 0
            const int t0 = se.x < 0 ? 0 : (se.x + slot_w < n ? se.x + slot_w : se.x);
            const uint4 *bp = blocks + (size_t)t0 * bu4;
            h = bp[0]; c0 = bp[1]; c1 = bp[2]; c2 = bp[3]; c3 = bp[4]; c4 = bp[5]; c5 = bp[6]; c6 = bp[7];
        }
        for (int lv = 0; lv < a.n_levels; ++lv) {
            const int beg = level_off[lv], end = level_off[lv + 1];
            const int Lsz = end - beg;
            const int npass = Lsz > wave * NS ? (Lsz - wave * NS + nwaves * NS - 1) / (nwaves * NS) : 0;
            for (int p = 0; p < npass; ++p, ++q) {
                // Prefetch the next pass of this wave's stream (read-only graph
                // data); past the end of the stream it reloads slot 0.
                const int2 sn = stream[q + 1];
                const int tn = sn.x < 0 ? 0 : (sn.x + slot_w < n ? sn.x + slot_w : sn.x);
                const uint4 *bpn = blocks + (size_t)tn * bu4;
                const uint4 nh = bpn[0], n0 = bpn[1], n1 = bpn[2], n2 = bpn[3], n3 = bpn[4], n4 = bpn[5],
                            n5 = bpn[6], n6 = bpn[7];
                if ((q & 3) == 0) {
                    // Draws for passes q..q+3: every lane computes one Philox call.
                    const int2 e = stream[q + fill_pass];
                    const int t2 = e.x + fill_slot;
                    const uint32_t i2 = (e.x >= 0 && t2 < n) ? (uint32_t)sched16[t2] : 0u;
                    const U4 o = philox10(U4{i2, (uint32_t)s, k, rgrp}, a.seed_lo, a.seed_hi);
                    *reinterpret_cast<uint4 *>(dbuf + 4 * lane) = make_uint4(o.x, o.y, o.z, o.w);
                    __builtin_amdgcn_wave_barrier();
                }
                const int t = se.x + slot_w;
                const bool active = t < end;
                const uint32_t noff = h.x;
                const int d = (int)h.y;
                const int md = se.y;
                // Count neighbours with w_ij x_j = +1 (padding reads the zero word).
                int cnt = 0;
#define PA_NB(off) (int)__builtin_amdgcn_ubfe(lds_word<W>((off) + half4), bitpos, 1)
#define PA_CHUNK(v) cnt += PA_NB(v.x) + PA_NB(v.y) + PA_NB(v.z) + PA_NB(v.w)
                PA_CHUNK(c0);
                if (md > 4) {
                    PA_CHUNK(c1);
                    if (md > 8) {
                        PA_CHUNK(c2);
                        if (md > 12) {
                            PA_CHUNK(c3);
                            if (md > 16) {
                                PA_CHUNK(c4);
                                if (md > 20) {
                                    PA_CHUNK(c5);
                                    if (md > 24) {
                                        PA_CHUNK(c6);
                                        if (md > kRegCols) {
                                            const uint32_t *rest = reinterpret_cast<const uint32_t *>(
                                                blocks + (size_t)(active ? t : se.x) * bu4) + 4;
                                            for (int kk = kRegCols; kk < md; ++kk) cnt += PA_NB(rest[kk]);
                                        }
                                    }
                                }
                            }
                        }
                    }
                }
#undef PA_CHUNK
#undef PA_NB
                const uint32_t word = lds_word<W>(noff + half4);
                const int bi = (int)__builtin_amdgcn_ubfe(word, bitpos, 1);
                const int u = bi ? cnt : d - cnt;   // edges with w_ij x_i x_j = +1
                const int m = d - 2 * u;            // flip changes E by 2m
                const int mm = m > 0 ? m : 0;       // T[0] = 2^32: downhill always accepted
                const uint32_t dr = dbuf[(q & 3) * 64 + lane];
                const int accept = (active && (uint64_t)dr < T[mm]) ? 1 : 0;
                const int up = (m > 0 && active) ? real : 0;
                att += (unsigned)up;
                acc += (unsigned)(up & accept);
                dE += accept ? 2 * m : 0;
                const unsigned long long bal = __ballot(accept);
                if (active) {
                    uint32_t fm;
                    if constexpr (W == 64) fm = rl < 32 ? (uint32_t)bal : (uint32_t)(bal >> 32);
                    else if constexpr (W == 32) fm = slot_w ? (uint32_t)(bal >> 32) : (uint32_t)bal;
                    else fm = (uint32_t)(bal >> (16 * slot_w)) & 0xFFFFu;
                    const uint32_t nw = word ^ fm;
                    lds_put<W>(noff + half4, nw);
                    if constexpr (SIGNED) lds_put<W>(comp + noff + half4, ~nw);
                }
                se = sn;
                h = nh; c0 = n0; c1 = n1; c2 = n2; c3 = n3; c4 = n4; c5 = n5; c6 = n6;
            }
            __syncthreads();
        }
        // Energies after sweep s and the block's best candidate.
        part[tid] = dE;
        dE = 0;
        __syncthreads();
        if (tid < W) {
            int sum = 0;
            for (int w = 0; w < nwaves; ++w)
                for (int qq = 0; qq < NS; ++qq) sum += part[w * 64 + qq * W + tid];
            Eblk[tid] += sum;
        }
        __syncthreads();
        if (tid == 0) {
            long long be = misc[0];
            int arg = -1;
            for (int qq = 0; qq < W && r0 + qq < a.R; ++qq)
                if ((long long)Eblk[qq] < be) {
                    be = Eblk[qq];
                    arg = qq;
                }
            misc[2] = arg;
            if (arg >= 0) {
                misc[0] = be;
                misc[1] = (long long)((((unsigned long long)((uint32_t)be ^ 0x80000000u)) << 32) |
                                      ((unsigned long long)s << 15) | (unsigned long long)(r0 + arg));
            }
        }
        __syncthreads();
        const int sq = (int)misc[2];
        if (sq >= 0) {
            uint32_t *dst = a.snap + (size_t)blk * a.nw32;
            const uint32_t sh4 = W == 64 ? 4u * (uint32_t)(sq >> 5) : 0u;
            for (int w = tid; w < a.nw32; w += blockDim.x) {
                uint32_t bits = 0;
                const int ib = w * 32;
                for (int b = 0; b < 32 && ib + b < n; ++b)
                    bits |= __builtin_amdgcn_ubfe(lds_word<W>(((uint32_t)(ib + b) << SH) + sh4), sq & 31, 1) << b;
                dst[w] = bits;
            }
        }
        __syncthreads();
    }

    for (int i = tid; i < n; i += blockDim.x) {
        const uint32_t off = (uint32_t)i << SH;
        if constexpr (W == 64) Xg[i] = ((uint64_t)lds_word<W>(off + 4) << 32) | lds_word<W>(off);
        else if constexpr (W == 32) reinterpret_cast<uint32_t *>(Xg + i)[sub] = lds_word<W>(off);
        else reinterpret_cast<uint16_t *>(Xg + i)[sub] = (uint16_t)lds_word<W>(off);
    }
    if (tid < W && r0 + tid < a.R) a.E[r0 + tid] = Eblk[tid];
    // Uphill counters: wave sums gathered in LDS, one global atomic per
    // workgroup on the two step-wide counters.
    const long long at = wave_sum_ll((long long)att), ac = wave_sum_ll((long long)acc);
    if (lane == 0) {
        if (at) atomicAdd(reinterpret_cast<unsigned long long *>(&misc[12]), (unsigned long long)at);
        if (ac) atomicAdd(reinterpret_cast<unsigned long long *>(&misc[13]), (unsigned long long)ac);
    }
    __syncthreads();
    if (tid == 0) {
        if (misc[12]) atomicAdd(&a.counters[0], (unsigned long long)misc[12]);
        if (misc[13]) atomicAdd(&a.counters[1], (unsigned long long)misc[13]);
        a.cand[blk] = (unsigned long long)misc[1];
    }
}

// ---------------------------------------------------------------------------
// Node-per-lane sweep kernel (multi-spin coding over W replicas).
//
// A workgroup owns W = 4, 8 or 16 replicas for a whole step. LDS holds one
// W-byte record per node (byte b = spin of block replica b, 1 for +1), for
// signed graphs a complemented record per node (so a negative edge reads
// "w_ij x_j = +1" directly), and an all-zero record for padding. Each lane
// handles one node of the current dependency level for all W replicas at
// once: the neighbours' records are added bytewise (one LDS read and W/4
// adds per neighbour give the W counts), and the per-replica Metropolis
// tests run on the packed bytes. A lane computes exactly the W/4 Philox
// calls its replicas need (one call = 4 consecutive replicas at one node).
// Adjacency blocks are read once per node and prefetched one round ahead
// into the other of two register buffers.
//
// The tests work on the bytes 0x80 + (m - 1), m = d - 2u the half energy
// change of a flip (u: edges the flip would break): bit 7 marks an uphill
// move, and the byte itself indexes the 256-entry 32-bit threshold table that
// sits at LDS address 0, T[m] at entry 0x80 + m - 1 (for m >= 1 and beta > 0,
// T[m] < 2^32; a row where every uphill threshold is 2^32 carries an
// accept-all flag instead). Bytewise
// arithmetic keeps 0x7F + d inside a byte, so this path serves graphs with
// maximum degree <= 127; the per-replica energy changes are gathered in byte
// accumulators that are widened into registers before they can overflow.
// ---------------------------------------------------------------------------
struct BytesLds {
    size_t rec, edelta, misc, total;
};

__host__ __device__ inline BytesLds bytes_lds_layout(int W, int sgn, int n, int /*dmax*/)
{
    BytesLds L;
    const size_t recs = (size_t)(sgn ? 2 * n : n) + 1;
    L.rec = kBytesRecBase;                        // [0, 1024): 256 u32 thresholds
    L.edelta = L.rec + align16(recs * (size_t)W);
    L.misc = L.edelta + 64 * 4;
    L.total = L.misc + 16 * 8;
    return L;
}

int sweep_bytes_lds(int W, int sgn, int n, int dmax)
{
    return (int)bytes_lds_layout(W, sgn, n, dmax).total;
}

typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) u32x2 lds_u2;
typedef __attribute__((address_space(3))) u32x4 lds_u4;

// Spread the low 4 bits of v into the low bit of 4 bytes.
__device__ __forceinline__ uint32_t spread4(uint32_t v)
{
    return ((v & 0xFu) * 0x00204081u) & 0x01010101u;
}

// 0xFF in every byte that holds 1 (bytes hold 0 or 1): v_perm_b32 selector
// 12 yields 0x00 and 13 yields 0xFF (a multiply by 0xFF would be quarter rate).
__device__ __forceinline__ uint32_t byte_mask(uint32_t v)
{
    return __builtin_amdgcn_perm(0u, 0u, v + 0x0C0C0C0Cu);
}

// Gather bit 0 of 4 bytes into 4 bits (byte b -> bit b).
__device__ __forceinline__ uint32_t gather4(uint32_t v)
{
    return (((v & 0x01010101u) * 0x01020408u) >> 24) & 0xFu;
}

template <int NR>
struct Rec {
    uint32_t v[NR];
};

template <int NR>
__device__ __forceinline__ Rec<NR> rec_load(uint32_t off)
{
    Rec<NR> r;
    if constexpr (NR == 1) {
        r.v[0] = *(lds_u32 *)(uintptr_t)off;
    } else if constexpr (NR == 2) {
        const u32x2 t = *(lds_u2 *)(uintptr_t)off;
        r.v[0] = t.x; r.v[1] = t.y;
    } else {
        const u32x4 t = *(lds_u4 *)(uintptr_t)off;
        r.v[0] = t.x; r.v[1] = t.y; r.v[2] = t.z; r.v[3] = t.w;
    }
    return r;
}

template <int NR>
__device__ __forceinline__ void rec_store(uint32_t off, const Rec<NR> &r)
{
    if constexpr (NR == 1) *(lds_u32 *)(uintptr_t)off = r.v[0];
    else if constexpr (NR == 2) *(lds_u2 *)(uintptr_t)off = u32x2{r.v[0], r.v[1]};
    else *(lds_u4 *)(uintptr_t)off = u32x4{r.v[0], r.v[1], r.v[2], r.v[3]};
}

// Adjacency block head held in registers: u16 {node, degree, 30 neighbour
// record indices} = 64 bytes; longer rows continue in global memory.
struct Blk {
    uint4 b0, b1, b2, b3;
};

constexpr int kBlkCols = 30;

__device__ __forceinline__ void blk_load(Blk &b, const uint4 *p)
{
    b.b0 = p[0]; b.b1 = p[1]; b.b2 = p[2]; b.b3 = p[3];
}

// Sum over the 64 lanes of a wave with DPP row shifts and row broadcasts
// (every lane active); the total is read from lane 63.
__device__ __forceinline__ int wave_sum_dpp(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);   // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);   // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// SG: 0 = all weights positive; 1 = negative edges read a complemented copy of
// the neighbour's record (records twice as many); 2 = negative edges carry a
// sign bit in their block entry and the record is complemented on reading
// (half the LDS of mode 1, one XOR per neighbour).
// One workgroup's step: tile `blk` (replicas blk*W .. blk*W + W - 1) of a run
// whose sweep launch has `nblk` tiles.
template <int W, int SG, bool DIRECT>
__device__ __forceinline__ void sweep_bytes_tile(const SweepArgs &a, const int4 *__restrict__ rounds,
                                                 const uint4 *__restrict__ blocks, const int blk,
                                                 const int nblk, const bool prio)
{
    constexpr bool SIGNED = SG == 1;     // complemented records in LDS
    constexpr bool SBIT = SG == 2;       // sign bits in the block entries
    const int gk = a.adapt ? a.as_state[3] : a.k;     // grid point of this step
    if (gk >= a.K) {
        // A finished run (adaptive steps past the last grid point): carry the
        // population over to the output buffer unchanged (the parent list is
        // the identity then), each workgroup a slice.
        const size_t words = (size_t)((a.R + 63) >> 6) * a.n;
        const size_t per = (words + nblk - 1) / nblk;
        const size_t w0 = (size_t)blk * per, w1 = w0 + per < words ? w0 + per : words;
        for (size_t w = w0 + threadIdx.x; w < w1; w += blockDim.x) a.X[w] = a.Xin[w];
        const int rper = (a.R + nblk - 1) / nblk;
        const int e0 = blk * rper, e1 = e0 + rper < a.R ? e0 + rper : a.R;
        for (int r = e0 + (int)threadIdx.x; r < e1; r += blockDim.x) a.E[r] = a.Ein[r];
        return;
    }
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NR = W / 4;
    const int n = a.n;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int nt = blockDim.x;
    const int r0 = blk * W;
    const int grp = r0 >> 6;
    const int sub = (r0 & 63) / W;

    const BytesLds L = bytes_lds_layout(W, SIGNED ? 1 : 0, n, a.dmax);
    uint32_t *T = reinterpret_cast<uint32_t *>(smem);               // T[m] at index 0x80 + m - 1
    int *Ed = reinterpret_cast<int *>(smem + L.edelta);
    long long *misc = reinterpret_cast<long long *>(smem + L.misc);
    int *Eblk = reinterpret_cast<int *>(misc + 4);
    constexpr uint32_t RB = kBytesRecBase;                        // LDS address of record 0
    const uint32_t comp = (uint32_t)n * W;                        // complemented records
    const uint32_t zrec = RB + (uint32_t)(SIGNED ? 2 * n : n) * W;  // zero record

    uint64_t *Xg = a.X + (size_t)grp * n;            // output words of this block's group
    // The block's replica slots take the spins of their resampling parents
    // (identity before the first resampling). Systematic resampling hands
    // out slots in parent order, so the parents of a block normally sit in
    // one or two 64-replica words: those are read once per node.
    const bool ident = a.parent == nullptr;
    int pr[W];
    int gA = 1 << 30, gB = -1;
#pragma unroll
    for (int b = 0; b < W; ++b) {
        const int r = r0 + b < a.R ? r0 + b : r0;
        pr[b] = ident ? r : a.parent[r];
        gA = (pr[b] >> 6) < gA ? (pr[b] >> 6) : gA;
        gB = (pr[b] >> 6) > gB ? (pr[b] >> 6) : gB;
    }
    const bool two = gB - gA <= 1;
    const uint64_t *XA = a.Xin + (size_t)gA * n, *XB = a.Xin + (size_t)gB * n;
    // Step tables and block state first, so that their loads overlap the
    // population loads below.
    if (tid < NR) *(lds_u32 *)(uintptr_t)(zrec + 4 * tid) = 0u;
    const int level = a.as_state[0];
    const uint32_t *trow = a.thr32 + ((size_t)gk * a.lmax1 + level) * (size_t)(a.dmax + 1);
    // Move byte 0x80 + (m - 1) of an uphill move indexes T[m]; the lower half
    // (downhill moves, accepted by mask) stays zero.
    for (int m = tid; m < 256; m += nt) T[m] = m >= 128 && m - 128 < a.dmax ? trow[m - 128] : 0u;
    // Accept-all row (exp(-beta * 2m) rounds to 1 for every uphill move).
    const uint32_t allm = trow[a.dmax] ? 0x01010101u : 0u;
    if (tid < W) {
        Eblk[tid] = (r0 + tid < a.R) ? a.Ein[ident ? r0 + tid : a.parent[r0 + tid]] : 0;
        Ed[tid] = 0;
    }
    if (prio && tid == 0) {
        // Sweeps in which this workgroup's waves take the higher issue
        // priority, as bits of s mod 10: the second workgroup on a compute
        // unit (slot 1, TG_ID of the HW_ID register) in sweeps 0, 2, 4, 5, 7
        // and 9 of every ten.
        const uint32_t slot = (__builtin_amdgcn_s_getreg((31 << 11) | 4) >> 16) & 15u;
        misc[14] = slot == 1 ? 0x2B5u : 0u;
    }
    if (tid == 0) {
        misc[0] = a.best_E[0];
        misc[1] = -1;  // no candidate (reads back as ~0ull)
        misc[12] = 0;  // uphill attempts and accepts of this workgroup
        misc[13] = 0;
    }
    if constexpr (W == 8) {
        // Expand the block's spin bits into byte records, LB nodes per lane and
        // pass (their loads in flight together). With resampling parents in two
        // words, slot b's spin is one bit of one 32-bit half of those words, the
        // same for every node: the half is picked by a uniform branch per slot,
        // so a spin costs one bit extract.
        constexpr int LB = W >= 8 ? 4 : 8;
        int psel[W];
#pragma unroll
        for (int b = 0; b < W; ++b)
            psel[b] = __builtin_amdgcn_readfirstlane(((pr[b] >> 6) == gA ? 0 : 2) + ((pr[b] & 63) >= 32 ? 1 : 0));
        for (int base = 0; base < n; base += LB * nt) {
            uint64_t va[LB], vb[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int i = base + u * nt + tid;
                va[u] = i < n ? XA[i] : 0ull;
                vb[u] = i < n && !ident && two ? XB[i] : 0ull;
            }
            Rec<NR> rc[LB];
            if (ident) {
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    const uint64_t v = field_of<W>(va[u], sub);
#pragma unroll
                    for (int q = 0; q < NR; ++q) rc[u].v[q] = spread4((uint32_t)(v >> (4 * q)));
                }
            } else if (two) {
#pragma unroll
                for (int u = 0; u < LB; ++u)
#pragma unroll
                    for (int q = 0; q < NR; ++q) rc[u].v[q] = 0u;
#pragma unroll
                for (int b = 0; b < W; ++b) {
                    const uint32_t sh = (uint32_t)__builtin_amdgcn_readfirstlane(pr[b] & 31);
                    const int q = b >> 2, bs = 8 * (b & 3);
                    if (psel[b] == 0) {
#pragma unroll
                        for (int u = 0; u < LB; ++u) rc[u].v[q] |= (((uint32_t)va[u] >> sh) & 1u) << bs;
                    } else if (psel[b] == 1) {
#pragma unroll
                        for (int u = 0; u < LB; ++u) rc[u].v[q] |= (((uint32_t)(va[u] >> 32) >> sh) & 1u) << bs;
                    } else if (psel[b] == 2) {
#pragma unroll
                        for (int u = 0; u < LB; ++u) rc[u].v[q] |= (((uint32_t)vb[u] >> sh) & 1u) << bs;
                    } else {
#pragma unroll
                        for (int u = 0; u < LB; ++u) rc[u].v[q] |= (((uint32_t)(vb[u] >> 32) >> sh) & 1u) << bs;
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    const int i = base + u * nt + tid;
                    uint64_t v = 0;
                    if (i < n) {
#pragma unroll
                        for (int b = 0; b < W; ++b)
                            v |= ((a.Xin[(size_t)(pr[b] >> 6) * n + i] >> (pr[b] & 63)) & 1ull) << b;
                    }
#pragma unroll
                    for (int q = 0; q < NR; ++q) rc[u].v[q] = spread4((uint32_t)(v >> (4 * q)));
                }
            }
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int i = base + u * nt + tid;
                if (i >= n) break;
                rec_store<NR>(RB + (uint32_t)i * W, rc[u]);
                if constexpr (SIGNED) {
                    Rec<NR> cc;
#pragma unroll
                    for (int q = 0; q < NR; ++q) cc.v[q] = rc[u].v[q] ^ 0x01010101u;
                    rec_store<NR>(RB + comp + (uint32_t)i * W, cc);
                }
            }
        }
    } else {
        // Expand the block's spin bits into byte records, 8 loads in flight per lane.
        for (int base = 0; base < n; base += 8 * nt) {
            uint64_t va[8], vb[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = base + u * nt + tid;
                va[u] = i < n ? XA[i] : 0ull;
                vb[u] = i < n && !ident && two ? XB[i] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = base + u * nt + tid;
                if (i >= n) break;
                uint64_t v = 0;
                if (ident) {
                    v = field_of<W>(va[u], sub);
                } else if (two) {
#pragma unroll
                    for (int b = 0; b < W; ++b) {
                        const uint64_t w = (pr[b] >> 6) == gA ? va[u] : vb[u];
                        v |= ((w >> (pr[b] & 63)) & 1ull) << b;
                    }
                } else {
#pragma unroll
                    for (int b = 0; b < W; ++b)
                        v |= ((a.Xin[(size_t)(pr[b] >> 6) * n + i] >> (pr[b] & 63)) & 1ull) << b;
                }
                Rec<NR> rc;
#pragma unroll
                for (int q = 0; q < NR; ++q) rc.v[q] = spread4((uint32_t)(v >> (4 * q)));
                rec_store<NR>(RB + (uint32_t)i * W, rc);
                if constexpr (SIGNED) {
#pragma unroll
                    for (int q = 0; q < NR; ++q) rc.v[q] ^= 0x01010101u;
                    rec_store<NR>(RB + comp + (uint32_t)i * W, rc);
                }
            }
        }
    }
    // Bytes of real (non-padding) replicas, as 0x80 markers for the counters.
    uint32_t real80[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) {
        uint32_t m = 0;
        for (int b = 0; b < 4; ++b)
            if (r0 + 4 * q + b < a.R) m |= 0x80u << (8 * b);
        real80[q] = m;
    }
    __syncthreads();

    const uint32_t k = (uint32_t)a.k;
    // rounds[] = {first slot, level end, 1 if last round of its level, 0}. The
    // read-only tables are separate restrict arguments so that the uniform
    // round reads become scalar loads and never wait on the block prefetch.
    const int bu4 = a.block_u4;
    const int nrounds = a.n_rounds;
    const uint32_t rgrp0 = (uint32_t)(r0 >> 2) | (a.inst << 16);

    uint32_t YA[NR], ZA[NR];
#pragma unroll
    for (int q = 0; q < NR; ++q) { YA[q] = 0; ZA[q] = 0; }
    unsigned int att = 0, acc = 0;
    constexpr int SHW = W == 4 ? 2 : (W == 8 ? 3 : 4);   // record index -> LDS byte offset
    constexpr int SHC = DIRECT ? 0 : SHW;                // block entry -> LDS byte offset
    // A 16-bit block entry names a neighbour record: an LDS byte offset
    // (DIRECT) or a record index. With sign bits, bit 0 of an offset (records
    // are at least 4-byte aligned) or bit 15 of an index marks a negative
    // edge, whose record is read complemented (0x01 in every byte).
    auto ent_off = [](uint32_t e) -> uint32_t {
        if constexpr (!SBIT) return e << SHC;
        else if constexpr (DIRECT) return e & 0xFFFEu;
        else return (e & 0x7FFFu) << SHW;
    };
    auto ent_neg = [](uint32_t e) -> uint32_t {
        if constexpr (!SBIT) return 0u;
        else if constexpr (DIRECT) return (e & 1u) * 0x01010101u;
        else return (e >> 15) * 0x01010101u;
    };
    const uint32_t zent = DIRECT ? zrec : zrec >> SHW;   // entry of the zero record

    Blk bufA, bufB;
    int4 rd = rounds[0];                          // the current round
    int4 nd = rounds[nrounds > 1 ? 1 : 0];        // the next round
    // Lane tid reads the block of slot (first slot of the round + tid): a
    // uniform base plus a per-lane constant offset. Slots past a level's end
    // belong to later levels or to the padding blocks after the last node;
    // those lanes only read.
    const uint32_t lane_off = (uint32_t)tid * (uint32_t)bu4 * 16u;
    auto blk_at = [&](int first) {
        return reinterpret_cast<const uint4 *>(reinterpret_cast<const unsigned char *>(blocks) +
                                               (size_t)(uint32_t)first * (uint32_t)(bu4 * 16) + lane_off);
    };
    const int wbase = __builtin_amdgcn_readfirstlane(tid & ~63);   // first thread of this wave
    blk_load(bufA, blk_at(rd.x));

    // Per-replica energy changes of this lane: byte accumulators (YA: d - u,
    // ZA: u, per accepted flip; the flip changes E by 2(d - 2u)) are widened
    // into E32 before a byte can overflow, and E32 is summed over the
    // workgroup once per sweep.
    int E32[W];
#pragma unroll
    for (int r = 0; r < W; ++r) E32[r] = 0;
    auto widen = [&]() {
#pragma unroll
        for (int q = 0; q < NR; ++q) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int y = (int)((YA[q] >> (8 * b)) & 0xFFu);
                const int z = (int)((ZA[q] >> (8 * b)) & 0xFFu);
                E32[4 * q + b] += 2 * (y - z);       // sum of 2m over accepted flips
            }
            YA[q] = 0;
            ZA[q] = 0;
        }
    };
    auto flush = [&]() {
        widen();
#pragma unroll
        for (int r = 0; r < W; ++r) {
            const int v = wave_sum_dpp(E32[r]);
            if (lane == 0 && v != 0) atomicAdd(&Ed[r], v);
            E32[r] = 0;
        }
    };

    auto step = [&](int s, int rho, Blk &cur, Blk &nxt, int4 &n2) {
        // The header of the round after next is loaded now and used one
        // iteration later; this lane's block of the next round is prefetched
        // (sweeps wrap to round 0; past the last round these are harmless
        // reloads).
        {
            int r2 = rho + 2;
            if (r2 >= nrounds) r2 -= nrounds;
            if (r2 >= nrounds) r2 -= nrounds;
            n2 = rounds[r2];
        }
        blk_load(nxt, blk_at(nd.x));
        const int t = rd.x + tid;
        if (rd.x + wbase < rd.y) {          // some lane of this wave has a node
            const bool active = tid < rd.y - rd.x;
            const uint32_t node = cur.b0.x & 0xFFFFu;
            const uint32_t noff = active ? RB + (node << SHW) : zrec;
            const int d = active ? (int)(cur.b0.x >> 16) : 0;
            // Levels are sorted by decreasing degree: the wave's first lane has its largest degree.
            const int md = __builtin_amdgcn_readfirstlane(d);
            // The own record and the first four neighbours are read before the
            // draws are computed, so that their LDS latency overlaps the Philox
            // arithmetic (the scheduling barriers and the empty asm keep the
            // compiler from moving the draws after the first use of the reads).
            // Lanes past their degree read the zero record.
            const Rec<NR> X = rec_load<NR>(noff);
            const uint32_t e0 = cur.b0.y & 0xFFFFu, e1 = cur.b0.y >> 16;
            const uint32_t e2 = cur.b0.z & 0xFFFFu, e3 = cur.b0.z >> 16;
            const Rec<NR> g0 = rec_load<NR>(ent_off(e0));
            const Rec<NR> g1 = rec_load<NR>(ent_off(e1));
            const Rec<NR> g2 = rec_load<NR>(ent_off(e2));
            const Rec<NR> g3 = rec_load<NR>(ent_off(e3));
            __builtin_amdgcn_sched_barrier(0);
            uint32_t dr[NR][4];
#pragma unroll
            for (int q = 0; q < NR; ++q) {
                const U4 o = philox10(U4{node, (uint32_t)s, k, rgrp0 + (uint32_t)q}, a.seed_lo, a.seed_hi);
                dr[q][0] = o.x; dr[q][1] = o.y; dr[q][2] = o.z; dr[q][3] = o.w;
                asm volatile("" ::"v"(dr[q][0]), "v"(dr[q][1]), "v"(dr[q][2]), "v"(dr[q][3]));
            }
            __builtin_amdgcn_sched_barrier(0);
            uint32_t C[NR];
#pragma unroll
            for (int q = 0; q < NR; ++q)
                C[q] = ((g0.v[q] ^ ent_neg(e0)) + (g1.v[q] ^ ent_neg(e1))) +
                       ((g2.v[q] ^ ent_neg(e2)) + (g3.v[q] ^ ent_neg(e3)));
#define PA_NB(ent)                                              \
    {                                                           \
        const uint32_t e_ = (ent);                              \
        const Rec<NR> nb = rec_load<NR>(ent_off(e_));           \
        const uint32_t m_ = ent_neg(e_);                        \
        _Pragma("unroll") for (int q = 0; q < NR; ++q) C[q] += nb.v[q] ^ m_; \
    }
#define PA_W(w) PA_NB((w) & 0xFFFFu) PA_NB((w) >> 16)
            {
                if (md > 4) {
                    PA_W(cur.b0.w) PA_W(cur.b1.x)
                    if (md > 8) {
                        PA_W(cur.b1.y) PA_W(cur.b1.z)
                        if (md > 12) {
                            PA_W(cur.b1.w) PA_W(cur.b2.x)
                            if (md > 16) {
                                PA_W(cur.b2.y) PA_W(cur.b2.z)
                                if (md > 20) {
                                    PA_W(cur.b2.w) PA_W(cur.b3.x)
                                    if (md > 24) {
                                        PA_W(cur.b3.y) PA_W(cur.b3.z)
                                        if (md > 28) {
                                            PA_W(cur.b3.w)
                                            if (md > kBlkCols) {
                                                const uint16_t *rest = reinterpret_cast<const uint16_t *>(
                                                    blocks + (size_t)(active ? t : rd.x) * bu4) + 2;
                                                for (int kk = kBlkCols; kk < md; ++kk) {
                                                    const uint32_t ent = active ? (uint32_t)rest[kk] : zent;
                                                    PA_NB(ent)
                                                }
                                            }
                                        }
                                    }
                                }
                            }
                        }
                    }
                }
            }
#undef PA_W
#undef PA_NB
            if (active) {
                const uint32_t Dm = __builtin_amdgcn_perm(0u, (uint32_t)d, 0u);   // d in every byte
                Rec<NR> Xn;
                // Every byte's threshold is requested before any is compared,
                // so the reads of all NR words are in flight together.
                uint32_t Uq[NR], wq[NR], th[NR][4];
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    // u = x ? c : d - c  (edges with w_ij x_i x_j = +1), per byte
                    const uint32_t msk = byte_mask(X.v[q]);
                    Uq[q] = (C[q] & msk) | ((Dm - C[q]) & ~msk);
                    // w = 0x80 + (m - 1) per byte with m = d - 2u
                    wq[q] = (0x7F7F7F7Fu + Dm) - 2u * Uq[q];
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        // T[m] sits at LDS word 0x80 + (m - 1): the move byte itself.
                        th[q][b] = *(lds_u32 *)(uintptr_t)(((wq[q] >> (8 * b)) & 0xFFu) << 2);
                }
#pragma unroll
                for (int q = 0; q < NR; ++q) {
                    const uint32_t U = Uq[q], w = wq[q];
                    uint32_t A = ((~w >> 7) & 0x01010101u) | allm;   // m <= 0 always accepts
#pragma unroll
                    for (int b = 0; b < 4; ++b) A |= (dr[q][b] < th[q][b] ? 1u : 0u) << (8 * b);
                    Xn.v[q] = X.v[q] ^ A;
                    const uint32_t up = w & real80[q];           // uphill markers
                    att += __builtin_popcount(up);
                    acc += __builtin_popcount(up & (A << 7));
                    const uint32_t Am = byte_mask(A);
                    YA[q] += (Dm - U) & Am;                      // d - u of accepted flips
                    ZA[q] += U & Am;                             // u of accepted flips
                }
                rec_store<NR>(noff, Xn);
                if constexpr (SIGNED) {
                    Rec<NR> Xc;
#pragma unroll
                    for (int q = 0; q < NR; ++q) Xc.v[q] = Xn.v[q] ^ 0x01010101u;
                    rec_store<NR>(comp + noff, Xc);
                }
            }
        }
        // Level ends need a barrier; the sweep's last one is taken after the
        // energy flush (sweep_done).
        if (rd.z && rho != nrounds - 1) __syncthreads();
    };

    // End of sweep s: the energy changes are summed over the workgroup, then
    // the block's best candidate is taken.
    // Issue priority for sweep s (scheduling only; launches with prio_mode 1):
    // bit s mod 10 of the workgroup's turn mask, set at the start.
    auto prio_turn = [&](int s) {
        if (!prio) return;
        const uint32_t turns = (uint32_t)misc[14];
        if (turns != 0u) {
            if ((turns >> (s % 10)) & 1u) __builtin_amdgcn_s_setprio(2);
            else __builtin_amdgcn_s_setprio(0);
        }
    };
    auto sweep_done = [&](int s) {
        flush();
        __syncthreads();
        {
            // Energies after sweep s and the block's best candidate, in wave 0
            // (lowest energy, then lowest replica; strict improvement only).
            if (tid < 64) {
                unsigned long long key = ~0ull;
                if (tid < W) {
                    const int e = Eblk[tid] + Ed[tid];
                    Eblk[tid] = e;
                    Ed[tid] = 0;
                    if (r0 + tid < a.R)
                        key = ((unsigned long long)((uint32_t)e ^ 0x80000000u) << 32) | (unsigned)tid;
                }
                key = wave_min_u64(key);
                if (tid == 0) {
                    int arg = -1;
                    if (key != ~0ull) {
                        const long long be = (long long)(int)((uint32_t)(key >> 32) ^ 0x80000000u);
                        if (be < misc[0]) {
                            arg = (int)(key & 0xFFFFFFFFu);
                            misc[0] = be;
                            misc[1] = (long long)(((key >> 32) << 32) | ((unsigned long long)s << 15) |
                                                  (unsigned long long)(r0 + arg));
                        }
                    }
                    misc[2] = arg;
                }
            }
            __syncthreads();
            prio_turn(s + 1);
            const int sq = (int)misc[2];
            if (sq >= 0) {
                // Snapshot of the improving replica; the next round may only
                // rewrite records after every lane has read them.
                uint32_t *dst = a.snap + (size_t)blk * a.nw32;
                const unsigned char *rb = smem + RB;
                for (int w = tid; w < a.nw32; w += nt) {
                    uint32_t bits = 0;
                    const int ib = w * 32;
                    for (int b = 0; b < 32 && ib + b < n; ++b)
                        bits |= (uint32_t)(rb[(size_t)(ib + b) * W + sq] & 1u) << b;
                    dst[w] = bits;
                }
                __syncthreads();
            }
        }
    };

    // The next round's block is loaded into one buffer while the other is
    // processed; rounds go in pairs with the two buffers' roles swapped, so no
    // registers are copied between rounds. The byte accumulators are widened
    // after every chunk of flush_every rounds (an even count, at most
    // 255 / d_max, so no byte can overflow) and at the end of each sweep.
    auto round = [&](int s, int rho, Blk &cur, Blk &nxt) {
        int4 n2;
        step(s, rho, cur, nxt, n2);
        rd = nd;
        nd = n2;
    };
    prio_turn(0);
    for (int s = 0; s < a.S; ++s) {
        for (int rho = 0; rho < nrounds;) {
            const int cnt = min(a.flush_every, nrounds - rho);
            int j = 0;
            for (; j + 2 <= cnt; j += 2) {
                round(s, rho + j, bufA, bufB);
                round(s, rho + j + 1, bufB, bufA);
            }
            if (j < cnt) {                          // odd tail at the end of a sweep
                round(s, rho + j, bufA, bufB);
                bufA = bufB;
            }
            rho += cnt;
            if (rho < nrounds) widen();
            else sweep_done(s);
        }
    }

    auto field = [&](int i) {
        const Rec<NR> rc = rec_load<NR>(RB + (uint32_t)i * W);
        uint64_t v = 0;
#pragma unroll
        for (int q = 0; q < NR; ++q) v |= (uint64_t)gather4(rc.v[q]) << (4 * q);
        return v;
    };
    if constexpr (W >= 8) {
        for (int i = tid; i < n; i += nt) {
            const uint64_t v = field(i);
            if constexpr (W == 16) reinterpret_cast<uint16_t *>(Xg + i)[sub] = (uint16_t)v;
            else reinterpret_cast<uint8_t *>(Xg + i)[sub] = (uint8_t)v;
        }
    } else {
        // 4-bit fields share a byte with the neighbouring block: flip the
        // changed bits atomically. Only this block writes these 4 bits during
        // the launch, so the words can be read first, 8 per lane in flight.
        const int sh = 4 * (sub & 7);
        for (int base = 0; base < n; base += 8 * nt) {
            uint32_t old[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = base + u * nt + tid;
                old[u] = i < n ? reinterpret_cast<const unsigned int *>(Xg + i)[sub >> 3] : 0u;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = base + u * nt + tid;
                if (i >= n) break;
                const unsigned delta = (((unsigned)field(i) ^ (old[u] >> sh)) & 0xFu) << sh;
                if (delta) atomicXor(reinterpret_cast<unsigned int *>(Xg + i) + (sub >> 3), delta);
            }
        }
    }
    if (tid < W && r0 + tid < a.R) a.E[r0 + tid] = Eblk[tid];
    // Uphill counters: wave sums gathered in LDS, one global atomic per
    // workgroup (not per wave) on the two step-wide counters.
    const long long at = wave_sum_ll((long long)att), ac = wave_sum_ll((long long)acc);
    if (lane == 0) {
        if (at) atomicAdd(reinterpret_cast<unsigned long long *>(&misc[12]), (unsigned long long)at);
        if (ac) atomicAdd(reinterpret_cast<unsigned long long *>(&misc[13]), (unsigned long long)ac);
    }
    __syncthreads();
    if (tid == 0) {
        if (misc[12]) atomicAdd(&a.counters[0], (unsigned long long)misc[12]);
        if (misc[13]) atomicAdd(&a.counters[1], (unsigned long long)misc[13]);
        a.cand[blk] = (unsigned long long)misc[1];
    }
}

template <int W, int SG, bool DIRECT, bool PRIO>
__global__ __launch_bounds__(1024) void sweep_bytes_kernel(SweepArgs a, const int4 *__restrict__ rounds,
                                                          const uint4 *__restrict__ blocks)
{
    // Workgroups are dispatched round-robin over the 8 XCDs. For 8- and
    // 16-replica tiles (plain byte stores) each XCD takes a contiguous range
    // of tiles, so tiles sharing a 64-replica word share an L2; 4-replica
    // tiles keep the plain order (their nibble stores are atomic XORs, which
    // would then contend within one XCD).
    const int nb = gridDim.x;
    const int blk = [nb] {
        const int b = blockIdx.x;
        if constexpr (W < 8) return b;
        const int x = b & 7, q = nb >> 3, rem = nb & 7;
        return x * q + (x < rem ? x : rem) + (b >> 3);
    }();
    sweep_bytes_tile<W, SG, DIRECT>(a, rounds, blocks, blk, nb, PRIO);
}

// One step of many runs in one launch: workgroup b takes the tile work[b] =
// {run, tile} (run < 0: an empty slot), with the run's arguments from
// runs[run]. Launch index t is step t - k_off of a run; its population
// buffers follow from the parity of that step (the initial population is in
// X0/E0), and step 0 reads no resampling parents. Runs outside their steps
// do nothing.
template <int W, int SG, bool DIRECT>
__global__ __launch_bounds__(1024) void sweep_bytes_multi_kernel(const MultiRun *__restrict__ runs,
                                                                const int2 *__restrict__ work, int t)
{
    const int2 wk = work[blockIdx.x];
    if (wk.x < 0) return;
    const MultiRun &m = runs[wk.x];
    const int k = t - m.k_off;
    if (k < 0 || k >= m.steps) return;
    SweepArgs a = m.sweep;
    const bool even = (k & 1) == 0;
    a.k = k;
    a.Xin = even ? m.X0 : m.X1;
    a.X = even ? m.X1 : m.X0;
    a.Ein = even ? m.E0 : m.E1;
    a.E = even ? m.E1 : m.E0;
    a.parent = k == 0 ? nullptr : m.epi.parent;
    sweep_bytes_tile<W, SG, DIRECT>(a, a.rounds, a.blocks, wk.y, m.nblk, false);
}

// ---------------------------------------------------------------------------
// Step epilogue (one workgroup): best-candidate reduction, population best
// check, noise-level update, statistics, reweighting and systematic
// resampling counts -> parent list.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t sys_f(uint64_t c, uint64_t R, uint64_t u, uint64_t S)
{
    const uint64_t rc = R * c;
    return rc <= u ? 0 : (rc - u + S - 1) / S;
}

__device__ __forceinline__ void epilogue_body(const EpiArgs &a)
{
    extern __shared__ int Esh[];       // [R] energies (when the population is read)
    __shared__ unsigned long long w_cand[16], w_key[16], w_scan[16];
    __shared__ long long w_sum[16];
    __shared__ long long par_total;
    __shared__ int admissible[kMaxJump + 1];
    const int g = a.adapt ? a.as_state[3] : a.k;   // grid point of this step's inverse temperature
    if (g >= a.K) return;                          // finished run (adaptive steps)
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nt = blockDim.x, nwv = nt >> 6;
    const int R = a.R;
    // Thread tid owns the contiguous replicas [lo, hi) (the scan order).
    const int per = (R + nt - 1) / nt;
    const int lo = tid * per < R ? tid * per : R;
    const int hi = lo + per < R ? lo + per : R;
    const bool need_e = a.do_pop || a.do_rest;
    // Best so far (uniform; thread 0 keeps the full record) and the improved flag.
    int bE = a.best[0], bvalid = a.best[4];
    int brec[5] = {0, 0, 0, 0, 0};
    if (tid == 0)
        for (int q = 0; q < 5; ++q) brec[q] = a.best[q];
    int simp = a.as_state[2];
    // Loads needed after the reductions, issued now.
    const bool resample = a.do_rest && g < a.K - 1;
    int off = resample && !a.adapt ? a.wtab_off[g] : 0, len = resample && !a.adapt ? a.wtab_len[g] : 0;
    int level_used = 0, stall0 = 0;
    unsigned long long att = 0, acc = 0;
    if (tid == 0 && a.do_rest) {
        level_used = a.as_state[0];
        stall0 = a.as_state[1];
        att = a.counters[0];
        acc = a.counters[1];
        par_total = 0;
    }

    // One reduction for the block candidates, the population minimum
    // (energy, then lowest replica) and the energy sum.
    unsigned long long kc = ~0ull, ke = ~0ull;
    long long es = 0;
    if (a.do_cand)
        for (int b = tid; b < a.nblk; b += nt) kc = a.cand[b] < kc ? a.cand[b] : kc;
    if (need_e)
        for (int r0 = tid; r0 < R; r0 += 4 * nt) {
            int v[4];       // four independent loads in flight
#pragma unroll
            for (int c = 0; c < 4; ++c) v[c] = r0 + c * nt < R ? a.E[r0 + c * nt] : 0;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int r = r0 + c * nt;
                if (r >= R) break;
                Esh[r] = v[c];
                const unsigned long long kk =
                    ((unsigned long long)((uint32_t)v[c] ^ 0x80000000u) << 32) | (unsigned)r;
                ke = kk < ke ? kk : ke;
                es += v[c];
            }
        }
    kc = wave_min_u64(kc);
    ke = wave_min_u64(ke);
    es = wave_sum_ll(es);
    if (lane == 0) {
        w_cand[wv] = kc;
        w_key[wv] = ke;
        w_sum[wv] = es;
    }
    __syncthreads();
    kc = ~0ull;
    ke = ~0ull;
    es = 0;
    for (int v = 0; v < nwv; ++v) {
        kc = w_cand[v] < kc ? w_cand[v] : kc;
        ke = w_key[v] < ke ? w_key[v] : ke;
        es += w_sum[v];
    }

    if (a.do_cand && kc != ~0ull) {
        const int E = (int)((uint32_t)(kc >> 32) ^ 0x80000000u);
        if (!bvalid || E < bE) {
            const int sw = (int)((kc >> 15) & 0xFFFFull);
            const int r = (int)(kc & 0x7FFFull);
            const uint32_t *src = a.snap + (size_t)(r / a.W) * a.nw32;
            for (int w = tid; w < a.nw32; w += nt) a.best_x[w] = src[w];
            if (tid == 0) {
                brec[0] = E; brec[1] = a.k; brec[2] = sw; brec[3] = r; brec[4] = 1;
            }
            bE = E;
            bvalid = 1;
            simp = 1;
        }
    }
    if (a.do_pop) {
        const int E = (int)((uint32_t)(ke >> 32) ^ 0x80000000u);
        const int r = (int)(ke & 0xFFFFFFFFull);
        if (!bvalid || E < bE) {
            const uint64_t *Xr = a.X + (size_t)(r >> 6) * a.n;
            const int b = r & 63;
            for (int w = tid; w < a.nw32; w += nt) {
                uint32_t bits = 0;
                for (int q = 0; q < 32 && w * 32 + q < a.n; ++q)
                    bits |= (uint32_t)((Xr[w * 32 + q] >> b) & 1ull) << q;
                a.best_x[w] = bits;
            }
            if (tid == 0) {
                brec[0] = E; brec[1] = a.pop_step; brec[2] = a.pop_sweep; brec[3] = r; brec[4] = 1;
            }
            bE = E;
            bvalid = 1;
            if (a.pop_step >= 0) simp = 1;
        }
    }

    if (a.do_rest) {
        const int emin = (int)((uint32_t)(ke >> 32) ^ 0x80000000u);
        long long *st = a.stats + (size_t)a.k * kStatFields;
        if (tid == 0) {
            int level = level_used, stall = stall0;
            if (a.as_enable) {
                if (simp) {
                    level = 0;
                    stall = 0;
                } else {
                    stall += 1;
                    if (stall >= a.as_stall &&
                        (unsigned __int128)(unsigned)a.as_frozen_inv * acc < (unsigned __int128)att) {
                        level = level + 1 < a.as_lmax ? level + 1 : a.as_lmax;
                        stall = 0;
                    }
                }
            }
            a.as_state[0] = level;
            a.as_state[1] = stall;
            a.counters[0] = 0;
            a.counters[1] = 0;
            st[0] = emin; st[1] = es; st[2] = (long long)att; st[3] = (long long)acc;
            st[4] = level_used; st[5] = bE;
            st[6] = 0; st[7] = 0;
            st[8] = g; st[9] = 0;
            if (!resample) a.as_state[3] = a.K;            // the last grid point: run finished
        }
        int jump = 1;
        if (resample && a.adapt) {
            // Largest jump j (<= adapt_jump, within the grid) whose weights
            // keep den (sum W)^2 >= num R sum W^2; wave wv tries j = jmax - wv,
            // jmax - wv - nwv, ... (128-bit sums), jump 1 needs no test.
            const int jmax = a.adapt_jump < a.K - 1 - g ? a.adapt_jump : a.K - 1 - g;
            for (int j = jmax - wv; j >= 2; j -= nwv) {
                const int oj = a.wtab_off[j - 1], lj = a.wtab_len[j - 1];
                unsigned long long s1 = 0, q_lo = 0, q_hi = 0;    // sum W, sum W^2 (128 bit)
                for (int r0 = lane; r0 < R; r0 += 8 * 64) {
                    unsigned long long wv[8];      // eight table reads in flight
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int r = r0 + 64 * c;
                        const int nn = r < R ? Esh[r < R ? r : r0] - emin : lj;
                        wv[c] = nn < lj ? a.wtab[oj + nn] : 0ull;
                    }
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const unsigned long long w = wv[c];
                        s1 += w;
                        const unsigned __int128 w2 = (unsigned __int128)w * w;
                        const unsigned long long l2 = q_lo + (unsigned long long)w2;
                        q_hi += (unsigned long long)(w2 >> 64) + (l2 < q_lo ? 1ull : 0ull);
                        q_lo = l2;
                    }
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) {
                    s1 += __shfl_xor(s1, o, 64);
                    const unsigned long long lo2 = __shfl_xor(q_lo, o, 64), hi2 = __shfl_xor(q_hi, o, 64);
                    const unsigned long long l2 = q_lo + lo2;
                    q_hi += hi2 + (l2 < q_lo ? 1ull : 0ull);
                    q_lo = l2;
                }
                if (lane == 0) {
                    const unsigned __int128 S2 = ((unsigned __int128)q_hi << 64) | q_lo;
                    admissible[j] = (unsigned __int128)s1 * s1 * (uint32_t)a.adapt_den >=
                                    (unsigned __int128)(uint32_t)a.adapt_num * (uint32_t)R * S2;
                }
            }
            __syncthreads();
            for (int j = jmax; j >= 2; --j)
                if (admissible[j]) {
                    jump = j;
                    break;
                }
            off = a.wtab_off[jump - 1];
            len = a.wtab_len[jump - 1];
        }
        if (!resample) {
            // No resampling after the last grid point: the next population is
            // this one (identity parents).
            for (int r = lo; r < hi; ++r) a.parent[r] = r;
        }
        if (resample) {
            // The weights of this thread's replicas, read 8 at a time so that
            // the table reads of a chunk are in flight together.
            constexpr int CH = 8;
            auto weights = [&](int r0, uint64_t (&wv)[CH]) {
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int r = r0 + c < hi ? r0 + c : r0;
                    const int nn = r0 + c < hi ? Esh[r] - emin : len;
                    wv[c] = nn < len ? a.wtab[off + nn] : 0ull;
                }
            };
            // The first chunk's weights stay in registers for the walk below
            // (with R <= 8 x threads it is the thread's only chunk).
            uint64_t w0[CH];
            weights(lo, w0);
            uint64_t ws = 0;
#pragma unroll
            for (int c = 0; c < CH; ++c) ws += w0[c];
            for (int r0 = lo + CH; r0 < hi; r0 += CH) {
                uint64_t wv[CH];
                weights(r0, wv);
#pragma unroll
                for (int c = 0; c < CH; ++c) ws += wv[c];
            }
            // Exclusive scan of the per-thread sums: wave scan, then the wave totals.
            uint64_t inc = ws;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint64_t t = __shfl_up(inc, o, 64);
                if (lane >= o) inc += t;
            }
            if (lane == 63) w_scan[wv] = inc;
            __syncthreads();
            uint64_t before = 0, S = 0;
            for (int v = 0; v < nwv; ++v) {
                const uint64_t x = w_scan[v];
                before += v < wv ? x : 0ull;
                S += x;
            }
            const uint64_t excl = before + inc - ws;
            const U4 o = philox10(U4{0u, 2u << 16, (uint32_t)a.k, a.inst << 16}, a.seed_lo, a.seed_hi);
            const uint64_t U = (uint64_t)o.x | ((uint64_t)o.y << 32);
            const uint64_t u = __umul64hi(U, S);
            // f(c) counts the sampling points u + j S below R c: one division
            // for this thread's first replica, then walk the points (each step
            // is one copy written), so no division per replica.
            uint64_t f = sys_f(excl, (uint64_t)R, u, S);
            uint64_t pt = u + f * S;                    // next sampling point
            uint64_t RC = (uint64_t)R * excl;
            long long parents = 0;
            for (int r0 = lo; r0 < hi; r0 += CH) {
                uint64_t wv[CH];
                if (r0 == lo) {
#pragma unroll
                    for (int c = 0; c < CH; ++c) wv[c] = w0[c];
                } else {
                    weights(r0, wv);
                }
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int r = r0 + c;
                    if (r >= hi) break;
                    RC += (uint64_t)R * wv[c];
                    const uint64_t f0 = f;
                    while (pt < RC) {
                        a.parent[f] = r;
                        ++f;
                        pt += S;
                    }
                    if (a.counts_rec) a.counts_rec[(size_t)a.k * R + r] = (int)(f - f0);
                    parents += f > f0;
                }
            }
            parents = wave_sum_ll(parents);
            if (lane == 0 && parents) atomicAdd((unsigned long long *)&par_total, (unsigned long long)parents);
            __syncthreads();
            if (tid == 0) {
                st[6] = par_total;
                st[7] = (long long)S;
                st[9] = jump;
                a.as_state[3] = g + jump;
            }
        }
    }
    if (tid == 0) {
        for (int q = 0; q < 5; ++q) a.best[q] = brec[q];
        a.as_state[2] = a.do_rest ? 0 : simp;
    }
}

__global__ __launch_bounds__(1024) void epilogue_kernel(EpiArgs a) { epilogue_body(a); }

// The epilogue of one step of many runs in one launch, one workgroup per run
// (launch index t is step t - k_off of a run; the population after step k's
// sweeps is in X1/E1 for even k).
__global__ __launch_bounds__(1024) void epilogue_multi_kernel(const MultiRun *__restrict__ runs, int t)
{
    const MultiRun &m = runs[blockIdx.x];
    const int k = t - m.k_off;
    if (k < 0 || k >= m.steps) return;
    EpiArgs a = m.epi;
    const bool even = (k & 1) == 0;
    a.k = k;
    a.E = even ? m.E1 : m.E0;
    a.X = even ? m.X1 : m.X0;
    a.do_cand = 1;
    a.do_pop = 0;
    a.do_rest = 1;
    epilogue_body(a);
}

// ---------------------------------------------------------------------------
// Resampling gather: slot q takes the spins and energy of parent(q). The
// parents of consecutive slots are non-decreasing, so a wave's 64 loads hit
// one or two groups.
// ---------------------------------------------------------------------------
constexpr int kGatherNodesPerWave = 64;

__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = blockIdx.y;
    const int q = g * 64 + lane;
    const int p = q < a.R ? a.parent[q] : -1;
    const int i0 = (blockIdx.x * 4 + wave) * kGatherNodesPerWave;
    const int pb = p & 63;
    // Systematic resampling hands out slots in parent order, so the lanes of
    // a wave usually read one or two parent words per node, which the memory
    // pipeline merges into one or two cache-line requests.
    const uint64_t *src = a.Xin + (size_t)(p >= 0 ? p >> 6 : 0) * a.n;
    // Batches of 16 loads in flight; indices past the last node are clamped
    // (their words are never stored).
    uint64_t out = 0;
    for (int t0 = 0; t0 < kGatherNodesPerWave; t0 += 16) {
        uint64_t w[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int i = i0 + t0 + u;
            w[u] = src[i < a.n ? i : a.n - 1];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const unsigned long long mask = __ballot(p >= 0 && ((w[u] >> pb) & 1ull));
            if (lane == t0 + u) out = mask;
        }
    }
    // Lane t holds the word of node i0 + t: one coalesced store per wave.
    if (lane < kGatherNodesPerWave && i0 + lane < a.n) a.Xout[(size_t)g * a.n + i0 + lane] = out;
    if (blockIdx.x == 0 && wave == 0 && q < a.R) a.Eout[q] = a.Ein[p];
}

// ---------------------------------------------------------------------------
// Non-local move: Houdayer cluster move on the pair (p, p + R/2). One
// workgroup per pair finds the connected component of the seed node inside
// the disagreement set D with a union-find over the edge list (parents in
// LDS), computes the energy change of replica a from the edges that cross
// the cluster boundary, and writes the cluster bitmap; icm_apply_kernel then
// flips the clusters of all pairs in the population words.
// ---------------------------------------------------------------------------

typedef volatile __attribute__((address_space(3))) uint32_t lds_vu32;

// LDS compare-and-swap on an LDS-typed pointer (a generic pointer would become a FLAT atomic).
__device__ __forceinline__ bool lds_cas(lds_vu32 *p, uint32_t expected, uint32_t desired)
{
    return __atomic_compare_exchange_n(p, &expected, desired, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
}

// Root of x with path halving. Roots are only ever hooked under smaller
// roots and halving links x to an ancestor, so P[x] <= x always holds and
// every step strictly decreases x: the walk ends within n steps.
__device__ __forceinline__ uint32_t uf_find(lds_vu32 *P, uint32_t x)
{
    for (;;) {
        const uint32_t px = P[x];
        if (px >= x) return x;
        const uint32_t ppx = P[px];
        if (ppx != px) P[x] = ppx;
        x = ppx;
    }
}

// Roots of x and y, both paths walked together (one LDS round trip serves a
// step of each), with path halving on both; a walk already at its root
// stays there (its reads return the root itself), and every pass moves the
// other one strictly down, so this ends as uf_find does.
__device__ __forceinline__ void uf_find2(lds_vu32 *P, uint32_t &x, uint32_t &y)
{
    for (;;) {
        const uint32_t px = P[x], py = P[y];
        if (px >= x && py >= y) return;
        const uint32_t ppx = P[px], ppy = P[py];
        if (ppx != px) P[x] = ppx;
        if (ppy != py) P[y] = ppy;
        x = ppx;
        y = ppy;
    }
}

// Bitmap words of nodes base .. base + blockDim.x - 1 from one flag per
// thread (lanes 0 and 32 of each wave write its two words).
__device__ __forceinline__ void label_words(uint32_t *V, int nw, int base, bool in)
{
    const int tid = threadIdx.x, lane = tid & 63;
    const unsigned long long m = __ballot(in);
    const int w0 = (base + (tid & ~63)) >> 5;
    if (lane == 0 && w0 < nw) V[w0] = (uint32_t)m;
    if (lane == 32 && w0 + 1 < nw) V[w0 + 1] = (uint32_t)(m >> 32);
}

// Merge the sets of x and y (lock-free: a failed hook means another lane
// hooked that root, which happens at most once per root).
__device__ __forceinline__ void uf_unite(lds_vu32 *P, uint32_t x, uint32_t y)
{
    for (;;) {
        uf_find2(P, x, y);
        if (x == y) return;
        if (x > y) {
            const uint32_t t = x;
            x = y;
            y = t;
        }
        if (lds_cas(&P[y], y, x)) return;
    }
}

constexpr int kIcmThreads = 512;

int icm_lds_bytes(int n, int nw32)
{
    return (n + 3 * nw32) * 4;
}

__global__ __launch_bounds__(kIcmThreads) void icm_kernel(IcmArgs a)
{
    if (a.adapt && a.as_state[3] >= a.K) return;      // finished run
    // LDS: P = union-find parents [n], bitmaps A = spins of replica a,
    // D = disagreement set, V = cluster (nw words each).
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ long long red_l[16];
    __shared__ int scan_i[kIcmThreads];
    __shared__ uint32_t root_s;
    const int tid = threadIdx.x, lane = tid & 63, nt = blockDim.x;
    const int n = a.g.n, nw = a.nw32;
    lds_vu32 *P = (lds_vu32 *)lds;
    uint32_t *A = lds + n, *D = A + nw, *V = D + nw;
    const int p = blockIdx.x, half = a.R / 2;
    const int ra = p, rb = p + half;
    const int ba = ra & 63, bb = rb & 63;
    const uint64_t *Xa = a.X + (size_t)(ra >> 6) * n;
    const uint64_t *Xb = a.X + (size_t)(rb >> 6) * n;
    uint32_t *Vout = a.vout + (size_t)p * nw;

    // Spins of a, the disagreement set and singleton parents; 4 independent
    // loads per replica in flight per lane.
    int cnt = 0;
    for (int base = 0; base < nw * 32; base += 4 * nt) {
        uint64_t va[4], vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * nt + tid;
            va[u] = i < n ? Xa[i] : 0ull;
            vb[u] = i < n ? Xb[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * nt + tid;
            if (i < n) P[i] = (uint32_t)i;
            const int xa = (int)((va[u] >> ba) & 1ull);
            const int dd = i < n ? xa ^ (int)((vb[u] >> bb) & 1ull) : 0;
            const unsigned long long ma = __ballot(xa), md = __ballot(dd);
            const int w0 = (base + u * nt + (tid & ~63)) >> 5;
            if (lane == 0 && w0 < nw) { A[w0] = (uint32_t)ma; D[w0] = (uint32_t)md; }
            if (lane == 32 && w0 + 1 < nw) { A[w0 + 1] = (uint32_t)(ma >> 32); D[w0 + 1] = (uint32_t)(md >> 32); }
            cnt += dd;
        }
    }
    const long long total = block_sum_ll(cnt, red_l);
    if (total == 0) {
        for (int w = tid; w < nw; w += nt) Vout[w] = 0u;
        return;
    }
    auto inD = [&](uint32_t i) { return (D[i >> 5] >> (i & 31)) & 1u; };
    // Components of the subgraph induced by D. A small D (at most n/16 nodes)
    // walks the adjacency rows of its own nodes; otherwise all edges are
    // scanned (the edge list is in shuffled order, so that the lanes of a
    // wave seldom contend for one root). Both give the same components.
    const uint32_t *edges = a.g.edges;
    const int ne = a.g.ne;
    const bool sparse = total * 16 <= n;
    if (sparse) {
        // Half a bitmap word per thread (all threads busy on small graphs);
        // a row's neighbours are read 8 at a time before any of them is
        // united, so the loads overlap instead of waiting one by one.
        for (int u = tid; u < 2 * nw; u += nt) {
            const int w = u >> 1;
            uint32_t bits = D[w] & ((u & 1) ? 0xFFFF0000u : 0x0000FFFFu);
            while (bits) {
                const uint32_t i = (uint32_t)(w * 32 + __ffs(bits) - 1);
                bits &= bits - 1;
                const int e0 = a.g.row_ptr[i], e1 = a.g.row_ptr[i + 1];
                for (int e = e0; e < e1; e += 8) {
                    uint32_t jv[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) jv[q] = e + q < e1 ? (uint32_t)a.g.col[e + q] : 0u;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (e + q < e1 && jv[q] > i && inD(jv[q])) uf_unite(P, i, jv[q]);
                }
            }
        }
    } else {
        for (int e0 = tid; e0 < ne; e0 += 8 * nt) {
            uint32_t ev[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = e0 + u * nt;
                ev[u] = idx < ne ? edges[idx] : 0u;
            }
            // Only the edges inside D: the wave then runs as many unions as
            // its busiest lane has, not one per edge slot.
            uint32_t pend = 0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t i = ev[u] & 0x7FFFu, j = (ev[u] >> 15) & 0x7FFFu;
                if (e0 + u * nt < ne && inD(i) && inD(j)) pend |= 1u << u;
            }
            while (pend) {
                const int u = __ffs(pend) - 1;
                pend &= pend - 1;
                uint32_t e = ev[0];
#pragma unroll
                for (int v = 1; v < 8; ++v) e = u == v ? ev[v] : e;
                uf_unite(P, e & 0x7FFFu, (e >> 15) & 0x7FFFu);
            }
        }
    }
    // Seed node: the pick-th element of D in node order (scan of per-thread word chunks).
    const uint32_t d = draw(a.seed_lo, a.seed_hi, a.inst, 3, 0, (uint32_t)a.k, 0u, (uint32_t)p);
    const int pick = (int)(((uint64_t)d * (uint64_t)total) >> 32);
    const int per = (nw + nt - 1) / nt;
    const int w_lo = tid * per < nw ? tid * per : nw, w_hi = w_lo + per < nw ? w_lo + per : nw;
    int mine = 0;
    for (int w = w_lo; w < w_hi; ++w) mine += __popc(D[w]);
    scan_i[tid] = mine;
    __syncthreads();        // also completes the unions
    for (int o = 1; o < nt; o <<= 1) {
        const int v = tid >= o ? scan_i[tid - o] : 0;
        __syncthreads();
        scan_i[tid] += v;
        __syncthreads();
    }
    const int before = scan_i[tid] - mine;
    if (pick >= before && pick < before + mine) {
        int c = before, w = w_lo;
        for (; w < w_hi; ++w) {
            const int pc = __popc(D[w]);
            if (c + pc > pick) break;
            c += pc;
        }
        uint32_t bits = D[w];
        for (int t = c; t < pick; ++t) bits &= bits - 1;
        root_s = uf_find(P, (uint32_t)(w * 32 + __ffs(bits) - 1));
    }
    __syncthreads();
    const uint32_t root = root_s;
    // Cluster = the seed's component: two nodes per thread and pass, their
    // roots walked together (nodes outside D start at the root itself).
    for (int base = 0; base < nw * 32; base += 2 * nt) {
        const int i0 = base + tid, i1 = i0 + nt;
        const bool c0 = i0 < n && inD((uint32_t)i0), c1 = i1 < n && inD((uint32_t)i1);
        uint32_t x = c0 ? (uint32_t)i0 : root, y = c1 ? (uint32_t)i1 : root;
        uf_find2(P, x, y);
        label_words(V, nw, base, c0 && x == root);
        label_words(V, nw, base + nt, c1 && y == root);
    }
    __syncthreads();
    // Energy change of replica a: the edges with one end in the cluster
    // change sign (an edge from the cluster to D - cluster cannot exist).
    long long dEa = 0;
    auto bitA = [&](uint32_t i) { return (int)((A[i >> 5] >> (i & 31)) & 1u); };
    if (sparse) {
        for (int u = tid; u < 2 * nw; u += nt) {
            const int w = u >> 1;
            uint32_t bits = V[w] & ((u & 1) ? 0xFFFF0000u : 0x0000FFFFu);
            while (bits) {
                const uint32_t i = (uint32_t)(w * 32 + __ffs(bits) - 1);
                bits &= bits - 1;
                const int e0 = a.g.row_ptr[i], e1 = a.g.row_ptr[i + 1], em = e0 + a.g.npos[i];
                for (int e = e0; e < e1; e += 8) {
                    uint32_t jv[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q) jv[q] = e + q < e1 ? (uint32_t)a.g.col[e + q] : 0u;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const uint32_t j = jv[q];
                        if (e + q >= e1 || ((V[j >> 5] >> (j & 31)) & 1u)) continue;
                        dEa += -2 * (1 - 2 * (bitA(i) ^ bitA(j) ^ (e + q >= em ? 1 : 0)));
                    }
                }
            }
        }
    }
    for (int e0 = tid; e0 < (sparse ? 0 : ne); e0 += 8 * nt) {
        uint32_t ev[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = e0 + u * nt;
            ev[u] = idx < ne ? edges[idx] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = ev[u] & 0x7FFFu, j = (ev[u] >> 15) & 0x7FFFu;
            const uint32_t vi = (V[i >> 5] >> (i & 31)) & 1u, vj = (V[j >> 5] >> (j & 31)) & 1u;
            if (e0 + u * nt < ne && vi != vj) {
                const int bi = (int)((A[i >> 5] >> (i & 31)) & 1u), bj = (int)((A[j >> 5] >> (j & 31)) & 1u);
                const int neg = (int)((ev[u] >> 30) & 1u);
                dEa += -2 * (1 - 2 * (bi ^ bj ^ neg));
            }
        }
    }
    dEa = block_sum_ll(dEa, red_l);
    for (int w = tid; w < nw; w += nt) Vout[w] = V[w];
    if (tid == 0) {
        a.E[ra] += (int)dEa;
        a.E[rb] -= (int)dEa;
    }
}

// ---------------------------------------------------------------------------
// Non-local move, single-replica kind: Wolff's cluster update of every
// replica (couplings J = -w of either sign). One workgroup per replica: the
// satisfied bonds (w_ij x_i x_j < 0) are activated with the step's bond
// threshold, a union-find over the active bonds (LDS parents, as above) gives
// the components, the seed's component is the cluster; the energy change
// comes from the edges that cross its boundary. Bond {i < j} of replica r
// draws word (r & 3) of Philox(key = seed, ctr = (i, j | 5 << 16, k,
// (r >> 2) | inst << 16)); the seed is floor(u N / 2^32) for the tag-4 draw u.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kIcmThreads) void wolff_kernel(IcmArgs a)
{
    if (a.adapt && a.as_state[3] >= a.K) return;      // finished run
    // LDS: P = union-find parents [n], A = spins of the replica, V = cluster.
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ long long red_l[16];
    __shared__ uint32_t root_s;
    const int tid = threadIdx.x, lane = tid & 63, nt = blockDim.x;
    const int n = a.g.n, nw = a.nw32;
    lds_vu32 *P = (lds_vu32 *)lds;
    uint32_t *A = lds + n, *V = A + nw;
    const int r = blockIdx.x, br = r & 63;
    const uint64_t *Xr = a.X + (size_t)(r >> 6) * n;
    uint32_t *Vout = a.vout + (size_t)r * nw;

    for (int base = 0; base < nw * 32; base += 4 * nt) {
        uint64_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * nt + tid;
            v[u] = i < n ? Xr[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * nt + tid;
            if (i < n) P[i] = (uint32_t)i;
            const unsigned long long m = __ballot(i < n && ((v[u] >> br) & 1ull));
            const int w0 = (base + u * nt + (tid & ~63)) >> 5;
            if (lane == 0 && w0 < nw) A[w0] = (uint32_t)m;
            if (lane == 32 && w0 + 1 < nw) A[w0 + 1] = (uint32_t)(m >> 32);
        }
    }
    __syncthreads();
    const uint64_t q = a.qtab[(size_t)(a.adapt ? a.as_state[3] : a.k) * a.lmax1 + a.as_state[0]];
    auto bit = [&](const uint32_t *B, uint32_t i) { return (B[i >> 5] >> (i & 31)) & 1u; };
    // Active bonds: a lane takes 8 edges of the (shuffled) edge list and draws
    // only for the satisfied ones.
    const uint32_t *edges = a.g.edges;
    const int ne = a.g.ne;
    for (int e0 = tid; e0 < ne; e0 += 8 * nt) {
        uint32_t ev[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = e0 + u * nt;
            ev[u] = idx < ne ? edges[idx] : 0u;
        }
        uint32_t pend = 0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = ev[u] & 0x7FFFu, j = (ev[u] >> 15) & 0x7FFFu;
            const uint32_t sat = bit(A, i) ^ bit(A, j) ^ ((ev[u] >> 30) & 1u);
            if (e0 + u * nt < ne && sat) pend |= 1u << u;
        }
        while (pend) {
            const int u = __ffs(pend) - 1;
            pend &= pend - 1;
            uint32_t e = ev[0];
#pragma unroll
            for (int v = 1; v < 8; ++v) e = u == v ? ev[v] : e;
            const uint32_t i = e & 0x7FFFu, j = (e >> 15) & 0x7FFFu;
            // A bond whose ends are already joined cannot change the
            // components: its draw is skipped.
            uint32_t x = i, y = j;
            uf_find2(P, x, y);
            if (x == y) continue;
            const uint32_t d = draw(a.seed_lo, a.seed_hi, a.inst, 5, j, (uint32_t)a.k, i, (uint32_t)r);
            if ((uint64_t)d < q) uf_unite(P, x, y);
        }
    }
    __syncthreads();
    if (tid == 0) {
        const uint32_t d = draw(a.seed_lo, a.seed_hi, a.inst, 4, 0, (uint32_t)a.k, 0u, (uint32_t)r);
        root_s = uf_find(P, (uint32_t)(((uint64_t)d * (uint64_t)n) >> 32));
    }
    __syncthreads();
    const uint32_t root = root_s;
    for (int base = 0; base < nw * 32; base += 2 * nt) {
        const int i0 = base + tid, i1 = i0 + nt;
        uint32_t x = i0 < n ? (uint32_t)i0 : root, y = i1 < n ? (uint32_t)i1 : root;
        uf_find2(P, x, y);
        label_words(V, nw, base, i0 < n && x == root);
        label_words(V, nw, base + nt, i1 < n && y == root);
    }
    __syncthreads();
    // Energy change: each edge with one end in the cluster changes sign.
    long long dE = 0;
    for (int e0 = tid; e0 < ne; e0 += 8 * nt) {
        uint32_t ev[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int idx = e0 + u * nt;
            ev[u] = idx < ne ? edges[idx] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = ev[u] & 0x7FFFu, j = (ev[u] >> 15) & 0x7FFFu;
            if (e0 + u * nt < ne && bit(V, i) != bit(V, j)) {
                const int s = (int)(bit(A, i) ^ bit(A, j) ^ ((ev[u] >> 30) & 1u));
                dE += -2 * (1 - 2 * s);
            }
        }
    }
    dE = block_sum_ll(dE, red_l);
    for (int w = tid; w < nw; w += nt) Vout[w] = V[w];
    if (tid == 0) a.E[r] += (int)dE;
}

// Flip every pair's cluster in both of its replicas (kind 0), or every
// replica's own cluster (kind 1): wave (word w, group g) gathers the 64
// replicas' bits of nodes 32w..32w+31 with ballots.
__global__ __launch_bounds__(256) void icm_apply_kernel(IcmArgs a)
{
    if (a.adapt && a.as_state[3] >= a.K) return;      // finished run
    const int lane = threadIdx.x & 63;
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int g = blockIdx.y;
    if (w >= a.nw32) return;
    const int q = g * 64 + lane, half = a.R / 2;
    const int pr = q < a.R ? (a.kind == 1 ? q : (q < half ? q : q - half)) : -1;
    const uint32_t v = pr >= 0 ? a.vout[(size_t)pr * a.nw32 + w] : 0u;
    uint64_t out = 0;
#pragma unroll
    for (int b = 0; b < 32; ++b) {
        const unsigned long long m = __ballot((v >> b) & 1u);
        if (lane == b) out = m;
    }
    const int i = w * 32 + lane;
    if (lane < 32 && i < a.g.n && out) a.X[(size_t)g * a.g.n + i] ^= out;
}

__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long v, long long count)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static thread_local char g_err[256];

static int check(const char *what)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
        return -1;
    }
    return 0;
}

// Dynamic LDS beyond the default must be allowed per kernel on each device.
// `cfg` holds, per device, the largest size allowed so far for one kernel; the
// mutex keeps concurrent launches from lowering another's setting.
constexpr int kMaxDevices = 64;
static std::mutex g_lds_mu;

static int allow_lds(const void *fn, int *cfg, int lds, const char *what)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return check(what);
    if (dev < 0 || dev >= kMaxDevices) {
        snprintf(g_err, sizeof g_err, "%s: device %d beyond the %d supported", what, dev, kMaxDevices);
        return -1;
    }
    std::lock_guard<std::mutex> lock(g_lds_mu);
    if (cfg[dev] >= lds) return 0;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess)
        return check(what);
    cfg[dev] = lds;
    return 0;
}

const char *last_hip_error() { return g_err; }

int launch_fill_u64(unsigned long long *p, unsigned long long v, long long count, void *stream)
{
    if (count <= 0) return 0;
    const int tb = 256;
    const long long nb = (count + tb - 1) / tb;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)nb), dim3(tb), 0, (hipStream_t)stream, p, v,
                       count);
    return check("fill");
}

int launch_init(const InitArgs &a, void *stream)
{
    const int per_block = 4 * kInitNodesPerWave;
    dim3 grid((a.g.n + per_block - 1) / per_block, a.G);
    hipLaunchKernelGGL(init_kernel, grid, dim3(256), 0, (hipStream_t)stream, a);
    return check("init_kernel");
}

int launch_energy(const InitArgs &a, void *stream)
{
    if (launch_fill_u64(reinterpret_cast<unsigned long long *>(a.E), 0ull, (long long)a.G * 32,
                        stream))
        return -1;
    const int per_block = 4 * kInitNodesPerWave;
    dim3 grid((a.g.n + per_block - 1) / per_block, a.G);
    hipLaunchKernelGGL(energy_kernel, grid, dim3(256), 0, (hipStream_t)stream, a);
    return check("energy_kernel");
}

template <int W, bool SG>
static int launch_sweep_t(int threads, int nblk, const SweepArgs &a, void *stream)
{
    const int lds = sweep_lds_bytes(W, SG ? 1 : 0, a.n, a.dmax, threads);
    static int configured[kMaxDevices] = {};
    if (allow_lds(reinterpret_cast<const void *>(&sweep_kernel<W, SG>), configured, lds,
                  "hipFuncSetAttribute(sweep)"))
        return -1;
    hipLaunchKernelGGL((sweep_kernel<W, SG>), dim3(nblk), dim3(threads), lds, (hipStream_t)stream, a,
                       a.stream, a.level_off, a.blocks);
    return check("sweep_kernel");
}

int launch_sweep(int W, int sgn, int threads, int nblk, const SweepArgs &a, void *stream)
{
    switch (W) {
    case 16: return sgn ? launch_sweep_t<16, true>(threads, nblk, a, stream)
                        : launch_sweep_t<16, false>(threads, nblk, a, stream);
    case 32: return sgn ? launch_sweep_t<32, true>(threads, nblk, a, stream)
                        : launch_sweep_t<32, false>(threads, nblk, a, stream);
    case 64: return sgn ? launch_sweep_t<64, true>(threads, nblk, a, stream)
                        : launch_sweep_t<64, false>(threads, nblk, a, stream);
    default:
        snprintf(g_err, sizeof g_err, "unsupported tile width %d", W);
        return -1;
    }
}

template <int W, int SG, bool D>
static int launch_bytes_t(int threads, int nblk, const SweepArgs &a, void *stream)
{
    const int lds = sweep_bytes_lds(W, SG == 1 ? 1 : 0, a.n, a.dmax);
    // The issue-priority turns are compiled only into 8-replica tiles.
    constexpr bool kHasPrio = W == 8;
    const bool prio = kHasPrio && a.prio_mode == 1;
    const void *fn = prio ? reinterpret_cast<const void *>(&sweep_bytes_kernel<W, SG, D, kHasPrio>)
                          : reinterpret_cast<const void *>(&sweep_bytes_kernel<W, SG, D, false>);
    static int configured[kMaxDevices] = {}, configured_p[kMaxDevices] = {};
    if (allow_lds(fn, prio ? configured_p : configured, lds, "hipFuncSetAttribute(sweep_bytes)")) return -1;
    if (prio)
        hipLaunchKernelGGL((sweep_bytes_kernel<W, SG, D, kHasPrio>), dim3(nblk), dim3(threads), lds,
                           (hipStream_t)stream, a, a.rounds, a.blocks);
    else
        hipLaunchKernelGGL((sweep_bytes_kernel<W, SG, D, false>), dim3(nblk), dim3(threads), lds,
                           (hipStream_t)stream, a, a.rounds, a.blocks);
    return check("sweep_bytes_kernel");
}

template <int W>
static int launch_bytes_w(int sgn, int threads, int nblk, const SweepArgs &a, void *stream)
{
    if (sgn == 2) return a.direct ? launch_bytes_t<W, 2, true>(threads, nblk, a, stream)
                                  : launch_bytes_t<W, 2, false>(threads, nblk, a, stream);
    if (sgn == 1) return a.direct ? launch_bytes_t<W, 1, true>(threads, nblk, a, stream)
                                  : launch_bytes_t<W, 1, false>(threads, nblk, a, stream);
    return a.direct ? launch_bytes_t<W, 0, true>(threads, nblk, a, stream)
                    : launch_bytes_t<W, 0, false>(threads, nblk, a, stream);
}

int launch_sweep_bytes(int W, int sgn, int threads, int nblk, const SweepArgs &a, void *stream)
{
    switch (W) {
    case 4: return launch_bytes_w<4>(sgn, threads, nblk, a, stream);
    case 8: return launch_bytes_w<8>(sgn, threads, nblk, a, stream);
    case 16: return launch_bytes_w<16>(sgn, threads, nblk, a, stream);
    default:
        snprintf(g_err, sizeof g_err, "unsupported byte-tile width %d", W);
        return -1;
    }
}

template <int W, int SG, bool D>
static int launch_multi_t(int threads, int blocks, int lds, const MultiRun *runs, const int2 *work, int k,
                          void *stream)
{
    static int configured[kMaxDevices] = {};
    if (allow_lds(reinterpret_cast<const void *>(&sweep_bytes_multi_kernel<W, SG, D>), configured, lds,
                  "hipFuncSetAttribute(sweep_bytes_multi)"))
        return -1;
    hipLaunchKernelGGL((sweep_bytes_multi_kernel<W, SG, D>), dim3(blocks), dim3(threads), lds,
                       (hipStream_t)stream, runs, work, k);
    return check("sweep_bytes_multi_kernel");
}

template <int W>
static int launch_multi_w(int sgn, bool direct, int threads, int blocks, int lds, const MultiRun *runs,
                          const int2 *work, int k, void *stream)
{
    if (sgn == 2) return direct ? launch_multi_t<W, 2, true>(threads, blocks, lds, runs, work, k, stream)
                                : launch_multi_t<W, 2, false>(threads, blocks, lds, runs, work, k, stream);
    return direct ? launch_multi_t<W, 0, true>(threads, blocks, lds, runs, work, k, stream)
                  : launch_multi_t<W, 0, false>(threads, blocks, lds, runs, work, k, stream);
}

int launch_sweep_multi(int W, int sgn, bool direct, int threads, int blocks, int lds, const MultiRun *runs,
                       const int2 *work, int k, void *stream)
{
    if (sgn == 1) {
        snprintf(g_err, sizeof g_err, "multi-run sweeps take unsigned records or sign bits");
        return -1;
    }
    switch (W) {
    case 4: return launch_multi_w<4>(sgn, direct, threads, blocks, lds, runs, work, k, stream);
    case 8: return launch_multi_w<8>(sgn, direct, threads, blocks, lds, runs, work, k, stream);
    case 16: return launch_multi_w<16>(sgn, direct, threads, blocks, lds, runs, work, k, stream);
    default:
        snprintf(g_err, sizeof g_err, "unsupported byte-tile width %d", W);
        return -1;
    }
}

int launch_epilogue_multi(int runs_count, int max_R, const MultiRun *runs, int k, void *stream)
{
    const int lds = max_R * 4;
    static int configured[kMaxDevices] = {};
    if (allow_lds(reinterpret_cast<const void *>(&epilogue_multi_kernel), configured, lds,
                  "hipFuncSetAttribute(epilogue_multi)"))
        return -1;
    hipLaunchKernelGGL(epilogue_multi_kernel, dim3(runs_count), dim3(kMaxThreads), lds, (hipStream_t)stream,
                       runs, k);
    return check("epilogue_multi_kernel");
}

int launch_epilogue(const EpiArgs &a, void *stream)
{
    const int lds = a.R * 4;
    static int configured[kMaxDevices] = {};
    if (allow_lds(reinterpret_cast<const void *>(&epilogue_kernel), configured, lds,
                  "hipFuncSetAttribute(epilogue)"))
        return -1;
    hipLaunchKernelGGL(epilogue_kernel, dim3(1), dim3(kMaxThreads), lds, (hipStream_t)stream, a);
    return check("epilogue_kernel");
}

int launch_gather(const GatherArgs &a, void *stream)
{
    const int per_block = 4 * kGatherNodesPerWave;
    dim3 grid((a.n + per_block - 1) / per_block, a.G);
    hipLaunchKernelGGL(gather_kernel, grid, dim3(256), 0, (hipStream_t)stream, a);
    return check("gather_kernel");
}

int launch_icm(const IcmArgs &a, void *stream)
{
    const int lds = icm_lds_bytes(a.g.n, a.nw32);
    static int configured[2][kMaxDevices] = {};
    const void *fn = a.kind == 1 ? reinterpret_cast<const void *>(&wolff_kernel)
                                 : reinterpret_cast<const void *>(&icm_kernel);
    if (allow_lds(fn, configured[a.kind == 1 ? 1 : 0], lds, "hipFuncSetAttribute(cluster move)")) return -1;
    if (a.kind == 1) {
        hipLaunchKernelGGL(wolff_kernel, dim3(a.R), dim3(kIcmThreads), lds, (hipStream_t)stream, a);
        if (int st = check("wolff_kernel")) return st;
    } else {
        hipLaunchKernelGGL(icm_kernel, dim3(a.R / 2), dim3(kIcmThreads), lds, (hipStream_t)stream, a);
        if (int st = check("icm_kernel")) return st;
    }
    hipLaunchKernelGGL(icm_apply_kernel, dim3((a.nw32 + 3) / 4, a.G), dim3(256), 0, (hipStream_t)stream, a);
    return check("icm_apply_kernel");
}

// ---------------------------------------------------------------------------
// Static device workspace for callers that cannot allocate device memory
// (pa_run_static). Every device the library runs on holds one copy until the
// process ends. In host code `scratch` names a host-side stand-in, not device
// memory: its device address on the current device comes from
// hipGetSymbolAddress, taken once per device and kept, and only that address
// is ever handed to kernels or copies.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void **ptr)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return check("hipGetDevice(static scratch)");
    if (dev < 0 || dev >= kMaxDevices) {
        snprintf(g_err, sizeof g_err, "static scratch: device %d beyond the %d supported", dev, kMaxDevices);
        return -1;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            snprintf(g_err, sizeof g_err, "hipGetSymbolAddress(static scratch) on device %d: %s", dev,
                     hipGetErrorString(e));
            (void)hipGetLastError();
            return -1;
        }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return 0;
}

}  // namespace pa
