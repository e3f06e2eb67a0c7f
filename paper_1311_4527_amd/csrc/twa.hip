// twa.hip -- gfx950 kernels and host runtime of the three-weight
// message-passing trajectory planner behind the C ABI of include/twa.h.
//
// One iteration (App. B, steps 1-7) is three launches on the solver stream:
//   k_stream  coalesced walk over all factors.  Collision factors by
//             columns: a wave holds one chunk of 64 pairs (i, j0..j0+63) of
//             the pair triangle across several break-point intervals; wall,
//             energy, velocity-limit and fixed factors one lane each.
//             Collision and wall factors get the closest-approach /
//             segment-distance activity test on n = z - u (Sec. 3.3.1-3.3.2
//             weight rule); factors that are active, or were active last
//             iteration, are appended to a work queue (one wave-aggregated
//             atomic, the collision queue sharded over 32 counters).
//             Energy, velocity-limit and fixed factors finish here.
//   k_queue   one wave per workgroup over the queue: the full non-convex
//             minimiser (App. C, D, I; a wall factor on two lanes), the u
//             update of the previous iteration (fused, see below),
//             m = x + u, and the consensus sums.
//   k_nodes   one lane per break-point node: z = weighted mean (step 5),
//             <-rho (step 6), clear the sums.
// The u update (step 7) of iteration k needs z^{k+1}, so it is deferred
// into the next iteration: the queue keeps x^k of the factors active in
// iteration k, the energy factors recompute it from (z^{k-1}, u^{k-1}) --
// bitwise the same arithmetic -- and u is updated in registers, so it is
// read once and written once per iteration.
// Consensus sums are accumulated as exact 64-bit fixed-point integers with
// atomics, so the result does not depend on the order of the additions.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/twa.h"
#include "prox.h"
#include "solver.h"

using namespace twa;
using twa_rt::Params;

// ------------------------------------------------------------------ device memory provider
namespace twa_rt {

namespace {
std::mutex g_alloc_mutex;
twa_alloc_fn g_alloc = nullptr;
twa_free_fn g_release = nullptr;
void *g_alloc_ctx = nullptr;
} // namespace

Allocator current_allocator(int device) {
    std::lock_guard<std::mutex> lock(g_alloc_mutex);
    Allocator a;
    a.alloc = g_alloc;
    a.release = g_release;
    a.ctx = g_alloc_ctx;
    a.device = device;
    return a;
}

void *Allocator::get(size_t bytes, hipStream_t stream) const {
    void *p = nullptr;
    if (alloc) {
        p = alloc(bytes, device, stream, ctx);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    return p;
}

void Allocator::put(void *ptr, size_t bytes, hipStream_t stream) const {
    if (!ptr) return;
    if (release) release(ptr, bytes, device, stream, ctx);
    else (void)hipFree(ptr);
}

} // namespace twa_rt

extern "C" twa_status twa_set_allocator(twa_alloc_fn alloc, twa_free_fn release, void *ctx) {
    if ((alloc == nullptr) != (release == nullptr)) return TWA_E_INVALID;
    std::lock_guard<std::mutex> lock(twa_rt::g_alloc_mutex);
    twa_rt::g_alloc = alloc;
    twa_rt::g_release = release;
    twa_rt::g_alloc_ctx = alloc ? ctx : nullptr;
    return TWA_OK;
}

#define TWA_VERSION "twa-mi355x 0.1"

namespace {

constexpr int kBlock = 256;

// The collision queue is cut into kShards shards with their lengths 256 B
// apart: a wave of the factor stream appends to shard (wave mod kShards), so
// the appends of the whole grid do not serialise on one address.  A shard
// holds every factor its waves could append (no overflow is possible).
constexpr int kShards = 32;
constexpr int kQueueStride = 64;

enum Mode : int { M_FIRST = 0, M_FUSED = 1, M_FINAL = 2 };

// what the per-segment factors are (twa_create flags)
enum Cost : int { COST_ENERGY = 0, COST_NONE = 1, COST_MAXVEL = 2, COST_MINVEL = 3 };

// queue entry flags
constexpr unsigned kPrev = 0x80000000u; // factor was active last iteration: recompute and update u
constexpr unsigned kIdx = 0x7fffffffu;

// Where the per-factor code reads node records: this and last iteration's
// (global memory, or a workgroup's copy in LDS in the batched kernel).
struct Rec {
    const float4 *cur, *prev;
};



using twa_rt::wval;

__device__ __forceinline__ int wcode(float4 r) { return (int)r.w; }

// wave-aggregated append of `val` where pred holds; all lanes must call
__device__ __forceinline__ void push(unsigned *q, int *len, bool pred, unsigned val) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return;
    int lane = __lane_id();
    int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(len, __popcll(mask));
    base = __shfl(base, leader);
    if (pred) q[base + __popcll(mask & ((1ull << lane) - 1ull))] = val;
}

__device__ __forceinline__ void count_wave(int *ctr, bool pred) {
    unsigned long long mask = __ballot(pred);
    if (mask && __lane_id() == __ffsll((long long)mask) - 1) atomicAdd(ctr, __popcll(mask));
}

// One edge's m into the exact fixed-point consensus sums of its node.  A
// value beyond the headroom (or not finite) raises the sticky overflow flag
// that twa_check_finite and twa_get_stats report: up to a node's degree of
// contributions below sat_lim cannot wrap the 64-bit sum.
__device__ __forceinline__ void contribute(const Params &P, long long node, int kind, const float *m, int D) {
    for (int k = 0; k < D; ++k) {
        float v = m[k] * P.scalef;
        if (!(fabsf(v) <= P.sat_lim)) P.counters[5] = 1;
        v = fminf(fmaxf(v, -4.0e18f), 4.0e18f);
        long long q = __float2ll_rn(v);
        atomicAdd(&P.acc[((long long)kind * D + k) * P.N + node], (unsigned long long)q);
    }
    atomicAdd(&P.cnt[(long long)kind * P.N + node], 1);
}

// The consensus contributions of one queued minimiser (up to four nodes),
// handed from the minimiser to the wave-level sum below.
struct Contrib {
    int n = 0;         // nodes contributed to (0, 2 or 4)
    unsigned skip = 0; // slot k is left out where bit k is set (fixed_node)
    long long nd[4];
    float m[4][3];
};

// Break-point s of every agent is a fixed start or goal: its fixed factor
// sends weight infinity in every iteration (App. B step 5 then takes z from
// that edge alone), so an ordinary (rho0) contribution to such a node never
// enters z, its <-rho or the adjoint's mean sets and is not made.  Standard
// ADMM sends rho0 from the fixed factors too; a VO epoch's reference end is
// soft.
__device__ __forceinline__ bool fixed_node(const Params &P, int s) {
    return !P.admm && (s == 0 || (s == P.eta && !P.vo));
}

// Contributions of every lane of a wave (all lanes call it; lanes with
// k >= c.n, or with slot k skipped, give nothing).  Slots 0 and 1 are agent i's nodes (s, i) and
// (s+1, i), which the queued collision factors of one pair-row chunk, and
// the wall factors of one agent and interval, share: there the lanes with
// the same node are summed across the wave first, so the node takes one
// atomic per component per group instead of one per lane (up to two groups
// are formed, the second only if the first had company; the remaining
// lanes add directly).  Slots 2 and 3 (agent j, a
// different node on every lane of a chunk) add directly.  The sums are exact
// integers, so the result does not depend on the grouping.
template <bool GROUP>
__device__ __forceinline__ void contribute_wave(const Params &P, const Contrib &c, int D) {
    const int lane = __lane_id();
    for (int k = 0; k < 4; ++k) {
        bool pred = k < c.n && !((c.skip >> k) & 1u);
        if (__ballot(pred) == 0ull) continue;
        const long long node = pred ? c.nd[k] : -1;
        long long q[3] = {0, 0, 0};
        if (pred)
            for (int d = 0; d < D; ++d) {
                float v = c.m[k][d] * P.scalef;
                if (!(fabsf(v) <= P.sat_lim)) P.counters[5] = 1;
                v = fminf(fmaxf(v, -4.0e18f), 4.0e18f);
                q[d] = __float2ll_rn(v);
            }
        for (int g = 0; g < (GROUP && k < 2 ? 2 : 0); ++g) {
            const unsigned long long pending = __ballot(pred);
            if (pending == 0ull) break;
            const int leader = __ffsll((long long)pending) - 1;
            const long long key = __shfl(node, leader);
            const bool mine = pred && node == key;
            const unsigned long long peers = __ballot(mine);
            long long sum[3];
            for (int d = 0; d < 3; ++d) sum[d] = mine ? q[d] : 0;
            if (__popcll(peers) > 1)
                for (int o = 1; o < 64; o <<= 1)
                    for (int d = 0; d < D; ++d) sum[d] += __shfl_xor(sum[d], o);
            if (lane == leader) {
                for (int d = 0; d < D; ++d) atomicAdd(&P.acc[(long long)d * P.N + key], (unsigned long long)sum[d]);
                atomicAdd(&P.cnt[key], (int)__popcll(peers));
            }
            pred = pred && !mine;
            if (__popcll(peers) == 1) break; // the nodes are spread: the rest add directly
        }
        if (pred) {
            for (int d = 0; d < D; ++d) atomicAdd(&P.acc[(long long)d * P.N + node], (unsigned long long)q[d]);
            atomicAdd(&P.cnt[node], 1);
        }
    }
}

// Finalizing pass only: fold |x - z| of an edge whose u is updated (both
// weights rho0) into the residual maximum (non-negative floats order as
// their bit patterns).
__device__ __forceinline__ void residual(const Params &P, const float *x, const float *z, int D) {
    float d2 = 0.f;
    for (int c = 0; c < D; ++c) d2 += (x[c] - z[c]) * (x[c] - z[c]);
    atomicMax(P.resid, __float_as_uint(sqrtf(d2)));
}

// (s, i, j) of factor f0 + k given (s, i, j) of f0: walk along the rows of
// the upper triangle (row i holds p-1-i pairs); 32-bit adds only.
__device__ __forceinline__ void advance_pair(int p, int k, int &s, int &i, int &j) {
    int c = j - i - 1 + k;
    int L = p - 1 - i;
    while (c >= L) {
        c -= L;
        if (++i >= p - 1) {
            i = 0;
            ++s;
        }
        L = p - 1 - i;
    }
    j = i + 1 + c;
}

// (s, i, w) of wall factor f0 + k given (s, i, w) of f0
__device__ __forceinline__ void advance_wall(int p, int W, int k, int &s, int &i, int &w) {
    int c = w + k;
    while (c >= W) {
        c -= W;
        if (++i >= p) {
            i = 0;
            ++s;
        }
    }
    w = c;
}

template <int D>
__device__ __forceinline__ void load_u_coll(const Params &P, long long f, float *u) {
    float4 a = P.u_coll[f];
    float4 b = P.u_coll[P.Fc + f];
    u[0] = a.x, u[1] = a.y, u[2] = a.z, u[3] = a.w;
    u[4] = b.x, u[5] = b.y, u[6] = b.z, u[7] = b.w;
    if constexpr (D == 3) {
        float4 c = P.u_coll[2 * P.Fc + f];
        u[8] = c.x, u[9] = c.y, u[10] = c.z, u[11] = c.w;
    }
}
template <int D>
__device__ __forceinline__ void load_x_coll(const Params &P, long long f, float *x) {
    float4 a = P.x_coll[f];
    float4 b = P.x_coll[P.Fc + f];
    x[0] = a.x, x[1] = a.y, x[2] = a.z, x[3] = a.w;
    x[4] = b.x, x[5] = b.y, x[6] = b.z, x[7] = b.w;
    if constexpr (D == 3) {
        float4 c = P.x_coll[2 * P.Fc + f];
        x[8] = c.x, x[9] = c.y, x[10] = c.z, x[11] = c.w;
    }
}
template <int D>
__device__ __forceinline__ void store_x_coll(const Params &P, long long f, const float *x) {
    P.x_coll[f] = make_float4(x[0], x[1], x[2], x[3]);
    P.x_coll[P.Fc + f] = make_float4(x[4], x[5], x[6], x[7]);
    if constexpr (D == 3) P.x_coll[2 * P.Fc + f] = make_float4(x[8], x[9], x[10], x[11]);
}
template <int D>
__device__ __forceinline__ void store_u_coll(const Params &P, long long f, const float *u) {
    P.u_coll[f] = make_float4(u[0], u[1], u[2], u[3]);
    P.u_coll[P.Fc + f] = make_float4(u[4], u[5], u[6], u[7]);
    if constexpr (D == 3) P.u_coll[2 * P.Fc + f] = make_float4(u[8], u[9], u[10], u[11]);
}

// four node records of a collision factor: (i,s), (i,s+1), (j,s), (j,s+1)
__device__ __forceinline__ void coll_nodes(const Params &P, int s, int i, int j, long long *nd) {
    nd[0] = (long long)s * P.p + i;
    nd[1] = (long long)(s + 1) * P.p + i;
    nd[2] = (long long)s * P.p + j;
    nd[3] = (long long)(s + 1) * P.p + j;
}

template <int D>
__device__ __forceinline__ bool coll_active(const float *n, float R) {
    // n: 4 edges x D; relative positions agent j - agent i at s and s+1
    f3 d0{n[2 * D + 0] - n[0], n[2 * D + 1] - n[1], D == 3 ? n[2 * D + 2] - n[2] : 0.f};
    f3 d1{n[3 * D + 0] - n[D + 0], n[3 * D + 1] - n[D + 1], D == 3 ? n[3 * D + 2] - n[D + 2] : 0.f};
    return cpa_below(d0, d1, R * R);
}

__device__ __forceinline__ void node_xyz(float4 r, float *z, int D) {
    z[0] = r.x, z[1] = r.y;
    if (D == 3) z[2] = r.z;
}

// ------------------------------------------------------------------ per-factor work
// Node record read through the scalar cache: for an address that is the
// same for the whole wave (agent i of a collision column).  Only for arrays
// the running kernel does not write.
__device__ __forceinline__ float4 load_uniform(const float4 *p, long long idx) {
    const __attribute__((address_space(4))) float *q = (const __attribute__((address_space(4))) float *)p + 4 * idx;
    return make_float4(q[0], q[1], q[2], q[3]);
}
__device__ __forceinline__ float load_uniform(const float *p, long long idx) {
    return ((const __attribute__((address_space(4))) float *)p)[idx];
}
__device__ __forceinline__ unsigned long long load_uniform(const unsigned long long *p, long long idx) {
    return ((const __attribute__((address_space(4))) unsigned long long *)p)[idx];
}
__device__ __forceinline__ int load_uniform(const int *p, long long idx) {
    return ((const __attribute__((address_space(4))) int *)p)[idx];
}

// Collision factor f given its four node records ((i,s), (i,s+1), (j,s),
// (j,s+1): current, and the previous iteration's for the dense form) and
// its u as loaded: activity test on n = z - u and the queue decision.
// word: the chunk's activity bits.
template <int D, int MODE, bool DENSE>
__device__ __forceinline__ bool coll_factor(const Params &P, long long f, float R, const float4 *rc, const float4 *rp,
                                            float *u, unsigned long long word, int lane, unsigned *val) {
    constexpr bool dense = DENSE;
    bool push_prev = false, push_new = false;
    float n[4 * D];
    bool check_cur = true;
    if (MODE == M_FIRST) {
        // u as loaded
    } else if (dense && P.admm) {
        // standard ADMM: every factor sent weight rho0 last iteration
        push_prev = true;
        check_cur = false;
    } else if (dense) {
        float zz[3];
        for (int e = 0; e < 4; ++e) {
            node_xyz(rp[e], zz, D);
            for (int k = 0; k < D; ++k) n[e * D + k] = zz[k] - u[e * D + k];
        }
        if (coll_active<D>(n, R)) {
            push_prev = true;
            check_cur = false;
        } else {
            // zero weight resets u; a u that is zero already (the common
            // case) is not written again, so the pass only reads u
            unsigned nz = 0u;
            for (int k = 0; k < 4 * D; ++k) nz |= __float_as_uint(u[k]);
            for (int k = 0; k < 4 * D; ++k) u[k] = 0.f;
            if (nz) store_u_coll<D>(P, f, u);
        }
    } else {
        if ((word >> lane) & 1ull) {
            push_prev = true;
            check_cur = false;
        } else {
            for (int k = 0; k < 4 * D; ++k) u[k] = 0.f;
        }
    }
    if (MODE == M_FINAL) {
        check_cur = false;
        if (!dense && !push_prev) store_u_coll<D>(P, f, u); // zero
    }
    if (check_cur) {
        float zz[3];
        for (int e = 0; e < 4; ++e) {
            node_xyz(rc[e], zz, D);
            for (int k = 0; k < D; ++k) n[e * D + k] = zz[k] - u[e * D + k];
        }
        push_new = P.admm || coll_active<D>(n, R);
        if (!push_new && P.dbg_rho) {
            long long e0 = P.e_coll + 4 * f;
            if (P.dbg_x)
                for (int k = 0; k < 4 * D; ++k) P.dbg_x[e0 * D + k] = n[k];
            P.dbg_rho[P.f_coll + f] = W_ZERO;
        }
    }
    *val = (unsigned)f | (push_prev ? kPrev : 0u);
    return push_prev || push_new;
}

// Collision column col: the pairs (i, j0 + lane) of one chunk of row i of
// the pair triangle (rows are cut into chunks of 64, so i is the same for
// the whole wave), over the break-point intervals s0 <= s < s1 <= s0 + CPW.
// Every load of the column (node records of break-points s0..s1, agent i's
// through the scalar cache when SCALAR_I, i.e. when Z points to global
// memory; the chunks' activity words; u where it is read) is issued before
// any factor is evaluated.  With clear_bits each chunk's activity word is
// cleared after it was read (the minimisers set it again for the factors
// active in this iteration).  Queued factors are appended to qs (length
// *qlen).
template <int D, int MODE, int CPW, bool DENSE, bool SCALAR_I>
__device__ __forceinline__ void coll_column(const Params &P, const Rec &Z, int col, int s0, int s1, int lane,
                                            bool clear_bits, unsigned *qs, int *qlen) {
    constexpr bool need_prev = DENSE && MODE != M_FIRST;
    constexpr bool need_u = DENSE || MODE == M_FIRST;
    constexpr bool need_word = !DENSE && MODE != M_FIRST;
    const int cu = __builtin_amdgcn_readfirstlane(col);
    const unsigned long long pk = load_uniform(P.chunk_coll, cu);
    const int i = (int)(pk >> 24), j0 = (int)(pk & 0xffffffull);
    const int p = P.p;
    const int j = j0 + lane;
    const bool valid = j < p;
    const int jj = valid ? j : j0; // in-bounds address for idle lanes
    const float R = load_uniform(P.radii, i) + P.radii[jj];
    // canonical index of (s, i, j) is s p(p-1)/2 + fr (all factor indices
    // fit in 31 bits): row i of the triangle holds the pairs (i, j > i)
    const unsigned fr = (unsigned)((long long)i * (2 * p - i - 1) / 2 + (j - i - 1));
    const unsigned P2 = (unsigned)P.P2;
    const float4 *ci = Z.cur + (long long)s0 * p + i, *cj = Z.cur + (long long)s0 * p + jj;
    const float4 *pi_ = Z.prev + (long long)s0 * p + i, *pj_ = Z.prev + (long long)s0 * p + jj;
    float4 ri[CPW + 1], rj[CPW + 1], pi[CPW + 1], pj[CPW + 1];
    unsigned long long word[CPW];
    float u[CPW][4 * D];
#pragma unroll
    for (int k = 0; k <= CPW; ++k) {
        if (s0 + k <= s1) {
            ri[k] = SCALAR_I ? load_uniform(ci, k * p) : ci[k * p];
            rj[k] = cj[k * p];
            if (need_prev) {
                pi[k] = SCALAR_I ? load_uniform(pi_, k * p) : pi_[k * p];
                pj[k] = pj_[k * p];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
        word[k] = 0ull;
        for (int q = 0; q < 4 * D; ++q) u[k][q] = 0.f;
        if (s0 + k < s1) {
            if (need_word) word[k] = P.bits_coll[(s0 + k) * (int)P.cps + cu];
            if (need_u && valid) load_u_coll<D>(P, (s0 + k) * P2 + fr, u[k]);
        }
    }
    // every factor of the column first, then the stores: the activity words
    // and the queue appends do not wait on each other's round trips
    bool q[CPW];
    unsigned val[CPW];
#pragma unroll
    for (int k = 0; k < CPW; ++k) {
        q[k] = false;
        val[k] = 0u;
        if (s0 + k < s1 && valid) {
            const float4 rc[4] = {ri[k], ri[k + 1], rj[k], rj[k + 1]};
            const float4 rp[4] = {pi[k], pi[k + 1], pj[k], pj[k + 1]};
            q[k] = coll_factor<D, MODE, DENSE>(P, (s0 + k) * P2 + fr, R, rc, rp, u[k], word[k], lane, &val[k]);
        }
    }
    if (clear_bits && lane == 0) {
#pragma unroll
        for (int k = 0; k < CPW; ++k)
            if (s0 + k < s1) P.bits_coll[(s0 + k) * (int)P.cps + cu] = 0ull;
    }
    bool any = false;
#pragma unroll
    for (int k = 0; k < CPW; ++k) any = any || q[k];
    if (__ballot(any) == 0ull) return; // nothing to queue: the common case
#pragma unroll
    for (int k = 0; k < CPW; ++k)
        if (s0 + k < s1) push(qs, qlen, q[k], val[k]);
}

// Collision factors f0 + k step (k < U) of a flat walk over the canonical
// order (64 consecutive factors per wave, rows mixed): the batched kernel's
// form for small instances, whose rows are shorter than a wave.  Every load
// of the U factors is issued before any is evaluated.  Reads each factor's
// activity bit from its row chunk's word without clearing it (the words are
// cleared in a separate pass once every factor has read its bit); queued
// factors are appended to the one queue of length *qlen.
template <int D, int MODE, int U>
__device__ __forceinline__ void coll_flat(const Params &P, const Rec &Z, long long f0, long long step, int *qlen) {
    const bool dense = P.dense != 0;
    long long f[U];
    bool valid[U];
    int s[U], i[U], j[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        f[k] = f0 + k * step;
        valid[k] = f[k] < P.Fc;
        const int fw = __builtin_amdgcn_readfirstlane((int)f[k]);
        const unsigned long long pk = fw < P.Fc ? P.wbase_coll[fw >> 6] : 0ull;
        s[k] = (int)(pk >> 48), i[k] = (int)((pk >> 24) & 0xffffffull), j[k] = (int)(pk & 0xffffffull);
        if (valid[k]) advance_pair(P.p, (int)(f[k] - fw), s[k], i[k], j[k]);
    }
    float4 rc[U][4], rp[U][4];
    float u[U][4 * D];
    unsigned long long word[U];
    float R[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        word[k] = 0ull;
        R[k] = 0.f;
        for (int q = 0; q < 4 * D; ++q) u[k][q] = 0.f;
        if (valid[k]) {
            long long nd[4];
            coll_nodes(P, s[k], i[k], j[k], nd);
            for (int e = 0; e < 4; ++e) rc[k][e] = Z.cur[nd[e]];
            for (int e = 0; e < 4; ++e) rp[k][e] = rc[k][e];
            if (dense || MODE == M_FIRST) load_u_coll<D>(P, f[k], u[k]);
            if (dense && MODE != M_FIRST)
                for (int e = 0; e < 4; ++e) rp[k][e] = Z.prev[nd[e]];
            const int r = j[k] - i[k] - 1;
            if (!dense && MODE != M_FIRST)
                word[k] = P.bits_coll[(long long)s[k] * P.cps + P.rowchunk[i[k]] + (r >> 6)] >> (r & 63);
            R[k] = P.radii[i[k]] + P.radii[j[k]];
        }
    }
    bool q[U];
    unsigned val[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        q[k] = false;
        val[k] = 0u;
        if (valid[k]) {
            if (dense) q[k] = coll_factor<D, MODE, true>(P, f[k], R[k], rc[k], rp[k], u[k], word[k], 0, &val[k]);
            else q[k] = coll_factor<D, MODE, false>(P, f[k], R[k], rc[k], rp[k], u[k], word[k], 0, &val[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) push(P.qc, qlen, q[k], val[k]);
}

// Where wall factor f sits: (s, i, wall), its two node records, the wall's
// end points and agent i's radius.
struct WallAt {
    long long f;
    int s, i, w;
    long long na, nb;
    float4 wl;
    float r;
};

__device__ __forceinline__ WallAt wall_at(const Params &P, long long f, unsigned long long pk, int k) {
    WallAt a;
    a.f = f;
    a.s = (int)(pk >> 48), a.i = (int)((pk >> 24) & 0xffffffull), a.w = (int)(pk & 0xffffffull);
    advance_wall(P.p, P.W, k, a.s, a.i, a.w);
    a.na = (long long)a.s * P.p + a.i;
    a.nb = a.na + P.p;
    a.wl = P.walls[a.w];
    a.r = P.radii[a.i];
    return a;
}

// Wall factor a: activity test (segment distance) and queue decision.  bit:
// the factor's activity bit (read only in the activity-bit form after the
// first iteration).
template <int MODE>
__device__ __forceinline__ bool wall_test(const Params &P, const Rec &Z, const WallAt &a, bool bit, unsigned *val) {
    const bool dense = P.dense != 0;
    const long long f = a.f;
    bool push_prev = false, push_new = false;
    const float4 wl = a.wl;
    f2 xa = mk(wl.x, wl.y), xb = mk(wl.z, wl.w);
    const float r = a.r;
    float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
    bool check_cur = true;
    if (MODE == M_FIRST) {
        u = P.u_wall[f];
    } else if (dense && P.admm) {
        push_prev = true;
        check_cur = false;
    } else if (dense) {
        u = P.u_wall[f];
        float4 za = Z.prev[a.na], zb = Z.prev[a.nb];
        f2 n0 = mk(za.x - u.x, za.y - u.y), n1 = mk(zb.x - u.z, zb.y - u.w);
        if (segseg_sq(n0, n1, xa, xb) < r * r) {
            push_prev = true;
            check_cur = false;
        } else {
            const unsigned nz = __float_as_uint(u.x) | __float_as_uint(u.y) | __float_as_uint(u.z) |
                                __float_as_uint(u.w);
            u = make_float4(0.f, 0.f, 0.f, 0.f);
            if (nz) P.u_wall[f] = u;
        }
    } else if (bit) {
        push_prev = true;
        check_cur = false;
    }
    if (MODE == M_FINAL) {
        check_cur = false;
        if (!dense && !push_prev) P.u_wall[f] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (check_cur) {
        float4 za = Z.cur[a.na], zb = Z.cur[a.nb];
        f2 n0 = mk(za.x - u.x, za.y - u.y), n1 = mk(zb.x - u.z, zb.y - u.w);
        push_new = P.admm || segseg_sq(n0, n1, xa, xb) < r * r;
        if (!push_new && P.dbg_rho) {
            long long e0 = P.e_wall + 2 * f;
            if (P.dbg_x) {
                P.dbg_x[e0 * 2 + 0] = n0.x, P.dbg_x[e0 * 2 + 1] = n0.y;
                P.dbg_x[e0 * 2 + 2] = n1.x, P.dbg_x[e0 * 2 + 3] = n1.y;
            }
            P.dbg_rho[P.f_wall + f] = W_ZERO;
        }
    }
    *val = (unsigned)f | (push_prev ? kPrev : 0u);
    return push_prev || push_new;
}

// Wall factor f of the stream (lanes of a wave take consecutive factors).
template <int MODE>
__device__ __forceinline__ void wall_stream(const Params &P, const Rec &Z, long long f, bool valid, bool *q,
                                            unsigned *val) {
    int fw = __builtin_amdgcn_readfirstlane((int)f);
    // (a wave whose first factor is past the end has no valid lane)
    unsigned long long pk = fw < P.Fw ? P.wbase_wall[fw >> 6] : 0ull;
    *q = false;
    *val = (unsigned)f;
    if (valid) {
        const WallAt a = wall_at(P, f, pk, (int)(f - fw));
        const bool bit = P.dense == 0 && MODE != M_FIRST && ((P.bits_wall[f >> 5] >> (f & 31)) & 1u);
        *q = wall_test<MODE>(P, Z, a, bit, val);
    }
}

// Per-segment factor of agent i between break-points s and s+1: the energy
// minimiser (App. E, always weight rho0), a velocity limit (App. F, G:
// weight rho0 while the limit binds, else zero and x = n) or no cost at all
// (feasibility only: weight zero).  Returns x in x[] and whether the factor
// sends weight rho0.
template <int D>
__device__ __forceinline__ bool segment_prox(const Params &P, float C, const float *n, int ka, int kb, float rho,
                                             float *x) {
    if (P.cost == COST_ENERGY) {
        for (int c = 0; c < D; ++c)
            energy_prox(n[c], n[D + c], wval(ka, rho), wval(kb, rho), ka, kb, C, x[c], x[D + c]);
        return true;
    }
    if (P.cost == COST_NONE) {
        for (int q = 0; q < 2 * D; ++q) x[q] = n[q];
        return P.admm != 0;
    }
    const bool bind = vel_prox<D>(n, n + D, wval(ka, rho), wval(kb, rho), ka, kb, C, P.cost == COST_MINVEL, x, x + D);
    return bind || P.admm;
}

// Per-segment factor f: finished here.
template <int D, int MODE>
__device__ __forceinline__ void energy_stream(const Params &P, const Rec &Z, long long f) {
    int i = (int)f / P.eta, s = (int)f - i * P.eta;
    long long na = (long long)s * P.p + i, nb = na + P.p;
    float C = P.C[f];
    float *up = P.u_energy + f * 2 * D;
    float u[6], n[6];
    for (int q = 0; q < 2 * D; ++q) u[q] = up[q];
    float4 ca = Z.cur[na], cb = Z.cur[nb];
    float zc[6];
    node_xyz(ca, zc, D);
    node_xyz(cb, zc + D, D);
    int ka = wcode(ca), kb = wcode(cb);
    if (MODE != M_FIRST) {
        // recompute x^k and ->rho^k from (z^{k-1}, u^{k-1}), then u^k
        float4 pa = Z.prev[na], pb = Z.prev[nb];
        float zp[6];
        node_xyz(pa, zp, D);
        node_xyz(pb, zp + D, D);
        float xk[6];
        for (int q = 0; q < 2 * D; ++q) n[q] = zp[q] - u[q];
        const bool sent = segment_prox<D>(P, C, n, wcode(pa), wcode(pb), P.rho_prev, xk);
        for (int c = 0; c < D; ++c) {
            u[c] = (sent && ka == W_STD) ? u[c] + P.step_prev * (xk[c] - zc[c]) : 0.f;
            u[D + c] = (sent && kb == W_STD) ? u[D + c] + P.step_prev * (xk[D + c] - zc[D + c]) : 0.f;
        }
        for (int q = 0; q < 2 * D; ++q) up[q] = u[q];
        if (MODE == M_FINAL) {
            if (sent && ka == W_STD) residual(P, xk, zc, D);
            if (sent && kb == W_STD) residual(P, xk + D, zc + D, D);
            return;
        }
    }
    float x[6], m[6];
    for (int q = 0; q < 2 * D; ++q) n[q] = zc[q] - u[q];
    const bool send = segment_prox<D>(P, C, n, ka, kb, P.rho, x);
    if (send) {
        for (int q = 0; q < 2 * D; ++q) m[q] = x[q] + u[q];
        if (!fixed_node(P, s)) contribute(P, na, 0, m, D);
        if (!fixed_node(P, s + 1)) contribute(P, nb, 0, m + D, D);
    }
    if (P.dbg_rho) {
        long long e0 = P.e_energy + 2 * f;
        if (P.dbg_x)
            for (int q = 0; q < 2 * D; ++q) P.dbg_x[e0 * D + q] = x[q];
        P.dbg_rho[P.f_energy + f] = send ? W_STD : W_ZERO;
    }
}

// Goal factor of a velocity-obstacle epoch (Sec. 5, App. H): the VO cost
// c |x - x^ref|^2 as the energy minimiser with its reference end certain
// (eq. minimizer_rvo_cost), always weight rho0.
template <int D>
__device__ __forceinline__ void vo_cost_prox(const float4 &xref, float C, const float *n, int k, float rho, float *x) {
    const float r[3] = {xref.x, xref.y, xref.z};
    for (int c = 0; c < D; ++c) {
        float lo;
        energy_prox(r[c], n[c], 0.f, wval(k, rho), W_INF, k, C, lo, x[c]);
    }
}

template <int D, int MODE>
__device__ __forceinline__ void vo_goal_stream(const Params &P, const Rec &Z, long long f) {
    const int i = (int)(f >> 1);
    const long long nd = (long long)P.eta * P.p + i;
    const float C = P.C[i];
    const float4 xr = P.xfix[f];
    float *up = P.u_fixed + f * D;
    float u[3], n[3], x[3], m[3], zc[3];
    for (int c = 0; c < D; ++c) u[c] = up[c];
    const float4 rc = Z.cur[nd];
    node_xyz(rc, zc, D);
    const int k = wcode(rc);
    if (MODE != M_FIRST) {
        // recompute x^k from (z^{k-1}, u^{k-1}), then u^k (weight rho0 both ways)
        const float4 rp = Z.prev[nd];
        float zp[3], xk[3];
        node_xyz(rp, zp, D);
        for (int c = 0; c < D; ++c) n[c] = zp[c] - u[c];
        vo_cost_prox<D>(xr, C, n, wcode(rp), P.rho_prev, xk);
        for (int c = 0; c < D; ++c) u[c] = (k == W_STD) ? u[c] + P.step_prev * (xk[c] - zc[c]) : 0.f, up[c] = u[c];
        if (MODE == M_FINAL) {
            if (k == W_STD) residual(P, xk, zc, D);
            return;
        }
    }
    for (int c = 0; c < D; ++c) n[c] = zc[c] - u[c];
    vo_cost_prox<D>(xr, C, n, k, P.rho, x);
    for (int c = 0; c < D; ++c) m[c] = x[c] + u[c];
    contribute(P, nd, 0, m, D);
    if (P.dbg_rho) {
        if (P.dbg_x)
            for (int c = 0; c < D; ++c) P.dbg_x[f * D + c] = x[c];
        P.dbg_rho[f] = W_STD;
    }
}

// Fixed start/goal factor f: x = const, weight infinity.
template <int D, int MODE>
__device__ __forceinline__ void fixed_stream(const Params &P, const Rec &Z, long long f) {
    if (P.vo && (f & 1)) {
        vo_goal_stream<D, MODE>(P, Z, f);
        return;
    }
    int i = (int)(f >> 1);
    int s = (f & 1) ? P.eta : 0;
    long long nd = (long long)s * P.p + i;
    float *up = P.u_fixed + f * D;
    float u[3];
    for (int c = 0; c < D; ++c) u[c] = up[c];
    float4 xf = P.xfix[f];
    float x[3] = {xf.x, xf.y, xf.z}, m[3];
    if (MODE != M_FIRST) {
        if (P.admm) {
            // weight rho0 both ways: the ordinary update with z^k
            float zc[3];
            node_xyz(Z.cur[nd], zc, D);
            for (int c = 0; c < D; ++c) u[c] = u[c] + P.step_prev * (x[c] - zc[c]), up[c] = u[c];
            if (MODE == M_FINAL) residual(P, x, zc, D);
        } else {
            // ->rho^{k-1} = infinity, so u^k = 0
            for (int c = 0; c < D; ++c) u[c] = 0.f, up[c] = 0.f;
        }
        if (MODE == M_FINAL) return;
    }
    for (int c = 0; c < D; ++c) m[c] = x[c] + u[c];
    contribute(P, nd, P.admm ? 0 : 1, m, D);
    if (!P.admm) P.inf_val[nd] = make_float4(m[0], m[1], D == 3 ? m[2] : 0.f, 0.f);
    if (P.dbg_rho) {
        if (P.dbg_x)
            for (int c = 0; c < D; ++c) P.dbg_x[f * D + c] = x[c];
        P.dbg_rho[f] = P.admm ? W_STD : W_INF;
    }
}

// Where collision factor f sits: (s, i, j), its four node records and the
// radius sum.
struct CollAt {
    long long f;
    int s, i, j;
    long long nd[4];
    float R;
};

__device__ __forceinline__ CollAt coll_at(const Params &P, long long f) {
    CollAt c;
    c.f = f;
    unsigned long long pk = P.wbase_coll[f >> 6];
    c.s = (int)(pk >> 48), c.i = (int)((pk >> 24) & 0xffffffull), c.j = (int)(pk & 0xffffffull);
    advance_pair(P.p, (int)(f & 63), c.s, c.i, c.j);
    coll_nodes(P, c.s, c.i, c.j, c.nd);
    c.R = P.radii[c.i] + P.radii[c.j];
    return c;
}

// Collision factor c taken from the queue (prev: it was active last
// iteration): deferred u update, full minimiser, consensus contributions.
// SET_BITS: mark the factor active in its chunk's activity word.
template <int D, int MODE, bool SET_BITS = true>
__device__ __forceinline__ bool coll_minimise(const Params &P, const Rec &Z, const CollAt &c, bool prev, float *nout,
                                              Contrib &out, const float4 *rc_in = nullptr) {
    const bool dense = P.dense != 0;
    const long long f = c.f;
    const int s = c.s, i = c.i, j = c.j;
    const long long *nd = c.nd;
    const float R = c.R;
    float u[4 * D], zc[4 * D], n[4 * D], x[4 * D], w[4];
    int k[4];
    float4 rc[4];
    // rc_in: the four current records as the caller already loaded them
    for (int q = 0; q < 4; ++q) {
        rc[q] = rc_in ? rc_in[q] : Z.cur[nd[q]];
        node_xyz(rc[q], zc + q * D, D);
        k[q] = wcode(rc[q]);
    }
    if (prev) {
        // x^k was stored when the factor was active last iteration
        load_u_coll<D>(P, f, u);
        load_x_coll<D>(P, f, x);
        for (int q = 0; q < 4; ++q)
            for (int c = 0; c < D; ++c)
                u[q * D + c] =
                    (k[q] == W_STD) ? u[q * D + c] + P.step_prev * (x[q * D + c] - zc[q * D + c]) : 0.f;
        if (MODE == M_FINAL) {
            store_u_coll<D>(P, f, u);
            for (int q = 0; q < 4; ++q)
                if (k[q] == W_STD) residual(P, x + q * D, zc + q * D, D);
            return false;
        }
    } else if (MODE == M_FIRST) {
        load_u_coll<D>(P, f, u);
    } else {
        for (int q = 0; q < 4 * D; ++q) u[q] = 0.f;
    }
    for (int q = 0; q < 4 * D; ++q) n[q] = zc[q] - u[q];
    if (P.adj_pool)
        for (int q = 0; q < 4 * D; ++q) nout[q] = n[q];
    bool act = coll_active<D>(n, R);
    if (act) {
        for (int q = 0; q < 4; ++q) w[q] = wval(k[q], P.rho);
        coll_prox<D>(n, w, k, R, x);
        out.n = 4;
        out.skip = (fixed_node(P, s) ? 5u : 0u) | (fixed_node(P, s + 1) ? 10u : 0u);
        for (int q = 0; q < 4; ++q) {
            out.nd[q] = nd[q];
            for (int c = 0; c < D; ++c) out.m[q][c] = x[q * D + c] + u[q * D + c];
        }
        store_x_coll<D>(P, f, x);
        if (SET_BITS) {
            const int r = j - i - 1;
            atomicOr(&P.bits_coll[(long long)s * P.cps + P.rowchunk[i] + (r >> 6)], 1ull << (r & 63));
        }
    } else {
        for (int q = 0; q < 4 * D; ++q) x[q] = n[q];
        if (P.admm) {
            // standard ADMM: x = n still carries weight rho0 (no fixed nodes)
            out.n = 4;
            for (int q = 0; q < 4; ++q) {
                out.nd[q] = nd[q];
                for (int c = 0; c < D; ++c) out.m[q][c] = x[q * D + c] + u[q * D + c];
            }
            store_x_coll<D>(P, f, x);
        }
    }
    if (MODE == M_FUSED && ((prev && (dense || act)) || (!prev && !dense))) store_u_coll<D>(P, f, u);
    if (P.dbg_rho) {
        long long e0 = P.e_coll + 4 * f;
        if (P.dbg_x)
            for (int q = 0; q < 4 * D; ++q) P.dbg_x[e0 * D + q] = x[q];
        P.dbg_rho[P.f_coll + f] = (act || P.admm) ? W_STD : W_ZERO;
    }
    return act;
}

// Queued collision factor (entry e)
template <int D, int MODE>
__device__ __forceinline__ bool coll_queue(const Params &P, const Rec &Z, unsigned e, float *nout, Contrib &out) {
    return coll_minimise<D, MODE>(P, Z, coll_at(P, e & kIdx), (e & kPrev) != 0, nout, out);
}

// The same minimiser on two lanes (lanes 2k and 2k+1 hold the same factor,
// `piece` = lane & 1): each lane solves one smooth piece of the capsule, the
// two results meet by a lane exchange, and both lanes finish identically.
// Bitwise equal to capsule_prox: the exchange keeps piece 0's candidate on
// equal F, as the sequential order does.  Device only; both lanes of a pair
// must call it together.
__device__ __forceinline__ void capsule_prox_pair(const Capsule C, f2 n0, f2 n1, float w0, float w1, int k0, int k1,
                                                  int piece, f2 &x0, f2 &x1) {
    bool i0 = k0 == W_INF, i1 = k1 == W_INF;
    if ((i0 && i1) || i0 || i1) {
        capsule_prox(C, n0, n1, w0, w1, k0, k1, x0, x1);
        return;
    }
    f2 d = sub(C.b, C.a);
    float L2 = dot(d, d);
    bool seg = L2 > 0.f;
    f2 sw = seg ? scl(perp(d), inv_sqrt(L2)) : mk(0.f, 1.f);
    CapBest mine;
    if (piece == 0 || seg) capsule_piece(C, n0, n1, w0, w1, piece, d, seg, mine);
    CapBest other;
    other.F = __shfl_xor(mine.F, 1);
    other.u.x = __shfl_xor(mine.u.x, 1);
    other.u.y = __shfl_xor(mine.u.y, 1);
    other.kind = __shfl_xor(mine.kind, 1);
    other.ctr = __shfl_xor(mine.ctr, 1);
    const CapBest &a = piece ? other : mine, &b = piece ? mine : other;
    CapBest bb = a;
    if (b.kind != CH_NONE && (b.F < bb.F || bb.kind == CH_NONE)) bb = b;
    capsule_finish(C, n0, n1, w0, w1, d, L2, seg, sw, bb, x0, x1, nullptr);
}

// Wall factor a taken from the queue (prev: it was active last iteration).
// piece < 0: one lane; 0 or 1: the two lanes of a pair share the minimiser
// (capsule_prox_pair) and lane 0 writes.  SET_BITS: mark the factor active in
// its activity word.
template <int MODE, bool SET_BITS = true>
__device__ __forceinline__ bool wall_minimise(const Params &P, const Rec &Z, const WallAt &a, bool prev, int piece,
                                              float *nout, Contrib &out) {
    const bool writer = piece <= 0;
    const bool dense = P.dense != 0;
    const long long f = a.f, na = a.na, nb = a.nb;
    const float4 wl = a.wl;
    Capsule Cw{mk(wl.x, wl.y), mk(wl.z, wl.w), a.r};
    float4 ca = Z.cur[na], cb = Z.cur[nb];
    int ka = wcode(ca), kb = wcode(cb);
    float4 u = make_float4(0.f, 0.f, 0.f, 0.f);
    if (prev) {
        // x^k was stored when the factor was active last iteration
        u = P.u_wall[f];
        float4 xs = P.x_wall[f];
        f2 x0 = mk(xs.x, xs.y), x1 = mk(xs.z, xs.w);
        u.x = (ka == W_STD) ? u.x + P.step_prev * (x0.x - ca.x) : 0.f;
        u.y = (ka == W_STD) ? u.y + P.step_prev * (x0.y - ca.y) : 0.f;
        u.z = (kb == W_STD) ? u.z + P.step_prev * (x1.x - cb.x) : 0.f;
        u.w = (kb == W_STD) ? u.w + P.step_prev * (x1.y - cb.y) : 0.f;
        if (MODE == M_FINAL) {
            if (writer) {
                P.u_wall[f] = u;
                const float za[2] = {ca.x, ca.y}, zb[2] = {cb.x, cb.y}, xa[2] = {x0.x, x0.y}, xb[2] = {x1.x, x1.y};
                if (ka == W_STD) residual(P, xa, za, 2);
                if (kb == W_STD) residual(P, xb, zb, 2);
            }
            return false;
        }
    } else if (MODE == M_FIRST) {
        u = P.u_wall[f];
    }
    f2 n0 = mk(ca.x - u.x, ca.y - u.y), n1 = mk(cb.x - u.z, cb.y - u.w);
    if (P.adj_pool) nout[0] = n0.x, nout[1] = n0.y, nout[2] = n1.x, nout[3] = n1.y;
    bool act = segseg_sq(n0, n1, Cw.a, Cw.b) < Cw.r * Cw.r;
    f2 x0 = n0, x1 = n1;
    if (act) {
        if (piece < 0) capsule_prox(Cw, n0, n1, wval(ka, P.rho), wval(kb, P.rho), ka, kb, x0, x1);
        else capsule_prox_pair(Cw, n0, n1, wval(ka, P.rho), wval(kb, P.rho), ka, kb, piece, x0, x1);
    }
    if (!writer) return act;
    if (act || P.admm) {
        // (standard ADMM: x = n still carries weight rho0)
        P.x_wall[f] = make_float4(x0.x, x0.y, x1.x, x1.y);
        out.n = 2;
        out.skip = (fixed_node(P, a.s) ? 1u : 0u) | (fixed_node(P, a.s + 1) ? 2u : 0u);
        out.nd[0] = na, out.nd[1] = nb;
        out.m[0][0] = x0.x + u.x, out.m[0][1] = x0.y + u.y;
        out.m[1][0] = x1.x + u.z, out.m[1][1] = x1.y + u.w;
        if (SET_BITS && act) atomicOr(&P.bits_wall[f >> 5], 1u << (f & 31));
    }
    if (MODE == M_FUSED && ((prev && (dense || act)) || (!prev && !dense))) P.u_wall[f] = u;
    if (P.dbg_rho) {
        long long e0 = P.e_wall + 2 * f;
        if (P.dbg_x) {
            P.dbg_x[e0 * 2 + 0] = x0.x, P.dbg_x[e0 * 2 + 1] = x0.y;
            P.dbg_x[e0 * 2 + 2] = x1.x, P.dbg_x[e0 * 2 + 3] = x1.y;
        }
        P.dbg_rho[P.f_wall + f] = (act || P.admm) ? W_STD : W_ZERO;
    }
    return act;
}

// Queued wall factor (entry e)
template <int MODE>
__device__ __forceinline__ bool wall_queue(const Params &P, const Rec &Z, unsigned e, int piece, float *nout,
                                           Contrib &out) {
    const long long f = e & kIdx;
    return wall_minimise<MODE>(P, Z, wall_at(P, f, P.wbase_wall[f >> 6], (int)(f & 63)), (e & kPrev) != 0, piece,
                               nout, out);
}

// Node nd: z and <-rho of the next iteration, shift records, clear sums.
template <int D>
__device__ __forceinline__ void node_update(const Params &P, long long nd) {
    int ci = P.cnt[P.N + nd], cs = P.cnt[nd];
    float4 cur = P.zr_cur[nd];
    float4 nw = cur;
    if (ci == 1) {
        // a single certain edge (the fixed start or goal): z is its m exactly
        float4 v = P.inf_val[nd];
        nw.x = v.x;
        nw.y = v.y;
        if (D == 3) nw.z = v.z;
        nw.w = (float)W_INF;
    } else if (ci > 0 || cs > 0) {
        int kind = ci > 0 ? 1 : 0;
        double den = (double)(ci > 0 ? ci : cs) * P.scale;
        float z[3];
        for (int c = 0; c < D; ++c) {
            long long a = (long long)P.acc[((long long)kind * D + c) * P.N + nd];
            z[c] = (float)((double)a / den);
        }
        nw.x = z[0];
        nw.y = z[1];
        if (D == 3) nw.z = z[2];
        nw.w = (float)(ci > 0 ? W_INF : W_STD);
    } else {
        // every incoming weight zero: each m equals z (x = n for an inactive
        // factor), so the mean of step 5 is z itself
        nw.w = (float)W_ZERO;
    }
    P.zr_prev[nd] = cur;
    P.zr_cur[nd] = nw;
    if (P.dbg_l) {
        const long long i = nd % P.p, s = nd / P.p;
        P.dbg_l[i * (P.eta + 1) + s] = (unsigned char)(int)nw.w;
        P.dbg_cnt[i * (P.eta + 1) + s] = ci > 0 ? ci : cs;
    }
    for (int kind = 0; kind < 2; ++kind) {
        for (int c = 0; c < D; ++c) P.acc[((long long)kind * D + c) * P.N + nd] = 0ull;
        P.cnt[(long long)kind * P.N + nd] = 0;
    }
}

// ------------------------------------------------------------------ plain kernels
// DENSE: the literal dense form (u of every edge read; written where it
// changes); it walks four break-point intervals per wave, the activity-bit
// form eight.
template <int D, int MODE, bool DENSE>
__device__ __forceinline__ void stream_block(const Params &P, long long b) {
    constexpr int CPW = DENSE ? 4 : 8;
    const bool clear_bits = MODE != M_FINAL && P.dense == 0;
    const Rec Z{P.zr_cur, P.zr_prev};
    if (b < P.nbc) {
        // wave -> (column, block of CPW break-point intervals); consecutive
        // waves take consecutive columns of the same intervals
        const unsigned wave = (unsigned)b * (kBlock / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const unsigned cps = (unsigned)P.cps;
        const int col = (int)(wave % cps), s0 = (int)(wave / cps) * CPW;
        const int shard = (int)(wave % kShards);
        if (s0 < P.eta)
            coll_column<D, MODE, CPW, DENSE, true>(P, Z, col, s0, min(s0 + CPW, P.eta), threadIdx.x & 63, clear_bits,
                                                   P.qc + (long long)shard * P.qcap, &P.qcnt[shard * kQueueStride]);
    } else if (b < P.nbc + P.nbw) {
        long long f = (b - P.nbc) * kBlock + threadIdx.x;
        bool valid = f < P.Fw, q;
        unsigned val;
        wall_stream<MODE>(P, Z, f, valid, &q, &val);
        if (clear_bits) {
            __syncthreads();
            if (valid && (f & 31) == 0) P.bits_wall[f >> 5] = 0u;
        }
        push(P.qw, &P.counters[1], q, val);
    } else if (b < P.nbc + P.nbw + P.nbe) {
        long long f = (b - P.nbc - P.nbw) * kBlock + threadIdx.x;
        if (f < P.Fe) energy_stream<D, MODE>(P, Z, f);
    } else {
        long long f = (b - P.nbc - P.nbw - P.nbe) * kBlock + threadIdx.x;
        if (f < P.Ff) fixed_stream<D, MODE>(P, Z, f);
    }
}

template <int D, int MODE, bool DENSE>
__global__ __launch_bounds__(kBlock) void k_stream(Params P) {
    stream_block<D, MODE, DENSE>(P, blockIdx.x);
}

// twa_backward's recompute: append (factor, n) of the lanes whose factor sent
// weight rho0 from its minimiser, one atomic per wave.  All lanes call it.
template <int D>
__device__ __forceinline__ void adj_append(const Params &P, bool pred, unsigned f, bool wall, const float *n) {
    const unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return;
    const int lane = __lane_id(), leader = __ffsll((long long)mask) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(P.adj_cursor, (unsigned)__popcll(mask));
    base = __shfl(base, leader);
    const unsigned idx = base + (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
    if (pred && idx < P.adj_cap) {
        twa_rt::AdjRec r;
        r.f = f;
        r.wall = wall ? 1u : 0u;
        for (int q = 0; q < 8; ++q) r.n[q] = (wall && q >= 4) ? 0.f : n[q];
        P.adj_pool[idx] = r;
    }
}

// One queue entry per lane of a wave-uniform loop: collision entries first,
// wall entries from the next multiple of 64 (a wave never mixes the two
// minimisers, whose run times differ several-fold); piece: which lane of a
// wall entry's pair (-1: the entry has one lane).  GROUP: sum agent i's
// contributions across the wave first (the grid-wide queue kernels; in one
// workgroup with the sums in LDS, or few waves, direct atomics are cheaper).
template <int D, int MODE, bool GROUP>
__device__ __forceinline__ void queue_entry(const Params &P, const Rec &Z, bool is_coll, bool is_wall, unsigned e,
                                            int piece) {
    bool ac = false, aw = false;
    float n[4 * D];
    Contrib c;
    if (is_coll) ac = coll_queue<D, MODE>(P, Z, e, n, c);
    else if (is_wall) aw = wall_queue<MODE>(P, Z, e, piece, n, c) && piece <= 0;
    if (MODE != M_FINAL) contribute_wave<GROUP>(P, c, D);
    count_wave(&P.counters[2], ac);
    count_wave(&P.counters[3], aw);
    if (P.adj_pool) adj_append<D>(P, ac || aw, e & kIdx, aw, n);
}

// One wave per workgroup: the few busy waves land on different compute
// units instead of sharing one unit's scalar pipeline and caches.  Entry t
// of the collision queue is entry t - pre[q] of shard q, where pre holds the
// prefix sums of the shard lengths and pre[q] <= t < pre[q + 1].
template <int D, int MODE>
__device__ __forceinline__ void queue_block(const Params &P, long long qb, long long nqb) {
    __shared__ int pre[kShards + 1];
    const int lane = threadIdx.x;
    int v = lane < kShards ? P.qcnt[lane * kQueueStride] : 0;
    for (int d = 1; d < kShards; d <<= 1) {
        const int o = __shfl_up(v, d);
        if (lane >= d) v += o;
    }
    if (lane < kShards) pre[lane + 1] = v;
    if (lane == 0) pre[0] = 0;
    const int nqc = __shfl(v, kShards - 1);
    __syncthreads();
    const int nqw = P.counters[1];
    // wall entries take two lanes each (capsule_prox_pair)
    const long long wall0 = ((long long)nqc + 63) & ~63LL, total = wall0 + 2LL * nqw;
    const long long stride = nqb * 64;
    const Rec Z{P.zr_cur, P.zr_prev};
    for (long long t0 = qb * 64; t0 < total; t0 += stride) {
        const long long t = t0 + lane;
        const bool is_coll = t < nqc, is_wall = t >= wall0 && t < total;
        unsigned e = 0u;
        if (is_coll) {
            int lo = 0, hi = kShards;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (pre[mid] <= t) lo = mid;
                else hi = mid;
            }
            e = P.qc[(long long)lo * P.qcap + (t - pre[lo])];
        } else if (is_wall) {
            e = P.qw[(t - wall0) >> 1];
        }
        queue_entry<D, MODE, true>(P, Z, is_coll, is_wall, e, (int)((t - wall0) & 1));
    }
}

template <int D, int MODE>
__global__ __launch_bounds__(64) void k_queue(Params P) {
    queue_block<D, MODE>(P, blockIdx.x, gridDim.x);
}

// counters of this iteration -> stats, then reset for the next one (the
// first `shards` collision queue shards were in use)
__device__ __forceinline__ void close_counters(const Params &P, int shards) {
    int nq = P.counters[1];
    for (int q = 0; q < shards; ++q) {
        nq += P.qcnt[q * kQueueStride];
        P.qcnt[q * kQueueStride] = 0;
    }
    P.stats[0] = P.counters[2];
    P.stats[1] = P.counters[3];
    P.stats[2] = nq;
    P.counters[1] = P.counters[2] = P.counters[3] = 0;
}

// close_counters by the first wave of a block, one lane per queue shard
__device__ __forceinline__ void close_counters_wave(const Params &P) {
    const int lane = threadIdx.x & 63;
    int v = 0;
    if (lane < kShards) {
        v = P.qcnt[lane * kQueueStride];
        P.qcnt[lane * kQueueStride] = 0;
    }
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
    if (lane == 0) {
        P.stats[0] = P.counters[2];
        P.stats[1] = P.counters[3];
        P.stats[2] = v + P.counters[1];
        P.counters[1] = P.counters[2] = P.counters[3] = 0;
        if (P.adj_offs) *P.adj_offs = *P.adj_cursor;
    }
}

template <int D>
__device__ __forceinline__ void nodes_block(const Params &P, long long b) {
    long long nd = b * kBlock + threadIdx.x;
    if (b == 0 && threadIdx.x < 64) close_counters_wave(P);
    if (nd < P.N) node_update<D>(P, nd);
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_nodes(Params P) {
    nodes_block<D>(P, blockIdx.x);
}

// A batched kernel's instance parameters, copied into LDS by the block: read
// through a pointer into global memory, every field used after a store
// would be fetched again (the compiler cannot tell that the stores leave
// them alone); in LDS they are cheap to reread.
template <int T>
__device__ __forceinline__ const Params &params_lds(const Params *src, Params *dst) {
    static_assert(sizeof(Params) % 4 == 0, "Params is copied as 32-bit words");
    constexpr int n = (int)(sizeof(Params) / 4);
    for (int t = threadIdx.x; t < n; t += T) reinterpret_cast<int *>(dst)[t] = reinterpret_cast<const int *>(src)[t];
    __syncthreads();
    return *dst;
}

// ------------------------------------------------------------------ batched persistent kernel
// One workgroup owns a bin of whole instances and runs all K iterations of
// each of them; the three phases of an iteration are separated by
// workgroup barriers only (instances are independent), so no workgroup
// ever waits for another.  The per-factor work is the plain solver's, so a
// batched instance evolves bitwise as it would on its own.  The instance's
// node records are copied into LDS at the start of each of its iterations
// when they fit (this iteration's, and last iteration's too in the dense
// form), so the walk and the minimisers read them from there; the queue
// lengths are workgroup-local counters.
constexpr int kBatchLdsNodes = 4000; // 62.5 KiB of node records per workgroup

template <int D, int MODE, int BLOCK>
__device__ __forceinline__ void batch_instance(const Params &P, float4 *zs, int *len) {
    const bool clear_bits = P.dense == 0;
    const bool stage = P.N <= kBatchLdsNodes;
    const bool stage_prev = P.dense && MODE != M_FIRST && 2 * P.N <= kBatchLdsNodes;
    if (stage)
        for (long long nd = threadIdx.x; nd < P.N; nd += BLOCK) zs[nd] = P.zr_cur[nd];
    if (stage_prev)
        for (long long nd = threadIdx.x; nd < P.N; nd += BLOCK) zs[P.N + nd] = P.zr_prev[nd];
    if (threadIdx.x == 0) len[0] = len[1] = 0;
    __syncthreads();
    const Rec Z{stage ? zs : P.zr_cur, stage_prev ? zs + P.N : P.zr_prev};
    if (P.p >= 64) {
        // rows of at least 64 pairs for the most part: the column walk of
        // the plain factor stream, wave by wave over (column, intervals)
        const unsigned w0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        const unsigned cps = (unsigned)P.cps;
        if (P.dense) {
            const unsigned nw = cps * (unsigned)((P.eta + 1) / 2);
            for (unsigned w = w0; w < nw; w += BLOCK / 64) {
                const int s0 = (int)(w / cps) * 2;
                coll_column<D, MODE, 2, true, false>(P, Z, (int)(w % cps), s0, min(s0 + 2, P.eta), threadIdx.x & 63,
                                                     false, P.qc, &len[0]);
            }
        } else {
            const unsigned nw = cps * (unsigned)((P.eta + 3) / 4);
            for (unsigned w = w0; w < nw; w += BLOCK / 64) {
                const int s0 = (int)(w / cps) * 4;
                coll_column<D, MODE, 4, false, false>(P, Z, (int)(w % cps), s0, min(s0 + 4, P.eta), threadIdx.x & 63,
                                                      false, P.qc, &len[0]);
            }
        }
    } else {
        for (long long base = 0; base < P.Fc; base += 2 * BLOCK)
            coll_flat<D, MODE, 2>(P, Z, base + threadIdx.x, BLOCK, &len[0]);
    }
    // The wall, energy and fixed factors start at the first wave the kinds
    // before them leave idle in their first round (whole waves, so each wave
    // still takes consecutive factors): in a small instance the kinds run
    // side by side instead of one after another on the first waves.
    auto round64 = [](long long n) { return (int)((std::min<long long>(n, BLOCK) + 63) / 64 * 64); };
    const long long lanes_c =
        P.p >= 64 ? 64LL * P.cps * (P.dense ? (P.eta + 1) / 2 : (P.eta + 3) / 4) : P.Fc;
    const int shift_w = round64(lanes_c) % BLOCK;
    const int shift_e = (shift_w + round64(P.Fw)) % BLOCK;
    const int shift_f = (shift_e + round64(P.Fe)) % BLOCK;
    const int tw = (threadIdx.x + BLOCK - shift_w) % BLOCK, te = (threadIdx.x + BLOCK - shift_e) % BLOCK,
              tf = (threadIdx.x + BLOCK - shift_f) % BLOCK;
    for (long long base = 0; base < P.Fw; base += BLOCK) {
        long long f = base + tw;
        bool valid = f < P.Fw, q;
        unsigned val;
        wall_stream<MODE>(P, Z, f, valid, &q, &val);
        push(P.qw, &len[1], q, val);
    }
    for (long long f = te; f < P.Fe; f += BLOCK) energy_stream<D, MODE>(P, Z, f);
    for (long long f = tf; f < P.Ff; f += BLOCK) fixed_stream<D, MODE>(P, Z, f);
    __syncthreads();
    if (clear_bits) {
        // every factor has read its activity bit: clear the words for the queue
        for (long long w = threadIdx.x; w < P.nch; w += BLOCK) P.bits_coll[w] = 0ull;
        for (long long w = threadIdx.x; w < (P.Fw + 31) / 32; w += BLOCK) P.bits_wall[w] = 0u;
        __syncthreads();
    }
    const int nqc = len[0], nqw = len[1];
    const long long wall0 = ((long long)nqc + 63) & ~63LL, total = wall0 + nqw;
    for (long long t0 = threadIdx.x & ~63; t0 < total; t0 += BLOCK) {
        const long long t = t0 + (threadIdx.x & 63);
        const bool is_coll = t < nqc, is_wall = t >= wall0 && t < total;
        queue_entry<D, MODE, false>(P, Z, is_coll, is_wall, is_coll ? P.qc[t] : is_wall ? P.qw[t - wall0] : 0u, -1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        P.qcnt[0] = nqc;
        P.counters[1] = nqw;
        close_counters(P, 1);
    }
    for (long long nd = threadIdx.x; nd < P.N; nd += BLOCK) node_update<D>(P, nd);
    __syncthreads();
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch(const Params *insts, const int *bin_start, const int *bin_items,
                                                  int K, int first) {
    __shared__ float4 zs[kBatchLdsNodes];
    __shared__ int len[2];
    __shared__ Params sp;
    const int g = blockIdx.x;
    const int q0 = bin_start[g], q1 = bin_start[g + 1];
    for (int it = 0; it < K; ++it) {
        const bool fst = first && it == 0;
        for (int q = q0; q < q1; ++q) {
            const Params &P = params_lds<BLOCK>(insts + bin_items[q], &sp);
            if (P.dim == 2) {
                if (fst) batch_instance<2, M_FIRST, BLOCK>(P, zs, len);
                else batch_instance<2, M_FUSED, BLOCK>(P, zs, len);
            } else {
                if (fst) batch_instance<3, M_FIRST, BLOCK>(P, zs, len);
                else batch_instance<3, M_FUSED, BLOCK>(P, zs, len);
            }
        }
    }
}

// ------------------------------------------------------------------ clearance measures
// squared distance from q to the segment [a, b] (planar)
__device__ __forceinline__ double pt_seg2(double qx, double qy, double ax, double ay, double bx, double by) {
    const double ex = bx - ax, ey = by - ay, ee = ex * ex + ey * ey;
    double t = 0.0;
    if (ee > 0.0) t = fmin(fmax(((qx - ax) * ex + (qy - ay) * ey) / ee, 0.0), 1.0);
    const double vx = qx - (ax + t * ex), vy = qy - (ay + t * ey);
    return vx * vx + vy * vy;
}

// twice the signed area of (a, b, c)
__device__ __forceinline__ double cross3(double ax, double ay, double bx, double by, double cx, double cy) {
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

// Clearance of agents i and j over one interval: closest approach of the two
// constant-velocity motions a -> b minus ri + rj (Sec. 2).
__device__ __forceinline__ double pair_clearance(float4 ai, float4 bi, float4 aj, float4 bj, double ri, double rj) {
    // relative position at the interval's ends; closest approach over the interval
    const double d0x = (double)aj.x - ai.x, d0y = (double)aj.y - ai.y, d0z = (double)aj.z - ai.z;
    const double ex = ((double)bj.x - bi.x) - d0x, ey = ((double)bj.y - bi.y) - d0y, ez = ((double)bj.z - bi.z) - d0z;
    const double ee = ex * ex + ey * ey + ez * ez;
    double a = 0.0;
    if (ee > 0.0) a = fmin(fmax(-(d0x * ex + d0y * ey + d0z * ez) / ee, 0.0), 1.0);
    const double vx = d0x + a * ex, vy = d0y + a * ey, vz = d0z + a * ez;
    return sqrt(vx * vx + vy * vy + vz * vz) - (ri + rj);
}

// Clearance of agent i's interval a -> b from a wall (planar): segment
// distance minus ri (Sec. 3.2).
__device__ __forceinline__ double wall_clearance(float4 ai, float4 bi, float4 wl, double ri) {
    const double px = ai.x, py = ai.y, qx = bi.x, qy = bi.y;
    const double o1 = cross3(px, py, qx, qy, wl.x, wl.y), o2 = cross3(px, py, qx, qy, wl.z, wl.w);
    const double o3 = cross3(wl.x, wl.y, wl.z, wl.w, px, py), o4 = cross3(wl.x, wl.y, wl.z, wl.w, qx, qy);
    double d2;
    if (o1 * o2 < 0.0 && o3 * o4 < 0.0) {
        d2 = 0.0; // proper crossing
    } else {
        d2 = fmin(fmin(pt_seg2(px, py, wl.x, wl.y, wl.z, wl.w), pt_seg2(qx, qy, wl.x, wl.y, wl.z, wl.w)),
                  fmin(pt_seg2(wl.x, wl.y, px, py, qx, qy), pt_seg2(wl.z, wl.w, px, py, qx, qy)));
    }
    return sqrt(d2) - ri;
}

// ------------------------------------------------------------------ LDS-resident tiny instance
// A tiny instance alone in one workgroup keeps its whole mutable state (node
// records, u, x, activity bits, consensus sums, counters) in LDS for the K
// iterations of a launch: loaded at the start, written back at the end.
// Every access of an iteration then stays on the compute unit.  Each lane
// owns one collision or wall factor for the whole launch (tiny_iteration),
// on a copy of the parameters whose pointers are redirected into LDS.
enum TinyArr {
    TA_ZPREV, TA_ZCUR, TA_UC, TA_XC, TA_UW, TA_XW, TA_UE, TA_UF, TA_BC, TA_BW, TA_CTR, TA_ACC, TA_CNT, TA_INF,
    TA_QC, TA_QW, TA_QCNT, kTinyArrays
};
constexpr int kTinyCopied = TA_QC; // arrays before it are loaded and written back; the rest is scratch

struct TinyLds {
    unsigned off[kTinyArrays];   // byte offset in the dynamic LDS (16-aligned)
    unsigned bytes[kTinyArrays]; // multiple of 4
    unsigned total;
};

__device__ __forceinline__ void tiny_arrays(const Params &P, void **a) {
    a[TA_ZPREV] = P.zr_prev, a[TA_ZCUR] = P.zr_cur, a[TA_UC] = P.u_coll, a[TA_XC] = P.x_coll;
    a[TA_UW] = P.u_wall, a[TA_XW] = P.x_wall, a[TA_UE] = P.u_energy, a[TA_UF] = P.u_fixed;
    a[TA_BC] = P.bits_coll, a[TA_BW] = P.bits_wall, a[TA_CTR] = P.counters, a[TA_ACC] = P.acc;
    a[TA_CNT] = P.cnt, a[TA_INF] = P.inf_val, a[TA_QC] = P.qc, a[TA_QW] = P.qw, a[TA_QCNT] = P.qcnt;
}

__device__ __forceinline__ void tiny_redirect(Params &P, char *b, const TinyLds &L) {
    P.zr_prev = reinterpret_cast<float4 *>(b + L.off[TA_ZPREV]);
    P.zr_cur = reinterpret_cast<float4 *>(b + L.off[TA_ZCUR]);
    P.u_coll = reinterpret_cast<float4 *>(b + L.off[TA_UC]);
    P.x_coll = reinterpret_cast<float4 *>(b + L.off[TA_XC]);
    P.u_wall = reinterpret_cast<float4 *>(b + L.off[TA_UW]);
    P.x_wall = reinterpret_cast<float4 *>(b + L.off[TA_XW]);
    P.u_energy = reinterpret_cast<float *>(b + L.off[TA_UE]);
    P.u_fixed = reinterpret_cast<float *>(b + L.off[TA_UF]);
    P.bits_coll = reinterpret_cast<unsigned long long *>(b + L.off[TA_BC]);
    P.bits_wall = reinterpret_cast<unsigned *>(b + L.off[TA_BW]);
    P.counters = reinterpret_cast<int *>(b + L.off[TA_CTR]);
    P.acc = reinterpret_cast<unsigned long long *>(b + L.off[TA_ACC]);
    P.cnt = reinterpret_cast<int *>(b + L.off[TA_CNT]);
    P.inf_val = reinterpret_cast<float4 *>(b + L.off[TA_INF]);
    P.qc = reinterpret_cast<unsigned *>(b + L.off[TA_QC]);
    P.qw = reinterpret_cast<unsigned *>(b + L.off[TA_QW]);
    P.qcnt = reinterpret_cast<int *>(b + L.off[TA_QCNT]);
}

// The factors a lane of k_tiny owns for the whole launch (a collision factor
// on waves 0-3, or 0-7 for more than 256 of them, a wall factor on waves
// 4-7), decoded once; act: the factor
// was active in the last iteration (its activity bit, kept in a register
// between iterations), ever: active in some iteration of the launch.
struct TinyOwn {
    CollAt c;
    WallAt w;
    bool act_c = false, act_w = false, ever_c = false, ever_w = false;
};

// One iteration of an LDS-resident tiny instance.  Every lane runs its own
// factors through the same per-factor code as the plain kernels (activity
// test, then the minimiser where the factor is queued) with no queue in
// between, so the iteration has two barriers: factors, then nodes.  The
// consensus sums are exact integers, so the order in which lanes add to them
// does not matter and the instance evolves bitwise as in the plain solver.
// The activity words are not read or written here: the owner lanes keep the
// bits (tiny_bits writes them back at the end of the launch).
template <int D, int MODE, int BLOCK>
__device__ __forceinline__ void tiny_iteration(const Params &P, int *len, TinyOwn &o) {
    const Rec Z{P.zr_cur, P.zr_prev};
    const bool dense = P.dense != 0;
    {
        bool q = false, act = false;
        Contrib out;
        if (o.c.f >= 0) {
            float4 rc[4], rp[4];
            float u[4 * D], n[4 * D];
            for (int k = 0; k < 4 * D; ++k) u[k] = 0.f;
            for (int e = 0; e < 4; ++e) rc[e] = Z.cur[o.c.nd[e]];
            for (int e = 0; e < 4; ++e) rp[e] = rc[e];
            if (dense || MODE == M_FIRST) load_u_coll<D>(P, o.c.f, u);
            if (dense && MODE != M_FIRST)
                for (int e = 0; e < 4; ++e) rp[e] = Z.prev[o.c.nd[e]];
            unsigned val;
            if (dense) q = coll_factor<D, MODE, true>(P, o.c.f, o.c.R, rc, rp, u, 0ull, 0, &val);
            else q = coll_factor<D, MODE, false>(P, o.c.f, o.c.R, rc, rp, u, o.act_c ? 1ull : 0ull, 0, &val);
            if (q) act = coll_minimise<D, MODE, false>(P, Z, o.c, (val & kPrev) != 0, n, out, rc);
        }
        count_wave(&len[0], q);
        contribute_wave<false>(P, out, D);
        count_wave(&P.counters[2], act);
        o.act_c = act;
        o.ever_c = o.ever_c || act;
    }
    if (P.Fw > 0) {
        bool q = false, act = false;
        Contrib out;
        if (o.w.f >= 0) {
            unsigned val;
            q = wall_test<MODE>(P, Z, o.w, o.act_w, &val);
            float n[4];
            if (q) act = wall_minimise<MODE, false>(P, Z, o.w, (val & kPrev) != 0, -1, n, out);
        }
        count_wave(&len[1], q);
        contribute_wave<false>(P, out, D);
        count_wave(&P.counters[3], act);
        o.act_w = act;
        o.ever_w = o.ever_w || act;
    }
    // per-segment and fixed factors from wave 4 on (beside the collision owners)
    auto round64 = [](long long n) { return (int)((std::min<long long>(n, BLOCK) + 63) / 64 * 64); };
    const int shift_e = 256 % BLOCK, shift_f = (shift_e + round64(P.Fe)) % BLOCK;
    const int te = (threadIdx.x + BLOCK - shift_e) % BLOCK, tf = (threadIdx.x + BLOCK - shift_f) % BLOCK;
    for (long long f = te; f < P.Fe; f += BLOCK) energy_stream<D, MODE>(P, Z, f);
    for (long long f = tf; f < P.Ff; f += BLOCK) fixed_stream<D, MODE>(P, Z, f);
    __syncthreads();
    if (threadIdx.x == 0) {
        P.qcnt[0] = len[0];
        P.counters[1] = len[1];
        close_counters(P, 1);
        len[0] = len[1] = 0;
    }
    for (long long nd = threadIdx.x; nd < P.N; nd += BLOCK) node_update<D>(P, nd);
    __syncthreads();
}

// Activity words at the end of a launch: in the activity-bit form the factors
// active in the last iteration (every word cleared first), in the dense form
// (where the words only accumulate) those active in any iteration added.
__device__ __forceinline__ void tiny_bits(const Params &P, const TinyOwn &o, int block) {
    const bool dense = P.dense != 0;
    if (!dense) {
        for (long long w = threadIdx.x; w < P.nch; w += block) P.bits_coll[w] = 0ull;
        for (long long w = threadIdx.x; w < (P.Fw + 31) / 32; w += block) P.bits_wall[w] = 0u;
        __syncthreads();
    }
    if (o.c.f >= 0 && (dense ? o.ever_c : o.act_c)) {
        const int r = o.c.j - o.c.i - 1;
        atomicOr(&P.bits_coll[(long long)o.c.s * P.cps + P.rowchunk[o.c.i] + (r >> 6)], 1ull << (r & 63));
    }
    if (o.w.f >= 0 && (dense ? o.ever_w : o.act_w)) atomicOr(&P.bits_wall[o.w.f >> 5], 1u << (o.w.f & 31));
    __syncthreads();
}

// every > 0: after every `every` iterations and after the last one, the
// smallest clearance of the current break-points (the measure of
// twa_get_quality, from the same functions) is taken over the workgroup; the
// launch stops after the first check that reaches bar.  ctl[0] accumulates
// the iterations run, ctl[1] is set once the bar is met (later launches of
// the same call then do nothing).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_tiny(const Params *src, TinyLds L, int K, int first, int every, double bar,
                                                int *ctl) {
    static_assert(BLOCK == 512, "the owner lanes take waves 0-3 and 4-7");
    if (ctl && ctl[1]) return;
    extern __shared__ __align__(16) char lds[];
    __shared__ int len[2];
    __shared__ double wmin[BLOCK / 64];
    // The parameters live in registers, their state pointers redirected into
    // LDS: the compiler then sees those pointers address LDS and accesses
    // them with LDS instructions.
    const Params &G = *src;
    void *ga[kTinyArrays];
    tiny_arrays(G, ga);
#pragma unroll
    for (int a = 0; a < kTinyCopied; ++a) {
        const unsigned *g = static_cast<const unsigned *>(ga[a]);
        unsigned *d = reinterpret_cast<unsigned *>(lds + L.off[a]);
        for (unsigned t = threadIdx.x; t < L.bytes[a] / 4; t += BLOCK) d[t] = g[t];
    }
    if (threadIdx.x == 0) {
        reinterpret_cast<int *>(lds + L.off[TA_QCNT])[0] = 0;
        len[0] = len[1] = 0;
    }
    __syncthreads();
    Params sp = G;
    tiny_redirect(sp, lds, L);
    TinyOwn o;
    o.c.f = o.w.f = -1;
    // collision factors spread over waves 0-3 (one per SIMD), wall factors
    // over waves 4-7, ceil(F / 4) lanes of each (F <= 256); more than 256
    // collision factors (no walls then) over all eight waves
    const int wv = (int)(threadIdx.x >> 6), ln = (int)(threadIdx.x & 63);
    const int wc = sp.Fc > 256 ? 8 : 4;
    const int per_c = (int)((sp.Fc + wc - 1) / wc), per_w = (int)((sp.Fw + 3) / 4);
    if (wv < wc && ln < per_c && wv * per_c + ln < sp.Fc) {
        o.c = coll_at(sp, wv * per_c + ln);
        const int r = o.c.j - o.c.i - 1;
        o.act_c = (sp.bits_coll[(long long)o.c.s * sp.cps + sp.rowchunk[o.c.i] + (r >> 6)] >> (r & 63)) & 1ull;
    } else if (wv >= 4 && ln < per_w && (wv - 4) * per_w + ln < sp.Fw) {
        const long long f = (wv - 4) * per_w + ln;
        o.w = wall_at(sp, f, sp.wbase_wall[f >> 6], (int)(f & 63));
        o.act_w = (sp.bits_wall[f >> 5] >> (f & 31)) & 1u;
    }
    int ran = K;
    bool met = false;
    for (int it = 0; it < K; ++it) {
        const bool fst = first && it == 0;
        if (sp.dim == 2) {
            if (fst) tiny_iteration<2, M_FIRST, BLOCK>(sp, len, o);
            else tiny_iteration<2, M_FUSED, BLOCK>(sp, len, o);
        } else {
            if (fst) tiny_iteration<3, M_FIRST, BLOCK>(sp, len, o);
            else tiny_iteration<3, M_FUSED, BLOCK>(sp, len, o);
        }
        if (every > 0 && ((it + 1) % every == 0 || it + 1 == K)) {
            // (the iteration ended with a barrier: the records are complete)
            const float4 *z = sp.zr_cur;
            double best = INFINITY;
            if (o.c.f >= 0)
                best = pair_clearance(z[o.c.nd[0]], z[o.c.nd[1]], z[o.c.nd[2]], z[o.c.nd[3]], (double)sp.radii[o.c.i],
                                      (double)sp.radii[o.c.j]);
            if (o.w.f >= 0 && sp.dim == 2)
                best = fmin(best, wall_clearance(z[o.w.na], z[o.w.nb], o.w.wl, (double)o.w.r));
            for (int d = 32; d >= 1; d >>= 1) best = fmin(best, __shfl_xor(best, d));
            if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = best;
            __syncthreads();
            double m = wmin[0];
            for (int w = 1; w < BLOCK / 64; ++w) m = fmin(m, wmin[w]);
            // (wmin is written again only after the next iteration's barriers)
            if (m >= bar) {
                ran = it + 1;
                met = true;
                break;
            }
        }
    }
    if (ctl && threadIdx.x == 0) {
        ctl[0] += ran;
        if (met) ctl[1] = 1;
    }
    tiny_bits(sp, o, BLOCK);
    // write the state back
#pragma unroll
    for (int a = 0; a < kTinyCopied; ++a) {
        const unsigned *d = reinterpret_cast<const unsigned *>(lds + L.off[a]);
        unsigned *g = static_cast<unsigned *>(ga[a]);
        for (unsigned t = threadIdx.x; t < L.bytes[a] / 4; t += BLOCK) g[t] = d[t];
    }
}

__global__ void k_reset_counters(Params P) {
    if (threadIdx.x < 4) P.counters[threadIdx.x] = 0;
    if (threadIdx.x < kShards) P.qcnt[threadIdx.x * kQueueStride] = 0;
}

// ------------------------------------------------------------------ phased batch
// The other batched form: one launch per phase of an iteration over every
// instance of the batch.  A host-built map sends each block to (instance,
// block of that instance's own launch), so a large instance spreads over
// many compute units; the per-block bodies are the plain kernels', hence
// the same bitwise evolution.
template <int MODE, bool DENSE>
__global__ __launch_bounds__(kBlock) void kp_stream(const Params *insts, const int2 *map) {
    __shared__ Params sp;
    const int2 m = map[blockIdx.x];
    const Params &P = params_lds<kBlock>(insts + m.x, &sp);
    if (P.dim == 2) stream_block<2, MODE, DENSE>(P, m.y);
    else stream_block<3, MODE, DENSE>(P, m.y);
}

// map: (instance, qb | nqb << 16), block qb of the nqb that share its queue
template <int MODE>
__global__ __launch_bounds__(64) void kp_queue(const Params *insts, const int2 *map) {
    __shared__ Params sp;
    const int2 m = map[blockIdx.x];
    const Params &P = params_lds<64>(insts + m.x, &sp);
    if (P.dim == 2) queue_block<2, MODE>(P, m.y & 0xffff, m.y >> 16);
    else queue_block<3, MODE>(P, m.y & 0xffff, m.y >> 16);
}

__global__ __launch_bounds__(kBlock) void kp_nodes(const Params *insts, const int2 *map) {
    __shared__ Params sp;
    const int2 m = map[blockIdx.x];
    const Params &P = params_lds<kBlock>(insts + m.x, &sp);
    if (P.dim == 2) nodes_block<2>(P, m.y);
    else nodes_block<3>(P, m.y);
}

// ------------------------------------------------------------------ layout conversion
// canonical [p][eta+1][dim] <-> time-major node records
__global__ void k_z_import(float4 *zr, const float *z, int p, int eta, int D, const unsigned char *lrho, int keep_w,
                           int startcode, int goalcode) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long N = (long long)p * (eta + 1);
    if (t >= N) return;
    int i = (int)(t / (eta + 1)), s = (int)(t % (eta + 1));
    long long nd = (long long)s * p + i;
    float4 r = zr[nd];
    r.x = z[t * D + 0];
    r.y = z[t * D + 1];
    r.z = D == 3 ? z[t * D + 2] : 0.f;
    if (lrho) r.w = (float)lrho[t];
    else if (!keep_w) r.w = (float)(s == 0 ? startcode : (s == eta ? goalcode : W_STD));
    zr[nd] = r;
}
__global__ void k_z_export(const float4 *zr, float *z, unsigned char *lrho, int p, int eta, int D) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long N = (long long)p * (eta + 1);
    if (t >= N) return;
    int i = (int)(t / (eta + 1)), s = (int)(t % (eta + 1));
    float4 r = zr[(long long)s * p + i];
    if (z) {
        z[t * D + 0] = r.x;
        z[t * D + 1] = r.y;
        if (D == 3) z[t * D + 2] = r.z;
    }
    if (lrho) lrho[t] = (unsigned char)(int)r.w;
}

// ------------------------------------------------------------------ quality
// Measures of the current break-points z, in double precision from the FP32
// node records: the energy objective sum C_is |z_i(s+1) - z_i(s)|^2 (Sec. 3.1),
// the smallest clearance over every pair and interval (closest approach of
// the two constant-velocity agents minus r_i + r_j, Sec. 2) and over every
// interval and wall (segment distance minus r_i, Sec. 3.2), and the largest
// move of a break-point in the last iteration.

// unsigned key whose order is the order of the doubles (for atomicMin)
__device__ __forceinline__ unsigned long long order_key(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// one workgroup of 1024 lanes: objective and largest move, reduced in a
// fixed order; also arms the clearance minimum for k_quality_clearance
__global__ __launch_bounds__(1024) void k_quality_sums(const float4 *zr, const float4 *zp, const float *C, int p,
                                                       int eta, double *out, unsigned long long *min_key) {
    __shared__ double part[2][1024];
    double obj = 0.0, mv = 0.0;
    const long long S = (long long)p * eta, N = (long long)p * (eta + 1);
    for (long long t = threadIdx.x; t < S; t += 1024) {
        const int i = (int)(t / eta), s = (int)(t % eta);
        const float4 a = zr[(long long)s * p + i], b = zr[(long long)(s + 1) * p + i];
        const double dx = (double)b.x - a.x, dy = (double)b.y - a.y, dz = (double)b.z - a.z;
        obj += (double)C[t] * (dx * dx + dy * dy + dz * dz);
    }
    for (long long nd = threadIdx.x; nd < N; nd += 1024) {
        const float4 a = zr[nd], b = zp[nd];
        const double dx = (double)a.x - b.x, dy = (double)a.y - b.y, dz = (double)a.z - b.z;
        mv = fmax(mv, sqrt(dx * dx + dy * dy + dz * dz));
    }
    part[0][threadIdx.x] = obj;
    part[1][threadIdx.x] = mv;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            part[0][threadIdx.x] += part[0][threadIdx.x + h];
            part[1][threadIdx.x] = fmax(part[1][threadIdx.x], part[1][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = part[0][0];
        out[1] = part[1][0];
        *min_key = order_key(INFINITY);
    }
}

// rows (s, i) of the pair triangle, one per workgroup pass; lanes over j > i
// and over the walls; one atomicMin per workgroup
__global__ __launch_bounds__(256) void k_quality_clearance(const float4 *zr, const float *radii, const float4 *walls,
                                                           int p, int eta, int W, int dim,
                                                           unsigned long long *min_key) {
    __shared__ double wmin[4];
    double best = INFINITY;
    const long long rows = (long long)p * eta;
    for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
        const int s = (int)(row / p), i = (int)(row % p);
        const float4 ai = zr[(long long)s * p + i], bi = zr[(long long)(s + 1) * p + i];
        const double ri = radii[i];
        for (int j = i + 1 + (int)threadIdx.x; j < p; j += 256)
            best = fmin(best, pair_clearance(ai, bi, zr[(long long)s * p + j], zr[(long long)(s + 1) * p + j], ri,
                                             (double)radii[j]));
        if (dim == 2)
            for (int w = (int)threadIdx.x; w < W; w += 256) best = fmin(best, wall_clearance(ai, bi, walls[w], ri));
    }
    for (int d = 32; d >= 1; d >>= 1) best = fmin(best, __shfl_xor(best, d));
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmin(fmin(wmin[0], wmin[1]), fmin(wmin[2], wmin[3]));
        atomicMin(min_key, order_key(m));
    }
}
// u: canonical [E][dim] <-> per-kind layouts.  dir 0: import, 1: export
__global__ void k_u_convert(Params P, float *u, int D, int dir) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    long long E = P.e_wall + 2 * P.Fw;
    if (t >= E) return;
    for (int c = 0; c < D; ++c) {
        float *dst = nullptr;
        float *src = u + t * D + c;
        if (t < P.e_energy) {
            dst = P.u_fixed + t * D + c;
        } else if (t < P.e_coll) {
            dst = P.u_energy + (t - P.e_energy) * D + c;
        } else if (t < P.e_wall) {
            long long r = t - P.e_coll;
            long long f = r >> 2;
            int slot = (int)(r & 3);
            int q = slot * D + c;          // position inside the factor's 4*D vector
            int plane = q >> 2, lane = q & 3;
            dst = reinterpret_cast<float *>(P.u_coll + plane * P.Fc + f) + lane;
        } else {
            long long r = t - P.e_wall;
            long long f = r >> 1;
            int slot = (int)(r & 1);
            dst = reinterpret_cast<float *>(P.u_wall + f) + slot * 2 + c;
        }
        if (dir == 0) *dst = *src;
        else *src = *dst;
    }
}
__global__ void k_fix_ends(float4 *zr, const float4 *xfix, int p, int eta, int startcode, int goalcode) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p) return;
    float4 a = xfix[2 * i], b = xfix[2 * i + 1];
    a.w = (float)startcode;
    b.w = (float)goalcode;
    zr[i] = a;
    zr[(long long)eta * p + i] = b;
}
__global__ void k_fill_bits(unsigned *bits, long long nwords, unsigned v) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nwords) bits[t] = v;
}
__global__ void k_finite(const float4 *zr, long long N, const float *u, long long nu, int *bad) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < N) {
        float4 r = zr[t];
        if (!isfinite(r.x) || !isfinite(r.y) || !isfinite(r.z)) atomicOr(bad, 1);
    }
    for (long long q = t; q < nu; q += (long long)gridDim.x * blockDim.x)
        if (!isfinite(u[q])) atomicOr(bad, 1);
}

} // namespace

// ============================================================================
// host runtime
// ============================================================================

namespace twa_rt {

twa_status fail(twa_solver *s, twa_status st, const std::string &msg) {
    if (s) {
        s->err = msg;
        if (st == TWA_E_DEVICE) s->latched = TWA_E_DEVICE;
    }
    return st;
}

twa_status check_alive(twa_solver *s) {
    if (!s) return TWA_E_INVALID;
    if (s->latched != TWA_OK) return s->latched;
    return TWA_OK;
}

float rho_at(const twa_solver *s, long long k) { return k < s->n_warm ? s->rho0_init : s->rho0; }

} // namespace twa_rt

using twa_rt::check_alive;
using twa_rt::fail;
using twa_rt::rho_at;

namespace {

constexpr int kGraphIters = 1 << (twa_solver::kGraphSizes - 1); // largest graph: 32 iterations
// twa_iterate_timed times its last kTimedTail iterations, launched on their
// own, each kernel with a start and a stop event attached to its own dispatch
// (hipExtLaunchKernel), so an event pair spans the kernel alone.  Once an
// event is recorded on the stream, every later launch of the same call runs
// slower (graph replays by about a third), so no event comes before the
// untimed replays.
constexpr int kTimedTail = 2;

// Two events of the solver's pool for the next timed kernel (false: none).
bool take_events(twa_solver *s, hipEvent_t *e0, hipEvent_t *e1) {
    while (s->events.size() < s->events_used + 2) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return false;
        s->events.push_back(e);
    }
    *e0 = s->events[s->events_used++];
    *e1 = s->events[s->events_used++];
    return true;
}

// Launch one kernel on the solver's stream; while timing, with events.
template <typename Kern, typename... Args>
void launch(twa_solver *s, Kern kernel, dim3 grid, dim3 block, Args... args) {
    hipEvent_t e0, e1;
    if (s->timing == 1 && take_events(s, &e0, &e1))
        hipExtLaunchKernelGGL(kernel, grid, block, 0, s->stream, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, s->stream, args...);
}


template <class T>
twa_status dev_alloc(twa_solver *s, T **ptr, size_t count) {
    size_t bytes = std::max<size_t>(count * sizeof(T), 16);
    void *p = s->mem.get(bytes, s->stream);
    if (!p) return fail(s, TWA_E_NOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    s->allocs.emplace_back(p, bytes);
    *ptr = static_cast<T *>(p);
    return TWA_OK;
}

template <class T>
twa_status to_host(twa_solver *s, std::vector<T> &dst, const T *src, size_t count) {
    dst.resize(count);
    if (count == 0) return TWA_OK;
    HIP_TRY(s, hipMemcpyAsync(dst.data(), src, count * sizeof(T), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return TWA_OK;
}


template <int D>
twa_status launch_iteration(twa_solver *s, int mode) {
    Params P = s->P;
    const dim3 g((unsigned)s->nblocks_stream), gq(s->nblocks_queue), gn((unsigned)((P.N + kBlock - 1) / kBlock));
    if (mode == M_FIRST) {
        if (P.dense) launch(s, k_stream<D, M_FIRST, true>, g, dim3(kBlock), P);
        else launch(s, k_stream<D, M_FIRST, false>, g, dim3(kBlock), P);
        launch(s, k_queue<D, M_FIRST>, gq, dim3(64), P);
    } else if (mode == M_FUSED) {
        if (P.dense) launch(s, k_stream<D, M_FUSED, true>, g, dim3(kBlock), P);
        else launch(s, k_stream<D, M_FUSED, false>, g, dim3(kBlock), P);
        launch(s, k_queue<D, M_FUSED>, gq, dim3(64), P);
    } else {
        if (P.dense) hipLaunchKernelGGL((k_stream<D, M_FINAL, true>), g, dim3(kBlock), 0, s->stream, P);
        else hipLaunchKernelGGL((k_stream<D, M_FINAL, false>), g, dim3(kBlock), 0, s->stream, P);
        hipLaunchKernelGGL((k_queue<D, M_FINAL>), gq, dim3(64), 0, s->stream, P);
        hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s->stream, P);
        HIP_TRY(s, hipGetLastError());
        return TWA_OK;
    }
    launch(s, k_nodes<D>, gn, dim3(kBlock), P);
    HIP_TRY(s, hipGetLastError());
    return TWA_OK;
}

twa_status run_iteration(twa_solver *s, int mode, float rho, float rho_prev) {
    // the warm-up's small rho0 enters the minimisers' weights only; the u
    // step is alpha / rho0 of the configuration throughout (App. B step 7
    // with Sec. 4's schedule: over the warm-up value it diverges)
    s->P.rho = rho;
    s->P.step = s->alpha / s->rho0;
    s->P.rho_prev = rho_prev;
    s->P.step_prev = s->alpha / s->rho0;
    s->P.dbg_x = (mode == M_FINAL) ? nullptr : s->dbg_x;
    s->P.dbg_rho = (mode == M_FINAL) ? nullptr : s->dbg_rho;
    s->P.adj_pool = (mode == M_FINAL) ? nullptr : s->adj_pool;
    s->P.adj_cursor = s->adj_cursor;
    s->P.adj_cap = s->adj_cap;
    s->P.adj_offs = (mode == M_FINAL) ? nullptr : s->adj_offs;
    s->P.dbg_l = (mode == M_FINAL) ? nullptr : s->dbg_l;
    s->P.dbg_cnt = s->dbg_cnt;
    twa_status st = s->dim == 2 ? launch_iteration<2>(s, mode) : launch_iteration<3>(s, mode);
    s->P.dbg_x = nullptr;
    s->P.dbg_rho = nullptr;
    s->P.adj_pool = nullptr;
    s->P.adj_offs = nullptr;
    s->P.dbg_l = nullptr;
    s->P.dbg_cnt = nullptr;
    return st;
}


// Capture graphs of 1, 2, 4, ..., kGraphIters fused iterations at the steady
// rho0, all at once (the first time a steady iteration is run), so later
// calls of any length replay without capturing.  Returns false if the
// stream cannot be captured.
bool capture_graphs(twa_solver *s) {
    if (s->graphs[0]) return true;
    if (s->graph_failed) return false;
    bool ok = true;
    for (int b = 0; b < twa_solver::kGraphSizes && ok; ++b) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            ok = false;
            break;
        }
        s->timing = 0;
        for (int it = 0; it < (1 << b) && ok; ++it) ok = run_iteration(s, M_FUSED, s->rho0, s->rho0) == TWA_OK;
        ok = (hipStreamEndCapture(s->stream, &g) == hipSuccess) && ok && g != nullptr;
        if (ok) ok = hipGraphInstantiate(&s->graphs[b], g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
    }
    if (!ok) {
        (void)hipGetLastError();
        for (hipGraphExec_t &e : s->graphs) {
            if (e) (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
        s->graph_failed = true;
        s->err.clear();
        s->latched = TWA_OK;
    }
    return ok;
}

// Instances this small (at most 256 collision + wall factors, or 512
// collision factors and no walls: one factor per lane of a 512-lane
// workgroup) run untimed iterations in one workgroup, all iterations of a
// call in one launch: three launches per iteration would cost more than the
// work.
constexpr long long kTinyFactors = 256;
constexpr int kTinyBlock = 512, kTinyChunk = 4096; // iterations per launch at most

bool tiny(const twa_solver *s) {
    return s->P.Fc + s->P.Fw <= kTinyFactors || (s->P.Fw == 0 && s->P.Fc <= 2 * kTinyFactors);
}

// LDS layout of a tiny instance's mutable state for k_tiny (the sizes of
// its device arrays); false when it does not fit kTinyLdsMax.
constexpr unsigned kTinyLdsMax = 56u << 10;

bool tiny_layout(const twa_solver *s, TinyLds *L) {
    const Params &P = s->P;
    const long long d = s->dim, N = P.N;
    long long bytes[kTinyArrays];
    bytes[TA_ZPREV] = bytes[TA_ZCUR] = 16 * N;
    bytes[TA_UC] = bytes[TA_XC] = 16 * std::max<long long>(1, d * P.Fc);
    bytes[TA_UW] = bytes[TA_XW] = 16 * std::max<long long>(1, P.Fw);
    bytes[TA_UE] = 4 * P.Fe * 2 * d;
    bytes[TA_UF] = 4 * P.Ff * d;
    bytes[TA_BC] = 8 * std::max<long long>(1, P.nch);
    bytes[TA_BW] = 4 * std::max<long long>(1, (P.Fw + 31) / 32);
    bytes[TA_CTR] = 4 * 8;
    bytes[TA_ACC] = 8 * 2 * d * N;
    bytes[TA_CNT] = 4 * 2 * N;
    bytes[TA_INF] = 16 * N;
    bytes[TA_QC] = bytes[TA_QW] = 4; // (no queues: each lane runs its own factors)
    bytes[TA_QCNT] = 4;
    long long off = 0;
    for (int a = 0; a < kTinyArrays; ++a) {
        L->off[a] = (unsigned)off;
        L->bytes[a] = (unsigned)bytes[a];
        off += (bytes[a] + 15) & ~15LL;
        if (off > (long long)kTinyLdsMax) return false;
    }
    L->total = (unsigned)off;
    return true;
}

// The device copy of a tiny instance's parameters that the persistent kernel
// reads (at the steady rho0, no debug capture) and its one-bin layout; made
// at create, so that iterating allocates and uploads nothing.
twa_status prepare_tiny(twa_solver *s) {
    Params c = s->P;
    c.rho = c.rho_prev = s->rho0;
    c.step = c.step_prev = s->alpha / s->rho0;
    c.dbg_x = nullptr;
    c.dbg_rho = nullptr;
    // bin_start {0, 1}, bin_items {0}; then the two control words of k_tiny's
    // clearance check (twa_iterate_until)
    const int bins[5] = {0, 1, 0, 0, 0};
    TRY(dev_alloc(s, &s->tiny_params, 1));
    TRY(dev_alloc(s, &s->tiny_bins, 5));
    HIP_TRY(s, hipMemcpyAsync(s->tiny_params, &c, sizeof(Params), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipMemcpyAsync(s->tiny_bins, bins, sizeof(bins), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream)); // the sources are on this stack
    return TWA_OK;
}

// k iterations of a tiny instance at the steady rho0 (bitwise the plain
// iterations: the same per-factor code).
twa_status iterate_tiny(twa_solver *s, int k) {
    TinyLds L;
    const bool resident = tiny_layout(s, &L);
    while (k > 0) {
        const int n = std::min(k, kTinyChunk);
        if (resident)
            hipLaunchKernelGGL(k_tiny<kTinyBlock>, dim3(1), dim3(kTinyBlock), L.total, s->stream,
                               (const Params *)s->tiny_params, L, n, s->pending ? 0 : 1, 0, 0.0, (int *)nullptr);
        else
            hipLaunchKernelGGL(k_batch<kTinyBlock>, dim3(1), dim3(kTinyBlock), 0, s->stream,
                               (const Params *)s->tiny_params, (const int *)s->tiny_bins,
                               (const int *)s->tiny_bins + 2, n, s->pending ? 0 : 1);
        HIP_TRY(s, hipGetLastError());
        s->pending = true;
        s->iter += n;
        k -= n;
    }
    return TWA_OK;
}

// Run k iterations; graph replays where possible.  timed: the last
// kTimedTail iterations are launched on their own, with events.
twa_status iterate_core(twa_solver *s, int k, bool timed) {
    const int tail = timed ? std::min(k, kTimedTail) : 0;
    // (steady rho0 throughout, the previous iteration's weights included)
    const bool settled = s->iter >= s->n_warm && (!s->pending || s->iter - 1 >= s->n_warm);
    if (s->tiny_params && k - tail > 0 && settled && !s->dbg_rho && !s->adj_pool) {
        TRY(iterate_tiny(s, k - tail));
        k = tail;
    }
    while (k > 0) {
        const bool steady = s->pending && s->iter - 1 >= s->n_warm && !s->dbg_rho && !s->adj_pool;
        // (a call that must not allocate replays graphs already captured but
        // captures none: instantiating a graph allocates)
        if (steady && k - tail > 0 && (s->graphs[0] || !s->no_capture) && capture_graphs(s)) {
            // the largest captured chunk that fits before the timed tail
            int b = twa_solver::kGraphSizes - 1;
            while ((1 << b) > k - tail) --b;
            HIP_TRY(s, hipGraphLaunch(s->graphs[b], s->stream));
            s->iter += 1 << b;
            s->graph_iters += 1 << b;
            k -= 1 << b;
            continue;
        }
        float rho = rho_at(s, s->iter);
        if (k <= tail) s->timing = 1;
        twa_status st;
        if (!s->pending) st = run_iteration(s, M_FIRST, rho, rho);
        else st = run_iteration(s, M_FUSED, rho, rho_at(s, s->iter - 1));
        s->timing = 0;
        if (st != TWA_OK) return st;
        s->pending = true;
        s->iter++;
        k--;
        s->dbg_x = nullptr;
        s->dbg_rho = nullptr;
        s->adj_pool = nullptr;
        s->adj_offs = nullptr;
        s->dbg_l = nullptr;
        s->dbg_cnt = nullptr;
    }
    return TWA_OK;
}

// Run k iterations; with a recording forward tape the call is cut at the
// tape's checkpoint iterations, each packed before the run goes on (only the
// last piece carries the timed tail).
twa_status iterate_impl(twa_solver *s, int k, bool timed) {
    if (!s->tape.ok || s->dbg_rho || s->adj_pool) return iterate_core(s, k, timed);
    while (k > 0) {
        TRY(twa_rt::tape_take(s));
        const long long since = s->iter - s->origin_iter;
        const int n = (int)std::min<long long>(k, s->tape.interval - since % s->tape.interval);
        TRY(iterate_core(s, n, timed && n == k));
        k -= n;
    }
    return TWA_OK;
}

bool same_capture(const twa_rt::SegCapture &a, const twa_rt::SegCapture &b) {
    return a.rout == b.rout && a.pool == b.pool && a.cursor == b.cursor && a.cap == b.cap && a.offs == b.offs &&
           a.lseg == b.lseg && a.cntseg == b.cntseg && a.F == b.F && a.N == b.N;
}

// pending -> canonical: materialise u^k
twa_status finalize(twa_solver *s) {
    if (!s->pending) return TWA_OK;
    HIP_TRY(s, hipMemsetAsync(s->resid_dev, 0, sizeof(unsigned), s->stream));
    TRY(run_iteration(s, M_FINAL, rho_at(s, s->iter), rho_at(s, s->iter - 1)));
    s->pending = false;
    s->resid_valid = true;
    return TWA_OK;
}

twa_status reset_state_buffers(twa_solver *s) {
    const Params &P = s->P;
    long long D = s->dim;
    HIP_TRY(s, hipMemsetAsync(P.u_coll, 0, sizeof(float4) * std::max<long long>(1, D * P.Fc), s->stream));
    HIP_TRY(s, hipMemsetAsync(P.u_wall, 0, sizeof(float4) * std::max<long long>(1, P.Fw), s->stream));
    HIP_TRY(s, hipMemsetAsync(P.u_energy, 0, sizeof(float) * std::max<long long>(1, P.Fe * 2 * D), s->stream));
    HIP_TRY(s, hipMemsetAsync(P.u_fixed, 0, sizeof(float) * std::max<long long>(1, P.Ff * D), s->stream));
    HIP_TRY(s, hipMemsetAsync(P.bits_coll, 0, sizeof(unsigned long long) * std::max<long long>(1, P.nch), s->stream));
    HIP_TRY(s, hipMemsetAsync(P.bits_wall, 0, sizeof(unsigned) * std::max<long long>(1, (P.Fw + 31) / 32), s->stream));
    HIP_TRY(s, hipMemsetAsync(P.acc, 0, sizeof(unsigned long long) * 2 * D * P.N, s->stream));
    HIP_TRY(s, hipMemsetAsync(P.cnt, 0, sizeof(int) * 2 * P.N, s->stream));
    HIP_TRY(s, hipMemsetAsync(P.counters, 0, sizeof(int) * 8, s->stream));
    HIP_TRY(s, hipMemsetAsync(P.qcnt, 0, sizeof(int) * kShards * kQueueStride, s->stream));
    HIP_TRY(s, hipMemsetAsync(s->stats_dev, 0, sizeof(int) * 4, s->stream));
    s->pending = false;
    s->resid_valid = false;
    return TWA_OK;
}

// canonical z, u, <-rho of a state without a pending u update
__global__ void k_z_export(const float4 *zr, float *z, unsigned char *lrho, int p, int eta, int D);
__global__ void k_u_convert(Params P, float *u, int D, int dir);

// TWA_F_TAPE: remember the current (settled) state as the start of the
// differentiated run
twa_status save_origin(twa_solver *s) {
    if (!(s->flags & TWA_F_TAPE)) return TWA_OK;
    unsigned nb = (unsigned)((s->P.N + 255) / 256);
    hipLaunchKernelGGL(k_z_export, dim3(nb), dim3(256), 0, s->stream, (const float4 *)s->P.zr_cur, s->origin_z,
                       s->origin_l, s->p, s->eta, s->dim);
    long long E = s->P.e_wall + 2 * s->P.Fw;
    hipLaunchKernelGGL(k_u_convert, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s->stream, s->P, s->origin_u,
                       s->dim, 1);
    HIP_TRY(s, hipGetLastError());
    s->origin_iter = s->iter;
    // a new run: the forward tape (if twa_backward made one) records it
    if (s->tape.mem) {
        HIP_TRY(s, hipMemsetAsync(s->tape.cursor, 0, sizeof(unsigned), s->stream));
        s->tape.count = 0;
        s->tape.ok = true;
    }
    return TWA_OK;
}

// Fixed-point scale of the consensus sums: a power of two such that the
// contributions of every edge of a node (degree 2(p-1) + 2 + 2 n_walls + 1),
// each with |m| <= 8 coord_max, sum below 2^62 (capped at 2^44, far below
// FP32's resolution at unit scale).  *limit: the largest |m| one contribution
// may carry before the overflow flag is raised (degree of them stay below
// 2^62 in magnitude, so the int64 sum cannot wrap).
void consensus_scale(int p, int n_walls, double coord_max, double *scale, double *limit) {
    const long long deg = 2LL * (p - 1) + 2 + 2LL * n_walls + 1;
    const double lim = std::ldexp(1.0, 62) / (8.0 * coord_max * (double)deg);
    const int S = std::min((int)std::floor(std::log2(lim)), 44);
    *scale = std::ldexp(1.0, S);
    *limit = std::ldexp(1.0, 62) / ((double)deg * *scale);
}

// Feasibility of the fixed end points (Sec. 1: non-strict separation):
// starts pairwise >= r_i + r_j apart and clear of every wall, goals too
// (a velocity-obstacle epoch's reference ends are preferences, not
// constraints).  FP32 positions left in contact may overlap by rounding: a
// 1e-5 relative slack.
twa_status check_ends(twa_solver *s, const std::vector<float> &h0, const std::vector<float> &hT) {
    const int p = s->p, dim = s->dim, n_walls = s->W;
    const std::vector<float> &hr = s->h_radii, &hw = s->h_walls;
    for (int which = 0; which < ((s->flags & TWA_F_VO) ? 1 : 2); ++which) {
        const std::vector<float> &X = which ? hT : h0;
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j) {
                double d2 = 0;
                for (int c = 0; c < dim; ++c) {
                    double d = (double)X[i * dim + c] - X[j * dim + c];
                    d2 += d * d;
                }
                double R = ((double)hr[i] + hr[j]) * (1.0 - 1e-5);
                if (d2 < R * R)
                    return fail(s, TWA_E_INFEASIBLE, std::string(which ? "goals " : "starts ") + std::to_string(i) +
                                                         " and " + std::to_string(j) + " overlap");
            }
        for (int i = 0; i < p && n_walls > 0; ++i)
            for (int w = 0; w < n_walls; ++w) {
                double ax = hw[w * 4 + 0], ay = hw[w * 4 + 1], bx = hw[w * 4 + 2], by = hw[w * 4 + 3];
                double qx = X[i * 2 + 0], qy = X[i * 2 + 1];
                double dx = bx - ax, dy = by - ay, L2 = dx * dx + dy * dy, t = 0;
                if (L2 > 0) t = std::min(1.0, std::max(0.0, ((qx - ax) * dx + (qy - ay) * dy) / L2));
                double ex = ax + t * dx - qx, ey = ay + t * dy - qy;
                if (ex * ex + ey * ey < (double)hr[i] * hr[i] * (1.0 - 2e-5))
                    return fail(s, TWA_E_INFEASIBLE, std::string(which ? "goal " : "start ") + std::to_string(i) +
                                                         " touches wall " + std::to_string(w));
            }
    }
    return TWA_OK;
}

// The constants of the fixed factors (start i, goal i as float4) and the
// straight-line state between them (<-rho infinity at certain ends, rho0
// elsewhere), time-major node records.
void build_ends(const twa_solver *s, const std::vector<float> &h0, const std::vector<float> &hT,
                std::vector<float4> &hfix, std::vector<float4> &hz) {
    const int p = s->p, eta = s->eta, dim = s->dim;
    const bool admm = s->P.admm != 0, vo = s->P.vo != 0;
    hfix.assign((size_t)2 * p, make_float4(0.f, 0.f, 0.f, 0.f));
    for (int i = 0; i < p; ++i) {
        hfix[2 * i] = make_float4(h0[i * dim], h0[i * dim + 1], dim == 3 ? h0[i * dim + 2] : 0.f, 0.f);
        hfix[2 * i + 1] = make_float4(hT[i * dim], hT[i * dim + 1], dim == 3 ? hT[i * dim + 2] : 0.f, 0.f);
    }
    hz.assign((size_t)(eta + 1) * p, make_float4(0.f, 0.f, 0.f, 0.f));
    for (int i = 0; i < p; ++i)
        for (int s2 = 0; s2 <= eta; ++s2) {
            float v[3] = {0.f, 0.f, 0.f};
            for (int c = 0; c < dim; ++c) {
                double a = h0[i * dim + c], b = hT[i * dim + c];
                v[c] = (s2 == 0) ? (float)a : (s2 == eta) ? (float)b : (float)(a + (double)s2 / eta * (b - a));
            }
            hz[(size_t)s2 * p + i] =
                make_float4(v[0], v[1], v[2], (float)(((s2 == 0 && !admm) || (s2 == eta && !admm && !vo)) ? W_INF : W_STD));
        }
}

bool finite_all(const std::vector<float> &v) {
    for (float x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

} // namespace

namespace twa_rt {

twa_status import_state(twa_solver *s, const float *z, const float *u, const unsigned char *lrho, long long iter) {
    TRY(check_alive(s));
    if (!z || !u || !lrho) return fail(s, TWA_E_INVALID, "null state array");
    if (iter < 0) return fail(s, TWA_E_INVALID, "iter must be >= 0");
    TRY(reset_state_buffers(s));
    unsigned nb = (unsigned)((s->P.N + 255) / 256);
    hipLaunchKernelGGL(k_z_import, dim3(nb), dim3(256), 0, s->stream, s->P.zr_cur, z, s->p, s->eta, s->dim, lrho, 1,
                       (int)W_INF, (int)W_INF);
    long long E = s->P.e_wall + 2 * s->P.Fw;
    hipLaunchKernelGGL(k_u_convert, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s->stream, s->P,
                       const_cast<float *>(u), s->dim, 0);
    HIP_TRY(s, hipGetLastError());
    HIP_TRY(s, hipMemcpyAsync(s->P.zr_prev, s->P.zr_cur, sizeof(float4) * s->P.N, hipMemcpyDeviceToDevice, s->stream));
    s->iter = iter;
    s->pending = false;
    return TWA_OK;
}

twa_status run_segment(twa_solver *s, long long len, const SegCapture &c, int slot) {
    auto capture_into = [&](long long t) {
        s->dbg_x = nullptr;
        s->dbg_rho = c.rout + t * c.F;
        s->adj_pool = c.pool;
        s->adj_cursor = c.cursor;
        s->adj_cap = c.cap;
        s->adj_offs = c.offs + t + 1;
        s->dbg_l = c.lseg + (t + 1) * c.N;
        s->dbg_cnt = c.cntseg + t * c.N;
    };
    auto capture_none = [&]() {
        s->dbg_rho = nullptr;
        s->adj_pool = nullptr;
        s->adj_offs = nullptr;
        s->dbg_l = nullptr;
        s->dbg_cnt = nullptr;
    };
    // every iteration at the configuration's rho0, the first from a settled state
    const bool steady = slot >= 0 && !s->pending && s->iter >= s->n_warm && len > 0;
    bool fits = steady && s->seg_graph[slot] && s->seg_len[slot] == len && same_capture(s->seg_key[slot], c);
    if (steady && !fits && !s->no_capture && !s->seg_failed) {
        if (s->seg_graph[slot]) (void)hipGraphExecDestroy(s->seg_graph[slot]);
        s->seg_graph[slot] = nullptr;
        hipGraph_t g = nullptr;
        bool ok = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        s->timing = 0;
        for (long long t = 0; t < len && ok; ++t) {
            capture_into(t);
            ok = run_iteration(s, t == 0 ? M_FIRST : M_FUSED, s->rho0, s->rho0) == TWA_OK;
        }
        capture_none();
        ok = (hipStreamEndCapture(s->stream, &g) == hipSuccess) && ok && g != nullptr;
        if (ok) ok = hipGraphInstantiate(&s->seg_graph[slot], g, nullptr, nullptr, 0) == hipSuccess;
        if (g) (void)hipGraphDestroy(g);
        if (ok) {
            s->seg_key[slot] = c;
            s->seg_len[slot] = len;
            fits = true;
        } else {
            (void)hipGetLastError();
            s->seg_graph[slot] = nullptr;
            s->seg_failed = true;
            s->err.clear();
            s->latched = TWA_OK;
        }
    }
    if (steady && fits) {
        HIP_TRY(s, hipGraphLaunch(s->seg_graph[slot], s->stream));
        s->iter += len;
        s->pending = true;
        return TWA_OK;
    }
    for (long long t = 0; t < len; ++t) {
        capture_into(t);
        TRY(iterate_impl(s, 1, false)); // (clears the capture pointers)
    }
    return TWA_OK;
}

twa_status export_lrho(twa_solver *s, unsigned char *lrho) {
    unsigned nb = (unsigned)((s->P.N + 255) / 256);
    hipLaunchKernelGGL(k_z_export, dim3(nb), dim3(256), 0, s->stream, (const float4 *)s->P.zr_cur, (float *)nullptr,
                       lrho, s->p, s->eta, s->dim);
    HIP_TRY(s, hipGetLastError());
    return TWA_OK;
}

} // namespace twa_rt

extern "C" {

const char *twa_version(void) { return TWA_VERSION; }

const char *twa_last_error(const twa_solver *s) { return s ? s->err.c_str() : "null solver"; }

void twa_destroy(twa_solver *s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (hipGraphExec_t e : s->graphs)
        if (e) (void)hipGraphExecDestroy(e);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    for (auto &a : s->allocs) s->mem.put(a.first, a.second, s->stream);
    s->mem.put(s->adj_ws, s->adj_ws_bytes, s->stream);
    s->mem.put(s->adj_arena, s->adj_arena_bytes, s->stream);
    s->mem.put(s->adj_pool_mem, s->adj_pool_bytes, s->stream);
    s->mem.put(s->tape.mem, s->tape.bytes, s->stream);
    if (s->adj_stream) {
        (void)hipStreamSynchronize(s->adj_stream);
        (void)hipStreamDestroy(s->adj_stream);
    }
    for (hipGraphExec_t e : s->seg_graph)
        if (e) (void)hipGraphExecDestroy(e);
    for (hipEvent_t e : s->adj_ev)
        if (e) (void)hipEventDestroy(e);
    if (s->adj_used) (void)hipHostFree(s->adj_used);
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    delete s;
}

twa_status twa_create(int p, int eta, int dim, const float *radii, const float *x0, const float *xT, int n_walls,
                      const float *walls, const float *C, float rho0, float alpha, unsigned flags,
                      void *hip_stream, twa_solver **out) {
    if (!out) return TWA_E_INVALID;
    *out = nullptr;
    twa_solver *s = new (std::nothrow) twa_solver();
    if (!s) return TWA_E_NOMEM;
    auto bail = [&](twa_status st) {
        std::string e = s->err;
        twa_destroy(s);
        (void)e;
        return st;
    };
    s->stream = static_cast<hipStream_t>(hip_stream);
    if (p < 1 || eta < 1 || (dim != 2 && dim != 3) || n_walls < 0) {
        fail(s, TWA_E_INVALID, "need p >= 1, eta >= 1, dim in {2,3}, n_walls >= 0");
        return bail(TWA_E_INVALID);
    }
    if (n_walls > 0 && dim != 2) {
        fail(s, TWA_E_INVALID, "walls are planar only (dim == 2)");
        return bail(TWA_E_INVALID);
    }
    if (!radii || !x0 || !xT || !C || (n_walls > 0 && !walls)) {
        fail(s, TWA_E_INVALID, "null array argument");
        return bail(TWA_E_INVALID);
    }
    if (!(rho0 > 0.f) || !(alpha > 0.f) || !std::isfinite(rho0) || !std::isfinite(alpha)) {
        fail(s, TWA_E_INVALID, "rho0 and alpha must be finite and > 0");
        return bail(TWA_E_INVALID);
    }
    const unsigned cost_flags = flags & (TWA_F_COST_NONE | TWA_F_COST_MAXVEL | TWA_F_COST_MINVEL);
    if ((cost_flags & (cost_flags - 1)) != 0) {
        fail(s, TWA_E_INVALID, "choose at most one TWA_F_COST_* flag");
        return bail(TWA_E_INVALID);
    }
    if ((flags & TWA_F_VO) && (cost_flags || eta != 1)) {
        fail(s, TWA_E_INVALID, "TWA_F_VO needs eta == 1 and no TWA_F_COST_* flag");
        return bail(TWA_E_INVALID);
    }
    if (flags & ~(unsigned)(TWA_F_DENSE | TWA_F_TAPE | TWA_F_ADMM | TWA_F_COST_NONE | TWA_F_COST_MAXVEL |
                            TWA_F_COST_MINVEL | TWA_F_VO)) {
        fail(s, TWA_E_INVALID, "unsupported flag");
        return bail(TWA_E_INVALID);
    }
    long long P2 = (long long)p * (p - 1) / 2;
    long long Fc = (long long)eta * P2, Fw = (long long)eta * p * n_walls, Fe = (long long)eta * p, Ff = 2LL * p;
    if (Fc >= (long long)kIdx || Fw >= (long long)kIdx || p >= (1 << 24) || eta >= (1 << 16) ||
        n_walls >= (1 << 24)) {
        fail(s, TWA_E_INVALID, "too many factors for one solver");
        return bail(TWA_E_INVALID);
    }
    s->p = p, s->eta = eta, s->dim = dim, s->W = n_walls;
    s->rho0 = s->rho0_init = rho0, s->alpha = alpha, s->flags = flags;
    if (hipGetDevice(&s->device) != hipSuccess) {
        (void)hipGetLastError();
        fail(s, TWA_E_DEVICE, "hipGetDevice failed");
        return bail(TWA_E_DEVICE);
    }
    s->mem = twa_rt::current_allocator(s->device);
    if (!s->stream) {
        // The null stream cannot be captured into graphs.  A stream made with
        // the default flags orders itself with the null stream both ways, so
        // the caller's null-stream work and the solver's stay in order.
        if (hipStreamCreate(&s->own_stream) != hipSuccess) {
            (void)hipGetLastError();
            fail(s, TWA_E_DEVICE, "hipStreamCreate failed");
            return bail(TWA_E_DEVICE);
        }
        s->stream = s->own_stream;
    }
    // --- host copies for validation
    std::vector<float> hr, h0, hT, hw, hC;
    if (to_host(s, hr, radii, p) || to_host(s, h0, x0, (size_t)p * dim) || to_host(s, hT, xT, (size_t)p * dim) ||
        to_host(s, hw, walls, (size_t)n_walls * 2 * dim) || to_host(s, hC, C, (size_t)p * eta))
        return bail(TWA_E_DEVICE);
    if (!finite_all(hr) || !finite_all(h0) || !finite_all(hT) || !finite_all(hw) || !finite_all(hC)) {
        fail(s, TWA_E_INVALID, "non-finite input");
        return bail(TWA_E_INVALID);
    }
    for (float r : hr)
        if (!(r > 0.f)) {
            fail(s, TWA_E_INVALID, "radii must be > 0");
            return bail(TWA_E_INVALID);
        }
    const bool vel = (flags & (TWA_F_COST_MAXVEL | TWA_F_COST_MINVEL | TWA_F_VO)) != 0;
    for (float c : hC)
        if (vel ? !(c > 0.f) : c < 0.f) {
            fail(s, TWA_E_INVALID,
                 vel ? "velocity limits and deviation costs must be > 0" : "energy coefficients must be >= 0");
            return bail(TWA_E_INVALID);
        }
    double Lmax = 1.0;
    for (float v : h0) Lmax = std::max(Lmax, (double)std::fabs(v));
    for (float v : hT) Lmax = std::max(Lmax, (double)std::fabs(v));
    for (float v : hw) Lmax = std::max(Lmax, (double)std::fabs(v));
    s->h_radii = hr;
    s->h_walls = hw;
    s->coord_max = Lmax;
    if (check_ends(s, h0, hT) != TWA_OK) return bail(TWA_E_INFEASIBLE);
    // --- device buffers
    Params &P = s->P;
    P.p = p, P.eta = eta, P.W = n_walls, P.dim = dim;
    P.Fc = Fc, P.Fw = Fw, P.Fe = Fe, P.Ff = Ff;
    P.N = (long long)p * (eta + 1);
    // break-point intervals per wave in k_stream (see k_stream)
    P.cpw = (flags & (TWA_F_DENSE | TWA_F_ADMM)) ? 4 : 8; // as k_stream<..., DENSE> (ADMM runs dense)
    // rows of the pair triangle cut into chunks of 64: chunk (s, i, j0)
    std::vector<int> hrowchunk((size_t)p, 0);
    for (int i = 0; i + 1 < p; ++i) hrowchunk[i + 1] = hrowchunk[i] + (p - 1 - i + 63) / 64;
    P.cps = p > 1 ? hrowchunk[p - 1] : 0;
    P.nch = (long long)eta * P.cps;
    P.P2 = P2;
    if (P.nch >= (1LL << 31)) {
        fail(s, TWA_E_INVALID, "too many factors for one solver");
        return bail(TWA_E_INVALID);
    }
    // (i, j0) of each chunk of a break-point interval (the same for every s)
    std::vector<unsigned long long> hchunk((size_t)std::max<long long>(1, P.cps));
    {
        long long c = 0;
        for (int i = 0; i + 1 < p; ++i)
            for (int j0 = i + 1; j0 < p; j0 += 64, ++c)
                hchunk[c] = ((unsigned long long)i << 24) | (unsigned long long)j0;
    }
    P.nbc = (P.cps * ((eta + P.cpw - 1) / P.cpw) + kBlock / 64 - 1) / (kBlock / 64);
    P.nbw = (Fw + kBlock - 1) / kBlock;
    P.nbe = (Fe + kBlock - 1) / kBlock;
    P.nbf = (Ff + kBlock - 1) / kBlock;
    s->nblocks_stream = P.nbc + P.nbw + P.nbe + P.nbf;
    s->nblocks_queue = 4096;
    {
        // a shard takes the appends of every kShards-th wave of the column walk
        long long waves = P.cps * ((eta + P.cpw - 1) / P.cpw);
        P.qcap = (waves + kShards - 1) / kShards * 64 * P.cpw;
    }
    P.e_energy = Ff;
    P.e_coll = Ff + 2 * Fe;
    P.e_wall = P.e_coll + 4 * Fc;
    P.f_energy = Ff;
    P.f_coll = Ff + Fe;
    P.f_wall = Ff + Fe + Fc;
    // standard ADMM keeps u on every edge: it runs in the dense form
    P.admm = (flags & TWA_F_ADMM) ? 1 : 0;
    P.vo = (flags & TWA_F_VO) ? 1 : 0;
    P.cost = (flags & (TWA_F_COST_NONE | TWA_F_VO)) ? COST_NONE
             : (flags & TWA_F_COST_MAXVEL) ? COST_MAXVEL
             : (flags & TWA_F_COST_MINVEL) ? COST_MINVEL
                                           : COST_ENERGY;
    P.dense = ((flags & TWA_F_DENSE) || P.admm) ? 1 : 0;
    {
        double lim_m = 0;
        consensus_scale(p, n_walls, Lmax, &P.scale, &lim_m);
        P.scalef = (float)P.scale;
        // per contribution, in scaled units, rounded down to a float
        P.sat_lim = std::nextafter((float)(lim_m * P.scale), 0.f);
    }
    float *radii_d, *C_d;
    float4 *walls_d, *xfix_d;
    unsigned long long *wbc_d, *wbw_d;
    if (dev_alloc(s, &P.zr_prev, P.N) || dev_alloc(s, &P.zr_cur, P.N) || dev_alloc(s, &radii_d, p) ||
        dev_alloc(s, &walls_d, std::max(1, n_walls)) || dev_alloc(s, &C_d, (size_t)p * eta) ||
        dev_alloc(s, &xfix_d, Ff) || dev_alloc(s, &P.u_coll, (size_t)std::max<long long>(1, dim * Fc)) ||
        dev_alloc(s, &P.u_wall, (size_t)std::max<long long>(1, Fw)) ||
        dev_alloc(s, &P.u_energy, (size_t)Fe * 2 * dim) || dev_alloc(s, &P.u_fixed, (size_t)Ff * dim) ||
        dev_alloc(s, &P.bits_coll, (size_t)std::max<long long>(1, P.nch)) ||
        dev_alloc(s, &P.bits_wall, (size_t)std::max<long long>(1, (Fw + 31) / 32)) ||
        dev_alloc(s, &P.qc, (size_t)std::max<long long>(1, std::max<long long>(Fc, kShards * P.qcap))) ||
        dev_alloc(s, &P.qw, (size_t)std::max<long long>(1, Fw)) || dev_alloc(s, &P.counters, 8) ||
        dev_alloc(s, &P.qcnt, (size_t)kShards * kQueueStride) ||
        dev_alloc(s, &P.acc, (size_t)2 * dim * P.N) || dev_alloc(s, &P.cnt, (size_t)2 * P.N) ||
        dev_alloc(s, &P.inf_val, (size_t)P.N) ||
        dev_alloc(s, &P.x_coll, (size_t)std::max<long long>(1, dim * Fc)) ||
        dev_alloc(s, &P.x_wall, (size_t)std::max<long long>(1, Fw)) ||
        dev_alloc(s, &wbc_d, (size_t)std::max<long long>(1, (Fc + 63) / 64)) ||
        dev_alloc(s, &wbw_d, (size_t)std::max<long long>(1, (Fw + 63) / 64)) ||
        dev_alloc(s, &s->stats_dev, 4) || dev_alloc(s, &s->bad_dev, 1) || dev_alloc(s, &s->quality_dev, 3) ||
        dev_alloc(s, &s->resid_dev, 1))
        return bail(TWA_E_NOMEM);
    unsigned long long *chunk_d;
    int *rowchunk_d;
    if (dev_alloc(s, &chunk_d, hchunk.size()) || dev_alloc(s, &rowchunk_d, hrowchunk.size()))
        return bail(TWA_E_NOMEM);
    P.chunk_coll = chunk_d, P.rowchunk = rowchunk_d;
    if ((flags & TWA_F_TAPE) &&
        (dev_alloc(s, &s->origin_z, (size_t)P.N * dim) ||
         dev_alloc(s, &s->origin_u, (size_t)(P.e_wall + 2 * Fw) * dim) || dev_alloc(s, &s->origin_l, (size_t)P.N)))
        return bail(TWA_E_NOMEM);
    P.radii = radii_d, P.C = C_d, P.walls = walls_d, P.xfix = xfix_d;
    P.wbase_coll = wbc_d, P.wbase_wall = wbw_d;
    // (s, i, j) / (s, i, w) of the first factor of every 64, in canonical order
    std::vector<unsigned long long> hwbc((size_t)std::max<long long>(1, (Fc + 63) / 64)),
        hwbw((size_t)std::max<long long>(1, (Fw + 63) / 64));
    {
        long long f = 0;
        for (int s2 = 0; s2 < eta && Fc > 0; ++s2)
            for (int i = 0; i < p; ++i)
                for (int j = i + 1; j < p; ++j, ++f)
                    if ((f & 63) == 0)
                        hwbc[f >> 6] = ((unsigned long long)s2 << 48) | ((unsigned long long)i << 24) | (unsigned long long)j;
        f = 0;
        for (int s2 = 0; s2 < eta && Fw > 0; ++s2)
            for (int i = 0; i < p; ++i)
                for (int w = 0; w < n_walls; ++w, ++f)
                    if ((f & 63) == 0)
                        hwbw[f >> 6] = ((unsigned long long)s2 << 48) | ((unsigned long long)i << 24) | (unsigned long long)w;
    }
    P.stats = s->stats_dev;
    P.resid = s->resid_dev;
    P.rho = P.rho_prev = rho0;
    P.step = P.step_prev = alpha / rho0;
    // constants
    std::vector<float4> hwall(std::max(1, n_walls)), hfix, hz;
    for (int w = 0; w < n_walls; ++w) hwall[w] = make_float4(hw[w * 4 + 0], hw[w * 4 + 1], hw[w * 4 + 2], hw[w * 4 + 3]);
    // initial state: straight lines, <-rho INF at the ends and STD inside
    build_ends(s, h0, hT, hfix, hz);
    s->xfix_dev = xfix_d;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(radii_d, hr.data(), sizeof(float) * p, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(walls_d, hwall.data(), sizeof(float4) * hwall.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(C_d, hC.data(), sizeof(float) * hC.size(), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(xfix_d, hfix.data(), sizeof(float4) * Ff, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(wbc_d, hwbc.data(), sizeof(unsigned long long) * hwbc.size(), hipMemcpyHostToDevice,
                           s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(chunk_d, hchunk.data(), sizeof(unsigned long long) * hchunk.size(), hipMemcpyHostToDevice,
                           s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(rowchunk_d, hrowchunk.data(), sizeof(int) * hrowchunk.size(), hipMemcpyHostToDevice,
                           s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(wbw_d, hwbw.data(), sizeof(unsigned long long) * hwbw.size(), hipMemcpyHostToDevice,
                           s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(P.zr_cur, hz.data(), sizeof(float4) * P.N, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(P.zr_prev, hz.data(), sizeof(float4) * P.N, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        fail(s, TWA_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
        return bail(TWA_E_DEVICE);
    }
    if (reset_state_buffers(s) != TWA_OK) return bail(TWA_E_DEVICE);
    if (save_origin(s) != TWA_OK) return bail(TWA_E_DEVICE);
    if (tiny(s)) {
        const twa_status st = prepare_tiny(s);
        if (st != TWA_OK) return bail(st);
    }
    if ((flags & TWA_F_TAPE) && twa_rt::tape_setup(s) != TWA_OK) return bail(TWA_E_DEVICE);
    if (hipStreamSynchronize(s->stream) != hipSuccess) return bail(TWA_E_DEVICE);
    *out = s;
    return TWA_OK;
}

twa_status twa_set_init(twa_solver *s, const float *z) {
    TRY(check_alive(s));
    if (!z) return fail(s, TWA_E_INVALID, "null z");
    long long N = s->P.N;
    unsigned nb = (unsigned)((N + 255) / 256);
    const int startcode = s->P.admm ? (int)W_STD : (int)W_INF;
    const int goalcode = (s->P.admm || s->P.vo) ? (int)W_STD : (int)W_INF;
    hipLaunchKernelGGL(k_z_import, dim3(nb), dim3(256), 0, s->stream, s->P.zr_cur, z, s->p, s->eta, s->dim,
                       (const unsigned char *)nullptr, 0, startcode, goalcode);
    HIP_TRY(s, hipGetLastError());
    // the end points are the constants x(0), x(T)
    hipLaunchKernelGGL(k_fix_ends, dim3((unsigned)((s->p + 255) / 256)), dim3(256), 0, s->stream, s->P.zr_cur,
                       (const float4 *)s->P.xfix, s->p, s->eta, startcode, goalcode);
    HIP_TRY(s, hipGetLastError());
    HIP_TRY(s, hipMemcpyAsync(s->P.zr_prev, s->P.zr_cur, sizeof(float4) * N, hipMemcpyDeviceToDevice, s->stream));
    TRY(reset_state_buffers(s));
    s->iter = 0;
    return save_origin(s);
}

twa_status twa_set_endpoints(twa_solver *s, const float *x0, const float *xT) {
    TRY(check_alive(s));
    if (!x0 || !xT) return fail(s, TWA_E_INVALID, "null x0 or xT");
    std::vector<float> h0, hT;
    TRY(to_host(s, h0, x0, (size_t)s->p * s->dim));
    TRY(to_host(s, hT, xT, (size_t)s->p * s->dim));
    if (!finite_all(h0) || !finite_all(hT)) return fail(s, TWA_E_INVALID, "non-finite end point");
    for (const std::vector<float> *v : {&h0, &hT})
        for (float c : *v)
            if (std::fabs((double)c) > s->coord_max)
                return fail(s, TWA_E_INVALID, "end point beyond the coordinate range the solver was created for");
    TRY(check_ends(s, h0, hT));
    build_ends(s, h0, hT, s->h_fix, s->h_z);
    HIP_TRY(s, hipMemcpyAsync(s->xfix_dev, s->h_fix.data(), sizeof(float4) * s->h_fix.size(), hipMemcpyHostToDevice,
                              s->stream));
    HIP_TRY(s, hipMemcpyAsync(s->P.zr_cur, s->h_z.data(), sizeof(float4) * s->P.N, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(s, hipMemcpyAsync(s->P.zr_prev, s->h_z.data(), sizeof(float4) * s->P.N, hipMemcpyHostToDevice, s->stream));
    TRY(reset_state_buffers(s));
    s->iter = 0;
    TRY(save_origin(s));
    HIP_TRY(s, hipStreamSynchronize(s->stream)); // the sources are host memory of the solver, reused next call
    return TWA_OK;
}

twa_status twa_set_schedule(twa_solver *s, float rho0_init, int n_warm) {
    TRY(check_alive(s));
    if (!(rho0_init > 0.f) || n_warm < 0) return fail(s, TWA_E_INVALID, "rho0_init > 0 and n_warm >= 0 required");
    s->rho0_init = rho0_init;
    s->n_warm = n_warm;
    return TWA_OK;
}

twa_status twa_iterate(twa_solver *s, int k) {
    TRY(check_alive(s));
    if (k < 0) return fail(s, TWA_E_INVALID, "k must be >= 0");
    return iterate_impl(s, k, false);
}

twa_status twa_iterate_until(twa_solver *s, int max_iter, int every, double min_clearance, int *done, int *met) {
    TRY(check_alive(s));
    if (!done || !met) return fail(s, TWA_E_INVALID, "null done or met");
    *done = 0;
    *met = 0;
    if (max_iter < 0 || every < 1 || std::isnan(min_clearance))
        return fail(s, TWA_E_INVALID, "max_iter >= 0, every >= 1 and a clearance bar required");
    if (max_iter == 0) return TWA_OK;
    TinyLds L;
    const bool settled = s->iter >= s->n_warm && (!s->pending || s->iter - 1 >= s->n_warm);
    if (s->tiny_params && settled && !s->dbg_rho && !s->adj_pool && !s->tape.ok && every <= kTinyChunk &&
        tiny_layout(s, &L)) {
        // the whole call on the device: launches of whole blocks of `every`
        // iterations, each stopping at the first check that meets the bar
        // (a launch after that returns at once); the host reads the outcome
        // after every 8 launches, so a large max_iter queues no more launches
        // than that beyond the one that met the bar
        int *ctl = s->tiny_bins + 3;
        HIP_TRY(s, hipMemsetAsync(ctl, 0, 2 * sizeof(int), s->stream));
        const int chunk = kTinyChunk / every * every;
        int left = max_iter, first = s->pending ? 0 : 1, h[2] = {0, 0};
        while (left > 0 && !h[1]) {
            for (int l = 0; l < 8 && left > 0; ++l, first = 0) {
                const int n = std::min(left, chunk);
                hipLaunchKernelGGL(k_tiny<kTinyBlock>, dim3(1), dim3(kTinyBlock), L.total, s->stream,
                                   (const Params *)s->tiny_params, L, n, first, every, min_clearance, ctl);
                HIP_TRY(s, hipGetLastError());
                left -= n;
            }
            HIP_TRY(s, hipMemcpyAsync(h, ctl, sizeof(h), hipMemcpyDeviceToHost, s->stream));
            HIP_TRY(s, hipStreamSynchronize(s->stream));
        }
        s->iter += h[0];
        s->pending = true;
        *done = h[0];
        *met = h[1];
        return TWA_OK;
    }
    while (*done < max_iter) {
        const int n = std::min(every, max_iter - *done);
        TRY(iterate_impl(s, n, false));
        *done += n;
        double clr;
        TRY(twa_get_quality(s, nullptr, &clr, nullptr));
        if (clr >= min_clearance) {
            *met = 1;
            break;
        }
    }
    return TWA_OK;
}

twa_status twa_iterate_timed(twa_solver *s, int k, double *kernel_ms) {
    TRY(check_alive(s));
    if (!kernel_ms) return fail(s, TWA_E_INVALID, "null kernel_ms");
    if (k < 0) return fail(s, TWA_E_INVALID, "k must be >= 0");
    s->events_used = 0;
    double acc[3] = {0, 0, 0};
    twa_status st = iterate_impl(s, k, true);
    hipError_t e = hipStreamSynchronize(s->stream);
    // timed iterations: a start and a stop event for each of the three kernels
    long long timed = 0;
    for (size_t q = 0; q + 5 < s->events_used && e == hipSuccess; q += 6, ++timed) {
        for (int kk = 0; kk < 3; ++kk) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s->events[q + 2 * kk], s->events[q + 2 * kk + 1]) == hipSuccess)
                acc[kk] += ms;
        }
    }
    s->events_used = 0;
    // the timed iterations stand for all k
    const double scale = timed > 0 ? (double)k / (double)timed : 0.0;
    for (int kk = 0; kk < 3; ++kk) kernel_ms[kk] = acc[kk] * scale;
    if (st != TWA_OK) return st;
    if (e != hipSuccess) return fail(s, TWA_E_DEVICE, std::string("timed iterate: ") + hipGetErrorString(e));
    return TWA_OK;
}

twa_status twa_capture_next(twa_solver *s, float *x_out, unsigned char *rho_out) {
    TRY(check_alive(s));
    if ((x_out == nullptr) != (rho_out == nullptr)) return fail(s, TWA_E_INVALID, "pass both buffers or neither");
    s->dbg_x = x_out;
    s->dbg_rho = rho_out;
    return TWA_OK;
}

twa_status twa_get_trajectories(twa_solver *s, float *z_out) {
    TRY(check_alive(s));
    if (!z_out) return fail(s, TWA_E_INVALID, "null z_out");
    unsigned nb = (unsigned)((s->P.N + 255) / 256);
    hipLaunchKernelGGL(k_z_export, dim3(nb), dim3(256), 0, s->stream, (const float4 *)s->P.zr_cur, z_out,
                       (unsigned char *)nullptr, s->p, s->eta, s->dim);
    HIP_TRY(s, hipGetLastError());
    return TWA_OK;
}

twa_status twa_get_state(twa_solver *s, float *z, float *u, unsigned char *lrho, long long *iter) {
    TRY(check_alive(s));
    TRY(finalize(s));
    unsigned nb = (unsigned)((s->P.N + 255) / 256);
    if (z || lrho)
        hipLaunchKernelGGL(k_z_export, dim3(nb), dim3(256), 0, s->stream, (const float4 *)s->P.zr_cur, z, lrho, s->p,
                           s->eta, s->dim);
    if (u) {
        long long E = s->P.e_wall + 2 * s->P.Fw;
        hipLaunchKernelGGL(k_u_convert, dim3((unsigned)((E + 255) / 256)), dim3(256), 0, s->stream, s->P, u, s->dim,
                           1);
    }
    HIP_TRY(s, hipGetLastError());
    if (iter) *iter = s->iter;
    return TWA_OK;
}

twa_status twa_set_state(twa_solver *s, const float *z, const float *u, const unsigned char *lrho, long long iter) {
    TRY(twa_rt::import_state(s, z, u, lrho, iter));
    return save_origin(s);
}

twa_status twa_get_stats(twa_solver *s, twa_stats *out) {
    TRY(check_alive(s));
    if (!out) return fail(s, TWA_E_INVALID, "null stats");
    TRY(finalize(s));
    int h[4] = {0, 0, 0, 0};
    unsigned r = 0;
    int overflow = 0;
    HIP_TRY(s, hipMemcpyAsync(h, s->stats_dev, sizeof(int) * 3, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipMemcpyAsync(&r, s->resid_dev, sizeof(unsigned), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipMemcpyAsync(&overflow, s->P.counters + 5, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    double obj = 0, clr = 0;
    TRY(twa_get_quality(s, &obj, &clr, nullptr)); // synchronises
    out->iter = s->iter;
    out->active_coll = h[0];
    out->active_wall = h[1];
    out->queued = h[2];
    out->tape_checkpoints = s->tape.ok ? s->tape.count : 0;
    float rf;
    std::memcpy(&rf, &r, sizeof(rf));
    out->residual = s->resid_valid ? (double)rf : 0.0;
    out->objective = obj;
    out->min_clearance = clr;
    out->graph_iterations = s->graph_iters;
    if (overflow) return fail(s, TWA_E_NUMERIC, "consensus sum beyond its fixed-point range (diverging iterates)");
    return TWA_OK;
}

twa_status twa_get_quality(twa_solver *s, double *objective, double *min_clearance, double *max_move) {
    TRY(check_alive(s));
    const Params &P = s->P;
    unsigned long long *min_key = reinterpret_cast<unsigned long long *>(s->quality_dev + 2);
    hipLaunchKernelGGL(k_quality_sums, dim3(1), dim3(1024), 0, s->stream, (const float4 *)P.zr_cur,
                       (const float4 *)P.zr_prev, P.C, s->p, s->eta, s->quality_dev, min_key);
    const long long rows = (long long)s->p * s->eta;
    hipLaunchKernelGGL(k_quality_clearance, dim3((unsigned)std::min<long long>(rows, 8192)), dim3(256), 0, s->stream,
                       (const float4 *)P.zr_cur, P.radii, P.walls, s->p, s->eta, s->W, s->dim, min_key);
    HIP_TRY(s, hipGetLastError());
    double h[3];
    HIP_TRY(s, hipMemcpyAsync(h, s->quality_dev, sizeof(h), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    unsigned long long k;
    std::memcpy(&k, &h[2], sizeof(k));
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    double m;
    std::memcpy(&m, &b, sizeof(m));
    if (objective) *objective = h[0];
    if (max_move) *max_move = h[1];
    if (min_clearance) *min_clearance = m;
    return TWA_OK;
}

twa_status twa_consensus_scale(int p, int n_walls, double coord_max, double *scale, double *limit) {
    if (p < 1 || n_walls < 0 || !(coord_max >= 1.0) || !std::isfinite(coord_max) || !scale || !limit)
        return TWA_E_INVALID;
    consensus_scale(p, n_walls, coord_max, scale, limit);
    return TWA_OK;
}

twa_status twa_sizes(const twa_solver *s, long long *n_factors, long long *n_edges) {
    if (!s) return TWA_E_INVALID;
    const Params &P = s->P;
    if (n_factors) *n_factors = P.Ff + P.Fe + P.Fc + P.Fw;
    if (n_edges) *n_edges = P.e_wall + 2 * P.Fw;
    return TWA_OK;
}

twa_status twa_check_finite(twa_solver *s) {
    TRY(check_alive(s));
    TRY(finalize(s));
    HIP_TRY(s, hipMemsetAsync(s->bad_dev, 0, sizeof(int), s->stream));
    unsigned nb = (unsigned)((s->P.N + 255) / 256);
    hipLaunchKernelGGL(k_finite, dim3(nb), dim3(256), 0, s->stream, (const float4 *)s->P.zr_cur, s->P.N,
                       (const float *)s->P.u_coll, (long long)(4 * s->dim * s->P.Fc), s->bad_dev);
    hipLaunchKernelGGL(k_finite, dim3(1), dim3(256), 0, s->stream, (const float4 *)s->P.zr_cur, 0LL,
                       (const float *)s->P.u_wall, (long long)(4 * s->P.Fw), s->bad_dev);
    hipLaunchKernelGGL(k_finite, dim3(1), dim3(256), 0, s->stream, (const float4 *)s->P.zr_cur, 0LL,
                       (const float *)s->P.u_energy, (long long)(2 * s->dim * s->P.Fe), s->bad_dev);
    HIP_TRY(s, hipGetLastError());
    int bad = 0, overflow = 0;
    HIP_TRY(s, hipMemcpyAsync(&bad, s->bad_dev, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipMemcpyAsync(&overflow, s->P.counters + 5, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    if (bad) return fail(s, TWA_E_NUMERIC, "non-finite value in z or u");
    if (overflow) return fail(s, TWA_E_NUMERIC, "consensus sum beyond its fixed-point range (diverging iterates)");
    return TWA_OK;
}


// ============================================================================
// batched instances: one persistent launch over many solvers
// ============================================================================

} // extern "C"

struct twa_batch {
    std::vector<twa_solver *> solvers;
    hipStream_t stream = nullptr;
    Params *insts_dev = nullptr;
    int *bin_start_dev = nullptr, *bin_items_dev = nullptr;
    int block = 256, groups = 0;       // block 0: the phased form
    int2 *map_dev = nullptr;           // phased form: stream, queue, node block maps
    int n_stream = 0, n_queue = 0, n_nodes = 0;
    hipGraphExec_t pexec = nullptr;    // phased form: kPhasedChunk iterations
    std::string err;
    twa_status latched = TWA_OK;
    hipGraphExec_t gexec = nullptr;
    int g_k = -1, g_first = -1;
    std::vector<Params> hparams;       // host copy of insts_dev
    hipStream_t own_stream = nullptr;  // made when the caller passes the null stream
    twa_rt::Allocator mem;             // where insts_dev, the bins and map_dev come from
    size_t map_bytes = 0;
};

namespace {

twa_status bfail(twa_batch *b, twa_status st, const std::string &msg) {
    if (b) {
        b->err = msg;
        if (st == TWA_E_DEVICE) b->latched = TWA_E_DEVICE;
    }
    return st;
}

#define BHIP_TRY(b, call)                                                                                      \
    do {                                                                                                       \
        hipError_t e_ = (call);                                                                                \
        if (e_ != hipSuccess) return bfail((b), TWA_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// cost of one iteration of a solver inside one workgroup of `block` lanes
double batch_cost(const twa_solver *s, int block) {
    const Params &P = s->P;
    auto ch = [block](long long n) { return (double)((n + block - 1) / block); };
    return ch(P.Fc) + ch(P.Fw) + ch(P.Fe) + ch(P.Ff) + ch(P.N) + 4.0;
}

void drop_graph(twa_batch *b) {
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
    b->g_k = b->g_first = -1;
}

twa_status batch_bins(twa_batch *b) {
    int n = (int)b->solvers.size();
    int G = std::max(1, std::min(b->groups > 0 ? b->groups : n, n));
    // longest processing time first onto the least-loaded bin
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::vector<double> cost(n);
    for (int i = 0; i < n; ++i) cost[i] = batch_cost(b->solvers[i], b->block);
    std::sort(order.begin(), order.end(), [&](int a, int c) { return cost[a] > cost[c]; });
    std::vector<double> load(G, 0.0);
    std::vector<std::vector<int>> bins(G);
    for (int i : order) {
        int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        bins[g].push_back(i);
        load[g] += cost[i];
    }
    std::vector<int> start(G + 1, 0), items;
    for (int g = 0; g < G; ++g) {
        start[g + 1] = start[g] + (int)bins[g].size();
        for (int i : bins[g]) items.push_back(i);
    }
    BHIP_TRY(b, hipMemcpyAsync(b->bin_start_dev, start.data(), sizeof(int) * (G + 1), hipMemcpyHostToDevice, b->stream));
    BHIP_TRY(b, hipMemcpyAsync(b->bin_items_dev, items.data(), sizeof(int) * n, hipMemcpyHostToDevice, b->stream));
    BHIP_TRY(b, hipStreamSynchronize(b->stream));
    b->groups = G;
    drop_graph(b);
    return TWA_OK;
}

constexpr int kPhasedChunk = 32;

void launch_batch(twa_batch *b, int k, int first) {
    if (b->block == 0) {
        const bool dense = b->solvers[0]->P.dense != 0;
        const Params *ins = (const Params *)b->insts_dev;
        const int2 *ms = b->map_dev, *mq = ms + b->n_stream, *mn = mq + b->n_queue;
        const dim3 gs(b->n_stream), gq(b->n_queue), gn(b->n_nodes);
        for (int it = 0; it < k; ++it) {
            if (first && it == 0) {
                if (dense) hipLaunchKernelGGL((kp_stream<M_FIRST, true>), gs, dim3(kBlock), 0, b->stream, ins, ms);
                else hipLaunchKernelGGL((kp_stream<M_FIRST, false>), gs, dim3(kBlock), 0, b->stream, ins, ms);
                hipLaunchKernelGGL(kp_queue<M_FIRST>, gq, dim3(64), 0, b->stream, ins, mq);
            } else {
                if (dense) hipLaunchKernelGGL((kp_stream<M_FUSED, true>), gs, dim3(kBlock), 0, b->stream, ins, ms);
                else hipLaunchKernelGGL((kp_stream<M_FUSED, false>), gs, dim3(kBlock), 0, b->stream, ins, ms);
                hipLaunchKernelGGL(kp_queue<M_FUSED>, gq, dim3(64), 0, b->stream, ins, mq);
            }
            hipLaunchKernelGGL(kp_nodes, gn, dim3(kBlock), 0, b->stream, ins, mn);
        }
        return;
    }
    dim3 grid(b->groups);
    if (b->block == 1024)
        hipLaunchKernelGGL(k_batch<1024>, grid, dim3(1024), 0, b->stream, (const Params *)b->insts_dev,
                           (const int *)b->bin_start_dev, (const int *)b->bin_items_dev, k, first);
    else if (b->block == 512)
        hipLaunchKernelGGL(k_batch<512>, grid, dim3(512), 0, b->stream, (const Params *)b->insts_dev,
                           (const int *)b->bin_start_dev, (const int *)b->bin_items_dev, k, first);
    else
        hipLaunchKernelGGL(k_batch<256>, grid, dim3(256), 0, b->stream, (const Params *)b->insts_dev,
                           (const int *)b->bin_start_dev, (const int *)b->bin_items_dev, k, first);
}

} // namespace

extern "C" {

const char *twa_batch_last_error(const twa_batch *b) { return b ? b->err.c_str() : "null batch"; }

void twa_batch_destroy(twa_batch *b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    for (twa_solver *s : b->solvers) twa_destroy(s);
    const size_t n = b->solvers.size();
    b->mem.put(b->insts_dev, sizeof(Params) * n, b->stream);
    b->mem.put(b->bin_start_dev, sizeof(int) * (n + 1), b->stream);
    b->mem.put(b->bin_items_dev, sizeof(int) * n, b->stream);
    b->mem.put(b->map_dev, b->map_bytes, b->stream);
    if (b->pexec) (void)hipGraphExecDestroy(b->pexec);
    if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
    delete b;
}

twa_status twa_batch_create(int n, const twa_instance *inst, unsigned flags, void *hip_stream, twa_batch **out) {
    if (!out || n < 1 || !inst) return TWA_E_INVALID;
    *out = nullptr;
    twa_batch *b = new (std::nothrow) twa_batch();
    if (!b) return TWA_E_NOMEM;
    b->stream = static_cast<hipStream_t>(hip_stream);
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return TWA_E_DEVICE;
    }
    b->mem = twa_rt::current_allocator(device);
    if (!b->stream) {
        // as twa_create: a capturable stream ordered with the null stream
        if (hipStreamCreate(&b->own_stream) != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return TWA_E_DEVICE;
        }
        b->stream = b->own_stream;
    }
    for (int i = 0; i < n; ++i) {
        const twa_instance &I = inst[i];
        twa_solver *s = nullptr;
        twa_status st = twa_create(I.p, I.eta, I.dim, I.radii, I.x0, I.xT, I.n_walls, I.walls, I.C, I.rho0, I.alpha,
                                   flags, b->stream, &s);
        if (st == TWA_OK && I.z0) {
            st = twa_set_init(s, I.z0);
            if (st != TWA_OK) twa_destroy(s);
        }
        if (st != TWA_OK) {
            twa_batch_destroy(b);
            return st;
        }
        b->solvers.push_back(s);
    }
    b->insts_dev = static_cast<Params *>(b->mem.get(sizeof(Params) * n, b->stream));
    b->bin_start_dev = static_cast<int *>(b->mem.get(sizeof(int) * (n + 1), b->stream));
    b->bin_items_dev = static_cast<int *>(b->mem.get(sizeof(int) * n, b->stream));
    if (!b->insts_dev || !b->bin_start_dev || !b->bin_items_dev) {
        twa_batch_destroy(b);
        return TWA_E_NOMEM;
    }
    std::vector<Params> &h = b->hparams;
    h.resize(n);
    for (int i = 0; i < n; ++i) {
        h[i] = b->solvers[i]->P;
        h[i].dbg_x = nullptr;
        h[i].dbg_rho = nullptr;
    }
    // block maps of the phased form: each instance's own stream and node
    // blocks, and one queue block per 256 factors (1..64: crowded instances
    // queue a good share of their factors, and a block's entries beyond the
    // first 64 wait for a whole minimiser each)
    // Queue blocks are ordered block-major (every instance's first block,
    // then every instance's second...): an instance's first blocks hold its
    // entries, and consecutive blocks land on different compute units, so
    // the busy ones spread over the chip instead of stacking up.
    std::vector<int2> ms, mq, mn;
    std::vector<int> nqb(n);
    for (int i = 0; i < n; ++i) {
        const twa_solver *s = b->solvers[i];
        for (long long lb = 0; lb < s->nblocks_stream; ++lb) ms.push_back(make_int2(i, (int)lb));
        nqb[i] = (int)std::min<long long>(64, std::max<long long>(1, (s->P.Fc + s->P.Fw + 255) / 256));
        for (long long lb = 0; lb < (s->P.N + kBlock - 1) / kBlock; ++lb) mn.push_back(make_int2(i, (int)lb));
    }
    for (int qb = 0; qb < 64; ++qb)
        for (int i = 0; i < n; ++i)
            if (qb < nqb[i]) mq.push_back(make_int2(i, qb | (nqb[i] << 16)));
    b->n_stream = (int)ms.size();
    b->n_queue = (int)mq.size();
    b->n_nodes = (int)mn.size();
    ms.insert(ms.end(), mq.begin(), mq.end());
    ms.insert(ms.end(), mn.begin(), mn.end());
    b->map_bytes = sizeof(int2) * ms.size();
    b->map_dev = static_cast<int2 *>(b->mem.get(b->map_bytes, b->stream));
    if (!b->map_dev) {
        twa_batch_destroy(b);
        return TWA_E_NOMEM;
    }
    if (hipMemcpyAsync(b->map_dev, ms.data(), sizeof(int2) * ms.size(), hipMemcpyHostToDevice, b->stream) !=
            hipSuccess ||
        hipMemcpyAsync(b->insts_dev, h.data(), sizeof(Params) * n, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        batch_bins(b) != TWA_OK) {
        twa_batch_destroy(b);
        return TWA_E_DEVICE;
    }
    *out = b;
    return TWA_OK;
}

twa_status twa_batch_config(twa_batch *b, int block, int groups) {
    if (!b) return TWA_E_INVALID;
    if (b->latched != TWA_OK) return b->latched;
    if (block == 0) {
        b->block = 0;
        drop_graph(b);
        return TWA_OK;
    }
    if (block != 256 && block != 512 && block != 1024)
        return bfail(b, TWA_E_INVALID, "block must be 0, 256, 512 or 1024");
    if (groups < 1) return bfail(b, TWA_E_INVALID, "groups must be >= 1");
    b->block = block;
    b->groups = groups;
    return batch_bins(b);
}

twa_status twa_batch_iterate(twa_batch *b, int k) {
    if (!b) return TWA_E_INVALID;
    if (b->latched != TWA_OK) return b->latched;
    if (k < 0) return bfail(b, TWA_E_INVALID, "k must be >= 0");
    if (k == 0) return TWA_OK;
    bool any_pending = false, all_pending = true, dbg = false;
    for (twa_solver *s : b->solvers) {
        if (s->latched != TWA_OK) return bfail(b, s->latched, "an instance has a latched device error");
        if (s->n_warm > 0 && s->iter < s->n_warm) return bfail(b, TWA_E_STATE, "batched instances take no rho0 schedule");
        // an iteration run at the warm-up rho0 whose u update is still
        // pending: settle it with its own weight and step (the batched
        // kernels run the steady rho0 only)
        if (s->pending && s->iter - 1 < s->n_warm && finalize(s) != TWA_OK)
            return bfail(b, TWA_E_DEVICE, "finalize: " + s->err);
        any_pending |= s->pending;
        all_pending &= s->pending;
        dbg |= s->dbg_rho != nullptr;
    }
    if (any_pending && !all_pending)
        for (twa_solver *s : b->solvers)
            if (finalize(s) != TWA_OK) return bfail(b, TWA_E_DEVICE, "finalize: " + s->err);
    int first = all_pending ? 0 : 1;
    if (dbg) {
        // twa_capture_next on a member: its first iteration runs on its own
        // launch with the capture buffers in the parameters the kernels read
        std::vector<Params> h = b->hparams;
        for (size_t i = 0; i < h.size(); ++i) {
            h[i].dbg_x = b->solvers[i]->dbg_x;
            h[i].dbg_rho = b->solvers[i]->dbg_rho;
        }
        BHIP_TRY(b, hipMemcpyAsync(b->insts_dev, h.data(), sizeof(Params) * h.size(), hipMemcpyHostToDevice, b->stream));
        launch_batch(b, 1, first);
        BHIP_TRY(b, hipGetLastError());
        BHIP_TRY(b, hipMemcpyAsync(b->insts_dev, b->hparams.data(), sizeof(Params) * h.size(), hipMemcpyHostToDevice,
                                   b->stream));
        BHIP_TRY(b, hipStreamSynchronize(b->stream)); // h lives on this stack
        for (twa_solver *s : b->solvers) {
            s->dbg_x = nullptr;
            s->dbg_rho = nullptr;
            s->pending = true;
            s->iter += 1;
        }
        first = 0;
        if (--k == 0) return TWA_OK;
    }
    if (b->block == 0) {
        // phased form: a first iteration on its own, then a captured graph
        // of kPhasedChunk iterations replayed, then the rest launched directly
        int left = k;
        if (first) {
            launch_batch(b, 1, 1);
            --left;
        }
        if (left >= kPhasedChunk && !b->pexec) {
            hipGraph_t g = nullptr;
            bool ok = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
            if (ok) {
                launch_batch(b, kPhasedChunk, 0);
                ok = hipStreamEndCapture(b->stream, &g) == hipSuccess && g != nullptr;
                if (ok) ok = hipGraphInstantiate(&b->pexec, g, nullptr, nullptr, 0) == hipSuccess;
                if (g) (void)hipGraphDestroy(g);
            }
            (void)hipGetLastError();
            if (!ok) b->pexec = nullptr;
        }
        for (; left >= kPhasedChunk && b->pexec; left -= kPhasedChunk) BHIP_TRY(b, hipGraphLaunch(b->pexec, b->stream));
        if (left > 0) launch_batch(b, left, 0);
        BHIP_TRY(b, hipGetLastError());
        for (twa_solver *s : b->solvers) {
            s->pending = true;
            s->iter += k;
        }
        return TWA_OK;
    }
    if (!b->gexec || b->g_k != k || b->g_first != first) {
        drop_graph(b);
        hipGraph_t g = nullptr;
        bool captured = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (captured) {
            launch_batch(b, k, first);
            captured = hipStreamEndCapture(b->stream, &g) == hipSuccess && g != nullptr;
            if (captured) captured = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0) == hipSuccess;
            if (g) (void)hipGraphDestroy(g);
        }
        (void)hipGetLastError();
        if (captured) {
            b->g_k = k;
            b->g_first = first;
        } else {
            b->gexec = nullptr;
        }
    }
    if (b->gexec) {
        BHIP_TRY(b, hipGraphLaunch(b->gexec, b->stream));
    } else {
        launch_batch(b, k, first);
        BHIP_TRY(b, hipGetLastError());
    }
    for (twa_solver *s : b->solvers) {
        s->pending = true;
        s->iter += k;
    }
    return TWA_OK;
}

twa_status twa_batch_iterate_timed(twa_batch *b, int k, double *ms) {
    if (!b || !ms) return TWA_E_INVALID;
    hipEvent_t e0, e1;
    BHIP_TRY(b, hipEventCreate(&e0));
    BHIP_TRY(b, hipEventCreate(&e1));
    (void)hipEventRecord(e0, b->stream);
    twa_status st = twa_batch_iterate(b, k);
    (void)hipEventRecord(e1, b->stream);
    hipError_t e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = t;
    if (st != TWA_OK) return st;
    if (e != hipSuccess) return bfail(b, TWA_E_DEVICE, std::string("batch timing: ") + hipGetErrorString(e));
    return TWA_OK;
}

twa_status twa_batch_size(const twa_batch *b, int *n) {
    if (!b || !n) return TWA_E_INVALID;
    *n = (int)b->solvers.size();
    return TWA_OK;
}

twa_status twa_batch_solver(twa_batch *b, int i, twa_solver **s) {
    if (!b || !s || i < 0 || i >= (int)b->solvers.size()) return TWA_E_INVALID;
    *s = b->solvers[i];
    return TWA_OK;
}

twa_status twa_batch_get_trajectories(twa_batch *b, int i, float *z_out) {
    if (!b || i < 0 || i >= (int)b->solvers.size()) return TWA_E_INVALID;
    return twa_get_trajectories(b->solvers[i], z_out);
}

} // extern "C"
