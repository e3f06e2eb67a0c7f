// solver.h -- state of one planner instance shared by the translation
// units of libtwa.so (forward iteration in twa.hip, adjoint in adjoint.hip).
// Internal: not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/twa.h"
#include "prox.h"

namespace twa_rt {

// a zero weight enters the minimisers as a small equal value (App. C-E)
constexpr float kZeroWeight = 1e-9f;

// weight value of a <-rho code under standard weight rho (infinity is
// carried by the code; its value slot is unused)
__host__ __device__ __forceinline__ float wval(int code, float rho) {
    return code == twa::W_STD ? rho : (code == twa::W_ZERO ? kZeroWeight * rho : 0.f);
}

// One active collision or wall factor of an iteration recomputed by
// twa_backward: its index (within its kind) and the minimiser input n of its
// edges (planar: 4 edges x 2 for a collision factor, 2 x 2 for a wall).
struct AdjRec {
    unsigned f, wall;
    float n[8];
};

struct Params {
    int p, eta, W, dim;
    long long Fc, Fw, Fe, Ff;
    long long nbc, nbw, nbe, nbf; // blocks per factor kind in k_stream
    int cpw;                      // break-point intervals per wave in k_stream
    // node records, time-major (s * p + i): x, y, z, <-rho code
    float4 *zr_prev, *zr_cur;
    const float *radii;  // [p]
    const float4 *walls; // [W] (xL.x, xL.y, xR.x, xR.y)
    const float *C;      // [p][eta]
    const float4 *xfix;  // [2p] start(i), goal(i)
    float4 *u_coll;      // [dim planes][Fc]
    float4 *u_wall;      // [Fw]
    float *u_energy;     // [Fe][2*dim]
    float *u_fixed;      // [2p][dim]
    unsigned long long *bits_coll;      // [nch] activity of each collision chunk's pairs
    unsigned *bits_wall;                // [Fw / 32] activity of wall factors
    const unsigned long long *chunk_coll; // [cps] (i, j0) of each chunk of an interval, packed 24|24 bits
    const int *rowchunk;                // [p] first chunk of row i within a break-point interval
    long long nch, cps, P2;             // chunks, chunks per interval, pairs p(p-1)/2
    unsigned *qc, *qw;
    int *qcnt;        // collision queue shard lengths, shard q at [q * kQueueStride]
    long long qcap;   // entries per collision queue shard
    int *counters; // [1] qw length, [2] active coll, [3] active wall, [5] consensus overflow (sticky)
    int *stats;    // last iteration: active coll, active wall, queued
    unsigned long long *acc; // [2 kinds][dim][N]  kind 0 = std, 1 = inf
    int *cnt;                // [2][N]
    float4 *inf_val;         // [N] m of a node's certain edge, kept exact when it is the only one
    float4 *x_coll;          // [dim planes][Fc] x of factors active in the last iteration
    float4 *x_wall;          // [Fw]
    const unsigned long long *wbase_coll; // per 64 factors: (s, i, j) of the first, packed 16|24|24 bits
    const unsigned long long *wbase_wall; // per 64 factors: (s, i, w) of the first
    long long N;
    double scale;
    float scalef;
    float sat_lim;   // largest |m| * scale one contribution may carry: degree of it cannot overflow int64
    unsigned *resid; // primal residual max |x - z| of the u updates run by the finalizing pass (float bits)
    float rho, step;      // this iteration: weight value of rho0, alpha/rho0
    float rho_prev, step_prev;
    int dense;
    int admm; // standard ADMM: every factor sends weight rho0 (TWA_F_ADMM)
    int cost; // per-segment factors: energy, none, maximum or minimum velocity
    int vo;   // one epoch of the velocity-obstacle planner (TWA_F_VO)
    // debug capture of this iteration
    float *dbg_x;
    unsigned char *dbg_rho;
    // adjoint capture of this iteration (twa_backward): n of every collision
    // and wall factor that sends weight rho0 is appended to adj_pool
    AdjRec *adj_pool;
    unsigned *adj_cursor; // appends attempted (those at index >= adj_cap are dropped)
    unsigned adj_cap;
    unsigned *adj_offs;   // the node pass stores the final cursor here
    unsigned char *dbg_l; // the node pass writes the new <-rho codes here, canonical [p][eta+1]
    int *dbg_cnt;         // and the size of each node's mean set (its edges of the winning weight)
    long long e_energy, e_coll, e_wall; // canonical edge offsets
    long long f_energy, f_coll, f_wall; // canonical factor offsets
};

// What the iterations of a segment recomputed by twa_backward capture:
// iteration t writes its ->rho to rout + t*F, appends a record per factor
// that sent rho0 to pool (cursor, cap), stores the cursor after it to
// offs[t + 1], and (node pass) the new <-rho codes to lseg + (t+1)*N and the
// mean-set sizes to cntseg + t*N.
struct SegCapture {
    unsigned char *rout;
    AdjRec *pool;
    unsigned *cursor;
    unsigned cap;
    unsigned *offs;
    unsigned char *lseg;
    int *cntseg;
    long long F, N;
};

// Device memory provider of one solver or batch: the process-wide pair of
// twa_set_allocator in effect at its create, else hipMalloc / hipFree.
struct Allocator {
    twa_alloc_fn alloc = nullptr;
    twa_free_fn release = nullptr;
    void *ctx = nullptr;
    int device = 0;
    // nullptr on failure (a HIP error it caused is cleared)
    void *get(size_t bytes, hipStream_t stream) const;
    // the caller has synchronised stream (or never used the memory)
    void put(void *ptr, size_t bytes, hipStream_t stream) const;
};
// the pair in effect now, for device
Allocator current_allocator(int device);

} // namespace twa_rt

struct twa_solver {
    int p = 0, eta = 0, dim = 0, W = 0;
    float rho0 = 1.f, alpha = 1.f, rho0_init = 1.f;
    int n_warm = 0;
    unsigned flags = 0;
    long long iter = 0;
    bool pending = false;
    hipStream_t stream = nullptr;
    twa_rt::Params P{};
    int *stats_dev = nullptr;
    double *quality_dev = nullptr; // twa_get_quality: objective, largest move, clearance key
    unsigned *resid_dev = nullptr;  // residual of the last finalized iteration (float bits)
    bool resid_valid = false;       // resid_dev holds the last iteration's residual
    int *bad_dev = nullptr;
    twa_rt::Allocator mem;                           // where every buffer below comes from
    std::vector<std::pair<void *, size_t>> allocs; // buffers of create (freed at destroy)
    std::string err;
    twa_status latched = TWA_OK;
    float *dbg_x = nullptr;
    unsigned char *dbg_rho = nullptr;
    twa_rt::AdjRec *adj_pool = nullptr; // adjoint capture of the next iteration
    unsigned *adj_cursor = nullptr;
    unsigned adj_cap = 0;
    unsigned *adj_offs = nullptr;
    unsigned char *dbg_l = nullptr;
    int *dbg_cnt = nullptr;
    long long nblocks_stream = 0;
    int nblocks_queue = 0;
    // event timing (twa_iterate_timed): 1 = kernels launched now take a
    // start and a stop event from the pool
    std::vector<hipEvent_t> events; // kept for the solver's life and reused
    size_t events_used = 0;
    int timing = 0;
    // HIP graphs of 1, 2, 4, ... kGraphIters fused iterations (graphs[b]
    // holds 2^b), so any count of steady iterations replays
    static constexpr int kGraphSizes = 6;
    hipGraphExec_t graphs[kGraphSizes] = {};
    bool graph_failed = false;
    long long graph_iters = 0;  // iterations run from graph replays
    hipStream_t own_stream = nullptr; // made at create when the caller passes the null stream
    bool no_capture = false;          // inside a call that allocates nothing: capture no new graph
    std::vector<float> h_radii, h_walls; // host copies for validating new end points
    double coord_max = 1.0;            // the coordinate range the consensus scale was chosen for
    float4 *xfix_dev = nullptr;        // the fixed factors' constants (P.xfix)
    std::vector<float4> h_fix, h_z;    // staging of twa_set_endpoints (kept, so later calls reuse it)
    int device = 0;                   // the HIP device current at create
    // tiny instances: the persistent batched kernel on this one instance
    // (a device copy of the parameters and its one-bin layout)
    twa_rt::Params *tiny_params = nullptr;
    int *tiny_bins = nullptr;
    // TWA_F_TAPE: the state the differentiated run starts from (canonical
    // layouts), saved by create / set_init / set_state
    float *origin_z = nullptr, *origin_u = nullptr;
    unsigned char *origin_l = nullptr;
    long long origin_iter = 0;
    // twa_backward's buffers: allocated at its first call, grown when a
    // later call needs more, kept until twa_destroy
    void *adj_ws = nullptr, *adj_arena = nullptr, *adj_pool_mem = nullptr;
    size_t adj_ws_bytes = 0, adj_arena_bytes = 0, adj_pool_bytes = 0;
    // twa_backward's second stream (a segment's reverse steps run on it while
    // the segment before it is recomputed on `stream`) and the events that
    // order the two: recomputed into, and reversed from, each capture copy
    hipStream_t adj_stream = nullptr;
    hipEvent_t adj_ev[4] = {};
    // graphs of a whole recomputed segment, one per capture copy, with the
    // segment length and capture buffers they were captured for
    hipGraphExec_t seg_graph[2] = {};
    twa_rt::SegCapture seg_key[2] = {};
    long long seg_len[2] = {0, 0};
    bool seg_failed = false;
    // Forward-time checkpoints for twa_backward (sized and allocated by its
    // first allocating call): from the next start of a differentiated run,
    // the state at every `interval` iterations since it is packed as
    // twa_backward packs its own checkpoints (z and <-rho dense, the fixed
    // and energy u dense, the collision/wall u as records), so a backward
    // call over a run the tape covers skips re-running the forward.
    struct Tape {
        int interval = 32;     // iterations between checkpoints
        int cap = 0;           // checkpoints it holds
        int count = 0;         // checkpoints taken since the run's start
        bool ok = false;       // recording (the run started after allocation, nothing lost)
        float *z = nullptr;    // [cap][N][2]
        unsigned char *l = nullptr; // [cap][N]
        float *us = nullptr;   // [cap][fixed + energy edges][2]
        unsigned *first = nullptr, *end = nullptr; // [cap] record ranges
        unsigned *cursor = nullptr;                // records appended (device)
        twa_rt::AdjRec *arena = nullptr;
        unsigned arena_cap = 0;
        float *u_tmp = nullptr; // [E][2] dense u of the state being packed
        void *mem = nullptr;
        size_t bytes = 0;
    } tape;
    unsigned *adj_used = nullptr; // pinned host [2]: records each recompute wanted
};

namespace twa_rt {

// record an error on the solver (device errors latch) and return st
twa_status fail(twa_solver *s, twa_status st, const std::string &msg);
// TWA_E_INVALID for NULL, the latched error if any, else TWA_OK
twa_status check_alive(twa_solver *s);
// weight value rho0 of iteration k under the warm-up schedule
float rho_at(const twa_solver *s, long long k);
// replace the state (canonical device arrays) without touching the start
// of the differentiated run
twa_status import_state(twa_solver *s, const float *z, const float *u, const unsigned char *lrho, long long iter);
// <-rho codes of the current node records, canonical [p][eta+1] (device
// array); leaves a pending u update pending
twa_status export_lrho(twa_solver *s, unsigned char *lrho);
// len iterations from a state just imported (no update pending), each
// capturing as c describes; replayed from the graph kept for capture copy
// `slot` (0 or 1; -1: no graph) when every iteration runs at the
// configuration's rho0 and the graph fits (captured now unless no_capture),
// else launched one by one
twa_status run_segment(twa_solver *s, long long len, const SegCapture &c, int slot);
// At a checkpoint iteration of a recording tape, pack the current state
// into it (twa_iterate calls it at multiples of the interval since the run's
// start); a no-op otherwise
twa_status tape_take(twa_solver *s);
// TWA_F_TAPE at create: look up the static scratch of twa_backward_noalloc
// on the solver's device, make twa_backward's second stream and its events
twa_status tape_setup(twa_solver *s);

} // namespace twa_rt

#define HIP_TRY(s, call)                                                                                       \
    do {                                                                                                       \
        hipError_t e_ = (call);                                                                                \
        if (e_ != hipSuccess)                                                                                  \
            return twa_rt::fail((s), TWA_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));         \
    } while (0)

#define TRY(x)                                                                                                 \
    do {                                                                                                       \
        twa_status st_ = (x);                                                                                  \
        if (st_ != TWA_OK) return st_;                                                                         \
    } while (0)
