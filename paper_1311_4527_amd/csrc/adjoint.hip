// adjoint.hip -- reverse-mode derivative of unrolled planner iterations
// (twa_backward of include/twa.h).
//
// One iteration k of App. B maps (z^k, u^k) to (z^{k+1}, u^{k+1}):
//   n = z - u                       (step 1, per edge)
//   x = g(n), ->rho                 (step 2, per factor)
//   m = x + u                       (step 4)
//   z' = mean of m over the edges of the node that carry the dominant weight
//        (infinity if any, else rho0; all edges if every weight is zero)
//   u' = u + (alpha/rho0)(x - z')   if ->rho and the new <-rho are both rho0,
//        else 0                     (steps 5-7)
// With every discrete decision held at the forward run's (the weights, the
// minimiser candidate) the map is differentiable, and its transpose runs
// backwards through the same steps, one reverse step per iteration:
//   k_adj_accum    per captured factor (one that sent rho0): its edges' count
//                  and kept cotangents du' per node
//   k_adj_select   per node: the class of the mean, and
//                  g = (dz' - s * sum of du' over kept edges) / |mean set|
//   k_adj_factors  per fixed / energy factor and per captured factor:
//                  dx = s du'[kept] + g[in mean set], dn = J_g^T dx (the
//                  minimiser derivatives from prox.h), du = du'[kept] +
//                  g[in mean set] - dn, dz += dn per node, radius and start /
//                  goal cotangents
// A factor that sent weight 0 carries no cotangent in the energy mode (see
// k_adj_accum), so a step's cost follows the active factors, not the edges.
// The forward decisions come from the solver itself: checkpoints every
// ceil(sqrt(K)) iterations (state in the canonical layouts, collision and
// wall u kept sparse: by the u rule of App. B step 7 it is zero on every
// factor that sent weight 0), and each segment recomputed with its weights
// and the minimiser inputs n of the factors that sent rho0 captured by the
// factor kernels themselves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/twa.h"
#include "prox.h"
#include "solver.h"

using namespace twa;
using twa_rt::AdjRec;
using twa_rt::wval;

namespace {

struct Adj {
    int p, eta, W;
    long long P2, N, E, F;
    long long e_energy, e_coll, e_wall, f_energy, f_coll, f_wall;
    const float *radii;
    const float4 *walls;
    const float *C;
    // decisions of iteration k
    const unsigned char *l;      // [N] <-rho^k
    const unsigned char *rout;   // [F] ->rho^k
    const unsigned char *lnext;  // [N] <-rho^{k+1}
    float rho, step;             // weight rho0 of iteration k; u step alpha / (configuration's rho0)
    // cotangents
    const float *zb_in;  // [N][2] dL/dz^{k+1}
    float *zb_out;       // [N][2] dL/dz^k: zeroed, then accumulated
    const float *ub_in;  // [E][2] dL/du^{k+1}
    float *ub_out;       // [E][2] dL/du^k: zeroed, then written where nonzero
    float *g;            // [N][2]
    unsigned char *cls;  // [N] weight class of the node's mean
    const int *cnt;      // [N] size of the node's mean set in iteration k (captured)
    const float *S_in;   // [N][2] sum of dL/du^{k+1} over the kept edges of captured factors
    float *S_next;       // [N][2] the same sum for iteration k-1, accumulated here
    const unsigned char *rout_prev; // [F] ->rho^{k-1}, or null when k-1 is not captured yet
    float *dx0, *dxT;    // [p][2], accumulated
    double *drd;         // [p], accumulated
};

__device__ __forceinline__ long long node_id(const Adj &A, int i, int s) { return (long long)i * (A.eta + 1) + s; }

__device__ __forceinline__ long long pair_index(int p, int a, int b) {
    return (long long)a * p - (long long)a * (a + 1) / 2 + (b - a - 1);
}

// (i, j) of collision factor q of a break-point interval (row-major i < j)
__device__ __forceinline__ void pair_of(int p, long long q, int &i, int &j) {
    double b = 2.0 * p - 1.0;
    i = (int)floor((b - sqrt(fmax(b * b - 8.0 * (double)q, 0.0))) * 0.5);
    i = max(0, min(i, p - 2));
    while (i > 0 && pair_index(p, i, i + 1) > q) --i;
    while (i < p - 2 && pair_index(p, i + 1, i + 2) <= q) ++i;
    j = (int)(q - pair_index(p, i, i + 1)) + i + 1;
}

// In the energy mode a collision or wall factor that sent weight 0 carries
// no cotangent: its edges are neither kept by the u update (that needs rho0)
// nor part of their node's mean (every node has a rho0 energy edge or an
// infinite fixed one, so the all-zero case never arises).  A reverse step
// therefore touches the fixed and energy edges and the captured factors only.

// S_in for the first reverse step of a segment (the step after it, which
// accumulates S for the others, belongs to the segment reversed before):
// per captured factor, its kept edges' dL/du^{k+1} into its nodes
__global__ __launch_bounds__(256) void k_adj_accum(Adj A, float *S, const AdjRec *pool, const unsigned *offs,
                                                   unsigned cap) {
    const unsigned b = offs[0], e = min(offs[1], cap);
    for (unsigned t = b + blockIdx.x * blockDim.x + threadIdx.x; t < e; t += gridDim.x * blockDim.x) {
        const AdjRec rec = pool[t];
        long long nd[4], ed[4];
        int ne;
        if (!rec.wall) {
            const long long fc = rec.f;
            int s = (int)(fc / A.P2), i, j;
            pair_of(A.p, fc - (long long)s * A.P2, i, j);
            nd[0] = node_id(A, i, s), nd[1] = nd[0] + 1, nd[2] = node_id(A, j, s), nd[3] = nd[2] + 1;
            const long long e0 = A.e_coll + 4 * fc;
            for (int k = 0; k < 4; ++k) ed[k] = e0 + k;
            ne = 4;
        } else {
            const long long fw = rec.f, per_s = (long long)A.p * A.W;
            const int s = (int)(fw / per_s), i = (int)((fw - (long long)s * per_s) / A.W);
            nd[0] = node_id(A, i, s), nd[1] = nd[0] + 1;
            ed[0] = A.e_wall + 2 * fw, ed[1] = ed[0] + 1;
            ne = 2;
        }
        for (int k = 0; k < ne; ++k)
            if (A.lnext[nd[k]] == W_STD) {
                atomicAdd(&S[2 * nd[k]], A.ub_in[2 * ed[k]]);
                atomicAdd(&S[2 * nd[k] + 1], A.ub_in[2 * ed[k] + 1]);
            }
    }
}

// Blocks [0, nb_nodes), per node: the class of its mean (infinite edges if
// any, else rho0 edges: the <-rho code the node pass gave it) and g = (dz' -
// s * sum of du' over kept edges) / |mean set|; and the node's entries of
// this step's output sums cleared.  The other blocks clear the output's u
// cotangents of the collision / wall factors captured two steps later (in
// forward order; records [clr[0], clr[1])), the last ones written there, so
// that only this step's writes remain.  Every fixed and energy edge is
// written at every step.
__global__ __launch_bounds__(256) void k_adj_select(Adj A, unsigned nb_nodes, const AdjRec *pool, const unsigned *clr,
                                                    unsigned cap) {
    if (blockIdx.x >= nb_nodes) {
        if (!clr) return;
        const unsigned b = clr[0], e = min(clr[1], cap), nblk = gridDim.x - nb_nodes;
        for (unsigned q = b + (blockIdx.x - nb_nodes) * blockDim.x + threadIdx.x; q < e; q += nblk * blockDim.x) {
            const AdjRec rec = pool[q];
            const long long e0 = rec.wall ? A.e_wall + 2 * (long long)rec.f : A.e_coll + 4 * (long long)rec.f;
            const int ne = rec.wall ? 2 : 4;
            for (int k = 0; k < ne; ++k) A.ub_out[2 * (e0 + k)] = A.ub_out[2 * (e0 + k) + 1] = 0.f;
        }
        return;
    }
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A.N) return;
    A.zb_out[2 * t] = A.zb_out[2 * t + 1] = 0.f;
    A.S_next[2 * t] = A.S_next[2 * t + 1] = 0.f;
    const int i = (int)(t / (A.eta + 1)), s = (int)(t % (A.eta + 1));
    const bool keep_node = A.lnext[t] == W_STD;
    float sx = A.S_in[2 * t], sy = A.S_in[2 * t + 1];
    auto edge = [&](long long f, long long e) {
        if (A.rout[f] == W_STD && keep_node) {
            sx += A.ub_in[2 * e];
            sy += A.ub_in[2 * e + 1];
        }
    };
    if (s == 0) edge(2LL * i, 2LL * i);
    if (s == A.eta) edge(2LL * i + 1, 2LL * i + 1);
    if (s > 0) {
        const long long fe = (long long)i * A.eta + s - 1;
        edge(A.f_energy + fe, A.e_energy + 2 * fe + 1);
    }
    if (s < A.eta) {
        const long long fe = (long long)i * A.eta + s;
        edge(A.f_energy + fe, A.e_energy + 2 * fe);
    }
    const float cnt = (float)A.cnt[t];
    A.cls[t] = A.lnext[t];
    A.g[2 * t] = (A.zb_in[2 * t] - A.step * sx) / cnt;
    A.g[2 * t + 1] = (A.zb_in[2 * t + 1] - A.step * sy) / cnt;
}

// dL/dx of edge e (node t) of a factor with weight r; also the part of
// dL/du^k that does not go through n.
__device__ __forceinline__ void edge_xbar(const Adj &A, int r, long long t, long long e, f2 &xb, f2 &up) {
    bool keep = r == W_STD && A.lnext[t] == W_STD;
    int c = A.cls[t];
    bool in_mean = c == W_INF ? r == W_INF : r == W_STD;
    f2 ubp = keep ? mk(A.ub_in[2 * e], A.ub_in[2 * e + 1]) : mk(0.f, 0.f);
    f2 gg = in_mean ? mk(A.g[2 * t], A.g[2 * t + 1]) : mk(0.f, 0.f);
    xb = add(scl(ubp, A.step), gg);
    up = add(ubp, gg);
}

// dL/du^k of edge e and dL/dn into its node's dL/dz^k.  kept_prev: the edge
// is kept by iteration k-1's u update (its factor sent rho0 there too and
// the node keeps rho0), so its dL/du^k enters that step's sum S.
__device__ __forceinline__ void edge_out(const Adj &A, long long t, long long e, f2 up, f2 nb, bool kept_prev = false) {
    const f2 uo = mk(up.x - nb.x, up.y - nb.y);
    A.ub_out[2 * e] = uo.x;
    A.ub_out[2 * e + 1] = uo.y;
    atomicAdd(&A.zb_out[2 * t], nb.x);
    atomicAdd(&A.zb_out[2 * t + 1], nb.y);
    if (kept_prev) {
        atomicAdd(&A.S_next[2 * t], uo.x);
        atomicAdd(&A.S_next[2 * t + 1], uo.y);
    }
}

// A fixed or energy factor (canonical factor index f < f_coll).
__device__ __forceinline__ void adj_small(const Adj &A, long long f) {
    const int r = A.rout[f];
    if (f < A.f_energy) {
        // fixed start / goal factor: x is the constant itself
        const int i = (int)(f >> 1);
        const int s = (f & 1) ? A.eta : 0;
        const long long t = node_id(A, i, s), e = f;
        f2 xb, up;
        edge_xbar(A, r, t, e, xb, up);
        float *dst = (f & 1) ? A.dxT : A.dx0;
        dst[2 * i] += xb.x;
        dst[2 * i + 1] += xb.y;
        edge_out(A, t, e, up, mk(0.f, 0.f));
    } else {
        // energy factor (App. E): linear in n
        const long long fe = f - A.f_energy;
        const int i = (int)(fe / A.eta), s = (int)(fe % A.eta);
        const long long t0 = node_id(A, i, s), t1 = t0 + 1;
        const long long e0 = A.e_energy + 2 * fe, e1 = e0 + 1;
        f2 xb0, up0, xb1, up1;
        edge_xbar(A, r, t0, e0, xb0, up0);
        edge_xbar(A, r, t1, e1, xb1, up1);
        const int k0 = A.l[t0], k1 = A.l[t1];
        const float w0 = wval(k0, A.rho), w1 = wval(k1, A.rho);
        const float C = A.C[fe];
        float nb[4] = {0.f, 0.f, 0.f, 0.f};
        energy_vjp(w0, w1, k0, k1, C, xb0.x, xb1.x, nb[0], nb[2]);
        energy_vjp(w0, w1, k0, k1, C, xb0.y, xb1.y, nb[1], nb[3]);
        edge_out(A, t0, e0, up0, mk(nb[0], nb[1]));
        edge_out(A, t1, e1, up1, mk(nb[2], nb[3]));
    }
}

// A collision or wall factor that sent rho0 (one captured record).
__device__ __forceinline__ void adj_active(const Adj &A, const AdjRec &rec) {
    if (!rec.wall) {
        // collision factor (App. C)
        const long long fc = rec.f;
        int s = (int)(fc / A.P2), i, j;
        pair_of(A.p, fc - (long long)s * A.P2, i, j);
        long long t[4] = {node_id(A, i, s), node_id(A, i, s + 1), node_id(A, j, s), node_id(A, j, s + 1)};
        long long e0 = A.e_coll + 4 * fc;
        float xb[8], w[4], nbv[8];
        int k[4];
        f2 up[4];
        for (int qq = 0; qq < 4; ++qq) {
            f2 x_b;
            edge_xbar(A, W_STD, t[qq], e0 + qq, x_b, up[qq]);
            xb[2 * qq] = x_b.x, xb[2 * qq + 1] = x_b.y;
            k[qq] = A.l[t[qq]];
            w[qq] = wval(k[qq], A.rho);
        }
        for (int qq = 0; qq < 8; ++qq) nbv[qq] = 0.f;
        float Rb = 0.f;
        coll_vjp2(rec.n, w, k, A.radii[i] + A.radii[j], xb, nbv, Rb);
        atomicAdd(&A.drd[i], (double)Rb);
        atomicAdd(&A.drd[j], (double)Rb);
        const bool prev = A.rout_prev && A.rout_prev[A.f_coll + fc] == W_STD;
        for (int qq = 0; qq < 4; ++qq)
            edge_out(A, t[qq], e0 + qq, up[qq], mk(nbv[2 * qq], nbv[2 * qq + 1]), prev && A.l[t[qq]] == W_STD);
    } else {
        // wall factor (App. D)
        const long long fw = rec.f;
        long long per_s = (long long)A.p * A.W;
        int s = (int)(fw / per_s);
        long long q = fw - (long long)s * per_s;
        int i = (int)(q / A.W), wi = (int)(q % A.W);
        long long t0 = node_id(A, i, s), t1 = t0 + 1;
        long long e0 = A.e_wall + 2 * fw, e1 = e0 + 1;
        f2 xb0, up0, xb1, up1;
        edge_xbar(A, W_STD, t0, e0, xb0, up0);
        edge_xbar(A, W_STD, t1, e1, xb1, up1);
        float4 wl = A.walls[wi];
        Capsule Cw{mk(wl.x, wl.y), mk(wl.z, wl.w), A.radii[i]};
        f2 n0 = mk(rec.n[0], rec.n[1]), n1 = mk(rec.n[2], rec.n[3]);
        int k0 = A.l[t0], k1 = A.l[t1];
        float w0 = wval(k0, A.rho), w1 = wval(k1, A.rho);
        f2 x0, x1;
        Choice ch;
        capsule_prox(Cw, n0, n1, w0, w1, k0, k1, x0, x1, &ch);
        f2 nb0 = mk(0.f, 0.f), nb1 = mk(0.f, 0.f);
        float rb = 0.f;
        capsule_vjp(Cw, n0, n1, w0, w1, k0, k1, ch, xb0, xb1, nb0, nb1, rb);
        atomicAdd(&A.drd[i], (double)rb);
        const bool prev = A.rout_prev && A.rout_prev[A.f_wall + fw] == W_STD;
        edge_out(A, t0, e0, up0, nb0, prev && A.l[t0] == W_STD);
        edge_out(A, t1, e1, up1, nb1, prev && A.l[t1] == W_STD);
    }
}

// The factors of one reverse step: blocks [0, nb_small) take the fixed and
// energy factors one lane each; the rest stride over the captured records
// [offs[0], offs[1]) (clipped to the pool's capacity), one lane each, so the
// non-linear derivatives run in full waves.
__global__ __launch_bounds__(256) void k_adj_factors(Adj A, unsigned nb_small, const AdjRec *pool, const unsigned *offs,
                                                     unsigned cap) {
    if (blockIdx.x < nb_small) {
        const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
        if (f < A.f_coll) adj_small(A, f);
        return;
    }
    const unsigned b = offs[0], e = min(offs[1], cap);
    const unsigned nblk = gridDim.x - nb_small;
    for (unsigned t = b + (blockIdx.x - nb_small) * blockDim.x + threadIdx.x; t < e; t += nblk * blockDim.x)
        adj_active(A, pool[t]);
}

// z^0 cotangent: its end points are the start and goal
__global__ void k_adj_finish(Adj A, float *dz0, float *dr) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < A.N) {
        int i = (int)(t / (A.eta + 1)), s = (int)(t % (A.eta + 1));
        bool end = s == 0 || s == A.eta;
        if (end) {
            float *dst = s == 0 ? A.dx0 : A.dxT;
            dst[2 * i] += A.zb_in[2 * t];
            dst[2 * i + 1] += A.zb_in[2 * t + 1];
        }
        if (dz0) {
            dz0[2 * t] = end ? 0.f : A.zb_in[2 * t];
            dz0[2 * t + 1] = end ? 0.f : A.zb_in[2 * t + 1];
        }
    }
    if (t < A.p) dr[t] = (float)A.drd[t];
}

// A state with its collision / wall u sparse (a checkpoint): z, <-rho and
// the u of the fixed and energy edges dense, then one record per collision
// or wall factor with a nonzero u (its index among all factors and its
// edges' u) in the record arena, from arena index *first to *end.
struct Sparse {
    float *z;          // [N][2]
    unsigned char *l;  // [N]
    float *u_small;    // [e_coll][2]: the fixed and energy edges
    unsigned *first, *end; // device
    AdjRec *arena;     // the record store [first, end) index (cap records)
    unsigned cap;
};

// canonical dense u -> arena records of the collision / wall factors with a
// nonzero u (appended at *cursor; those past cap are dropped, the cursor
// still counts them)
__global__ __launch_bounds__(256) void k_pack(const float *u, long long f_coll, long long nfac, long long e_coll,
                                              long long Fc, AdjRec *arena, unsigned cap, unsigned *cursor) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool nz = false;
    float v[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (q < nfac) {
        const bool wall = q >= Fc;
        const long long e0 = wall ? e_coll + 4 * Fc + 2 * (q - Fc) : e_coll + 4 * q;
        const int nv = wall ? 4 : 8;
        for (int c = 0; c < nv; ++c) {
            v[c] = u[2 * e0 + c];
            nz = nz || v[c] != 0.f;
        }
    }
    const unsigned long long mask = __ballot(nz);
    if (mask == 0ull) return;
    const int lane = __lane_id(), leader = __ffsll((long long)mask) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(cursor, (unsigned)__popcll(mask));
    base = __shfl(base, leader);
    const unsigned idx = base + (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
    if (nz && idx < cap) {
        AdjRec r;
        r.f = (unsigned)(f_coll + q);
        r.wall = q >= Fc;
        for (int c = 0; c < 8; ++c) r.n[c] = v[c];
        arena[idx] = r;
    }
}

// arena records [*first, *end) -> canonical dense u (zeroed before)
__global__ __launch_bounds__(256) void k_unpack(float *u, long long f_coll, long long e_coll, long long Fc,
                                                const AdjRec *arena, const unsigned *first, const unsigned *end,
                                                unsigned cap) {
    const unsigned b = *first, e = min(*end, cap);
    for (unsigned t = b + blockIdx.x * blockDim.x + threadIdx.x; t < e; t += gridDim.x * blockDim.x) {
        const AdjRec r = arena[t];
        const long long q = (long long)r.f - f_coll;
        const long long e0 = r.wall ? e_coll + 4 * Fc + 2 * (q - Fc) : e_coll + 4 * q;
        const int nv = r.wall ? 4 : 8;
        for (int c = 0; c < nv; ++c) u[2 * e0 + c] = r.n[c];
    }
}

__global__ void k_copy_u32(unsigned *dst, const unsigned *src) { *dst = *src; }

__global__ void k_fill_float(float *p, long long n) {
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (long long)gridDim.x * blockDim.x)
        p[t] = 0.f;
}

// ------------------------------------------------------------------ scratch
// The library's static scratch for twa_backward_noalloc (callers that cannot
// allocate): each device holds one copy, from the first load of the
// library's code on it until the process ends.  Host code reaches it only
// through the address looked up per device at solver creation (the array's
// own name is a host-side stand-in).  Calls on one device share it.
constexpr size_t kScratchBytes = 128ull << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// ------------------------------------------------------------------ workspace
// Bump allocation of one call's buffers from a region: the solver's own
// (allocated at its first call and kept), or the library's static scratch.
// With base == nullptr it only adds up the sizes.
struct Region {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    template <class T>
    T *take(size_t count) {
        const size_t off = (used + 255) & ~(size_t)255;
        const size_t bytes = std::max<size_t>(count * sizeof(T), 16);
        if (base && off + bytes > cap) return nullptr;
        used = off + bytes;
        return base ? reinterpret_cast<T *>(base + off) : reinterpret_cast<T *>(256);
    }
};

struct Shape {
    long long N, E, F, K, L, ncp, len_max, e_small, nfac;
    int p;
};

// tape_every > 0: the forward tape holds the checkpoints every tape_every
// iterations, and segments are a multiple of that near sqrt(K)
Shape shape_of(const twa_solver *s, int tape_every = 0) {
    const twa_rt::Params &P = s->P;
    Shape h;
    h.N = P.N, h.E = P.e_wall + 2 * P.Fw, h.F = P.Ff + P.Fe + P.Fc + P.Fw, h.p = s->p;
    h.e_small = P.e_coll, h.nfac = P.Fc + P.Fw;
    h.K = s->iter - s->origin_iter;
    const double root = std::sqrt((double)std::max<long long>(h.K, 0));
    if (tape_every > 0)
        h.L = tape_every * std::max<long long>(1, std::llround(root / tape_every));
    else
        h.L = std::max<long long>(1, (long long)std::ceil(root));
    h.ncp = h.K > 0 ? (h.K + h.L - 1) / h.L : 0;
    h.len_max = std::min(h.L, std::max<long long>(h.K, 1));
    return h;
}

// Everything a call needs besides the record arena and the capture pool.
// Checkpoint c's arrays are slices c of the ck_* arrays (no host-side table).
struct Buffers {
    Sparse cur;                   // the forward state at the call, restored at the end
    float *ck_z, *ck_us;          // [ncp][N][2], [ncp][e_small][2]
    unsigned char *ck_l;          // [ncp][N]
    unsigned *ck_first, *ck_end;  // [ncp]
    float *u_tmp;                 // [E][2] dense u of a state being packed or unpacked
    // two cotangent sets, alternately a reverse step's input and its output
    // (the output is cleared where the step before last wrote it, or whole
    // at a segment's first two steps): dL/du [E][2], dL/dz [N][2], and the
    // per-node sum S [N][2] that the step after it reads
    char *set[2];
    size_t set_bytes;
    float *g;                     // [N][2]
    unsigned char *cls;           // [N]
    double *drd;                  // [p]
    unsigned *arena_cursor;
    // What a segment's recompute captures, twice: segment c uses copy c & 1,
    // so that one segment is recomputed while the one after it is reversed.
    unsigned *pool_cursor[2];
    unsigned *offs[2];            // [len_max + 1] pool cursor before each iteration of a segment
    unsigned char *rout[2];       // [len_max][F] ->rho of each iteration of a segment
    unsigned char *lseg[2];       // [len_max + 1][N] <-rho before each iteration, and after the last
    int *cntseg[2];               // [len_max][N] size of each node's mean set in each iteration
    AdjRec *arena, *pool[2];
    unsigned arena_cap, pool_cap; // pool_cap: records of each of the two pools
    // pools_follow: the arena and the pools share one store of arena_cap
    // records; the pools take what the checkpoints leave (set after pass 1)
    bool pools_follow;
};

// Carve one cotangent set (see Buffers) from base; returns its size.
size_t set_layout(const Shape &h, char *base, float **ub = nullptr, float **zb = nullptr, float **S = nullptr) {
    Region R;
    R.base = base;
    R.cap = ~(size_t)0;
    float *a = R.take<float>((size_t)h.E * 2);
    float *b = R.take<float>((size_t)h.N * 2);
    float *c = R.take<float>((size_t)h.N * 2);
    if (ub) *ub = a, *zb = b, *S = c;
    return R.used;
}

bool layout(Region &R, const Shape &h, Buffers &B) {
    B.cur.z = R.take<float>((size_t)h.N * 2);
    B.cur.l = R.take<unsigned char>((size_t)h.N);
    B.cur.u_small = R.take<float>((size_t)h.e_small * 2);
    B.cur.first = R.take<unsigned>(1);
    B.cur.end = R.take<unsigned>(1);
    const size_t nc = (size_t)std::max<long long>(h.ncp, 1);
    B.ck_z = R.take<float>(nc * h.N * 2);
    B.ck_us = R.take<float>(nc * h.e_small * 2);
    B.ck_l = R.take<unsigned char>(nc * h.N);
    B.ck_first = R.take<unsigned>(nc);
    B.ck_end = R.take<unsigned>(nc);
    B.u_tmp = R.take<float>((size_t)h.E * 2);
    B.set_bytes = set_layout(h, nullptr);
    B.set[0] = R.take<char>(B.set_bytes);
    B.set[1] = R.take<char>(B.set_bytes);
    B.g = R.take<float>((size_t)h.N * 2);
    B.cls = R.take<unsigned char>((size_t)h.N);
    B.drd = R.take<double>((size_t)h.p);
    B.arena_cursor = R.take<unsigned>(1);
    bool ok = true;
    for (int b = 0; b < 2; ++b) {
        B.pool_cursor[b] = R.take<unsigned>(1);
        B.offs[b] = R.take<unsigned>((size_t)h.len_max + 1);
        B.rout[b] = R.take<unsigned char>((size_t)h.len_max * h.F);
        B.lseg[b] = R.take<unsigned char>((size_t)(h.len_max + 1) * h.N);
        B.cntseg[b] = R.take<int>((size_t)h.len_max * h.N);
        ok = ok && B.pool_cursor[b] && B.offs[b] && B.rout[b] && B.lseg[b] && B.cntseg[b];
    }
    return ok && B.cur.z && B.cur.l && B.cur.u_small && B.cur.first && B.cur.end && B.ck_z && B.ck_us && B.ck_l &&
           B.ck_first && B.ck_end && B.u_tmp && B.set[0] && B.set[1] && B.g && B.cls && B.drd && B.arena_cursor;
}

Sparse ckpt(const Buffers &B, const Shape &h, long long c) {
    Sparse q;
    q.z = B.ck_z + c * h.N * 2;
    q.l = B.ck_l + c * h.N;
    q.u_small = B.ck_us + c * h.e_small * 2;
    q.first = B.ck_first + c;
    q.end = B.ck_end + c;
    q.arena = B.arena;
    q.cap = B.arena_cap;
    return q;
}

// checkpoint c of the solver's forward tape
Sparse tape_slot(const twa_solver *s, long long c) {
    const twa_solver::Tape &T = s->tape;
    const long long N = s->P.N, es = s->P.e_coll;
    Sparse q;
    q.z = T.z + c * N * 2;
    q.l = T.l + c * N;
    q.u_small = T.us + c * es * 2;
    q.first = T.first + c;
    q.end = T.end + c;
    q.arena = T.arena;
    q.cap = T.arena_cap;
    return q;
}

unsigned grid_for(unsigned long long n) { return (unsigned)std::max<unsigned long long>(1, std::min<unsigned long long>((n + 255) / 256, 1024)); }

// the solver's current state into q: z and <-rho, the fixed and energy u
// dense, the collision / wall u as records appended to q's store at *cursor
// (u_tmp: [E][2] scratch)
twa_status pack_state(twa_solver *s, float *u_tmp, unsigned *cursor, const Sparse &q) {
    const long long e_small = s->P.e_coll, nfac = s->P.Fc + s->P.Fw;
    long long it = 0;
    TRY(twa_get_state(s, q.z, u_tmp, q.l, &it)); // settles the pending u update
    HIP_TRY(s, hipMemcpyAsync(q.u_small, u_tmp, sizeof(float) * 2 * e_small, hipMemcpyDeviceToDevice, s->stream));
    hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, s->stream, q.first, (const unsigned *)cursor);
    if (nfac > 0)
        hipLaunchKernelGGL(k_pack, dim3((unsigned)((nfac + 255) / 256)), dim3(256), 0, s->stream,
                           (const float *)u_tmp, s->P.f_coll, nfac, e_small, s->P.Fc, q.arena, q.cap, cursor);
    hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(1), 0, s->stream, q.end, (const unsigned *)cursor);
    HIP_TRY(s, hipGetLastError());
    return TWA_OK;
}

twa_status pack(twa_solver *s, const Shape &, Buffers &B, const Sparse &q) {
    return pack_state(s, B.u_tmp, B.arena_cursor, q);
}

// state q into the solver, at iteration k
twa_status unpack(twa_solver *s, const Shape &h, Buffers &B, const Sparse &q, long long k) {
    hipLaunchKernelGGL(k_fill_float, dim3(grid_for((unsigned long long)h.E * 2)), dim3(256), 0, s->stream, B.u_tmp,
                       h.E * 2);
    HIP_TRY(s, hipMemcpyAsync(B.u_tmp, q.u_small, sizeof(float) * 2 * h.e_small, hipMemcpyDeviceToDevice, s->stream));
    hipLaunchKernelGGL(k_unpack, dim3(grid_for(q.cap)), dim3(256), 0, s->stream, B.u_tmp, s->P.f_coll,
                       h.e_small, s->P.Fc, (const AdjRec *)q.arena, (const unsigned *)q.first,
                       (const unsigned *)q.end, q.cap);
    HIP_TRY(s, hipGetLastError());
    return twa_rt::import_state(s, q.z, B.u_tmp, q.l, k);
}

// what made an attempt stop short
enum { kDone = 0, kArenaFull = 1, kPoolFull = 2 };

// One attempt of the whole computation with the buffers of B.  *outcome is
// kDone, or which record store ran out (*need: the records it wanted); the
// solver's forward state is restored either way.
// grow_pool (may be null): make the capture pool hold `need` records, for
// the segment to be recomputed once more; without it an overflow ends the
// attempt.
using GrowPool = twa_status (*)(twa_solver *s, Buffers &B, unsigned need);

twa_status run_once(twa_solver *s, const Shape &h, Buffers &B, const float *dL_dz, float *dL_dx0, float *dL_dxT,
                    float *dL_dr, float *dL_dz0, int *outcome, unsigned *need, GrowPool grow_pool, bool use_tape,
                    unsigned *arena_used) {
    const twa_rt::Params &P = s->P;
    hipStream_t st = s->stream;
    *outcome = kDone;
    *need = 0;
    if (!s->adj_stream || !s->adj_used)
        return twa_rt::fail(s, TWA_E_STATE, "twa_backward: the solver has no reverse stream");
    // whatever way this returns, the reverse stream's work on B is over
    struct Join {
        hipStream_t rs;
        ~Join() { (void)hipStreamSynchronize(rs); }
    } join{s->adj_stream};
    HIP_TRY(s, hipMemsetAsync(B.arena_cursor, 0, sizeof(unsigned), st));
    const long long cur_iter = s->iter, it0 = s->origin_iter;
    B.cur.arena = B.arena;
    B.cur.cap = B.arena_cap;
    // checkpoint c: from the forward tape (every h.L / interval-th of its
    // checkpoints), or packed by pass 1
    const long long tape_step = use_tape ? h.L / s->tape.interval : 0;
    auto checkpoint = [&](long long c) { return use_tape ? tape_slot(s, c * tape_step) : ckpt(B, h, c); };
    TRY(pack(s, h, B, B.cur));
    unsigned used = 0;
    HIP_TRY(s, hipMemcpyAsync(&used, B.arena_cursor, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIP_TRY(s, hipStreamSynchronize(st));
    if (used > B.arena_cap) {
        // the forward state itself did not fit: nothing else was touched
        *outcome = kArenaFull;
        *need = used;
        return TWA_OK;
    }
    // pass 1: checkpoints every L iterations from the run's start (the tape
    // holds them already when it covers the run)
    if (!use_tape) {
        if (h.K > 0) TRY(twa_rt::import_state(s, s->origin_z, s->origin_u, s->origin_l, it0));
        for (long long c = 0; c < h.ncp; ++c) {
            TRY(pack(s, h, B, ckpt(B, h, c)));
            if (c + 1 < h.ncp) TRY(twa_iterate(s, (int)h.L));
        }
    }
    HIP_TRY(s, hipMemcpyAsync(&used, B.arena_cursor, sizeof(unsigned), hipMemcpyDeviceToHost, st));
    HIP_TRY(s, hipStreamSynchronize(st));
    if (used > B.arena_cap) {
        *outcome = kArenaFull;
        *need = used;
        return unpack(s, h, B, B.cur, cur_iter);
    }
    if (arena_used) *arena_used = used;
    if (B.pools_follow) {
        // nothing is appended to the arena after pass 1
        const unsigned start = (used + 63u) & ~63u;
        B.pool_cap = start < B.arena_cap ? (B.arena_cap - start) / 2 : 0u;
        B.pool[0] = B.arena + start;
        B.pool[1] = B.pool[0] + B.pool_cap;
        B.arena_cap = used;
    }

    Adj A{};
    A.p = s->p, A.eta = s->eta, A.W = s->W;
    A.P2 = (long long)s->p * (s->p - 1) / 2, A.N = h.N, A.E = h.E, A.F = h.F;
    A.e_energy = P.e_energy, A.e_coll = P.e_coll, A.e_wall = P.e_wall;
    A.f_energy = P.f_energy, A.f_coll = P.f_coll, A.f_wall = P.f_wall;
    A.radii = P.radii, A.walls = P.walls, A.C = P.C;
    A.g = B.g, A.cls = B.cls, A.dx0 = dL_dx0, A.dxT = dL_dxT, A.drd = B.drd;
    int in = 0; // the set holding dL/d(state after the step being reversed)
    {
        float *ub, *zb, *S;
        set_layout(h, B.set[in], &ub, &zb, &S);
        HIP_TRY(s, hipMemsetAsync(B.set[in], 0, B.set_bytes, st));
        HIP_TRY(s, hipMemcpyAsync(zb, dL_dz, sizeof(float) * h.N * 2, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(s, hipMemsetAsync(dL_dx0, 0, sizeof(float) * s->p * 2, st));
    HIP_TRY(s, hipMemsetAsync(dL_dxT, 0, sizeof(float) * s->p * 2, st));
    HIP_TRY(s, hipMemsetAsync(B.drd, 0, sizeof(double) * s->p, st));
    const unsigned nb_nodes = (unsigned)((h.N + 255) / 256), nb_small = (unsigned)((P.f_coll + 255) / 256);
    const unsigned nb_rec = 256; // blocks striding over the captured records
    const unsigned nb_clr = 64;  // blocks clearing a step's output sparsely

    // pass 2: segments in reverse, software-pipelined over two streams: a
    // segment is recomputed on the solver's stream, capturing its decisions
    // into capture copy c & 1, while the segment after it runs backwards on
    // the reverse stream.  Events: adj_ev[b] recomputed into copy b,
    // adj_ev[2 + b] copy b reversed (free for the next recompute).
    hipStream_t rs = s->adj_stream;
    HIP_TRY(s, hipEventRecord(s->adj_ev[2], st));
    HIP_TRY(s, hipStreamWaitEvent(rs, s->adj_ev[2], 0)); // the cotangent sets are set up
    auto recompute = [&](long long c) -> twa_status {
        const long long k0 = it0 + c * h.L, len = std::min(h.L, h.K - c * h.L);
        const int b = (int)(c & 1);
        // the reverse of segment c + 2 read this copy
        if (c + 2 < h.ncp) HIP_TRY(s, hipStreamWaitEvent(st, s->adj_ev[2 + b], 0));
        TRY(unpack(s, h, B, checkpoint(c), k0));
        HIP_TRY(s, hipMemsetAsync(B.pool_cursor[b], 0, sizeof(unsigned), st));
        HIP_TRY(s, hipMemsetAsync(B.offs[b], 0, sizeof(unsigned), st));
        TRY(twa_rt::export_lrho(s, B.lseg[b]));
        // each iteration's weights, its captured factors, and (from its node
        // pass) the new <-rho codes, the mean-set sizes and the capture
        // cursor; a full-length segment replays the graph kept for copy b
        twa_rt::SegCapture cap;
        cap.rout = B.rout[b];
        cap.pool = B.pool[b];
        cap.cursor = B.pool_cursor[b];
        cap.cap = B.pool_cap;
        cap.offs = B.offs[b];
        cap.lseg = B.lseg[b];
        cap.cntseg = B.cntseg[b];
        cap.F = h.F;
        cap.N = h.N;
        TRY(twa_rt::run_segment(s, len, cap, len == h.L ? b : -1));
        HIP_TRY(s, hipMemcpyAsync(s->adj_used + b, B.pool_cursor[b], sizeof(unsigned), hipMemcpyDeviceToHost, st));
        HIP_TRY(s, hipEventRecord(s->adj_ev[b], st));
        return TWA_OK;
    };
    if (h.ncp > 0) TRY(recompute(h.ncp - 1));
    for (long long c = h.ncp - 1; c >= 0; --c) {
        const long long k0 = it0 + c * h.L, len = std::min(h.L, h.K - c * h.L);
        const int b = (int)(c & 1);
        // segment c is recomputed (and nothing after it is queued on st)
        HIP_TRY(s, hipEventSynchronize(s->adj_ev[b]));
        while (s->adj_used[b] > B.pool_cap) {
            if (!grow_pool) {
                *outcome = kPoolFull;
                *need = s->adj_used[b];
                return unpack(s, h, B, B.cur, cur_iter);
            }
            // (the segment being reversed reads the other pool)
            HIP_TRY(s, hipStreamSynchronize(rs));
            TRY(grow_pool(s, B, s->adj_used[b]));
            TRY(recompute(c));
            HIP_TRY(s, hipEventSynchronize(s->adj_ev[b]));
        }
        // the segment before it goes on the solver's stream first, so that
        // the two run together
        if (c > 0) TRY(recompute(c - 1));
        HIP_TRY(s, hipStreamWaitEvent(rs, s->adj_ev[b], 0));
        for (long long t = len - 1; t >= 0; --t) {
            float *ub_in, *zb_in, *S_in, *ub_out, *zb_out, *S_out;
            set_layout(h, B.set[in], &ub_in, &zb_in, &S_in);
            set_layout(h, B.set[1 - in], &ub_out, &zb_out, &S_out);
            A.ub_in = ub_in, A.zb_in = zb_in, A.S_in = S_in;
            A.ub_out = ub_out, A.zb_out = zb_out, A.S_next = S_out;
            A.l = B.lseg[b] + t * h.N;
            A.lnext = B.lseg[b] + (t + 1) * h.N;
            A.cnt = B.cntseg[b] + t * h.N;
            A.rout = B.rout[b] + t * h.F;
            A.rout_prev = t > 0 ? B.rout[b] + (t - 1) * h.F : nullptr;
            A.rho = twa_rt::rho_at(s, k0 + t);
            A.step = s->alpha / s->rho0; // the u step ignores the warm-up's rho0
            const unsigned *offs = B.offs[b] + t;
            // the step after this one belongs to the segment reversed before
            // (or is the loss): it could not accumulate this step's S
            if (t == len - 1)
                hipLaunchKernelGGL(k_adj_accum, dim3(nb_rec), dim3(256), 0, rs, A, S_in, (const AdjRec *)B.pool[b],
                                   offs, B.pool_cap);
            // The output set holds what step t + 2 wrote.  Its records are in
            // this segment's pool if it belongs to the segment; otherwise
            // (it was reversed before, its pool is being refilled) the whole
            // set is cleared.
            const bool sparse = t + 2 < len;
            if (!sparse) HIP_TRY(s, hipMemsetAsync(B.set[1 - in], 0, B.set_bytes, rs));
            hipLaunchKernelGGL(k_adj_select, dim3(nb_nodes + (sparse ? nb_clr : 0u)), dim3(256), 0, rs, A, nb_nodes,
                               (const AdjRec *)B.pool[b], sparse ? B.offs[b] + t + 2 : nullptr, B.pool_cap);
            hipLaunchKernelGGL(k_adj_factors, dim3(nb_small + nb_rec), dim3(256), 0, rs, A, nb_small,
                               (const AdjRec *)B.pool[b], offs, B.pool_cap);
            HIP_TRY(s, hipGetLastError());
            in = 1 - in;
        }
        HIP_TRY(s, hipEventRecord(s->adj_ev[2 + b], rs));
    }
    {
        float *ub, *zb, *S;
        set_layout(h, B.set[in], &ub, &zb, &S);
        A.zb_in = zb;
    }
    const long long nfin = std::max<long long>(h.N, s->p);
    hipLaunchKernelGGL(k_adj_finish, dim3((unsigned)((nfin + 255) / 256)), dim3(256), 0, rs, A, dL_dz0, dL_dr);
    HIP_TRY(s, hipGetLastError());
    TRY(unpack(s, h, B, B.cur, cur_iter));
    HIP_TRY(s, hipStreamSynchronize(rs));
    HIP_TRY(s, hipStreamSynchronize(st));
    return TWA_OK;
}

// Does the forward tape hold every checkpoint of the current run (one at
// each multiple of its interval below K, none of their records dropped)?
// Synchronises the stream when it has to read the record count.
bool tape_covers(twa_solver *s) {
    const twa_solver::Tape &T = s->tape;
    const long long K = s->iter - s->origin_iter;
    if (!T.mem || !T.ok || K <= 0) return false;
    if (T.count < (K + T.interval - 1) / T.interval) return false;
    unsigned used = ~0u;
    if (hipMemcpyAsync(&used, T.cursor, sizeof(unsigned), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return used <= T.arena_cap;
}

// Allocate the forward tape after an allocating twa_backward, for runs like
// the one just differentiated: 64 checkpoints of every 32 iterations (runs
// up to 2,048 iterations), each with room for twice the records a
// checkpoint of this run held.  It records from the next start of a run.
twa_status tape_alloc(twa_solver *s, unsigned records_per_checkpoint) {
    twa_solver::Tape &T = s->tape;
    if (T.mem) return TWA_OK;
    const long long N = s->P.N, es = s->P.e_coll, E = s->P.e_wall + 2 * s->P.Fw;
    const int cap = 64;
    const size_t per = 2 * (size_t)records_per_checkpoint + 1024;
    const size_t recs = std::min<size_t>((size_t)cap * per, 0x7fffffffu);
    for (int pass = 0; pass < 2; ++pass) {
        Region R;
        if (pass == 1) {
            R.base = static_cast<char *>(T.mem);
            R.cap = T.bytes;
        }
        float *z = R.take<float>((size_t)cap * N * 2);
        unsigned char *l = R.take<unsigned char>((size_t)cap * N);
        float *us = R.take<float>((size_t)cap * es * 2);
        unsigned *first = R.take<unsigned>(cap), *end = R.take<unsigned>(cap), *cursor = R.take<unsigned>(1);
        float *u_tmp = R.take<float>((size_t)E * 2);
        AdjRec *arena = R.take<AdjRec>(recs);
        if (pass == 0) {
            T.bytes = R.used;
            T.mem = s->mem.get(T.bytes, s->stream);
            if (!T.mem) {
                T.bytes = 0;
                return TWA_OK; // no tape: later calls re-run the forward as this one did
            }
        } else {
            T.z = z, T.l = l, T.us = us, T.first = first, T.end = end, T.cursor = cursor, T.u_tmp = u_tmp;
            T.arena = arena;
            T.arena_cap = (unsigned)recs;
        }
    }
    T.cap = cap;
    T.count = 0;
    T.ok = false; // the run just differentiated was not recorded
    return TWA_OK;
}

twa_status check_args(twa_solver *s, const float *dL_dz, float *dL_dx0, float *dL_dxT, float *dL_dr) {
    using twa_rt::fail;
    TRY(twa_rt::check_alive(s));
    if (!(s->flags & TWA_F_TAPE)) return fail(s, TWA_E_STATE, "twa_backward needs TWA_F_TAPE at create");
    if (s->dim != 2) return fail(s, TWA_E_INVALID, "twa_backward supports dim == 2 only");
    if (s->P.admm) return fail(s, TWA_E_INVALID, "twa_backward supports the three-weight mode only");
    if (s->P.cost != 0) return fail(s, TWA_E_INVALID, "twa_backward supports the energy cost only");
    if (!dL_dz || !dL_dx0 || !dL_dxT || !dL_dr) return fail(s, TWA_E_INVALID, "null array argument");
    if (s->iter < s->origin_iter) return fail(s, TWA_E_STATE, "iteration count below the run's start");
    return TWA_OK;
}

twa_status ensure(twa_solver *s, void **buf, size_t *have, size_t want);

// the two capture pools, halves of one buffer
void set_pools(Buffers &B, void *mem, size_t bytes) {
    B.pool_cap = (unsigned)std::min<size_t>(bytes / 2 / sizeof(AdjRec), 0xffffffffu);
    B.pool[0] = static_cast<AdjRec *>(mem);
    B.pool[1] = B.pool[0] + B.pool_cap;
}

// the allocating path's pool growth (a quarter to spare)
twa_status grow_solver_pool(twa_solver *s, Buffers &B, unsigned need) {
    const size_t want = std::min<size_t>((size_t)need * 5 / 4 + 1024, 0xffffffffu) * sizeof(AdjRec);
    TRY(ensure(s, &s->adj_pool_mem, &s->adj_pool_bytes, 2 * want));
    set_pools(B, s->adj_pool_mem, s->adj_pool_bytes);
    return TWA_OK;
}

// grow-only device buffer owned by the solver
twa_status ensure(twa_solver *s, void **buf, size_t *have, size_t want) {
    if (*have >= want) return TWA_OK;
    if (*buf) {
        // the stream may still read the old buffer
        HIP_TRY(s, hipStreamSynchronize(s->stream));
        s->mem.put(*buf, *have, s->stream);
    }
    *buf = nullptr;
    *have = 0;
    *buf = s->mem.get(want, s->stream);
    if (!*buf)
        return twa_rt::fail(s, TWA_E_NOMEM, "twa_backward: allocation of " + std::to_string(want) + " bytes failed");
    *have = want;
    return TWA_OK;
}

} // namespace

namespace twa_rt {

twa_status tape_take(twa_solver *s) {
    twa_solver::Tape &T = s->tape;
    if (!T.ok || s->dbg_rho || s->adj_pool) return TWA_OK;
    const long long since = s->iter - s->origin_iter;
    if (since > (long long)T.count * T.interval) {
        T.ok = false; // iterations ran past a checkpoint (not through twa_iterate)
        return TWA_OK;
    }
    if (since % T.interval != 0 || since / T.interval != T.count) return TWA_OK;
    if (T.count >= T.cap) {
        T.ok = false; // the run outgrew the tape
        return TWA_OK;
    }
    TRY(pack_state(s, T.u_tmp, T.cursor, tape_slot(s, T.count)));
    ++T.count;
    return TWA_OK;
}

// the static scratch's address on the solver's device, the reverse stream
// and its events (set up at create)
twa_status tape_setup(twa_solver *s) {
    if (s->device < 0 || s->device >= kMaxDevices) return fail(s, TWA_E_DEVICE, "device index out of range");
    if (hipStreamCreate(&s->adj_stream) != hipSuccess) {
        (void)hipGetLastError();
        s->adj_stream = nullptr;
        return fail(s, TWA_E_DEVICE, "hipStreamCreate failed");
    }
    for (hipEvent_t &ev : s->adj_ev)
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            ev = nullptr;
            return fail(s, TWA_E_DEVICE, "hipEventCreate failed");
        }
    if (hipHostMalloc(reinterpret_cast<void **>(&s->adj_used), 2 * sizeof(unsigned), hipHostMallocDefault) !=
        hipSuccess) {
        (void)hipGetLastError();
        s->adj_used = nullptr;
        return fail(s, TWA_E_DEVICE, "hipHostMalloc failed");
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[s->device]) return TWA_OK;
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(s, TWA_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_ptr[s->device] = p;
    return TWA_OK;
}

} // namespace twa_rt

extern "C" twa_status twa_backward(twa_solver *s, const float *dL_dz, float *dL_dx0, float *dL_dxT, float *dL_dr,
                                   float *dL_dz0) {
    TRY(check_args(s, dL_dz, dL_dx0, dL_dxT, dL_dr));
    const bool use_tape = tape_covers(s);
    const Shape h = shape_of(s, use_tape ? s->tape.interval : 0);
    Region sz;
    Buffers B{};
    layout(sz, h, B);
    TRY(ensure(s, &s->adj_ws, &s->adj_ws_bytes, sz.used));
    Region R;
    R.base = static_cast<char *>(s->adj_ws);
    R.cap = s->adj_ws_bytes;
    layout(R, h, B);
    // record stores: sized from the last iteration's queue, grown on demand
    int queued = 0;
    HIP_TRY(s, hipMemcpyAsync(&queued, s->stats_dev + 2, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    const size_t per = 2 * (size_t)std::max(queued, 0) + 1024;
    const size_t packed = use_tape ? 1 : (size_t)h.ncp + 1; // checkpoints the arena takes
    size_t want_arena = std::max<size_t>(s->adj_arena_bytes, packed * per * sizeof(AdjRec));
    size_t want_pool = std::max<size_t>(s->adj_pool_bytes, 2 * (size_t)h.len_max * per * sizeof(AdjRec));
    for (int attempt = 0; attempt < 3; ++attempt) {
        const size_t cap_recs = (size_t)0xffffffffu * sizeof(AdjRec);
        TRY(ensure(s, &s->adj_arena, &s->adj_arena_bytes, std::min(want_arena, cap_recs)));
        TRY(ensure(s, &s->adj_pool_mem, &s->adj_pool_bytes, std::min(want_pool, cap_recs)));
        B.arena = static_cast<AdjRec *>(s->adj_arena);
        B.arena_cap = (unsigned)(s->adj_arena_bytes / sizeof(AdjRec));
        set_pools(B, s->adj_pool_mem, s->adj_pool_bytes);
        int outcome = kDone;
        unsigned need = 0, used = 0;
        TRY(run_once(s, h, B, dL_dz, dL_dx0, dL_dxT, dL_dr, dL_dz0, &outcome, &need, grow_solver_pool, use_tape,
                     &used));
        if (outcome == kDone)
            return use_tape ? TWA_OK : tape_alloc(s, (unsigned)(used / std::max<long long>(1, h.ncp + 1)));
        // the arena's need is exact (every checkpoint was counted): one more attempt
        want_arena = (size_t)need * sizeof(AdjRec) * 5 / 4 + 4096;
    }
    return twa_rt::fail(s, TWA_E_NOMEM, "twa_backward: record stores kept overflowing");
}

extern "C" twa_status twa_backward_noalloc(twa_solver *s, const float *dL_dz, float *dL_dx0, float *dL_dxT,
                                           float *dL_dr, float *dL_dz0) {
    using twa_rt::fail;
    TRY(check_args(s, dL_dz, dL_dx0, dL_dxT, dL_dr));
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (s->device >= 0 && s->device < kMaxDevices) base = g_scratch_ptr[s->device];
    }
    if (!base) return fail(s, TWA_E_STATE, "twa_backward_noalloc: no scratch on the solver's device");
    const bool use_tape = tape_covers(s);
    const Shape h = shape_of(s, use_tape ? s->tape.interval : 0);
    Region R;
    R.base = static_cast<char *>(base);
    R.cap = kScratchBytes;
    Buffers B{};
    if (!layout(R, h, B)) {
        Region sz;
        layout(sz, h, B);
        return fail(s, TWA_E_NOMEM, "twa_backward_noalloc: the run needs more than the " +
                                        std::to_string(kScratchBytes >> 20) + " MiB scratch (" +
                                        std::to_string(sz.used >> 20) + " MiB before its records)");
    }
    // the rest of the scratch holds the records: the checkpoints' first, the
    // two capture pools share what they leave (less an alignment pad)
    const size_t left = R.cap - std::min(R.cap, ((R.used + 255) & ~(size_t)255) + 256);
    B.arena_cap = (unsigned)std::min<size_t>(left / sizeof(AdjRec), 0xffffffffu);
    B.arena = R.take<AdjRec>(B.arena_cap);
    B.pools_follow = true;
    const unsigned total = B.arena_cap;
    if (!B.arena || B.arena_cap < 256)
        return fail(s, TWA_E_NOMEM, "twa_backward_noalloc: no scratch left for the records");
    const bool was = s->no_capture;
    s->no_capture = true; // replay graphs already captured, capture none (that would allocate)
    int outcome = kDone;
    unsigned need = 0;
    const twa_status st =
        run_once(s, h, B, dL_dz, dL_dx0, dL_dxT, dL_dr, dL_dz0, &outcome, &need, nullptr, use_tape, nullptr);
    s->no_capture = was;
    if (st != TWA_OK) return st;
    if (outcome == kArenaFull)
        return fail(s, TWA_E_NOMEM, "twa_backward_noalloc: the scratch holds " + std::to_string(total) +
                                        " records, the checkpoints need " + std::to_string(need));
    if (outcome != kDone)
        return fail(s, TWA_E_NOMEM, "twa_backward_noalloc: the checkpoints leave " + std::to_string(B.pool_cap) +
                                        " records of scratch to each capture pool, a segment needs " +
                                        std::to_string(need));
    return TWA_OK;
}
