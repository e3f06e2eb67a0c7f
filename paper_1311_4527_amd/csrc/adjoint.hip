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
// backwards through the same steps:
//   k_adj_select   per node: the class of the mean, and
//                  g = (dz' - s * sum of du' over kept edges) / |mean set|
//   k_adj_factors  per factor: dx = s du'[kept] + g[in mean set],
//                  dn = J_g^T dx (minimiser derivatives from prox.h),
//                  du = du'[kept] + g[in mean set] - dn, radius and start /
//                  goal cotangents
//   k_adj_gather   per node: dz = sum of dn over the node's edges
// State is read in the canonical layouts of the public header.  The forward
// states come from the solver itself: checkpoints every ceil(sqrt(K))
// iterations, and one segment at a time recomputed with every state kept.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/twa.h"
#include "prox.h"
#include "solver.h"

using namespace twa;
using twa_rt::wval;

namespace {

struct Adj {
    int p, eta, W;
    long long P2, N, E, F;
    long long e_energy, e_coll, e_wall, f_energy, f_coll, f_wall;
    const float *radii;
    const float4 *walls;
    const float *C;
    // forward state of iteration k (canonical layouts) and its decisions
    const float *z;              // [N][2]
    const float *u;              // [E][2]
    const unsigned char *l;      // [N] <-rho^k
    const unsigned char *rout;   // [F] ->rho^k
    const unsigned char *lnext;  // [N] <-rho^{k+1}
    float rho, step;             // rho0 of iteration k, alpha / rho0
    // cotangents
    float *zb;           // [N][2] dL/dz^{k+1} in, dL/dz^k out (k_adj_gather)
    float *ub;           // [E][2] dL/du^{k+1} in, dL/du^k out (k_adj_factors)
    float *g;            // [N][2]
    unsigned char *cls;  // [N] weight class of the node's mean
    float *nb;           // [E][2] dL/dn
    float *dx0, *dxT;    // [p][2], accumulated
    double *drd;         // [p], accumulated
};

__device__ __forceinline__ long long node_id(const Adj &A, int i, int s) { return (long long)i * (A.eta + 1) + s; }

__device__ __forceinline__ long long pair_index(int p, int a, int b) {
    return (long long)a * p - (long long)a * (a + 1) / 2 + (b - a - 1);
}

// Visit every edge of node (i, s) as fn(factor, edge); lanes of a wave
// split the collision and wall edges, lane 0 takes the fixed and energy ones.
template <class Fn>
__device__ __forceinline__ void for_node_edges(const Adj &A, int i, int s, int lane, Fn fn) {
    if (lane == 0) {
        if (s == 0) fn(2LL * i, 2LL * i);
        if (s == A.eta) fn(2LL * i + 1, 2LL * i + 1);
        if (s > 0) {
            long long fe = (long long)i * A.eta + s - 1;
            fn(A.f_energy + fe, A.e_energy + 2 * fe + 1);
        }
        if (s < A.eta) {
            long long fe = (long long)i * A.eta + s;
            fn(A.f_energy + fe, A.e_energy + 2 * fe);
        }
    }
    for (int j = lane; j < A.p; j += 64) {
        if (j == i) continue;
        int a = min(i, j), b = max(i, j);
        int base = (i == a) ? 0 : 2;
        long long pi = pair_index(A.p, a, b);
        if (s < A.eta) {
            long long fc = (long long)s * A.P2 + pi;
            fn(A.f_coll + fc, A.e_coll + 4 * fc + base);
        }
        if (s > 0) {
            long long fc = (long long)(s - 1) * A.P2 + pi;
            fn(A.f_coll + fc, A.e_coll + 4 * fc + base + 1);
        }
    }
    for (int w = lane; w < A.W; w += 64) {
        if (s < A.eta) {
            long long fw = ((long long)s * A.p + i) * A.W + w;
            fn(A.f_wall + fw, A.e_wall + 2 * fw);
        }
        if (s > 0) {
            long long fw = ((long long)(s - 1) * A.p + i) * A.W + w;
            fn(A.f_wall + fw, A.e_wall + 2 * fw + 1);
        }
    }
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// one wave per node
__global__ __launch_bounds__(256) void k_adj_select(Adj A) {
    int lane = threadIdx.x & 63;
    long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= A.N) return;
    int i = (int)(t / (A.eta + 1)), s = (int)(t % (A.eta + 1));
    bool keep_node = A.lnext[t] == W_STD;
    int ninf = 0, nstd = 0, deg = 0;
    float sx = 0.f, sy = 0.f;
    for_node_edges(A, i, s, lane, [&](long long f, long long e) {
        int r = A.rout[f];
        ninf += r == W_INF;
        nstd += r == W_STD;
        ++deg;
        if (r == W_STD && keep_node) {
            sx += A.ub[2 * e];
            sy += A.ub[2 * e + 1];
        }
    });
    ninf = wave_sum(ninf);
    nstd = wave_sum(nstd);
    deg = wave_sum(deg);
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) {
        int cnt = ninf ? ninf : (nstd ? nstd : deg);
        A.cls[t] = (unsigned char)(ninf ? W_INF : (nstd ? W_STD : W_ZERO));
        A.g[2 * t] = (A.zb[2 * t] - A.step * sx) / (float)cnt;
        A.g[2 * t + 1] = (A.zb[2 * t + 1] - A.step * sy) / (float)cnt;
    }
}

// one wave per node: dz^k = sum of dn over the node's edges
__global__ __launch_bounds__(256) void k_adj_gather(Adj A) {
    int lane = threadIdx.x & 63;
    long long t = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= A.N) return;
    int i = (int)(t / (A.eta + 1)), s = (int)(t % (A.eta + 1));
    float sx = 0.f, sy = 0.f;
    for_node_edges(A, i, s, lane, [&](long long, long long e) {
        sx += A.nb[2 * e];
        sy += A.nb[2 * e + 1];
    });
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) {
        A.zb[2 * t] = sx;
        A.zb[2 * t + 1] = sy;
    }
}

// dL/dx of edge e (node t) of a factor with weight r; also the part of
// dL/du^k that does not go through n.
__device__ __forceinline__ void edge_xbar(const Adj &A, int r, long long t, long long e, f2 &xb, f2 &up) {
    bool keep = r == W_STD && A.lnext[t] == W_STD;
    int c = A.cls[t];
    bool in_mean = c == W_INF ? r == W_INF : (c == W_STD ? r == W_STD : true);
    f2 ubp = keep ? mk(A.ub[2 * e], A.ub[2 * e + 1]) : mk(0.f, 0.f);
    f2 gg = in_mean ? mk(A.g[2 * t], A.g[2 * t + 1]) : mk(0.f, 0.f);
    xb = add(scl(ubp, A.step), gg);
    up = add(ubp, gg);
}

__device__ __forceinline__ f2 edge_n(const Adj &A, long long t, long long e) {
    return mk(A.z[2 * t] - A.u[2 * e], A.z[2 * t + 1] - A.u[2 * e + 1]);
}

__device__ __forceinline__ void edge_out(const Adj &A, long long e, f2 up, f2 nb) {
    A.ub[2 * e] = up.x - nb.x;
    A.ub[2 * e + 1] = up.y - nb.y;
    A.nb[2 * e] = nb.x;
    A.nb[2 * e + 1] = nb.y;
}

// one lane per factor, canonical factor order
__global__ __launch_bounds__(256) void k_adj_factors(Adj A) {
    long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= A.F) return;
    int r = A.rout[f];
    if (f < A.f_energy) {
        // fixed start / goal factor: x is the constant itself
        int i = (int)(f >> 1);
        int s = (f & 1) ? A.eta : 0;
        long long t = node_id(A, i, s), e = f;
        f2 xb, up;
        edge_xbar(A, r, t, e, xb, up);
        float *dst = (f & 1) ? A.dxT : A.dx0;
        dst[2 * i] += xb.x;
        dst[2 * i + 1] += xb.y;
        edge_out(A, e, up, mk(0.f, 0.f));
    } else if (f < A.f_coll) {
        // energy factor (App. E): linear in n
        long long fe = f - A.f_energy;
        int i = (int)(fe / A.eta), s = (int)(fe % A.eta);
        long long t0 = node_id(A, i, s), t1 = t0 + 1;
        long long e0 = A.e_energy + 2 * fe, e1 = e0 + 1;
        f2 xb0, up0, xb1, up1;
        edge_xbar(A, r, t0, e0, xb0, up0);
        edge_xbar(A, r, t1, e1, xb1, up1);
        int k0 = A.l[t0], k1 = A.l[t1];
        float w0 = wval(k0, A.rho), w1 = wval(k1, A.rho);
        float C = A.C[fe];
        float nb[4] = {0.f, 0.f, 0.f, 0.f};
        energy_vjp(w0, w1, k0, k1, C, xb0.x, xb1.x, nb[0], nb[2]);
        energy_vjp(w0, w1, k0, k1, C, xb0.y, xb1.y, nb[1], nb[3]);
        edge_out(A, e0, up0, mk(nb[0], nb[1]));
        edge_out(A, e1, up1, mk(nb[2], nb[3]));
    } else if (f < A.f_wall) {
        // collision factor (App. C): (s, i, j) from the triangular index
        long long fc = f - A.f_coll;
        int s = (int)(fc / A.P2);
        long long q = fc - (long long)s * A.P2;
        double b = 2.0 * A.p - 1.0;
        int i = (int)floor((b - sqrt(fmax(b * b - 8.0 * (double)q, 0.0))) * 0.5);
        i = max(0, min(i, A.p - 2));
        while (i > 0 && pair_index(A.p, i, i + 1) > q) --i;
        while (i < A.p - 2 && pair_index(A.p, i + 1, i + 2) <= q) ++i;
        int j = (int)(q - pair_index(A.p, i, i + 1)) + i + 1;
        long long t[4] = {node_id(A, i, s), node_id(A, i, s + 1), node_id(A, j, s), node_id(A, j, s + 1)};
        long long e0 = A.e_coll + 4 * fc;
        float xb[8], n[8], w[4], nbv[8];
        int k[4];
        f2 up[4];
        for (int qq = 0; qq < 4; ++qq) {
            f2 x_b;
            edge_xbar(A, r, t[qq], e0 + qq, x_b, up[qq]);
            xb[2 * qq] = x_b.x, xb[2 * qq + 1] = x_b.y;
            f2 nn = edge_n(A, t[qq], e0 + qq);
            n[2 * qq] = nn.x, n[2 * qq + 1] = nn.y;
            k[qq] = A.l[t[qq]];
            w[qq] = wval(k[qq], A.rho);
        }
        if (r == W_STD) {
            for (int qq = 0; qq < 8; ++qq) nbv[qq] = 0.f;
            float Rb = 0.f;
            coll_vjp2(n, w, k, A.radii[i] + A.radii[j], xb, nbv, Rb);
            atomicAdd(&A.drd[i], (double)Rb);
            atomicAdd(&A.drd[j], (double)Rb);
        } else {
            // inactive: x = n
            for (int qq = 0; qq < 8; ++qq) nbv[qq] = xb[qq];
        }
        for (int qq = 0; qq < 4; ++qq) edge_out(A, e0 + qq, up[qq], mk(nbv[2 * qq], nbv[2 * qq + 1]));
    } else {
        // wall factor (App. D)
        long long fw = f - A.f_wall;
        long long per_s = (long long)A.p * A.W;
        int s = (int)(fw / per_s);
        long long q = fw - (long long)s * per_s;
        int i = (int)(q / A.W), wi = (int)(q % A.W);
        long long t0 = node_id(A, i, s), t1 = t0 + 1;
        long long e0 = A.e_wall + 2 * fw, e1 = e0 + 1;
        f2 xb0, up0, xb1, up1;
        edge_xbar(A, r, t0, e0, xb0, up0);
        edge_xbar(A, r, t1, e1, xb1, up1);
        f2 nb0 = xb0, nb1 = xb1;
        if (r == W_STD) {
            float4 wl = A.walls[wi];
            Capsule Cw{mk(wl.x, wl.y), mk(wl.z, wl.w), A.radii[i]};
            f2 n0 = edge_n(A, t0, e0), n1 = edge_n(A, t1, e1);
            int k0 = A.l[t0], k1 = A.l[t1];
            float w0 = wval(k0, A.rho), w1 = wval(k1, A.rho);
            f2 x0, x1;
            Choice ch;
            capsule_prox(Cw, n0, n1, w0, w1, k0, k1, x0, x1, &ch);
            nb0 = mk(0.f, 0.f);
            nb1 = mk(0.f, 0.f);
            float rb = 0.f;
            capsule_vjp(Cw, n0, n1, w0, w1, k0, k1, ch, xb0, xb1, nb0, nb1, rb);
            atomicAdd(&A.drd[i], (double)rb);
        }
        edge_out(A, e0, up0, nb0);
        edge_out(A, e1, up1, nb1);
    }
}

// z^0 cotangent: its end points are the start and goal
__global__ void k_adj_finish(Adj A, float *dz0, float *dr) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < A.N) {
        int i = (int)(t / (A.eta + 1)), s = (int)(t % (A.eta + 1));
        bool end = s == 0 || s == A.eta;
        if (end) {
            float *dst = s == 0 ? A.dx0 : A.dxT;
            dst[2 * i] += A.zb[2 * t];
            dst[2 * i + 1] += A.zb[2 * t + 1];
        }
        if (dz0) {
            dz0[2 * t] = end ? 0.f : A.zb[2 * t];
            dz0[2 * t + 1] = end ? 0.f : A.zb[2 * t + 1];
        }
    }
    if (t < A.p) dr[t] = (float)A.drd[t];
}

// device buffers of one twa_backward call, freed on every exit path
struct Scratch {
    std::vector<void *> ptrs;
    ~Scratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    template <class T>
    bool get(T **out, size_t count) {
        void *p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(count * sizeof(T), 16)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        ptrs.push_back(p);
        *out = static_cast<T *>(p);
        return true;
    }
};

struct StateBuf {
    float *z = nullptr, *u = nullptr;
    unsigned char *l = nullptr;
};

} // namespace

extern "C" twa_status twa_backward(twa_solver *s, const float *dL_dz, float *dL_dx0, float *dL_dxT, float *dL_dr,
                                   float *dL_dz0) {
    using twa_rt::fail;
    TRY(twa_rt::check_alive(s));
    if (!(s->flags & TWA_F_TAPE)) return fail(s, TWA_E_STATE, "twa_backward needs TWA_F_TAPE at create");
    if (s->dim != 2) return fail(s, TWA_E_INVALID, "twa_backward supports dim == 2 only");
    if (s->P.admm) return fail(s, TWA_E_INVALID, "twa_backward supports the three-weight mode only");
    if (s->P.cost != 0) return fail(s, TWA_E_INVALID, "twa_backward supports the energy cost only");
    if (!dL_dz || !dL_dx0 || !dL_dxT || !dL_dr) return fail(s, TWA_E_INVALID, "null array argument");
    const twa_rt::Params &P = s->P;
    const long long N = P.N, E = P.e_wall + 2 * P.Fw, F = P.Ff + P.Fe + P.Fc + P.Fw;
    const long long K = s->iter - s->origin_iter;
    if (K < 0) return fail(s, TWA_E_STATE, "iteration count below the run's start");
    const int D = 2;
    const long long L = std::max<long long>(1, (long long)std::ceil(std::sqrt((double)K)));
    const long long ncp = K > 0 ? (K + L - 1) / L : 0;

    Scratch sc;
    auto state_buf = [&](StateBuf &b) {
        return sc.get(&b.z, (size_t)N * D) && sc.get(&b.u, (size_t)E * D) && sc.get(&b.l, (size_t)N);
    };
    StateBuf cur;
    std::vector<StateBuf> ckpt((size_t)ncp), seg((size_t)std::min(L, K));
    std::vector<unsigned char *> rout((size_t)std::min(L, K));
    unsigned char *lnext = nullptr, *cls = nullptr;
    float *xscr = nullptr, *zb = nullptr, *ub = nullptr, *g = nullptr, *nb = nullptr;
    double *drd = nullptr;
    bool ok = state_buf(cur) && sc.get(&lnext, (size_t)N) && sc.get(&cls, (size_t)N) &&
              sc.get(&xscr, (size_t)E * D) && sc.get(&zb, (size_t)N * D) && sc.get(&ub, (size_t)E * D) &&
              sc.get(&g, (size_t)N * D) && sc.get(&nb, (size_t)E * D) && sc.get(&drd, (size_t)s->p);
    for (auto &b : ckpt) ok = ok && state_buf(b);
    for (size_t q = 0; q < seg.size(); ++q) ok = ok && state_buf(seg[q]) && sc.get(&rout[q], (size_t)F);
    if (!ok) return fail(s, TWA_E_NOMEM, "twa_backward: checkpoint allocation failed");

    // keep the forward state to restore it at the end
    long long cur_iter = 0;
    TRY(twa_get_state(s, cur.z, cur.u, cur.l, &cur_iter));
    const long long it0 = s->origin_iter;

    // pass 1: checkpoints every L iterations from the run's start
    if (K > 0) TRY(twa_rt::import_state(s, s->origin_z, s->origin_u, s->origin_l, it0));
    for (long long c = 0; c < ncp; ++c) {
        long long dummy;
        TRY(twa_get_state(s, ckpt[c].z, ckpt[c].u, ckpt[c].l, &dummy));
        if (c + 1 < ncp) TRY(twa_iterate(s, (int)L));
    }

    Adj A{};
    A.p = s->p, A.eta = s->eta, A.W = s->W;
    A.P2 = (long long)s->p * (s->p - 1) / 2, A.N = N, A.E = E, A.F = F;
    A.e_energy = P.e_energy, A.e_coll = P.e_coll, A.e_wall = P.e_wall;
    A.f_energy = P.f_energy, A.f_coll = P.f_coll, A.f_wall = P.f_wall;
    A.radii = P.radii, A.walls = P.walls, A.C = P.C;
    A.zb = zb, A.ub = ub, A.g = g, A.cls = cls, A.nb = nb, A.dx0 = dL_dx0, A.dxT = dL_dxT, A.drd = drd;
    HIP_TRY(s, hipMemcpyAsync(zb, dL_dz, sizeof(float) * N * D, hipMemcpyDeviceToDevice, s->stream));
    HIP_TRY(s, hipMemsetAsync(ub, 0, sizeof(float) * E * D, s->stream));
    HIP_TRY(s, hipMemsetAsync(dL_dx0, 0, sizeof(float) * s->p * D, s->stream));
    HIP_TRY(s, hipMemsetAsync(dL_dxT, 0, sizeof(float) * s->p * D, s->stream));
    HIP_TRY(s, hipMemsetAsync(drd, 0, sizeof(double) * s->p, s->stream));
    const unsigned nb_nodes = (unsigned)((N + 3) / 4), nb_fac = (unsigned)((F + 255) / 256);

    // pass 2: segments in reverse; recompute each with every state kept
    for (long long c = ncp - 1; c >= 0; --c) {
        long long k0 = it0 + c * L, len = std::min(L, K - c * L);
        TRY(twa_rt::import_state(s, ckpt[c].z, ckpt[c].u, ckpt[c].l, k0));
        for (long long t = 0; t < len; ++t) {
            long long dummy;
            TRY(twa_get_state(s, seg[t].z, seg[t].u, seg[t].l, &dummy));
            TRY(twa_capture_next(s, xscr, rout[t]));
            TRY(twa_iterate(s, 1));
        }
        TRY(twa_get_state(s, nullptr, nullptr, lnext, nullptr));
        for (long long t = len - 1; t >= 0; --t) {
            A.z = seg[t].z, A.u = seg[t].u, A.l = seg[t].l, A.rout = rout[t];
            A.lnext = (t + 1 < len) ? seg[t + 1].l : lnext;
            A.rho = twa_rt::rho_at(s, k0 + t);
            A.step = s->alpha / A.rho;
            hipLaunchKernelGGL(k_adj_select, dim3(nb_nodes), dim3(256), 0, s->stream, A);
            hipLaunchKernelGGL(k_adj_factors, dim3(nb_fac), dim3(256), 0, s->stream, A);
            hipLaunchKernelGGL(k_adj_gather, dim3(nb_nodes), dim3(256), 0, s->stream, A);
            HIP_TRY(s, hipGetLastError());
        }
    }
    long long nfin = std::max<long long>(N, s->p);
    hipLaunchKernelGGL(k_adj_finish, dim3((unsigned)((nfin + 255) / 256)), dim3(256), 0, s->stream, A, dL_dz0,
                       dL_dr);
    HIP_TRY(s, hipGetLastError());
    // restore the forward state
    TRY(twa_rt::import_state(s, cur.z, cur.u, cur.l, cur_iter));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return TWA_OK;
}
