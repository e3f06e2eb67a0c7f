// Host build of the HIP library's FP32 minimisers (prox.h), so the CPU test
// suite can compare them case by case with the FP64 reference.
#include "../paper_1311_4527_amd/csrc/prox.h"
using namespace twa;
extern "C" {
// collision minimiser on the four n-messages of one factor (dim 2 or 3)
void h_coll(int dim, const float *n, const float *w, const int *k, float R, float *x) {
    if (dim == 2) coll_prox<2>(n, w, k, R, x);
    else coll_prox<3>(n, w, k, R, x);
}
void h_capsule(const float *ab, float r, const float *n, float w0, float w1, int k0, int k1, float *x) {
    Capsule C{mk(ab[0], ab[1]), mk(ab[2], ab[3]), r};
    f2 a, b;
    capsule_prox(C, mk(n[0], n[1]), mk(n[2], n[3]), w0, w1, k0, k1, a, b);
    x[0] = a.x, x[1] = a.y, x[2] = b.x, x[3] = b.y;
}
void h_energy(const float *nl, const float *nh, int dim, float wl, float wh, int kl, int kh, float C, float *xl,
              float *xh) {
    for (int c = 0; c < dim; ++c) energy_prox(nl[c], nh[c], wl, wh, kl, kh, C, xl[c], xh[c]);
}
}
extern "C" {
void h_coll_vjp(const float *n, const float *w, const int *k, float R, const float *xb, float *nb, float *Rb) {
    for (int q = 0; q < 8; ++q) nb[q] = 0.f;
    float r = 0.f;
    coll_vjp2(n, w, k, R, xb, nb, r);
    *Rb = r;
}
void h_capsule_vjp(const float *ab, float r, const float *n, float w0, float w1, int k0, int k1, const float *xb,
                   float *nb, float *rb) {
    Capsule C{mk(ab[0], ab[1]), mk(ab[2], ab[3]), r};
    f2 a, b;
    Choice ch;
    capsule_prox(C, mk(n[0], n[1]), mk(n[2], n[3]), w0, w1, k0, k1, a, b, &ch);
    f2 n0b = mk(0.f, 0.f), n1b = mk(0.f, 0.f);
    float rr = 0.f;
    capsule_vjp(C, mk(n[0], n[1]), mk(n[2], n[3]), w0, w1, k0, k1, ch, mk(xb[0], xb[1]), mk(xb[2], xb[3]), n0b, n1b, rr);
    nb[0] = n0b.x, nb[1] = n0b.y, nb[2] = n1b.x, nb[3] = n1b.y;
    *rb = rr;
}
void h_energy_vjp(float wl, float wh, int kl, int kh, float C, float xlb, float xhb, float *nlb, float *nhb) {
    float a = 0.f, b = 0.f;
    energy_vjp(wl, wh, kl, kh, C, xlb, xhb, a, b);
    *nlb = a, *nhb = b;
}
}
extern "C" {
int h_vel(int dim, const float *nl, const float *nh, float wl, float wh, int kl, int kh, float C, int minimum,
          float *xl, float *xh) {
    if (dim == 2) return vel_prox<2>(nl, nh, wl, wh, kl, kh, C, minimum != 0, xl, xh);
    return vel_prox<3>(nl, nh, wl, wh, kl, kh, C, minimum != 0, xl, xh);
}
}
