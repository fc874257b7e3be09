// Double-precision complex helpers and lattice indexing shared by the
// reduction kernels (inner products at t_in, BW integrands, the pair matrix).
#pragma once
#include "swf_dev.h"

namespace swf {

__device__ __forceinline__ double2 d2(double a, double b) { double2 r; r.x = a; r.y = b; return r; }
__device__ __forceinline__ double2 dmul(double2 a, double2 b) { return d2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 dcmul(double2 a, double2 b) { return d2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }  // conj(a) b
__device__ __forceinline__ double2 dadd(double2 a, double2 b) { return d2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 dsc(double2 a, double s) { return d2(a.x * s, a.y * s); }

template <class C> __device__ __forceinline__ double2 todbl(C a) { return d2((double)a.x, (double)a.y); }

// H0(K) psi = (alpha.K + beta) psi in double.
__device__ __forceinline__ void h0d(const double2 (&p)[4], double2 (&o)[4], double Kx, double Ky, double Kz) {
    const double2 km = d2(Kx, -Ky), kp = d2(Kx, Ky);
    o[0] = dadd(p[0], dadd(dsc(p[2], Kz), dmul(km, p[3])));
    o[1] = dadd(p[1], dadd(dmul(kp, p[2]), dsc(p[3], -Kz)));
    o[2] = dadd(dadd(dsc(p[0], Kz), dmul(km, p[1])), dsc(p[2], -1.0));
    o[3] = dadd(dadd(dmul(kp, p[0]), dsc(p[1], -Kz)), dsc(p[3], -1.0));
}

// (alpha.eps) psi for a real polarisation vector.
__device__ __forceinline__ void gam_eps(const double2 (&p)[4], double2 (&o)[4], const double* e) {
    const double2 em = d2(e[0], -e[1]), ep = d2(e[0], e[1]);
    o[0] = dadd(dsc(p[2], e[2]), dmul(em, p[3]));
    o[1] = dadd(dmul(ep, p[2]), dsc(p[3], -e[2]));
    o[2] = dadd(dsc(p[0], e[2]), dmul(em, p[1]));
    o[3] = dadd(dmul(ep, p[0]), dsc(p[1], -e[2]));
}

__device__ __forceinline__ void site_xyz(long long i, const SolveDev* S, int& x, int& y, int& z) {
    x = (int)(i % S->n[0]);
    const long long r = i / S->n[0];
    y = (int)(r % S->n[1]);
    z = (int)(r / S->n[1]);
}

__device__ __forceinline__ void site_k(const SolveDev* S, int x, int y, int z, double& Kx, double& Ky, double& Kz) {
    Kx = S->dk[0] * kindex(x, S->n[0]);
    Ky = S->dim >= 2 ? S->dk[1] * kindex(y, S->n[1]) : S->kap[1];
    Kz = S->dim >= 3 ? S->dk[2] * kindex(z, S->n[2]) : S->kap[2];
}

}  // namespace swf
