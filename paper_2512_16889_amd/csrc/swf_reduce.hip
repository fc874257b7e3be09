// Reductions of the SWF solver: the inner products at t_in (pair amplitude and
// marginals of eq. (Nmn), arXiv 2512.16889), the Breit-Wheeler vertex
// integrands of eq. (Mabfinite) evaluated at every RK4 stage, their RK4
// accumulation, the asymptotic-past term of eq. (MScatScatPast), diagnostics.
//
// Every reduction accumulates in double, per thread over a fixed grid-stride
// sequence, then over the block in a fixed tree; blocks write partial sums that
// are added in a fixed order afterwards.  No atomics: results are bitwise
// repeatable.
#include "swf_kernels.h"
#include "swf_reduce.h"
#include "swf_dmath.h"

namespace swf {

constexpr int RED_THREADS = 256;

template <int NV>
__device__ __forceinline__ void block_sum_store(double2 (&acc)[NV], double2* out) {
    __shared__ double2 sh[RED_THREADS][NV];
    const int tid = threadIdx.x;
#pragma unroll
    for (int v = 0; v < NV; ++v) sh[tid][v] = acc[v];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                sh[tid][v].x += sh[tid + s][v].x;
                sh[tid][v].y += sh[tid + s][v].y;
            }
        }
        __syncthreads();
    }
    if (tid < NV) out[(long long)blockIdx.x * NV + tid] = sh[0][tid];
}

// sum_k (Pi_sign(K) A(k))^dag (Pi_sign(K) B(k)), K the full momentum of A's
// lattice.  Equal to A^dag Pi B (Pi is an orthogonal projector); the projected
// vectors are formed first because the probabilities are exponentially small
// next to |A|^2 and the expanded form would cancel catastrophically.
template <class R>
__global__ void __launch_bounds__(RED_THREADS) kspace_proj_kernel(RedArgs a) {
    using C = cpx<R>;
    const SolveDev* SA = a.solves + a.sa;
    const SolveDev* SB = a.solves + a.sb;
    const C* A = reinterpret_cast<const C*>(SA->buf[a.ra]);
    const C* B = reinterpret_cast<const C*>(SB->buf[a.rb]);
    const bool same = (A == B);
    const long long ns = SA->nsites;
    double2 acc[1] = {d2(0, 0)};
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < ns; i += (long long)gridDim.x * RED_THREADS) {
        int x, y, z;
        site_xyz(i, SA, x, y, z);
        double Kx, Ky, Kz;
        site_k(SA, x, y, z, Kx, Ky, Kz);
        const double sg = a.sign / sqrt(1.0 + Kx * Kx + Ky * Ky + Kz * Kz);
        double2 pa[4], pb[4], h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) pa[q] = todbl(A[q * ns + i]);
        h0d(pa, h, Kx, Ky, Kz);
#pragma unroll
        for (int q = 0; q < 4; ++q) pa[q] = dsc(dadd(pa[q], dsc(h[q], sg)), 0.5);
        if (same) {
#pragma unroll
            for (int q = 0; q < 4; ++q) pb[q] = pa[q];
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) pb[q] = todbl(B[q * ns + i]);
            h0d(pb, h, Kx, Ky, Kz);
#pragma unroll
            for (int q = 0; q < 4; ++q) pb[q] = dsc(dadd(pb[q], dsc(h[q], sg)), 0.5);
        }
        double2 s = d2(0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) s = dadd(s, dcmul(pa[q], pb[q]));
        acc[0] = dadd(acc[0], s);
    }
    block_sum_store<1>(acc, a.out);
}

// Asymptotic-past (scat,scat) sum: A = FFT(U_s), B = FFT(V_s e^{i k.x}) so that
// B(kappa) = V~(kappa - k); sum over kappa, sigma, sigma' of
// (Pi_sigma(kappa) A)^dag (alpha.eps) (Pi_sigma'(kappa - k) B) / (i(sigma E - sigma' E' - k0)).
template <class R>
__global__ void __launch_bounds__(RED_THREADS) kspace_bwpast_kernel(RedArgs a) {
    using C = cpx<R>;
    const SolveDev* SA = a.solves + a.sa;
    const SolveDev* SB = a.solves + a.sb;
    const C* A = reinterpret_cast<const C*>(SA->buf[a.ra]);
    const C* B = reinterpret_cast<const C*>(SB->buf[a.rb]);
    const long long ns = SA->nsites;
    double2 acc[1] = {d2(0, 0)};
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < ns; i += (long long)gridDim.x * RED_THREADS) {
        int x, y, z;
        site_xyz(i, SA, x, y, z);
        double Kx, Ky, Kz;
        site_k(SA, x, y, z, Kx, Ky, Kz);
        const double Qx = Kx - a.kv[0], Qy = Ky - a.kv[1], Qz = Kz - a.kv[2];
        const double E = sqrt(1.0 + Kx * Kx + Ky * Ky + Kz * Kz);
        const double Ep = sqrt(1.0 + Qx * Qx + Qy * Qy + Qz * Qz);
        double2 pa[4], pb[4], ha[4], hb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pa[q] = todbl(A[q * ns + i]);
            pb[q] = todbl(B[q * ns + i]);
        }
        h0d(pa, ha, Kx, Ky, Kz);
        h0d(pb, hb, Qx, Qy, Qz);
        for (int sg = -1; sg <= 1; sg += 2) {
            double2 PA[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) PA[q] = dsc(dadd(pa[q], dsc(ha[q], sg / E)), 0.5);
            for (int sp = -1; sp <= 1; sp += 2) {
                double2 PB[4], GB[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) PB[q] = dsc(dadd(pb[q], dsc(hb[q], sp / Ep)), 0.5);
                gam_eps(PB, GB, a.eps);
                double2 s = d2(0, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) s = dadd(s, dcmul(PA[q], GB[q]));
                // s / (i w) = -i s / w
                const double w = sg * E - sp * Ep - a.k0;
                acc[0] = dadd(acc[0], d2(s.y / w, -s.x / w));
            }
        }
    }
    block_sum_store<1>(acc, a.out);
}

// F_q = sum_x psi_q(x) exp(-i kappa.x), x_j = -L_j/2 + i_j dx_j (continuum
// Fourier coefficient at a possibly off-lattice kappa).
template <class R>
__global__ void __launch_bounds__(RED_THREADS) xspace_fourier_kernel(RedArgs a) {
    using C = cpx<R>;
    const SolveDev* S = a.solves + a.sa;
    const C* A = reinterpret_cast<const C*>(S->buf[a.ra]);
    const long long ns = S->nsites;
    double2 acc[4] = {d2(0, 0), d2(0, 0), d2(0, 0), d2(0, 0)};
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < ns; i += (long long)gridDim.x * RED_THREADS) {
        int x, y, z;
        site_xyz(i, S, x, y, z);
        double ph = a.kv[0] * (a.x0[0] + x * a.dx[0]);
        if (S->dim >= 2) ph += a.kv[1] * (a.x0[1] + y * a.dx[1]);
        if (S->dim >= 3) ph += a.kv[2] * (a.x0[2] + z * a.dx[2]);
        double sn, cs;
        sincos(-ph, &sn, &cs);
        const double2 e = d2(cs, sn);
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = dadd(acc[q], dmul(todbl(A[q * ns + i]), e));
    }
    block_sum_store<4>(acc, a.out);
}

// (psi|psi), (psi_b|psi), max |component|, count of non-finite values.
template <class R>
__global__ void __launch_bounds__(RED_THREADS) xspace_diag_kernel(RedArgs a) {
    using C = cpx<R>;
    const SolveDev* S = a.solves + a.sa;
    const C* A = reinterpret_cast<const C*>(S->buf[a.ra]);
    const long long ns = S->nsites;
    double2 acc[3] = {d2(0, 0), d2(0, 0), d2(0, 0)};
    double mx = 0.0, bad = 0.0;
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < ns; i += (long long)gridDim.x * RED_THREADS) {
        int x, y, z;
        site_xyz(i, S, x, y, z);
        // psi_b = w exp(-i E t + i K.x); K: p for U, -p for V on the non-trivial axes
        double ph = -S->E * a.t + a.kv[0] * (a.x0[0] + x * a.dx[0]);
        if (S->dim >= 2) ph += a.kv[1] * (a.x0[1] + y * a.dx[1]);
        if (S->dim >= 3) ph += a.kv[2] * (a.x0[2] + z * a.dx[2]);
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double2 e = d2(cs, sn);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double2 p = todbl(A[q * ns + i]);
            if (!isfinite(p.x) || !isfinite(p.y)) bad += 1.0;
            mx = fmax(mx, fmax(fabs(p.x), fabs(p.y)));
            acc[0].x += p.x * p.x + p.y * p.y;
            const double2 b = dmul(d2(S->w[2 * q], S->w[2 * q + 1]), e);
            acc[1] = dadd(acc[1], dcmul(b, p));
        }
    }
    acc[2] = d2(mx, bad);
    // max and count do not add: reduce them separately
    __shared__ double shm[RED_THREADS], shb[RED_THREADS];
    shm[threadIdx.x] = mx;
    shb[threadIdx.x] = bad;
    block_sum_store<3>(acc, a.out);
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0, bb = 0.0;
        for (int j = 0; j < RED_THREADS; ++j) {
            m = fmax(m, shm[j]);
            bb += shb[j];
        }
        a.out[(long long)blockIdx.x * 3 + 2] = d2(m, bb);
    }
}

// Breit-Wheeler integrand of eq. (Mabfinite) at one RK4 stage, for a group of
// vertices with one photon and NU x NV solves (one group per blockIdx.y):
//   Mdot_ab = sum_x e^{-i(k0 t - k.x)} Ua^dag (alpha.eps) Vb  for (s,s), (b,s), (s,b).
// Per site the stage inputs of the V solves are read and multiplied by
// alpha.eps once, then each U solve is read once and dotted with every V.
// With psi_b = w e^{-iEt + iK.x} the spatial factors of the three terms are
//   (s,s): e^{ik.x},  (b,s): conj(e^{iK_U.x}) e^{ik.x},  (s,b): e^{iK_V.x} e^{ik.x},
// read from per-axis tables the host forms in double; the time factors
//   e^{-ik0 t},  conj(e^{-iE_U t}) e^{-ik0 t},  e^{-iE_V t} e^{-ik0 t}
// are constant over the sum and multiply the block sums.  Every pair (u, v) of
// the group is summed; the vertices take theirs.  Sites are visited in a fixed
// grid-stride order with 32-bit coordinates advanced by carries (a lattice has
// at most 1024^3 = 2^30 sites).
// s += conj(a) b and s += a b, four fused multiply-adds each
__device__ __forceinline__ void cmac_conj(double2& s, double2 a, double2 b) {
    s.x = fma(a.x, b.x, s.x);
    s.x = fma(a.y, b.y, s.x);
    s.y = fma(a.x, b.y, s.y);
    s.y = fma(-a.y, b.x, s.y);
}
__device__ __forceinline__ void cmac(double& sx, double& sy, double2 a, double2 b) {
    sx = fma(a.x, b.x, sx);
    sx = fma(-a.y, b.y, sx);
    sy = fma(a.x, b.y, sy);
    sy = fma(a.y, b.x, sy);
}
// (alpha.eps) p for real eps, three fused operations per real output
__device__ __forceinline__ void gam_eps_fma(const double2 (&p)[4], double2 (&o)[4], double e0, double e1, double e2) {
    // rows 0, 2: e2 p_{q+2} + (e0 - i e1) p_{q+3};  rows 1, 3: (e0 + i e1) p_{q+1} - e2 p_{q+2}  (indices mod 4)
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const double2 a = p[2 - 2 * h], b = p[3 - 2 * h];
        o[2 * h].x = fma(e1, b.y, fma(e0, b.x, e2 * a.x));
        o[2 * h].y = fma(-e1, b.x, fma(e0, b.y, e2 * a.y));
        o[2 * h + 1].x = fma(-e2, b.x, fma(-e1, a.y, e0 * a.x));
        o[2 * h + 1].y = fma(-e2, b.y, fma(e1, a.x, e0 * a.y));
    }
}

template <class R, int NU, int NV>
__global__ void __launch_bounds__(RED_THREADS) bw_stage_kernel(BwArgs a) {
    using C = cpx<R>;
    constexpr int NP = NU * NV;
    const VertexGroupDev* G = a.groups + blockIdx.y;
    const int role = a.stage == 0 ? BUF_Y : BUF_YS;
    const C* ctab = reinterpret_cast<const C*>(a.ctab);
    const SolveDev* S0 = a.solves + G->su[0];
    const unsigned n0 = (unsigned)S0->n[0], n1 = (unsigned)S0->n[1];
    const unsigned ns = (unsigned)S0->nsites;
    gptr<const nv2<R>> Up[NU], Vp[NV];
    const C* T1[NU];
    const C* T2[NV];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        Up[u] = cview<R>(a.solves[G->su[u]].buf[role]);
        T1[u] = ctab + G->t1[u];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        Vp[v] = cview<R>(a.solves[G->sv[v]].buf[role]);
        T2[v] = ctab + G->t2[v];
    }
    const C* TK = ctab + G->tk;
    const double e0 = G->eps[0], e1 = G->eps[1], e2 = G->eps[2];
    double acc[NP][3][2];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[p][c][0] = acc[p][c][1] = 0.0;
    const unsigned stride = gridDim.x * RED_THREADS;
    unsigned i = blockIdx.x * RED_THREADS + threadIdx.x;
    unsigned x = i % n0, y = (i / n0) % n1, z = (i / n0) / n1;
    const unsigned sx = stride % n0, sy = (stride / n0) % n1, sz = (stride / n0) / n1;
    for (; i < ns; i += stride) {
        const unsigned iy = n0 + y, iz = n0 + n1 + z;
        // V side: (alpha.eps) V_scat of each V solve, and its (s,b) factor
        double2 gy[NV][4], f2[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double2 yv[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) yv[q] = todbl(gload_nt<C>(Vp[v], (long long)q * ns + i));
            gam_eps_fma(yv, gy[v], e0, e1, e2);
            f2[v] = todbl(cmul(cmul(T2[v][x], T2[v][iy]), T2[v][iz]));
        }
        const double2 f0 = todbl(cmul(cmul(TK[x], TK[iy]), TK[iz]));
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            double2 yu[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) yu[q] = todbl(gload_nt<C>(Up[u], (long long)q * ns + i));
            const double2 f1 = todbl(cmul(cmul(T1[u][x], T1[u][iy]), T1[u][iz]));
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double2 ss = d2(0, 0), bs = d2(0, 0), sb = d2(0, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    cmac_conj(ss, yu[q], gy[v][q]);
                    cmac_conj(bs, d2(G->cu[u][2 * q], G->cu[u][2 * q + 1]), gy[v][q]);
                    cmac_conj(sb, yu[q], d2(G->cv[v][2 * q], G->cv[v][2 * q + 1]));
                }
                double (&A)[3][2] = acc[u * NV + v];
                cmac(A[0][0], A[0][1], f0, ss);
                cmac(A[1][0], A[1][1], f1, bs);
                cmac(A[2][0], A[2][1], f2[v], sb);
            }
        }
        x += sx;
        y += sy;
        z += sz;
        if (x >= n0) { x -= n0; ++y; }
        if (y >= n1) { y -= n1; ++z; }
    }
    // block sums of the 3 terms of every pair: a fixed butterfly within each
    // wave, then the waves in order; times the terms' time factors; partials
    // layout [vertex][stage][block][3]
    constexpr int NT = 3 * NP;
    constexpr int NW = RED_THREADS / 64;
    __shared__ double2 shw[NW][NT];
    const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double2 s = d2(acc[p][c][0], acc[p][c][1]);
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                s.x += __shfl_down(s.x, off, 64);
                s.y += __shfl_down(s.y, off, 64);
            }
            if (lane == 0) shw[wave][3 * p + c] = s;
        }
    __syncthreads();
    if (tid < 3 * G->nvx) {
        const int j = tid / 3, c = tid % 3;
        const int p = G->ui[j] * NV + G->vi[j];
        double2 s = shw[0][3 * p + c];
#pragma unroll
        for (int w = 1; w < NW; ++w) s = dadd(s, shw[w][3 * p + c]);
        const double ts = a.t_out - (double)(*a.step) * a.dt - a.cst * a.dt;
        // phase of the term: -(k0 + [E_V]) t for (s,s) / (s,b), (E_U - k0) t for (b,s)
        double w = -a.verts[G->vtx[0]].k0;
        if (c == 1) w += a.solves[G->su[G->ui[j]]].E;
        if (c == 2) w -= a.solves[G->sv[G->vi[j]]].E;
        double sn, cs;
        sincos(w * ts, &sn, &cs);
        a.part[(((long long)G->vtx[j] * a.nst + a.stage) * gridDim.x + blockIdx.x) * 3 + c] = dmul(d2(cs, sn), s);
    }
}

// (alpha.E) p for a complex polarisation vector E (the packet's field)
__device__ __forceinline__ void alpha_E(const double2 (&p)[4], double2 (&o)[4], const double2 (&E)[3]) {
    const double2 em = d2(E[0].x + E[1].y, E[0].y - E[1].x);   // E_x - i E_y
    const double2 ep = d2(E[0].x - E[1].y, E[0].y + E[1].x);   // E_x + i E_y
    o[0] = dadd(dmul(E[2], p[2]), dmul(em, p[3]));
    o[1] = dadd(dmul(ep, p[2]), dsc(dmul(E[2], p[3]), -1.0));
    o[2] = dadd(dmul(E[2], p[0]), dmul(em, p[1]));
    o[3] = dadd(dmul(ep, p[0]), dsc(dmul(E[2], p[1]), -1.0));
}

// The same integrand for a photon wave packet (one packet vertex per
// blockIdx.y): eps_mu e^{-ikx} is replaced by the packet's field
// E(t,x) = sum_m c_m e^{-i k0_m t} eps_m e^{i k_m.x}, assembled per site from the
// modes' phase tables.
template <class R>
__global__ void __launch_bounds__(RED_THREADS) bw_packet_stage_kernel(BwArgs a) {
    using C = cpx<R>;
    const VertexDev* V = a.verts + a.packets[blockIdx.y];
    const SolveDev* SU = a.solves + V->su;
    const SolveDev* SV = a.solves + V->sv;
    const int role = a.stage == 0 ? BUF_Y : BUF_YS;
    const double ts = a.t_out - (double)(*a.step) * a.dt - a.cst * a.dt;
    const C* ctab = reinterpret_cast<const C*>(a.ctab);
    const int nm = V->nmodes;
    // c_m e^{-i k0_m t} eps_m of every mode and its phase tables
    __shared__ double2 am[MAX_MODES][3];
    __shared__ long long phm[MAX_MODES];
    for (int m = threadIdx.x; m < nm; m += RED_THREADS) {
        const ModeDev* M = a.modes + V->mode0 + m;
        double sn, cs;
        sincos(-M->k0 * ts, &sn, &cs);
        const double2 cm = dmul(d2(M->c[0], M->c[1]), d2(cs, sn));
        for (int j = 0; j < 3; ++j) am[m][j] = dsc(cm, M->eps[j]);
        phm[m] = M->phk;
    }
    __syncthreads();
    double2 eu, ev;
    {
        double sn, cs;
        sincos(-SU->E * ts, &sn, &cs);
        eu = d2(cs, sn);
        sincos(-SV->E * ts, &sn, &cs);
        ev = d2(cs, sn);
    }
    const C* U = reinterpret_cast<const C*>(SU->buf[role]);
    const C* W = reinterpret_cast<const C*>(SV->buf[role]);
    const C* phU = ctab + SU->ph;
    const C* phV = ctab + SV->ph;
    const int n0 = SU->n[0], n1 = SU->n[1];
    const long long ns = SU->nsites;
    double2 acc[3] = {d2(0, 0), d2(0, 0), d2(0, 0)};
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < ns; i += (long long)gridDim.x * RED_THREADS) {
        const int x = (int)(i % n0);
        const long long r = i / n0;
        const int y = (int)(r % n1), z = (int)(r / n1);
        double2 E[3] = {d2(0, 0), d2(0, 0), d2(0, 0)};
        for (int m = 0; m < nm; ++m) {
            const C* t = ctab + phm[m];
            const double2 ph = todbl(cmul(cmul(t[x], t[n0 + y]), t[n0 + n1 + z]));
#pragma unroll
            for (int j = 0; j < 3; ++j) E[j] = dadd(E[j], dmul(am[m][j], ph));
        }
        const double2 pu = dmul(eu, todbl(cmul(cmul(phU[x], phU[n0 + y]), phU[n0 + n1 + z])));
        const double2 pv = dmul(ev, todbl(cmul(cmul(phV[x], phV[n0 + y]), phV[n0 + n1 + z])));
        double2 yu[4], yv[4], bu[4], bv[4], gyv[4], gbv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            yu[q] = todbl(U[q * ns + i]);
            yv[q] = todbl(W[q * ns + i]);
            bu[q] = dmul(d2(SU->w[2 * q], SU->w[2 * q + 1]), pu);
            bv[q] = dmul(d2(SV->w[2 * q], SV->w[2 * q + 1]), pv);
        }
        alpha_E(yv, gyv, E);
        alpha_E(bv, gbv, E);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc[0] = dadd(acc[0], dcmul(yu[q], gyv[q]));
            acc[1] = dadd(acc[1], dcmul(bu[q], gyv[q]));
            acc[2] = dadd(acc[2], dcmul(yu[q], gbv[q]));
        }
    }
    // partials layout [vertex][stage][block][3]
    double2* out = a.part + ((long long)a.packets[blockIdx.y] * a.nst + a.stage) * (long long)gridDim.x * 3;
    block_sum_store<3>(acc, out);
}

__global__ void bw_accum_kernel(BwArgs a, int nblk) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.nvert * 3) return;
    const int v = gid / 3, term = gid % 3;
    const SolveDev* SU = a.solves + a.verts[v].su;
    double2 s = d2(0, 0);
    for (int st = 0; st < a.nst; ++st) {
        const double2* p = a.part + ((long long)v * a.nst + st) * (long long)nblk * 3;
        double2 ss = d2(0, 0);
        for (int b = 0; b < nblk; ++b) ss = dadd(ss, p[(long long)b * 3 + term]);
        s = dadd(s, dsc(ss, a.wst[st]));
    }
    const double f = -a.dt * SU->dV;
    double2* M = a.M + (long long)v * 3 + term;
    *M = dadd(*M, dsc(s, f));
}

// ---------------------------------------------------------------------------
// Breit-Wheeler amplitude by partial integration in t (the paper's second
// route, eq. (MScatScat2) and its (back,scat), (scat,back) partners).  With
// the scattered waves split into energy-projected, phase-removed parts, the
// free evolution drops out mode by mode (Pi_sigma H0 = sigma E Pi_sigma), so
// every term becomes a time integral over [t_in, t_out] of products with the
// source S = -i V (psi_s + psi_b) alone.  Per RK4 stage:
//   (s,s): i e^{-i k0 t} dV/N sum_kappa sum_{sigma,sigma'}
//          [(Pi_sigma S~_U)^dag G Pi_sigma' V~' + (Pi_sigma U~)^dag G Pi_sigma' S~'_V] / Om,
//          Om = sigma E(kappa) - sigma' E(kappa - k) - k0, V~' = FFT(V e^{i k.x});
//   (b,s): i e^{i(p0-k0)t} sum_sigma' u^dag G Pi_sigma'(p-k) S_V,c(p-k) / (p0 - sigma' E(p-k) - k0);
//   (s,b): i e^{i(q0-k0)t} sum_sigma (Pi_sigma(k-q) S_U,c(k-q))^dag G v / (sigma E(k-q) + q0 - k0);
// G = alpha.eps, F_c(kappa) = dV sum_x F(x) e^{-i kappa.x}.  The transforms
// live in the A0 (state) and A1 (source) buffers of each vertex solve.

// x-space part: the 8 Fourier sums of S_V at p - k and S_U at k - q for every
// vertex (blockIdx.y), read from the A1 buffers while they hold S in x space.
template <class R>
__global__ void __launch_bounds__(RED_THREADS) bw2_src_kernel(BwArgs a) {
    using C = cpx<R>;
    const VertexDev* V = a.verts + blockIdx.y;
    const SolveDev* SU = a.solves + V->su;
    const SolveDev* SV = a.solves + V->sv;
    const C* SrcU = reinterpret_cast<const C*>(SU->buf[BUF_A1]);
    const C* SrcV = reinterpret_cast<const C*>(SV->buf[BUF_A1]);
    const long long ns = SU->nsites;
    double2 acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = d2(0, 0);
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < ns; i += (long long)gridDim.x * RED_THREADS) {
        int x, y, z;
        site_xyz(i, SU, x, y, z);
        const double X[3] = {V->x0[0] + x * V->dx[0], V->x0[1] + y * V->dx[1], V->x0[2] + z * V->dx[2]};
        double pb = 0.0, ps = 0.0;
        for (int j = 0; j < SU->dim; ++j) {
            pb += V->kbs[j] * X[j];
            ps += V->ksb[j] * X[j];
        }
        double sn, cs;
        sincos(-pb, &sn, &cs);
        const double2 eb = d2(cs, sn);
        sincos(-ps, &sn, &cs);
        const double2 es = d2(cs, sn);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc[q] = dadd(acc[q], dmul(todbl(SrcV[q * ns + i]), eb));
            acc[4 + q] = dadd(acc[4 + q], dmul(todbl(SrcU[q * ns + i]), es));
        }
    }
    double2* out = a.part2 + ((long long)blockIdx.y * 4 + a.stage) * 9 * (long long)gridDim.x + gridDim.x;
    block_sum_store<8>(acc, out);
}

// k-space (s,s) sum of vertex a.vtx (without the factor i e^{-i k0 t} dV/N).
template <class R>
__global__ void __launch_bounds__(RED_THREADS) bw2_kss_kernel(BwArgs a) {
    using C = cpx<R>;
    const VertexDev* V = a.verts + a.vtx;
    const SolveDev* SU = a.solves + V->su;
    const SolveDev* SV = a.solves + V->sv;
    const C* Uk = reinterpret_cast<const C*>(SU->buf[BUF_A0]);
    const C* SUk = reinterpret_cast<const C*>(SU->buf[BUF_A1]);
    const C* Vk = reinterpret_cast<const C*>(SV->buf[BUF_A0]);
    const C* SVk = reinterpret_cast<const C*>(SV->buf[BUF_A1]);
    const long long ns = SU->nsites;
    double2 acc[1] = {d2(0, 0)};
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < ns; i += (long long)gridDim.x * RED_THREADS) {
        int x, y, z;
        site_xyz(i, SU, x, y, z);
        double Kx, Ky, Kz;
        site_k(SU, x, y, z, Kx, Ky, Kz);
        const double Qx = Kx - V->k[0], Qy = Ky - V->k[1], Qz = Kz - V->k[2];
        const double E = sqrt(1.0 + Kx * Kx + Ky * Ky + Kz * Kz);
        const double Ep = sqrt(1.0 + Qx * Qx + Qy * Qy + Qz * Qz);
        double2 u[4], su[4], v[4], sv[4], hu[4], hsu[4], hv[4], hsv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            u[q] = todbl(Uk[q * ns + i]);
            su[q] = todbl(SUk[q * ns + i]);
            v[q] = todbl(Vk[q * ns + i]);
            sv[q] = todbl(SVk[q * ns + i]);
        }
        h0d(u, hu, Kx, Ky, Kz);
        h0d(su, hsu, Kx, Ky, Kz);
        h0d(v, hv, Qx, Qy, Qz);
        h0d(sv, hsv, Qx, Qy, Qz);
        for (int sg = -1; sg <= 1; sg += 2) {
            double2 PU[4], PSU[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                PU[q] = dsc(dadd(u[q], dsc(hu[q], sg / E)), 0.5);
                PSU[q] = dsc(dadd(su[q], dsc(hsu[q], sg / E)), 0.5);
            }
            for (int sp = -1; sp <= 1; sp += 2) {
                double2 PV[4], PSV[4], GV[4], GSV[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    PV[q] = dsc(dadd(v[q], dsc(hv[q], sp / Ep)), 0.5);
                    PSV[q] = dsc(dadd(sv[q], dsc(hsv[q], sp / Ep)), 0.5);
                }
                gam_eps(PV, GV, V->eps);
                gam_eps(PSV, GSV, V->eps);
                double2 s = d2(0, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) s = dadd(s, dadd(dcmul(PSU[q], GV[q]), dcmul(PU[q], GSV[q])));
                const double w = sg * E - sp * Ep - V->k0;
                acc[0] = dadd(acc[0], dsc(s, 1.0 / w));
            }
        }
    }
    double2* out = a.part2 + ((long long)a.vtx * 4 + a.stage) * 9 * (long long)gridDim.x;
    block_sum_store<1>(acc, out);
}

// Pi_sigma(K) f = (f + sigma H0(K) f / E(K)) / 2 at a (possibly off-lattice) K.
__device__ void proj_at(const double2 (&f)[4], double2 (&o)[4], const double* K, int sigma) {
    double2 h[4];
    h0d(f, h, K[0], K[1], K[2]);
    const double E = sqrt(1.0 + K[0] * K[0] + K[1] * K[1] + K[2] * K[2]);
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = dsc(dadd(f[q], dsc(h[q], sigma / E)), 0.5);
}

// M2_ab += (h/6) (d0 + 2 d1 + 2 d2 + d3) from the stage sums, in a fixed order;
// one thread per (vertex, term).
__global__ void bw2_accum_kernel(BwArgs a, int nblk) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.nvert * 3) return;
    const int v = gid / 3, term = gid % 3;
    const VertexDev* V = a.verts + v;
    const SolveDev* SU = a.solves + V->su;
    const SolveDev* SV = a.solves + V->sv;
    const double wst[4] = {1.0, 2.0, 2.0, 1.0};
    const int n = *a.step;
    double2 s = d2(0, 0);
    for (int st = 0; st < 4; ++st) {
        const double cst = st == 0 ? 0.0 : (st == 3 ? 1.0 : 0.5);
        const double t = a.t_out - (double)n * a.dt - cst * a.dt;
        const double2* p = a.part2 + ((long long)v * 4 + st) * 9 * (long long)nblk;
        double2 d;
        if (term == 0) {
            double2 ss = d2(0, 0);
            for (int b = 0; b < nblk; ++b) ss = dadd(ss, p[b]);
            double sn, cs;
            sincos(-V->k0 * t, &sn, &cs);
            // i e^{-i k0 t} dV/N
            d = dsc(dmul(d2(-sn, cs), ss), SU->dV * SU->inv_n);
        } else {
            // F_c = dV sum over blocks of the x-space sums
            const int o = term == 1 ? 0 : 4;
            double2 F[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double2 f = d2(0, 0);
                for (int b = 0; b < nblk; ++b) f = dadd(f, p[nblk + (long long)b * 8 + o + q]);
                F[q] = dsc(f, SU->dV);
            }
            double2 m = d2(0, 0);
            if (term == 1) {
                double2 u[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) u[q] = d2(SU->w[2 * q], SU->w[2 * q + 1]);
                const double Ek = sqrt(1.0 + V->kbs[0] * V->kbs[0] + V->kbs[1] * V->kbs[1] + V->kbs[2] * V->kbs[2]);
                for (int sp = -1; sp <= 1; sp += 2) {
                    double2 PF[4], GF[4];
                    proj_at(F, PF, V->kbs, sp);
                    gam_eps(PF, GF, V->eps);
                    double2 dot = d2(0, 0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) dot = dadd(dot, dcmul(u[q], GF[q]));
                    m = dadd(m, dsc(dot, 1.0 / (V->p0 - sp * Ek - V->k0)));
                }
                double sn, cs;
                sincos((V->p0 - V->k0) * t, &sn, &cs);
                d = dmul(d2(-sn, cs), m);   // i e^{i(p0-k0)t} m
            } else {
                double2 vs[4], gv[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) vs[q] = d2(SV->w[2 * q], SV->w[2 * q + 1]);
                gam_eps(vs, gv, V->eps);
                const double Ek = sqrt(1.0 + V->ksb[0] * V->ksb[0] + V->ksb[1] * V->ksb[1] + V->ksb[2] * V->ksb[2]);
                for (int sg = -1; sg <= 1; sg += 2) {
                    double2 PF[4];
                    proj_at(F, PF, V->ksb, sg);
                    double2 dot = d2(0, 0);
#pragma unroll
                    for (int q = 0; q < 4; ++q) dot = dadd(dot, dcmul(PF[q], gv[q]));
                    m = dadd(m, dsc(dot, 1.0 / (sg * Ek + V->q0 - V->k0)));
                }
                double sn, cs;
                sincos((V->q0 - V->k0) * t, &sn, &cs);
                d = dmul(d2(-sn, cs), m);   // i e^{i(q0-k0)t} m
            }
        }
        s = dadd(s, dsc(d, wst[st]));
    }
    double2* M = a.M2 + (long long)v * 3 + term;
    *M = dadd(*M, dsc(s, -a.dt / 6.0));
}

// In-loop check of the state: *flag becomes the largest ~((step << 32) | s)
// over the solves s whose psi_s (Y array) holds a NaN or an Inf, so the host
// reads back the first step and solve where one appeared (0: none so far).
// One read of every state, one atomic per wave that found a bad value.
template <class R>
__global__ void __launch_bounds__(RED_THREADS) finite_kernel(const SolveDev* solves, int nsolves, int step,
                                                            unsigned long long* flag) {
    for (int s = 0; s < nsolves; ++s) {
        const SolveDev* S = solves + s;
        const nv2<R>* y = reinterpret_cast<const nv2<R>*>(S->buf[BUF_Y]);
        const long long n = 4 * S->nsites;
        bool bad = false;
        for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < n;
             i += (long long)gridDim.x * RED_THREADS) {
            const nv2<R> v = y[i];
            bad = bad || !(isfinite(v.x) && isfinite(v.y));
        }
        if (__any(bad) && (threadIdx.x % warpSize) == 0)
            atomicMax(flag, ~(((unsigned long long)step << 32) | (unsigned)s));
    }
}

__global__ void tick_kernel(int* step, int n) {
    if (threadIdx.x == 0) __hip_atomic_fetch_add(step, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------------ launchers
template <class R>
static hipError_t launch_red(int kind, const RedArgs& a, int blocks, hipStream_t st) {
    dim3 g(blocks), b(RED_THREADS);
    switch (kind) {
        case RED_KPROJ: hipLaunchKernelGGL(kspace_proj_kernel<R>, g, b, 0, st, a); break;
        case RED_KBWPAST: hipLaunchKernelGGL(kspace_bwpast_kernel<R>, g, b, 0, st, a); break;
        case RED_XFOURIER: hipLaunchKernelGGL(xspace_fourier_kernel<R>, g, b, 0, st, a); break;
        case RED_XDIAG: hipLaunchKernelGGL(xspace_diag_kernel<R>, g, b, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduction(int fp64, int kind, const RedArgs& a, int blocks, hipStream_t st) {
    return fp64 ? launch_red<double>(kind, a, blocks, st) : launch_red<float>(kind, a, blocks, st);
}

template <class R>
static hipError_t bw_stage_shape(const BwArgs& a, dim3 g, int nu, int nv, hipStream_t st) {
    dim3 b(RED_THREADS);
    if (nu == 1 && nv == 1) hipLaunchKernelGGL((bw_stage_kernel<R, 1, 1>), g, b, 0, st, a);
    else if (nu == 1 && nv == 2) hipLaunchKernelGGL((bw_stage_kernel<R, 1, 2>), g, b, 0, st, a);
    else if (nu == 2 && nv == 1) hipLaunchKernelGGL((bw_stage_kernel<R, 2, 1>), g, b, 0, st, a);
    else if (nu == 2 && nv == 2) hipLaunchKernelGGL((bw_stage_kernel<R, 2, 2>), g, b, 0, st, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_bw_stage(int fp64, const BwArgs& a, int blocks, int nu, int nv, int ngroups, hipStream_t st) {
    const dim3 g(blocks, ngroups);
    return fp64 ? bw_stage_shape<double>(a, g, nu, nv, st) : bw_stage_shape<float>(a, g, nu, nv, st);
}

hipError_t launch_bw_packet_stage(int fp64, const BwArgs& a, int blocks, int npackets, hipStream_t st) {
    dim3 g(blocks, npackets), b(RED_THREADS);
    if (fp64) hipLaunchKernelGGL(bw_packet_stage_kernel<double>, g, b, 0, st, a);
    else hipLaunchKernelGGL(bw_packet_stage_kernel<float>, g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_bw_accum(const BwArgs& a, int nblk, hipStream_t st) {
    const int threads = 64;
    const int blocks = (a.nvert * 3 + threads - 1) / threads;
    hipLaunchKernelGGL(bw_accum_kernel, dim3(blocks), dim3(threads), 0, st, a, nblk);
    return hipGetLastError();
}

hipError_t launch_bw2_src(int fp64, const BwArgs& a, int blocks, hipStream_t st) {
    const dim3 g(blocks, a.nvert), b(RED_THREADS);
    if (fp64) hipLaunchKernelGGL(bw2_src_kernel<double>, g, b, 0, st, a);
    else hipLaunchKernelGGL(bw2_src_kernel<float>, g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_bw2_kss(int fp64, const BwArgs& a, int blocks, hipStream_t st) {
    const dim3 g(blocks), b(RED_THREADS);
    if (fp64) hipLaunchKernelGGL(bw2_kss_kernel<double>, g, b, 0, st, a);
    else hipLaunchKernelGGL(bw2_kss_kernel<float>, g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_bw2_accum(const BwArgs& a, int nblk, hipStream_t st) {
    const int threads = 64;
    const int blocks = (a.nvert * 3 + threads - 1) / threads;
    hipLaunchKernelGGL(bw2_accum_kernel, dim3(blocks), dim3(threads), 0, st, a, nblk);
    return hipGetLastError();
}

template <class R>
__global__ void __launch_bounds__(RED_THREADS) combo_kernel(ComboArgs a) {
    using C = cpx<R>;
    const int2 it = a.items[blockIdx.x];
    const SolveDev* __restrict__ S = a.solves + it.x;
    const int n0 = S->n[0], n1 = S->n[1], nrows = S->nrows;
    const long long ns = S->nsites;
    gptr<const nv2<R>> in[3];
    R c[2][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        in[i] = a.in[i] >= 0 ? cview<R>(S->buf[a.in[i]]) : cview<R>(S->buf[0]);
        c[0][i] = (R)a.c[0][i];
        c[1][i] = (R)a.c[1][i];
    }
    gptr<nv2<R>> o0 = wview<R>(S->buf[a.out[0] >= 0 ? a.out[0] : 0]);
    gptr<nv2<R>> o1 = wview<R>(S->buf[a.out[1] >= 0 ? a.out[1] : 0]);
    gptr<const R> rtab = glob(reinterpret_cast<const R*>(a.rtab));
    const bool mask = a.mask && S->mask >= 0;
    const int per = a.rows * n0;
    for (int e = threadIdx.x; e < 4 * per; e += RED_THREADS) {
        const int q = e / per, r = e % per;
        const int row = it.y * a.rows + r / n0, x = r % n0;
        if (row >= nrows) continue;
        const long long idx = (long long)q * ns + (long long)row * n0 + x;
        C v[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) v[i] = a.in[i] >= 0 ? gload_nt<C>(in[i], idx) : cmake<C>((R)0, (R)0);
        C w0 = cadd(cadd(cscale(v[0], c[0][0]), cscale(v[1], c[0][1])), cscale(v[2], c[0][2]));
        if (mask) w0 = cscale(w0, rtab[S->mask + x] * rtab[S->mask + n0 + row % n1] * rtab[S->mask + n0 + n1 + row / n1]);
        if (a.out[0] >= 0) gstore_nt<C>(o0, idx, w0);
        if (a.out[1] >= 0)
            gstore_nt<C>(o1, idx, cadd(cadd(cscale(v[0], c[1][0]), cscale(v[1], c[1][1])), cscale(v[2], c[1][2])));
    }
}

hipError_t launch_combo(int fp64, const ComboArgs& a, int nitems, hipStream_t st) {
    if (nitems <= 0) return hipSuccess;
    if (fp64) hipLaunchKernelGGL(combo_kernel<double>, dim3(nitems), dim3(RED_THREADS), 0, st, a);
    else hipLaunchKernelGGL(combo_kernel<float>, dim3(nitems), dim3(RED_THREADS), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_tick(int* step, hipStream_t st) { return launch_advance(step, 1, st); }

hipError_t launch_finite_check(int fp64, const SolveDev* solves, int nsolves, int step, unsigned long long* flag,
                               hipStream_t st) {
    if (fp64)
        hipLaunchKernelGGL(finite_kernel<double>, dim3(1024), dim3(RED_THREADS), 0, st, solves, nsolves, step, flag);
    else
        hipLaunchKernelGGL(finite_kernel<float>, dim3(1024), dim3(RED_THREADS), 0, st, solves, nsolves, step, flag);
    return hipGetLastError();
}

hipError_t launch_advance(int* step, int n, hipStream_t st) {
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(64), 0, st, step, n);
    return hipGetLastError();
}

}  // namespace swf
