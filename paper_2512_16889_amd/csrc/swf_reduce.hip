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

// Breit-Wheeler integrand of eq. (Mabfinite) at one RK4 stage for every vertex:
// Mdot_ab = sum_x e^{-i(k0 t - k.x)} Ua^dag (alpha.eps) Vb for (s,s), (b,s), (s,b).
template <class R>
__global__ void __launch_bounds__(RED_THREADS) bw_stage_kernel(BwArgs a) {
    using C = cpx<R>;
    const VertexDev* V = a.verts + blockIdx.y;
    const SolveDev* SU = a.solves + V->su;
    const SolveDev* SV = a.solves + V->sv;
    const int role = a.stage == 0 ? BUF_Y : BUF_YS;
    const C* U = reinterpret_cast<const C*>(SU->buf[role]);
    const C* W = reinterpret_cast<const C*>(SV->buf[role]);
    const C* ctab = reinterpret_cast<const C*>(a.ctab);
    const C* phU = ctab + SU->ph;
    const C* phV = ctab + SV->ph;
    const C* phK = ctab + V->phk;
    const int n = *a.step;
    const double cst = (a.stage == 0) ? 0.0 : (a.stage == 3 ? 1.0 : 0.5);
    const double ts = a.t_out - (double)n * a.dt - cst * a.dt;
    double2 wcU[4], wcV[4];
    {
        double sn, cs;
        sincos(-SU->E * ts, &sn, &cs);
        for (int q = 0; q < 4; ++q) wcU[q] = dmul(d2(SU->w[2 * q], SU->w[2 * q + 1]), d2(cs, sn));
        sincos(-SV->E * ts, &sn, &cs);
        for (int q = 0; q < 4; ++q) wcV[q] = dmul(d2(SV->w[2 * q], SV->w[2 * q + 1]), d2(cs, sn));
    }
    double snk, csk;
    sincos(-V->k0 * ts, &snk, &csk);
    const double2 ek = d2(csk, snk);
    const int n0 = SU->n[0], n1 = SU->n[1];
    const long long ns = SU->nsites;
    double2 acc[3] = {d2(0, 0), d2(0, 0), d2(0, 0)};
    for (long long i = (long long)blockIdx.x * RED_THREADS + threadIdx.x; i < ns; i += (long long)gridDim.x * RED_THREADS) {
        const int x = (int)(i % n0);
        const long long r = i / n0;
        const int y = (int)(r % n1), z = (int)(r / n1);
        const double2 pu = todbl(cmul(cmul(phU[x], phU[n0 + y]), phU[n0 + n1 + z]));
        const double2 pv = todbl(cmul(cmul(phV[x], phV[n0 + y]), phV[n0 + n1 + z]));
        const double2 pk = dmul(ek, todbl(cmul(cmul(phK[x], phK[n0 + y]), phK[n0 + n1 + z])));
        double2 yu[4], yv[4], bu[4], bv[4], gyv[4], gbv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            yu[q] = todbl(U[q * ns + i]);
            yv[q] = todbl(W[q * ns + i]);
            bu[q] = dmul(wcU[q], pu);
            bv[q] = dmul(wcV[q], pv);
        }
        gam_eps(yv, gyv, V->eps);
        gam_eps(bv, gbv, V->eps);
        double2 s0 = d2(0, 0), s1 = d2(0, 0), s2 = d2(0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            s0 = dadd(s0, dcmul(yu[q], gyv[q]));
            s1 = dadd(s1, dcmul(bu[q], gyv[q]));
            s2 = dadd(s2, dcmul(yu[q], gbv[q]));
        }
        acc[0] = dadd(acc[0], dmul(pk, s0));
        acc[1] = dadd(acc[1], dmul(pk, s1));
        acc[2] = dadd(acc[2], dmul(pk, s2));
    }
    // partials layout [vertex][stage][block][3]
    double2* out = a.part + ((long long)blockIdx.y * 4 + a.stage) * (long long)gridDim.x * 3;
    block_sum_store<3>(acc, out);
}

// M_ab += (h/6) dV (d0 + 2 d1 + 2 d2 + d3), partial sums added in a fixed order.
__global__ void bw_accum_kernel(BwArgs a, int nblk) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= a.nvert * 3) return;
    const int v = gid / 3, term = gid % 3;
    const SolveDev* SU = a.solves + a.verts[v].su;
    const double wst[4] = {1.0, 2.0, 2.0, 1.0};
    double2 s = d2(0, 0);
    for (int st = 0; st < 4; ++st) {
        const double2* p = a.part + ((long long)v * 4 + st) * (long long)nblk * 3;
        double2 ss = d2(0, 0);
        for (int b = 0; b < nblk; ++b) ss = dadd(ss, p[(long long)b * 3 + term]);
        s = dadd(s, dsc(ss, wst[st]));
    }
    const double f = -a.dt / 6.0 * SU->dV;
    double2* M = a.M + (long long)v * 3 + term;
    *M = dadd(*M, dsc(s, f));
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

hipError_t launch_bw_stage(int fp64, const BwArgs& a, int blocks, hipStream_t st) {
    dim3 g(blocks, a.nvert), b(RED_THREADS);
    if (fp64) hipLaunchKernelGGL(bw_stage_kernel<double>, g, b, 0, st, a);
    else hipLaunchKernelGGL(bw_stage_kernel<float>, g, b, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_bw_accum(const BwArgs& a, int nblk, hipStream_t st) {
    const int threads = 64;
    const int blocks = (a.nvert * 3 + threads - 1) / threads;
    hipLaunchKernelGGL(bw_accum_kernel, dim3(blocks), dim3(threads), 0, st, a, nblk);
    return hipGetLastError();
}

hipError_t launch_tick(int* step, hipStream_t st) { return launch_advance(step, 1, st); }

hipError_t launch_advance(int* step, int n, hipStream_t st) {
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(64), 0, st, step, n);
    return hipGetLastError();
}

}  // namespace swf
