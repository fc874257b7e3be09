// Kernel templates of the SWF solver (included by the per-size instantiation
// files and by swf_reduce.hip).
//
// One RK4 stage of the scattered-wave equation (eq. (scatDirac) of arXiv
// 2512.16889 multiplied by gamma^0),
//     k = IFFT[-i H0(k) FFT y_i] - i (A_0 + alpha^j A_j)(t_i) (y_i + psi_b(t_i)),
// is split into passes over the spinor-of-arrays state:
//   * column passes (axes y, z): forward transform, and on the last
//     non-trivial axis the -i H0(k)/N multiply and the inverse transform;
//   * one row pass (axis x): inverse transform, the stage epilogue (source
//     term, RK4 accumulation, absorber) and the forward x transform of the
//     next stage's input, so each stage costs one read and one write of the
//     FFT buffer per pass plus the RK4 state traffic.
#pragma once
#include "swf_dev.h"

namespace swf {

// Row-pass modes.
enum { ROW_FWD = 0, ROW_STAGE = 1, ROW_INV = 2, ROW_RHS = 3, ROW_FWDPH = 4 };
// Column-pass modes.
enum { COL_FWD = 0, COL_INV = 1, COL_H0 = 2 };

struct PassArgs {
    const SolveDev* solves;
    const TermDev* terms;
    const void* rtab;      // real tables (field profiles, masks)
    const void* ctab;      // complex tables (phases, twiddles)
    const int2* items;     // (solve, tile) per block
    const int* step;       // device step counter
    double t_out, dt;
    int stage;             // RK4 stage 0..3 (ROW_STAGE)
    int src, dst;          // buffer roles
    int h0row;             // 1: the row pass also applies -i H0 / N (dim == 1)
    double t_explicit;     // time of ROW_RHS
    long long ph2;         // ROW_FWDPH: complex offset of exp(i k_j x_j) tables
};

// ------------------------------------------------------------------ tile variants
// A pass kernel is instantiated for several tile shapes; the host times them on
// the actual problem (autotuner) and keeps the fastest.
//   row pass: T threads per x-line, ROWS lines per block, CG components per
//             LDS exchange round;
//   column pass: T threads per line, W adjacent x-columns per block, CG.
template <int N, int T> constexpr bool plan_ok() {
    if (T < 1 || N % T) return false;
    for (int j = 0; j < FftPlan<N>::NR; ++j)
        if ((N / FftPlan<N>::R[j]) % T || (N / T) % FftPlan<N>::R[j]) return false;
    return true;
}
template <int N> constexpr int half_t() {
    constexpr int T = FftPlan<N>::T;
    return (T % 2 == 0 && 2 * N / T <= 16 && plan_ok<N, T / 2>()) ? T / 2 : T;
}
constexpr int NVAR = 4;
template <int N> constexpr int nvar() { return N >= 256 ? NVAR : 1; }
constexpr size_t LDS_CAP = 72 * 1024;
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int cg_fit(size_t per_comp) { return 4 * per_comp <= LDS_CAP ? 4 : (2 * per_comp <= LDS_CAP ? 2 : 1); }

template <class R, int N, int V> struct RowVar {
    static constexpr int T = (V == 3) ? half_t<N>() : FftPlan<N>::T;
    static constexpr int ROWS = imax(1, (V == 2 ? 128 : 256) / T);
    static constexpr int THREADS = T * ROWS;
    using Lay = RowLay<N, ROWS>;
    static constexpr size_t PER_COMP = (size_t)ROWS * Lay::STRIDE * sizeof(cpx<R>);
    static constexpr int CG = V == 0 ? 1 : cg_fit(PER_COMP);
    static constexpr size_t BYTES = CG * PER_COMP;
};

template <class R, int N, int V> struct ColVar {
    static constexpr int WANT = sizeof(R) == 4 ? 16 : 8;
    static constexpr int T = (V >= 2) ? half_t<N>() : FftPlan<N>::T;
    static constexpr int W = imax(1, imin(V == 2 ? 2 * WANT : WANT, 512 / T));
    static constexpr int THREADS = T * W;
    static constexpr size_t PER_COMP = (size_t)N * W * sizeof(cpx<R>);
    static constexpr int CG = (V == 1 || V == 3) ? imin(2, cg_fit(PER_COMP)) : 1;
    static constexpr size_t BYTES = CG * PER_COMP;
};

// ------------------------------------------------------------------ row pass
template <class R, int N, int V, int MODE>
__global__ void __launch_bounds__((RowVar<R, N, V>::THREADS)) row_kernel(PassArgs a) {
    using C = cpx<R>;
    using VC = RowVar<R, N, V>;
    constexpr int T = VC::T;
    constexpr int ROWS = VC::ROWS;
    constexpr int E = N / T;
    using Lay = typename VC::Lay;
    constexpr int CG = VC::CG;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* lds = reinterpret_cast<C*>(smem_raw);
    __shared__ R sh_fyz[ROWS][MAX_TERMS];
    __shared__ int sh_mu[MAX_TERMS];
    __shared__ long long sh_tab[MAX_TERMS];
    __shared__ C sh_wc[4];
    __shared__ C sh_phyz[ROWS];

    const int tid = threadIdx.x;
    const int t = tid % T;
    const int line = tid / T;
    const int2 it = a.items[blockIdx.x];
    const SolveDev* __restrict__ S = a.solves + it.x;
    const int nrows = S->nrows;
    const int row = it.y * ROWS + line;
    const bool act = row < nrows;
    const int rowc = act ? row : 0;
    const long long base = (long long)rowc * N;
    const long long ns = S->nsites;
    const C* __restrict__ tw = reinterpret_cast<const C*>(a.ctab) + S->tw[0];
    const C* __restrict__ ctab = reinterpret_cast<const C*>(a.ctab);
    const R* __restrict__ rtab = reinterpret_cast<const R*>(a.rtab);
    const int n0 = S->n[0], n1 = S->n[1];
    const int yy = rowc % n1, zz = rowc / n1;
    C v[4][E];

    if constexpr (MODE == ROW_FWD || MODE == ROW_FWDPH) {
        const C* __restrict__ src = reinterpret_cast<const C*>(S->buf[a.src]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) v[q][m] = src[q * ns + base + t + T * m];
        if constexpr (MODE == ROW_FWDPH) {
            const C* ph = ctab + a.ph2;
            const C pyz = cmul(ph[n0 + yy], ph[n0 + n1 + zz]);
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const C p = cmul(ph[t + T * m], pyz);
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q][m] = cmul(v[q][m], p);
            }
        }
        fft_line<C, N, T, -1, 4, CG, Lay>(v, lds, t, line, tw);
        if (act) {
            C* __restrict__ dst = reinterpret_cast<C*>(S->buf[a.dst]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int m = 0; m < E; ++m) dst[q * ns + base + t + T * m] = v[q][m];
        }
        return;
    } else {
        // ---- inverse transform of the k-space buffer (optionally after -i H0 / N)
        const C* __restrict__ tb = reinterpret_cast<const C*>(S->buf[BUF_T]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) v[q][m] = tb[q * ns + base + t + T * m];
        if (a.h0row) {
            const R Ky = (R)S->kap[1], Kz = (R)S->kap[2], s = (R)S->inv_n;
            const double dk = S->dk[0];
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const R Kx = (R)(dk * kindex(t + T * m, N));
                apply_h0(v[0][m], v[1][m], v[2][m], v[3][m], Kx, Ky, Kz, s);
            }
        }
        fft_line<C, N, T, +1, 4, CG, Lay>(v, lds, t, line, tw);
        if constexpr (MODE == ROW_INV) {
            if (act) {
                C* __restrict__ dst = reinterpret_cast<C*>(S->buf[a.dst]);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int m = 0; m < E; ++m) dst[q * ns + base + t + T * m] = v[q][m];
            }
            return;
        } else {
            // ---- stage epilogue: k = K - i V(t_i) (y_i + psi_b(t_i))
            double ts;
            if constexpr (MODE == ROW_RHS) {
                ts = a.t_explicit;
            } else {
                const int n = *a.step;
                const double cst = (a.stage == 0) ? 0.0 : (a.stage == 3 ? 1.0 : 0.5);
                ts = a.t_out - (double)n * a.dt - cst * a.dt;
            }
            const int nterm = S->nterm;
            for (int j = t; j < nterm; j += T) {
                const TermDev tm = a.terms[S->term0 + j];
                const double coef = tm.amp * profile_t(tm.ft_type, tm.c, tm.w, tm.k, tm.phi, ts);
                sh_fyz[line][j] = (R)coef * rtab[tm.tab + n0 + yy] * rtab[tm.tab + n0 + n1 + zz];
                if (line == 0) {
                    sh_mu[j] = tm.mu;
                    sh_tab[j] = tm.tab;
                }
            }
            for (int q = tid; q < 4; q += VC::THREADS) {
                double sn, cs;
                sincos(-S->E * ts, &sn, &cs);
                const double wr = S->w[2 * q], wi = S->w[2 * q + 1];
                sh_wc[q] = cmake<C>((R)(wr * cs - wi * sn), (R)(wr * sn + wi * cs));
            }
            if (t == 0) {
                const C* ph = ctab + S->ph;
                sh_phyz[line] = cmul(ph[n0 + yy], ph[n0 + n1 + zz]);
            }
            __syncthreads();
            const C* __restrict__ phx = ctab + S->ph;
            const C wc0 = sh_wc[0], wc1 = sh_wc[1], wc2 = sh_wc[2], wc3 = sh_wc[3];
            const C phyz = sh_phyz[line];
            const R h = (R)(-a.dt);
            const R h2 = (R)(-0.5 * a.dt), h3 = (R)(-a.dt / 3.0), h6 = (R)(-a.dt / 6.0);
            C* __restrict__ Y = reinterpret_cast<C*>(S->buf[BUF_Y]);
            C* __restrict__ ACC = reinterpret_cast<C*>(S->buf[BUF_ACC]);
            C* __restrict__ YS = reinterpret_cast<C*>(S->buf[BUF_YS]);
            const C* __restrict__ YIN = reinterpret_cast<const C*>(S->buf[MODE == ROW_RHS ? a.src : (a.stage == 0 ? BUF_Y : BUF_YS)]);
            const long long mask = S->mask;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const int x = t + T * m;
                const long long o = base + x;
                R A0 = 0, A1 = 0, A2 = 0, A3 = 0;
                for (int j = 0; j < nterm; ++j) {
                    const R f = sh_fyz[line][j] * rtab[sh_tab[j] + x];
                    const int mu = sh_mu[j];
                    A0 += mu == 0 ? f : (R)0;
                    A1 += mu == 1 ? f : (R)0;
                    A2 += mu == 2 ? f : (R)0;
                    A3 += mu == 3 ? f : (R)0;
                }
                const C ph = cmul(phx[x], phyz);
                C s[4], yi[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) yi[q] = YIN[q * ns + o];
                s[0] = cadd(yi[0], cmul(wc0, ph));
                s[1] = cadd(yi[1], cmul(wc1, ph));
                s[2] = cadd(yi[2], cmul(wc2, ph));
                s[3] = cadd(yi[3], cmul(wc3, ph));
                C vs[4];
                apply_pot(s, vs, A0, A1, A2, A3);
                C k[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) k[q] = cadd(v[q][m], cmul_mi(vs[q]));
                if constexpr (MODE == ROW_RHS) {
                    if (act) {
                        C* dst = reinterpret_cast<C*>(S->buf[a.dst]);
#pragma unroll
                        for (int q = 0; q < 4; ++q) dst[q * ns + o] = k[q];
                    }
                } else {
                    if (a.stage == 0) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const C acc = cadd(yi[q], cscale(k[q], h6));
                            const C yn = cadd(yi[q], cscale(k[q], h2));
                            if (act) {
                                ACC[q * ns + o] = acc;
                                YS[q * ns + o] = yn;
                            }
                            v[q][m] = yn;
                        }
                    } else if (a.stage < 3) {
                        const R hc = a.stage == 1 ? h2 : h;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const C y0 = Y[q * ns + o];
                            const C acc = cadd(ACC[q * ns + o], cscale(k[q], h3));
                            const C yn = cadd(y0, cscale(k[q], hc));
                            if (act) {
                                ACC[q * ns + o] = acc;
                                YS[q * ns + o] = yn;
                            }
                            v[q][m] = yn;
                        }
                    } else {
                        R mk = (R)1;
                        if (mask >= 0)
                            mk = rtab[mask + x] * rtab[mask + n0 + yy] * rtab[mask + n0 + n1 + zz];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            C yn = cadd(ACC[q * ns + o], cscale(k[q], h6));
                            if (mask >= 0) yn = cscale(yn, mk);
                            if (act) Y[q * ns + o] = yn;
                            v[q][m] = yn;
                        }
                    }
                }
            }
            if constexpr (MODE == ROW_STAGE) {
                // forward x transform of the next stage's input
                fft_line<C, N, T, -1, 4, CG, Lay>(v, lds, t, line, tw);
                if (act) {
                    C* __restrict__ tbw = reinterpret_cast<C*>(S->buf[BUF_T]);
#pragma unroll
                    for (int q = 0; q < 4; ++q)
#pragma unroll
                        for (int m = 0; m < E; ++m) tbw[q * ns + base + t + T * m] = v[q][m];
                }
            }
        }
    }
}

// ------------------------------------------------------------------ column pass
template <class R, int N, int V, int MODE, int AXIS>
__global__ void __launch_bounds__((ColVar<R, N, V>::THREADS)) col_kernel(PassArgs a) {
    using C = cpx<R>;
    using VC = ColVar<R, N, V>;
    constexpr int T = VC::T;
    constexpr int W = VC::W;
    constexpr int CG = VC::CG;
    constexpr int E = N / T;
    using Lay = ColLay<N, W>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* lds = reinterpret_cast<C*>(smem_raw);

    const int tid = threadIdx.x;
    const int xl = tid % W;
    const int t = tid / W;
    const int2 it = a.items[blockIdx.x];
    const SolveDev* __restrict__ S = a.solves + it.x;
    const int n0 = S->n[0], n1 = S->n[1];
    const int ntx = (n0 + W - 1) / W;
    const int xt = it.y % ntx;
    const int other = it.y / ntx;
    const int x = xt * W + xl;
    const bool act = x < n0;
    const long long stride = AXIS == 1 ? (long long)n0 : (long long)n0 * n1;
    const long long obase = AXIS == 1 ? (long long)other * n0 * n1 : (long long)other * n0;
    const long long base = obase + (act ? x : 0);
    const long long ns = S->nsites;
    C* __restrict__ buf = reinterpret_cast<C*>(S->buf[a.dst]);
    const C* __restrict__ tw = reinterpret_cast<const C*>(a.ctab) + S->tw[AXIS];
    C v[4][E];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < E; ++m) v[q][m] = buf[q * ns + base + (long long)(t + T * m) * stride];
    if constexpr (MODE == COL_FWD || MODE == COL_H0) fft_line<C, N, T, -1, 4, CG, Lay>(v, lds, t, xl, tw);
    if constexpr (MODE == COL_H0) {
        const R s = (R)S->inv_n;
        const R Kx = (R)(S->dk[0] * kindex(act ? x : 0, n0));
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int idx = t + T * m;
            R Ky, Kz;
            if constexpr (AXIS == 1) {
                Ky = (R)(S->dk[1] * kindex(idx, N));
                Kz = (R)S->kap[2];
            } else {
                Ky = (R)(S->dk[1] * kindex(other, n1));
                Kz = (R)(S->dk[2] * kindex(idx, N));
            }
            apply_h0(v[0][m], v[1][m], v[2][m], v[3][m], Kx, Ky, Kz, s);
        }
    }
    if constexpr (MODE == COL_INV || MODE == COL_H0) fft_line<C, N, T, +1, 4, CG, Lay>(v, lds, t, xl, tw);
    if (act) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) buf[q * ns + base + (long long)(t + T * m) * stride] = v[q][m];
    }
}

// Kernel table of one (precision, N) instantiation.
struct RowVariant { const void* stage; int threads, rows; size_t lds; };
struct ColVariant { const void* fn[2][3]; int threads, w; size_t lds; };
struct SizeKernels {
    int nvar;
    RowVariant row[NVAR];          // the RK4 stage pass, by variant
    const void* row_other[5];      // other row modes (variant 0)
    int row0_threads, row0_rows;
    size_t row0_lds;
    ColVariant col[NVAR];
};

template <class R, int N, int V>
RowVariant make_row_variant() {
    using VC = RowVar<R, N, V>;
    return RowVariant{(const void*)row_kernel<R, N, V, ROW_STAGE>, VC::THREADS, VC::ROWS, VC::BYTES};
}
template <class R, int N, int V>
ColVariant make_col_variant() {
    using VC = ColVar<R, N, V>;
    ColVariant c;
    c.fn[0][COL_FWD] = (const void*)col_kernel<R, N, V, COL_FWD, 1>;
    c.fn[0][COL_INV] = (const void*)col_kernel<R, N, V, COL_INV, 1>;
    c.fn[0][COL_H0] = (const void*)col_kernel<R, N, V, COL_H0, 1>;
    c.fn[1][COL_FWD] = (const void*)col_kernel<R, N, V, COL_FWD, 2>;
    c.fn[1][COL_INV] = (const void*)col_kernel<R, N, V, COL_INV, 2>;
    c.fn[1][COL_H0] = (const void*)col_kernel<R, N, V, COL_H0, 2>;
    c.threads = VC::THREADS;
    c.w = VC::W;
    c.lds = VC::BYTES;
    return c;
}

template <class R, int N>
SizeKernels make_size_kernels() {
    SizeKernels k;
    k.nvar = nvar<N>();
    k.row[0] = make_row_variant<R, N, 0>();
    k.col[0] = make_col_variant<R, N, 0>();
    if constexpr (nvar<N>() > 1) {
        k.row[1] = make_row_variant<R, N, 1>();
        k.row[2] = make_row_variant<R, N, 2>();
        k.row[3] = make_row_variant<R, N, 3>();
        k.col[1] = make_col_variant<R, N, 1>();
        k.col[2] = make_col_variant<R, N, 2>();
        k.col[3] = make_col_variant<R, N, 3>();
    } else {
        for (int v = 1; v < NVAR; ++v) {
            k.row[v] = k.row[0];
            k.col[v] = k.col[0];
        }
    }
    k.row_other[ROW_FWD] = (const void*)row_kernel<R, N, 0, ROW_FWD>;
    k.row_other[ROW_STAGE] = (const void*)row_kernel<R, N, 0, ROW_STAGE>;
    k.row_other[ROW_INV] = (const void*)row_kernel<R, N, 0, ROW_INV>;
    k.row_other[ROW_RHS] = (const void*)row_kernel<R, N, 0, ROW_RHS>;
    k.row_other[ROW_FWDPH] = (const void*)row_kernel<R, N, 0, ROW_FWDPH>;
    k.row0_threads = RowVar<R, N, 0>::THREADS;
    k.row0_rows = RowVar<R, N, 0>::ROWS;
    k.row0_lds = RowVar<R, N, 0>::BYTES;
    return k;
}

}  // namespace swf
