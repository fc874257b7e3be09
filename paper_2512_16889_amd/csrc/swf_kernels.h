// Kernel templates of the SWF solver (included by the per-size instantiation
// files and by swf_reduce.hip).
//
// One RK4 stage of the scattered-wave equation (eq. (scatDirac) of arXiv
// 2512.16889 multiplied by gamma^0),
//     k = IFFT[-i H0(k) FFT y_i] - i (A_0 + alpha^j A_j)(t_i) (y_i + psi_b(t_i)),
// H0(k) = alpha.k + beta.  Spectral derivatives along different axes commute,
// so the kinetic term is a sum over axes,
//     IFFT[-i H0 FFT y] = -i sum_j alpha^j D_j y - i beta y,
//     D_j y = IFFT_j[k_j FFT_j y]   (a one-dimensional transform along axis j),
// and in the Dirac representation every alpha^j is a signed permutation of
// the four components: (alpha^1 y)_q = y_{3-q}, (alpha^2 y)_q = -+i y_{3-q}
// (- for even q), (alpha^3 y)_q = +-y_{q^2} (+ for q = 0, 2).  A stage is
// therefore split into passes over the spinor-of-arrays state that never mix
// components inside a transform:
//   * column passes (axes y, z): one component per block; D_j of the component
//     alpha^j takes, written (y) or added (z) into the G buffer at the
//     component it lands on, G = alpha^2 D_y y + alpha^3 D_z y;
//   * one row pass (axis x): D_x of the component alpha^1 takes, then the
//     stage epilogue (beta and trivial-axis terms, the source, the RK4
//     update, the absorber) for the thread's own component.
// Per RK4 step this reads and writes 36 state arrays in 3D (24 in 2D, 12 in
// 1D).  The other row and column kernels (forward / inverse transforms of a
// whole state, the full right-hand side) serve the t_in observables, the
// operator test hook and the Breit-Wheeler partial-integration route.
#pragma once
#include "swf_dev.h"

namespace swf {

// Row-pass modes.
// ROW_SRC writes the source term -i V(t) (y + psi_b(t)) of the RK4 stage
// `stage` alone, in x space (no transform).
enum { ROW_FWD = 0, ROW_STAGE = 1, ROW_INV = 2, ROW_RHS = 3, ROW_FWDPH = 4, ROW_SRC = 5, ROW_NMODES = 6 };
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
    int stage;             // RK4 stage 0..3 (ROW_STAGE, ROW_SRC)
    int src, dst;          // buffer roles
    int h0row;             // 1: the row pass also applies -i H0 / N (dim == 1)
    int expo;              // 1: the k-space multiply (COL_H0, h0row) is exp(-i H0 tau) / N instead
    double tau;            //    of -i H0 / N: the free evolution over tau (interaction picture)
    double t_explicit;     // time of ROW_RHS
    long long ph2;         // ROW_FWDPH: complex offset of exp(i k_j x_j) tables
    int nitems;            // work items of this launch
    int nsteps;            // line_kernel: RK4 steps per launch
};

// ------------------------------------------------------------------ tile variants
// A pass kernel is instantiated for several tile shapes; the host times them on
// the actual problem (autotuner) and keeps the fastest.
//   row pass: T threads per x-line, ROWS lines per block, CG components per
//             LDS exchange round;
//   column pass: T threads per line, W adjacent x-columns per block, CG.
template <int N, int T, class P = FftPlan<N>> constexpr bool plan_ok() {
    if (T < 1 || N % T) return false;
    for (int j = 0; j < P::NR; ++j)
        if ((N / P::R[j]) % T || (N / T) % P::R[j]) return false;
    return true;
}
// the plan of a variant: the default one, or the few-points-per-thread one
template <int N, bool SMALL> struct PlanSel { using type = FftPlan<N>; };
template <int N> struct PlanSel<N, true> { using type = typename SmallPlan<N>::type; };
template <int N> constexpr int half_t() {
    constexpr int T = FftPlan<N>::T;
    return (T % 2 == 0 && 2 * N / T <= 16 && plan_ok<N, T / 2>()) ? T / 2 : T;
}
constexpr int NVAR = 4;       // tile variants of the stepping passes (row and column)
template <int N> constexpr int nvar() { return N >= 256 ? NVAR : 1; }
constexpr size_t LDS_CAP = 72 * 1024;
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int cg_fit(size_t per_comp) { return 4 * per_comp <= LDS_CAP ? 4 : (2 * per_comp <= LDS_CAP ? 2 : 1); }

// Tile of the row kernel (whole-state transforms and right-hand side): the
// default plan, T threads per x-line, up to 256 threads per block.
template <class R, int N, int V> struct RowVar {
    using PL = FftPlan<N>;
    static constexpr int T = PL::T;
    static constexpr int ROWS = imax(1, 256 / T);
    static constexpr int THREADS = T * ROWS;
    using Lay = RowLay<N, ROWS>;
    static constexpr size_t PER_COMP = (size_t)ROWS * Lay::STRIDE * sizeof(cpx<R>);
    static constexpr int CG = 1;
    static constexpr size_t BYTES = CG * PER_COMP;
    static constexpr bool SEQ = false;
    static_assert(plan_ok<N, T, PL>(), "row variant violates the FFT plan constraints");
};

template <class R, int N, int V> struct ColVar {
    // columns per block:
    //   v0: a full 128-byte line (WANT columns) of the default plan, capped at
    //       512 threads;
    //   v1: narrower tiles (more, smaller blocks per CU; the host then groups
    //       the tiles of one line on one XCD);
    //   v2: the few-points-per-thread plan, capped at 512 threads;
    //   v3: the few-points-per-thread plan with up to 1024 threads, so that a
    //       tile still covers a full 128-byte line where T is large (N >= 512)
    static constexpr int WANT = sizeof(R) == 4 ? 16 : 8;
    static constexpr bool SMALL = (V == 2 || V == 3) && has_small_plan<N>();
    using PL = typename PlanSel<N, SMALL>::type;
    static constexpr int T = PL::T;
    static constexpr int W0 = imax(1, imin(WANT, (V == 3 ? 1024 : 512) / T));
    static constexpr int W = V == 1 ? imax(1, WANT / 4) : W0;
    static constexpr int THREADS = T * W;
    static constexpr size_t PER_COMP = (size_t)N * W * sizeof(cpx<R>);
    static constexpr int CG = 1;
    static constexpr size_t BYTES = CG * PER_COMP;
    static constexpr bool SEQ = false;
    static_assert(plan_ok<N, T, PL>(), "column variant violates the FFT plan constraints");
};

// Transform the four components of a line: together (shared exchange rounds,
// more registers live) or one component after another (SEQ: fewer registers,
// more barriers).
template <class C, int N, int T, int DIR, int CG, bool SEQ, class Lay, class P>
__device__ __forceinline__ void fft4(C (&v)[4][N / T], C* lds, int t, int line, const C* tw) {
    if constexpr (SEQ) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            fft_line<C, N, T, DIR, 1, 1, Lay, P>(reinterpret_cast<C(&)[1][N / T]>(v[q]), lds, t, line, tw);
    } else {
        fft_line<C, N, T, DIR, 4, CG, Lay, P>(v, lds, t, line, tw);
    }
}

// ------------------------------------------------------------------ row pass
// Global-address-space views of the state arrays (their pointers come from the
// solve descriptors, so the compiler cannot infer the address space itself and
// would otherwise emit flat memory instructions).
template <class T> using gptr = T __attribute__((address_space(1)))*;
template <class T> __device__ __forceinline__ gptr<T> glob(T* p) { return (gptr<T>)p; }
// complex numbers cross the global address space as native clang vectors
template <class R> using nv2 = R __attribute__((ext_vector_type(2)));
template <class C> __device__ __forceinline__ C gload(gptr<const nv2<decltype(C::x)>> p, long long i) {
    const nv2<decltype(C::x)> v = p[i];
    return cmake<C>(v.x, v.y);
}
template <class C> __device__ __forceinline__ void gstore(gptr<nv2<decltype(C::x)>> p, long long i, C c) {
    nv2<decltype(C::x)> v;
    v.x = c.x;
    v.y = c.y;
    p[i] = v;
}
// streaming (non-temporal) load and store for the stepping passes: they read
// and write each line once per launch, and nothing touches the line again
// before the whole batch has been swept, so caching it only evicts other data
// (the column tiles cover whole 128-byte lines).
template <class C> __device__ __forceinline__ C gload_nt(gptr<const nv2<decltype(C::x)>> p, long long i) {
    const nv2<decltype(C::x)> v = __builtin_nontemporal_load(&p[i]);
    return cmake<C>(v.x, v.y);
}
template <class C> __device__ __forceinline__ void gstore_nt(gptr<nv2<decltype(C::x)>> p, long long i, C c) {
    nv2<decltype(C::x)> v;
    v.x = c.x;
    v.y = c.y;
    __builtin_nontemporal_store(v, &p[i]);
}
template <class R> __device__ __forceinline__ gptr<const nv2<R>> cview(const void* p) {
    return (gptr<const nv2<R>>)(reinterpret_cast<const nv2<R>*>(p));
}
template <class R> __device__ __forceinline__ gptr<nv2<R>> wview(void* p) {
    return (gptr<nv2<R>>)(reinterpret_cast<nv2<R>*>(p));
}

template <class R, int N, int V, int MODE, int STAGE>
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
    __shared__ C tw[N];

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
    // twiddle table in LDS: the first twiddle read comes after the first
    // exchange's barriers, so no extra barrier is needed here
    gptr<const nv2<R>> ctab = cview<R>(a.ctab);
    gptr<const R> rtab = glob(reinterpret_cast<const R*>(a.rtab));
    for (int i = tid; i < N; i += VC::THREADS) tw[i] = gload<C>(ctab, S->tw[0] + i);
    const int n0 = S->n[0], n1 = S->n[1];
    const int yy = rowc % n1, zz = rowc / n1;

    auto load = [&](int role, C (&w)[4][E]) {
        gptr<const nv2<R>> p = cview<R>(S->buf[role]) + base + t;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) w[q][m] = gload_nt<C>(p, q * ns + T * m);
    };
    auto store = [&](int role, const C (&w)[4][E]) {
        if (!act) return;
        gptr<nv2<R>> p = wview<R>(S->buf[role]) + base + t;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) gstore_nt<C>(p, q * ns + T * m, w[q][m]);
    };

    C v[4][E];
    if constexpr (MODE == ROW_FWD || MODE == ROW_FWDPH) {
        load(a.src, v);
        if constexpr (MODE == ROW_FWDPH) {
            const long long ph = a.ph2;
            const C pyz = cmul(gload<C>(ctab, ph + n0 + yy), gload<C>(ctab, ph + n0 + n1 + zz));
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const C p = cmul(gload<C>(ctab, ph + t + T * m), pyz);
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q][m] = cmul(v[q][m], p);
            }
        }
        fft4<C, N, T, -1, CG, VC::SEQ, Lay, typename VC::PL>(v, lds, t, line, tw);
        store(a.dst, v);
        return;
    } else {
        if constexpr (MODE == ROW_SRC) {
            // no kinetic term: the epilogue below adds the source to zero
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int m = 0; m < E; ++m) v[q][m] = cmake<C>((R)0, (R)0);
        } else {
            // ---- inverse transform of the k-space buffer (optionally after -i H0 / N)
            load(BUF_T, v);
            if (a.h0row) {
                const R Ky = (R)S->kap[1], Kz = (R)S->kap[2], s = (R)S->inv_n;
                const double dk = S->dk[0];
                if (a.expo) {
#pragma unroll
                    for (int m = 0; m < E; ++m)
                        apply_expo(v[0][m], v[1][m], v[2][m], v[3][m], dk * kindex(t + T * m, N), S->kap[1], S->kap[2],
                                   a.tau, S->inv_n);
                } else {
#pragma unroll
                    for (int m = 0; m < E; ++m) {
                        const R Kx = (R)(dk * kindex(t + T * m, N));
                        apply_h0(v[0][m], v[1][m], v[2][m], v[3][m], Kx, Ky, Kz, s);
                    }
                }
            }
            fft4<C, N, T, +1, CG, VC::SEQ, Lay, typename VC::PL>(v, lds, t, line, tw);
        }
        if constexpr (MODE == ROW_INV) {
            store(a.dst, v);
            return;
        } else {
            // ---- stage epilogue: k = K - i V(t_i) (y_i + psi_b(t_i))
            double ts;
            if constexpr (MODE == ROW_RHS) {
                ts = a.t_explicit;
            } else {
                const double cst = a.stage == 0 ? 0.0 : (a.stage == 3 ? 1.0 : 0.5);
                ts = a.t_out - (double)(*a.step) * a.dt - cst * a.dt;
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
            if (t == 0) sh_phyz[line] = cmul(gload<C>(ctab, S->ph + n0 + yy), gload<C>(ctab, S->ph + n0 + n1 + zz));
            {
                // state loads are independent of the barrier below: issue them first
                C yi[4][E];
                load(a.src, yi);
                __syncthreads();
                // field A_mu on this line's points
                R A[4][E];
#pragma unroll
                for (int mu = 0; mu < 4; ++mu)
#pragma unroll
                    for (int m = 0; m < E; ++m) A[mu][m] = (R)0;
#pragma unroll
                for (int j = 0; j < MAX_TERMS; ++j) {
                    if (j < nterm) {
                        const R fyz = sh_fyz[line][j];
                        gptr<const R> tab = rtab + sh_tab[j] + t;
                        const int mu = sh_mu[j];
#pragma unroll
                        for (int m = 0; m < E; ++m) {
                            const R f = fyz * tab[T * m];
                            A[0][m] += mu == 0 ? f : (R)0;
                            A[1][m] += mu == 1 ? f : (R)0;
                            A[2][m] += mu == 2 ? f : (R)0;
                            A[3][m] += mu == 3 ? f : (R)0;
                        }
                    }
                }
                const long long phx = S->ph + t;
                const C wc[4] = {sh_wc[0], sh_wc[1], sh_wc[2], sh_wc[3]};
                const C phyz = sh_phyz[line];
#pragma unroll
                for (int m = 0; m < E; ++m) {
                    const C ph = cmul(gload<C>(ctab, phx + T * m), phyz);
                    C sv[4], vs[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) sv[q] = cadd(yi[q][m], cmul(wc[q], ph));
                    apply_pot(sv, vs, A[0][m], A[1][m], A[2][m], A[3][m]);
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q][m] = cadd(v[q][m], cmul_mi(vs[q]));   // v = k
                }
                store(a.dst, v);
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
    __shared__ C tw[N];

    const int tid = threadIdx.x;
    const int xl = tid % W;
    const int t = tid / W;

    // One tile = W adjacent columns of one solve at one fixed other-axis index.
    const int2 it = a.items[blockIdx.x];
    const SolveDev* __restrict__ S = a.solves + it.x;
    const int n0 = S->n[0], n1 = S->n[1];
    const int ntx = (n0 + W - 1) / W;
    const int other = it.y / ntx;
    const int x = (it.y % ntx) * W + xl;
    const bool act = x < n0;
    const long long stride = AXIS == 1 ? (long long)n0 : (long long)n0 * n1;
    const long long obase = AXIS == 1 ? (long long)other * n0 * n1 : (long long)other * n0;
    const long long base = obase + (act ? x : 0) + (long long)t * stride;
    const long long ns = S->nsites;

    gptr<const nv2<R>> ctab = cview<R>(a.ctab);
    for (int i = tid; i < N; i += VC::THREADS) tw[i] = gload<C>(ctab, S->tw[AXIS] + i);

    C v[4][E];
    {
        gptr<const nv2<R>> p = cview<R>(S->buf[a.dst]) + base;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) v[q][m] = gload<C>(p, q * ns + (long long)(T * m) * stride);
    }
    if constexpr (MODE == COL_FWD || MODE == COL_H0) fft4<C, N, T, -1, CG, VC::SEQ, Lay, typename VC::PL>(v, lds, t, xl, tw);
    if constexpr (MODE == COL_H0) {
        const double kx = S->dk[0] * kindex(act ? x : 0, n0);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int idx = t + T * m;
            double ky, kz;
            if constexpr (AXIS == 1) {
                ky = S->dk[1] * kindex(idx, N);
                kz = S->kap[2];
            } else {
                ky = S->dk[1] * kindex(other, n1);
                kz = S->dk[2] * kindex(idx, N);
            }
            if (a.expo) apply_expo(v[0][m], v[1][m], v[2][m], v[3][m], kx, ky, kz, a.tau, S->inv_n);
            else apply_h0(v[0][m], v[1][m], v[2][m], v[3][m], (R)kx, (R)ky, (R)kz, (R)S->inv_n);
        }
    }
    if constexpr (MODE == COL_INV || MODE == COL_H0) fft4<C, N, T, +1, CG, VC::SEQ, Lay, typename VC::PL>(v, lds, t, xl, tw);
    if (act) {
        gptr<nv2<R>> p = wview<R>(S->buf[a.dst]) + base;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) gstore<C>(p, q * ns + (long long)(T * m) * stride, v[q][m]);
    }
}

// ------------------------------------------------------------------ stepping passes
// Source component and phase of the alpha^j entries (Dirac representation):
// (alpha^1 y)_q = y_{3-q}; (alpha^2 y)_q = (-i for even q, +i for odd q) y_{3-q};
// (alpha^3 y)_q = (+1 for q = 0, 2; -1 for q = 1, 3) y_{q^2}; beta = diag(1, 1, -1, -1).
template <class C> __device__ __forceinline__ C alpha2_phase(int q, C v) { return (q & 1) ? cmul_i(v) : cmul_mi(v); }
template <class C> __device__ __forceinline__ C alpha3_phase(int q, C v) { return (q & 1) ? cmake<C>(-v.x, -v.y) : v; }

// Column derivative pass: the blocks of blockIdx.y = q transform the
// component alpha^j takes for output component q along axis j = AXIS (y or
// z), multiply by k_j / n_j, transform back, and write (ACCUM = 0) or add
// (ACCUM = 1) the result, with alpha^j's phase, into component q of the G
// buffer (a.dst).  a.src: the stage input.  One component per thread: E
// points of the transform in registers.
//   v0: default plan, one 128-byte line of x per tile;  v1: few-points plan, one line;
//   v2: few-points plan, two lines;                      v3: default plan, two lines.
template <class R, int N, int V> struct CdVar {
    static constexpr int WANT = sizeof(R) == 4 ? 16 : 8;   // columns per 128-byte line
    static constexpr bool SMALL = (V == 1 || V == 2) && has_small_plan<N>();
    using PL = typename PlanSel<N, SMALL>::type;
    static constexpr int T = PL::T;
    static constexpr int E = N / T;
    // widest power-of-two tile whose exchange buffer fits the LDS with the twiddles
    static constexpr int WFIT = (int)((163840 - N * sizeof(cpx<R>) - 1024) / (N * sizeof(cpx<R>)));
    static constexpr int WMAX = WFIT >= 32 ? 32 : (WFIT >= 16 ? 16 : (WFIT >= 8 ? 8 : (WFIT >= 4 ? 4 : 2)));
    static constexpr int W = imax(1, imin(imin(WANT * (V >= 2 ? 2 : 1), 1024 / T), WMAX));
    static constexpr int THREADS = T * W;
    static constexpr size_t BYTES = (size_t)N * W * sizeof(cpx<R>);
    // A tile whose exchange buffer and twiddles leave room for only one
    // workgroup per compute unit (160 KB of LDS) would leave HBM idle while it
    // transforms; those y passes run as a persistent loop over the tiles that
    // loads the next tile while this one is transformed.  Only where the
    // workgroup has at most 512 threads (with more, the prefetch would spill)
    // and the tile is at most 8 columns wide: every lattice length is a
    // multiple of 8, so such tiles are never partial.
    static constexpr bool PIPE = 2 * (BYTES + N * sizeof(cpx<R>)) > 163840 && THREADS <= 512 && 8 % W == 0;
    static_assert(plan_ok<N, T, PL>(), "column derivative variant violates the FFT plan constraints");
};

template <class R, int N, int V, int AXIS, int ACCUM>
__global__ void __launch_bounds__((CdVar<R, N, V>::THREADS)) col_d_kernel(PassArgs a) {
    using C = cpx<R>;
    using VC = CdVar<R, N, V>;
    constexpr int T = VC::T;
    constexpr int W = VC::W;
    constexpr int E = VC::E;
    using Lay = ColLay<N, W>;
    using PL = typename VC::PL;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* lds = reinterpret_cast<C*>(smem_raw);
    __shared__ C tw[N];

    const int tid = threadIdx.x;
    const int xl = tid % W;
    const int t = tid / W;
    const int q = blockIdx.y;                       // output component
    const int src = AXIS == 1 ? 3 - q : (q ^ 2);    // the component alpha^j takes
    // (the persistent loop only for the y pass: the z pass's partial sums would
    // double the registers a prefetch holds)
    constexpr bool PIPE = VC::PIPE && !ACCUM;
    if constexpr (!PIPE) {
        // one tile = W adjacent columns of one solve at one fixed other-axis index
        const int2 it = a.items[blockIdx.x];
        const SolveDev* __restrict__ S = a.solves + it.x;
        const int n0 = S->n[0], n1 = S->n[1];
        const int ntx = (n0 + W - 1) / W;
        const int other = it.y / ntx;
        const int x = (it.y % ntx) * W + xl;
        const bool act = x < n0;
        const long long stride = AXIS == 1 ? (long long)n0 : (long long)n0 * n1;
        const long long obase = AXIS == 1 ? (long long)other * n0 * n1 : (long long)other * n0;
        const long long base = obase + (act ? x : 0) + (long long)t * stride;
        const long long ns = S->nsites;
        gptr<const nv2<R>> ctab = cview<R>(a.ctab);
        for (int i = tid; i < N; i += VC::THREADS) tw[i] = gload<C>(ctab, S->tw[AXIS] + i);

        C v[1][E];
        C g[E];
        {
            gptr<const nv2<R>> p = cview<R>(S->buf[a.src]) + base + src * ns;
#pragma unroll
            for (int m = 0; m < E; ++m) v[0][m] = gload_nt<C>(p, (long long)(T * m) * stride);
            if constexpr (ACCUM) {
                // the partial sum of the earlier axis, loaded ahead of the transforms
                gptr<const nv2<R>> pg = cview<R>(S->buf[a.dst]) + base + q * ns;
#pragma unroll
                for (int m = 0; m < E; ++m) g[m] = gload_nt<C>(pg, (long long)(T * m) * stride);
            }
        }
        fft_line<C, N, T, -1, 1, 1, Lay, PL>(v, lds, t, xl, tw);
        const double kscale = S->dk[AXIS] / (double)N;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const C w = cscale(v[0][m], (R)(kscale * kindex(t + T * m, N)));
            v[0][m] = AXIS == 1 ? alpha2_phase(q, w) : alpha3_phase(q, w);
        }
        fft_line<C, N, T, +1, 1, 1, Lay, PL>(v, lds, t, xl, tw);
        if (act) {
            gptr<nv2<R>> p = wview<R>(S->buf[a.dst]) + base + q * ns;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                const C o = ACCUM ? cadd(g[m], v[0][m]) : v[0][m];
                gstore_nt<C>(p, (long long)(T * m) * stride, o);
            }
        }
    } else {
        // Every solve of a launch has the same lengths (so the same twiddles); a
        // tile's own descriptor words (its item and its solve's arrays) are read
        // through the constant address space, as scalar loads, which do not wait
        // for the previous tile's stores still in flight.
        const SolveDev* S0 = a.solves + a.items[blockIdx.x].x;
        const int n0 = S0->n[0], n1 = S0->n[1];
        const int ntx = (n0 + W - 1) / W;
        const long long ns = S0->nsites;
        const long long stride = AXIS == 1 ? (long long)n0 : (long long)n0 * n1;
        const double kscale = S0->dk[AXIS] / (double)N;
        gptr<const nv2<R>> ctab = cview<R>(a.ctab);
        for (int i = tid; i < N; i += VC::THREADS) tw[i] = gload<C>(ctab, S0->tw[AXIS] + i);
        using cword = const unsigned long long __attribute__((address_space(4)))*;
        struct Tile {
            unsigned long long src, dst;   // the solve's stage input and G arrays
            long long base;
            bool act;
        };
        auto tile = [&](int item) {
            const unsigned long long w = *(cword)(a.items + item);
            const int solve = (int)(unsigned)w, ty = (int)(w >> 32);
            const int other = ty / ntx;
            const int x = (ty % ntx) * W + xl;
            Tile u;
            // (no partial persistent tiles: their stores need no branch)
            u.act = PIPE || x < n0;
            const long long obase = AXIS == 1 ? (long long)other * n0 * n1 : (long long)other * n0;
            u.base = obase + (u.act ? x : 0) + (long long)t * stride;
            const SolveDev* S = a.solves + solve;
            u.src = *(cword)(&S->buf[a.src]);
            u.dst = *(cword)(&S->buf[a.dst]);
            return u;
        };
        auto load = [&](const Tile& u, C (&v)[E], C (&g)[E]) {
            gptr<const nv2<R>> p = cview<R>((const void*)u.src) + u.base + src * ns;
    #pragma unroll
            for (int m = 0; m < E; ++m) v[m] = gload_nt<C>(p, (long long)(T * m) * stride);
            if constexpr (ACCUM) {
                // the partial sum of the earlier axis, loaded ahead of the transforms
                gptr<const nv2<R>> pg = cview<R>((const void*)u.dst) + u.base + q * ns;
    #pragma unroll
                for (int m = 0; m < E; ++m) g[m] = gload_nt<C>(pg, (long long)(T * m) * stride);
            }
        };

        // Order of a persistent iteration: issue the next tile's loads, transform
        // this tile, store it, then take the next tile's values (waiting for its
        // loads but not for the stores just issued).  The first tile's loads are
        // waited for before the loop, so that at the loop's top only stores are
        // in flight and nothing there waits for them.
        int item = blockIdx.x;
        Tile u = tile(item);
        C v[1][E], g[E];
        load(u, v[0], g);
        if constexpr (PIPE) {
    #pragma unroll
            for (int m = 0; m < E; ++m) asm volatile("" ::"v"(v[0][m].x), "v"(v[0][m].y));
        }
        for (;;) {
            const int next = item + (int)gridDim.x;
            const bool more = PIPE && next < a.nitems;
            Tile un;
            C vn[E], gn[E];
            if (more) {
                un = tile(next);
                load(un, vn, gn);
            }
            fft_line<C, N, T, -1, 1, 1, Lay, PL>(v, lds, t, xl, tw);
    #pragma unroll
            for (int m = 0; m < E; ++m) {
                const C w = cscale(v[0][m], (R)(kscale * kindex(t + T * m, N)));
                v[0][m] = AXIS == 1 ? alpha2_phase(q, w) : alpha3_phase(q, w);
            }
            fft_line<C, N, T, +1, 1, 1, Lay, PL>(v, lds, t, xl, tw);
            if (u.act) {
                gptr<nv2<R>> p = wview<R>((void*)u.dst) + u.base + q * ns;
    #pragma unroll
                for (int m = 0; m < E; ++m) {
                    const C o = ACCUM ? cadd(g[m], v[0][m]) : v[0][m];
                    gstore_nt<C>(p, (long long)(T * m) * stride, o);
                }
            }
            if (!more) break;
            item = next;
            u = un;
    #pragma unroll
            for (int m = 0; m < E; ++m) {
                v[0][m] = vn[m];
                g[m] = gn[m];
            }
        }
    }
}

// Row (x) stage pass: the RK4 stage STAGE for one spinor component per
// thread.  T threads share a component line (E = N/T points each), 4T a
// grid line.  A thread reads its own component of the stage input y_i and
// exchanges it through LDS for the two it also needs (3 - q and q ^ 2, the
// partners alpha^j couples q to), transforms component 3 - q along x,
// multiplies by k_x / n_0 and transforms back, which gives (alpha^1 D_x y)_q,
// and then finishes its own component at its points:
//     k_q = -i [alpha^1 D_x y + G + (beta y) + sum over trivial axes kappa_j (alpha^j y)
//               + (A_0 + alpha^j A_j)(y + psi_b)]_q,
// the RK4 update of component q with the accumulator written once, and the
// absorber at the last stage.  STAGE 4..9 are the six stages of the
// fixed-step Dormand-Prince 5(4) stepper instead: the stage writes its slope
// k_s and the next stage input y + h sum_{j<=s} a_{s+1,j} k_j (reading the
// earlier slopes), the last one the step y + h sum_j b_j k_j.
//   v0 / v1: few-points plan, 256 / 128 threads per block;
//   v2 / v3 (SITE): few-points / default plan, 256 / 128 threads: the thread
//   reads component 3 - q of the stage input for the transform straight from
//   memory, leaves (alpha^1 D_x y)_q in LDS, and finishes whole sites (all
//   four components of the sites t + T m, m = q, q+4, ...), reading the
//   stage input there again, so the field and phase work is done once per site.
template <class R, int N, int V> struct RdVar {
    static constexpr bool SITE = V >= 2;
    static constexpr bool SMALL = (V <= 2) && has_small_plan<N>();
    using PL = typename PlanSel<N, SMALL>::type;
    static constexpr int T = PL::T;
    static constexpr int E = N / T;
    static constexpr int ROWS = imax(1, ((V % 2) == 0 ? 256 : 128) / (4 * T));
    static constexpr int THREADS = 4 * T * ROWS;
    using Lay = RowLay<N, 4 * ROWS>;
    static constexpr size_t BYTES = (size_t)4 * ROWS * Lay::STRIDE * sizeof(cpx<R>);
    // waves per SIMD the compiler is asked to fit: what the LDS of a compute
    // unit (160 KiB) allows, at most 2 in double (four components' worth of
    // points stay live) and 4 in single precision
    static constexpr int BLOCKS_PER_CU = (int)(163840 / (BYTES + N * sizeof(cpx<R>) + 512));
    static constexpr int WAVES = imax(1, imin(SITE ? 4 : (sizeof(R) == 8 ? 2 : 4), BLOCKS_PER_CU * (THREADS / 64) / 4));
    static_assert(plan_ok<N, T, PL>(), "row derivative variant violates the FFT plan constraints");
    static_assert(THREADS <= 1024, "row derivative block too large");
};

template <class R, int N, int V, int STAGE>
__global__ void __launch_bounds__((RdVar<R, N, V>::THREADS))
__attribute__((amdgpu_waves_per_eu(RdVar<R, N, V>::WAVES, 8))) row_d_kernel(PassArgs a) {
    using C = cpx<R>;
    using VC = RdVar<R, N, V>;
    constexpr int T = VC::T;
    constexpr int E = VC::E;
    constexpr int ROWS = VC::ROWS;
    using Lay = typename VC::Lay;
    using PL = typename VC::PL;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* lds = reinterpret_cast<C*>(smem_raw);
    __shared__ R sh_fyz[ROWS][MAX_TERMS];
    __shared__ int sh_mu[MAX_TERMS];
    __shared__ long long sh_tab[MAX_TERMS];
    __shared__ C sh_wc[4];
    __shared__ C sh_phyz[ROWS];
    __shared__ C tw[N];

    const int tid = threadIdx.x;
    const int t = tid % T;
    const int q = (tid / T) % 4;
    const int line = tid / (4 * T);
    const int qx = 3 - q, qz = q ^ 2;
    const int2 it = a.items[blockIdx.x];
    const SolveDev* __restrict__ S = a.solves + it.x;
    const int row = it.y * ROWS + line;
    const bool act = row < S->nrows;
    const int rowc = act ? row : 0;
    const long long base = (long long)rowc * N;
    const long long ns = S->nsites;
    gptr<const nv2<R>> ctab = cview<R>(a.ctab);
    gptr<const R> rtab = glob(reinterpret_cast<const R*>(a.rtab));
    for (int i = tid; i < N; i += VC::THREADS) tw[i] = gload<C>(ctab, S->tw[0] + i);
    const int n0 = S->n[0], n1 = S->n[1];
    const int yy = rowc % n1, zz = rowc / n1;

    // STAGE 0..3: classical RK4 stages; 4..9: Dormand-Prince stages 0..5
    constexpr bool DP = STAGE >= 4;
    constexpr int DS = DP ? STAGE - 4 : 0;
    constexpr bool FIRST = STAGE == 0 || STAGE == 4, LAST = STAGE == 3 || STAGE == 9;
    gptr<const nv2<R>> pin = cview<R>(S->buf[FIRST ? BUF_Y : BUF_YS]) + base;
    C v[1][E];
    C yq[E], yx[E], yz[E];
    if constexpr (VC::SITE) {
        // the component alpha^1 takes, straight from memory (read again by the epilogue)
#pragma unroll
        for (int m = 0; m < E; ++m) v[0][m] = gload<C>(pin, qx * ns + t + T * m);
    } else {
        // own component of the stage input
#pragma unroll
        for (int m = 0; m < E; ++m) yq[m] = gload_nt<C>(pin, q * ns + t + T * m);
    }
    // per-line constants of the stage time (read after the barriers below)
    constexpr double cst = DP ? dp5_c(DS) : (STAGE == 0 ? 0.0 : (STAGE == 3 ? 1.0 : 0.5));
    const double ts = a.t_out - (double)(*a.step) * a.dt - cst * a.dt;
    const int nterm = S->nterm;
    if (q == 0) {
        for (int j = t; j < nterm; j += T) {
            const TermDev tm = a.terms[S->term0 + j];
            const double coef = tm.amp * profile_t(tm.ft_type, tm.c, tm.w, tm.k, tm.phi, ts);
            sh_fyz[line][j] = (R)coef * rtab[tm.tab + n0 + yy] * rtab[tm.tab + n0 + n1 + zz];
            if (line == 0) {
                sh_mu[j] = tm.mu;
                sh_tab[j] = tm.tab;
            }
        }
        if (t == 0) sh_phyz[line] = cmul(gload<C>(ctab, S->ph + n0 + yy), gload<C>(ctab, S->ph + n0 + n1 + zz));
    }
    if (tid < 4) {
        double sn, cs;
        sincos(-S->E * ts, &sn, &cs);
        const double wr = S->w[2 * tid], wi = S->w[2 * tid + 1];
        sh_wc[tid] = cmake<C>((R)(wr * cs - wi * sn), (R)(wr * sn + wi * cs));
    }
    if constexpr (!VC::SITE) {
        // the partner components through LDS
#pragma unroll
        for (int m = 0; m < E; ++m) lds[Lay::addr(0, 4 * line + q, t + T * m)] = yq[m];
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) {
            yx[m] = lds[Lay::addr(0, 4 * line + qx, t + T * m)];
            yz[m] = lds[Lay::addr(0, 4 * line + qz, t + T * m)];
            v[0][m] = yx[m];
        }
    }
    // (alpha^1 D_x y)_q: the first exchange's barrier orders the reads above
    // before the transform reuses the LDS
    fft_line<C, N, T, -1, 1, 1, Lay, PL>(v, lds, t, 4 * line + q, tw);
    const double kscale = S->dk[0] / (double)N;
#pragma unroll
    for (int m = 0; m < E; ++m) v[0][m] = cscale(v[0][m], (R)(kscale * kindex(t + T * m, N)));
    fft_line<C, N, T, +1, 1, 1, Lay, PL>(v, lds, t, 4 * line + q, tw);

    // ---- stage epilogue
    const R h = (R)(-a.dt);
    const R h2 = (R)(-0.5 * a.dt), h6 = (R)(-a.dt / 6.0), third = (R)(1.0 / 3.0);
    const C phyz = sh_phyz[line];
    const R ky = (R)S->kap[1], kz = (R)S->kap[2];   // zero on non-trivial axes
    const bool has_g = S->dim >= 2;
    const long long mask = S->mask;
    const R myz = (LAST && mask >= 0) ? rtab[mask + n0 + yy] * rtab[mask + n0 + n1 + zz] : (R)1;
    // Dormand-Prince: slope k_j of the stage input's sum, at offset off of the line
    auto dp5_prev = [&](C acc, long long off) {
#pragma unroll
        for (int j = 0; j < DS; ++j)
            if (dp5_a(DS + 1, j) != 0.0)
                acc = cadd(acc, cscale(gload_nt<C>(cview<R>(S->buf[dp5_kbuf(j)]) + base, off), (R)(-a.dt * dp5_a(DS + 1, j))));
        return acc;
    };
    const R hk = (R)(-a.dt * dp5_a(DS + 1, DS));   // h a_{s+1,s} for the stage's own slope
    // field A_mu at point idx of this line
    auto field = [&](int idx, R (&A)[4]) {
        A[0] = A[1] = A[2] = A[3] = (R)0;
#pragma unroll
        for (int jt = 0; jt < MAX_TERMS; ++jt) {
            if (jt < nterm) {
                const R f = sh_fyz[line][jt] * rtab[sh_tab[jt] + idx];
                const int mu = sh_mu[jt];
                A[0] += mu == 0 ? f : (R)0;
                A[1] += mu == 1 ? f : (R)0;
                A[2] += mu == 2 ? f : (R)0;
                A[3] += mu == 3 ? f : (R)0;
            }
        }
    };
    if constexpr (VC::SITE) {
        // whole sites: (alpha^1 D_x y) of all four components through LDS
        __syncthreads();
#pragma unroll
        for (int m = 0; m < E; ++m) lds[Lay::addr(0, 4 * line + q, t + T * m)] = v[0][m];
        __syncthreads();
        const C wc[4] = {sh_wc[0], sh_wc[1], sh_wc[2], sh_wc[3]};
        gptr<const nv2<R>> pg = cview<R>(S->buf[BUF_T]) + base;
        gptr<const nv2<R>> pop = cview<R>(S->buf[STAGE == 3 ? BUF_ACC : BUF_Y]) + base;
        gptr<nv2<R>> wys = wview<R>(S->buf[BUF_YS]) + base;
        gptr<nv2<R>> wk = wview<R>(S->buf[dp5_kbuf(DS < 5 ? DS : 0)]) + base;
        gptr<nv2<R>> wacc = wview<R>(S->buf[BUF_ACC]) + base;
        gptr<nv2<R>> wy = wview<R>(S->buf[BUF_Y]) + base;
#pragma unroll
        for (int j = 0; j < (E + 3) / 4; ++j) {
            const int m = q + 4 * j;
            if (m < E) {
                const int idx = t + T * m;
                C y[4], g[4], y0[4], u[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    y[c] = gload_nt<C>(pin, c * ns + idx);
                    g[c] = has_g ? gload_nt<C>(pg, c * ns + idx) : cmake<C>((R)0, (R)0);
                    y0[c] = FIRST ? cmake<C>((R)0, (R)0) : gload_nt<C>(pop, c * ns + idx);
                }
                R A[4];
                field(idx, A);
                const C ph = cmul(gload<C>(ctab, S->ph + idx), phyz);
                C sv[4], vs[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) sv[c] = cadd(y[c], cmul(wc[c], ph));
                apply_pot(sv, vs, A[0], A[1], A[2], A[3]);
                const R mk = (LAST && mask >= 0) ? rtab[mask + idx] * myz : (R)1;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const R bc = c < 2 ? (R)1 : (R)-1;
                    C w = cadd(cadd(lds[Lay::addr(0, 4 * line + c, idx)], g[c]), cscale(y[c], bc));
                    w = cadd(w, cadd(cscale(alpha2_phase(c, y[3 - c]), ky), cscale(alpha3_phase(c, y[c ^ 2]), kz)));
                    u[c] = cmul_mi(cadd(w, vs[c]));   // k_c
                }
                // classical RK4 with the accumulator written once: with the stage
                // inputs y_2 = y + h/2 k1, y_3 = y + h/2 k2, y_4 = y + h k3,
                //   y_{n+1} = (y_2 + 2 y_3 - y)/3 + y_4/3 + h/6 k4,
                // so stage 1 stores acc = (y_2 + 2 y_3 - y)/3 and stage 3 finishes
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const C k = u[c];
                    if constexpr (DP) {
                        // Dormand-Prince: y_{s+1} = y + h sum_{j<=s} a_{s+1,j} k_j (row 6: the step)
                        const C yn = cadd(dp5_prev(DS == 0 ? y[c] : y0[c], c * ns + idx), cscale(k, hk));
                        if (act) {
                            if constexpr (DS < 5) {
                                gstore_nt<C>(wk, c * ns + idx, k);
                                gstore_nt<C>(wys, c * ns + idx, yn);
                            } else {
                                gstore_nt<C>(wy, c * ns + idx, cscale(yn, mk));
                            }
                        }
                    } else if constexpr (STAGE == 0) {
                        if (act) gstore_nt<C>(wys, c * ns + idx, cadd(y[c], cscale(k, h2)));             // y_2
                    } else if constexpr (STAGE == 1) {
                        const C y3 = cadd(y0[c], cscale(k, h2));                                          // y_3
                        if (act) {
                            gstore_nt<C>(wacc, c * ns + idx, cscale(csub(cadd(y[c], cscale(y3, (R)2)), y0[c]), third));
                            gstore_nt<C>(wys, c * ns + idx, y3);
                        }
                    } else if constexpr (STAGE == 2) {
                        if (act) gstore_nt<C>(wys, c * ns + idx, cadd(y0[c], cscale(k, h)));             // y_4
                    } else {
                        if (act) gstore_nt<C>(wy, c * ns + idx, cscale(cadd(cadd(y0[c], cscale(y[c], third)), cscale(k, h6)), mk));
                    }
                }
            }
        }
    } else {
        // component q at the thread's own points
        const C wq = sh_wc[q], wx = sh_wc[qx], wz = sh_wc[qz];
        const R bq = q < 2 ? (R)1 : (R)-1;
        gptr<const nv2<R>> pg = cview<R>(S->buf[BUF_T]) + base + q * ns + t;
        gptr<const nv2<R>> py = cview<R>(S->buf[BUF_Y]) + base + q * ns + t;
        gptr<const nv2<R>> pacc = cview<R>(S->buf[BUF_ACC]) + base + q * ns + t;
        gptr<nv2<R>> wys = wview<R>(S->buf[BUF_YS]) + base + q * ns + t;
        gptr<nv2<R>> wacc = wview<R>(S->buf[BUF_ACC]) + base + q * ns + t;
        gptr<nv2<R>> wy = wview<R>(S->buf[BUF_Y]) + base + q * ns + t;
        gptr<nv2<R>> wk = wview<R>(S->buf[dp5_kbuf(DS < 5 ? DS : 0)]) + base + q * ns + t;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int idx = t + T * m;
            const C g = has_g ? gload_nt<C>(pg, T * m) : cmake<C>((R)0, (R)0);
            C y0 = cmake<C>((R)0, (R)0);
            if constexpr (STAGE == 1 || STAGE == 2 || (DP && DS > 0)) y0 = gload_nt<C>(py, T * m);
            if constexpr (STAGE == 3) y0 = gload_nt<C>(pacc, T * m);
            R A[4];
            field(idx, A);
            const C ph = cmul(gload<C>(ctab, S->ph + idx), phyz);
            // y + psi_b on the three components
            const C sq = cadd(yq[m], cmul(wq, ph)), sx = cadd(yx[m], cmul(wx, ph)), sz = cadd(yz[m], cmul(wz, ph));
            // [alpha^1 D_x y + G + beta y + kappa terms + A0 s + (A1 alpha^1 + A2 alpha^2) s + A3 alpha^3 s]_q
            C u = cadd(cadd(v[0][m], g), cscale(yq[m], bq));
            u = cadd(u, cadd(cscale(alpha2_phase(q, yx[m]), ky), cscale(alpha3_phase(q, yz[m]), kz)));
            u = cadd(u, cscale(sq, A[0]));
            u = cadd(u, cadd(cscale(sx, A[1]), cscale(alpha2_phase(q, sx), A[2])));
            u = cadd(u, cscale(alpha3_phase(q, sz), A[3]));
            const C k = cmul_mi(u);
            // classical RK4 with the accumulator written once (as above)
            if constexpr (DP) {
                const C yn = cadd(dp5_prev(DS == 0 ? yq[m] : y0, q * ns + idx), cscale(k, hk));
                if (act) {
                    if constexpr (DS < 5) {
                        gstore_nt<C>(wk, T * m, k);
                        gstore_nt<C>(wys, T * m, yn);
                    } else {
                        const R mk = mask >= 0 ? rtab[mask + idx] * myz : (R)1;
                        gstore_nt<C>(wy, T * m, cscale(yn, mk));
                    }
                }
            } else if constexpr (STAGE == 0) {
                if (act) gstore_nt<C>(wys, T * m, cadd(yq[m], cscale(k, h2)));                    // y_2
            } else if constexpr (STAGE == 1) {
                const C y3 = cadd(y0, cscale(k, h2));                                              // y_3
                if (act) {
                    gstore_nt<C>(wacc, T * m, cscale(csub(cadd(yq[m], cscale(y3, (R)2)), y0), third));
                    gstore_nt<C>(wys, T * m, y3);
                }
            } else if constexpr (STAGE == 2) {
                if (act) gstore_nt<C>(wys, T * m, cadd(y0, cscale(k, h)));                          // y_4
            } else {
                const R mk = mask >= 0 ? rtab[mask + idx] * myz : (R)1;
                if (act) gstore_nt<C>(wy, T * m, cscale(cadd(cadd(y0, cscale(yq[m], third)), cscale(k, h6)), mk));
            }
        }
    }
}

// ------------------------------------------------------------------ 1D whole-loop kernel
// A (1+1)D solve is one line of at most 1024 points: its whole state fits on
// one compute unit.  line_kernel runs a.nsteps complete RK4 steps of one solve
// per workgroup without leaving the chip: the state y and the stage input stay
// in registers, the running RK4 sum in thread-private LDS slots, and each stage
// transforms the line forward, multiplies by -i H0(k)/N and transforms back
// through LDS.  Only the final state is written to the Y array.  The update is
// the classical y_{n+1} = y + h/6 (k1 + 2 k2 + 2 k3 + k4) with h = -dt,
// accumulated stage by stage.  Field profiles, background phases, the absorber
// mask and the twiddles are staged in LDS once per launch; the per-stage time
// factors are evaluated in double by a few lanes and broadcast through LDS.
// WIDE: the exchange rounds move CGW components at once (fewer barriers, more
// LDS); otherwise half as many.  The host takes the wide build where its LDS,
// with the field's profile tables, fits.
template <class R, int N, bool WIDE> struct LineVar {
    using PL = Plan4<N>;
    static constexpr int T = PL::T;
    static constexpr int E = N / T;
    using Lay = RowLay<N, 1>;
    static constexpr int CGW = sizeof(R) == 8 ? 2 : 4;
    static constexpr int CG = WIDE ? CGW : CGW / 2;
    static constexpr size_t XCH = CG * (size_t)Lay::STRIDE * sizeof(cpx<R>);
    // dynamic LDS without the field profiles: exchange, twiddles, phases,
    // RK4 sum, mask (the host adds nterm * N reals)
    static constexpr size_t BASE_BYTES = XCH + 2 * N * sizeof(cpx<R>) + 4 * N * sizeof(cpx<R>) + N * sizeof(R);
    static_assert(PL::NR >= 2, "the stage broadcast relies on the barriers of the exchanges");
    static_assert(plan_ok<N, T, PL>(), "line plan violates the FFT plan constraints");
};

// A zero the compiler cannot see through.  Offsetting the lane index with it
// once per transform keeps the (loop-invariant) exchange addresses from being
// hoisted out of the time loop into registers.
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

template <class R, int N, bool WIDE>
__global__ void __launch_bounds__((LineVar<R, N, WIDE>::T)) line_kernel(PassArgs a) {
    using C = cpx<R>;
    using VC = LineVar<R, N, WIDE>;
    constexpr int T = VC::T;
    constexpr int E = VC::E;
    constexpr int CG = VC::CG;
    using Lay = typename VC::Lay;
    using PL = typename VC::PL;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    C* xch = reinterpret_cast<C*>(smem_raw);
    C* tw = reinterpret_cast<C*>(smem_raw + VC::XCH);
    C* phx = tw + N;                               // exp(i K.x) on the line (trivial axes folded in)
    C* accl = phx + N;                             // RK4 sum, [q][m][lane]
    R* msk = reinterpret_cast<R*>(accl + 4 * N);   // absorber mask (1 if off)
    R* fx = msk + N;                               // spatial profile of each field term
    __shared__ R sh_coef[2][MAX_TERMS];            // amp * f_t(t) per term, double-buffered by stage
    __shared__ C sh_wc[2][4];                      // background spinor * exp(-i E t)
    __shared__ int sh_mu[MAX_TERMS];

    const int t = threadIdx.x;
    const SolveDev* __restrict__ S = a.solves + a.items[blockIdx.x].x;
    gptr<const nv2<R>> ctab = cview<R>(a.ctab);
    gptr<const R> rtab = glob(reinterpret_cast<const R*>(a.rtab));
    const int nterm = S->nterm;
    {
        // trivial axes (index 0 of each): constant factors of the tables
        const C phyz = cmul(gload<C>(ctab, S->ph + N), gload<C>(ctab, S->ph + N + 1));
        const long long mk = S->mask;
        const R myz = mk >= 0 ? rtab[mk + N] * rtab[mk + N + 1] : (R)1;
        for (int i = t; i < N; i += T) {
            tw[i] = gload<C>(ctab, S->tw[0] + i);
            phx[i] = cmul(gload<C>(ctab, S->ph + i), phyz);
            msk[i] = mk >= 0 ? rtab[mk + i] * myz : (R)1;
        }
        for (int j = 0; j < nterm; ++j) {
            const long long tb = a.terms[S->term0 + j].tab;
            const R fyz = rtab[tb + N] * rtab[tb + N + 1];
            for (int i = t; i < N; i += T) fx[j * N + i] = rtab[tb + i] * fyz;
        }
        if (t < nterm) sh_mu[t] = a.terms[S->term0 + t].mu;
    }
    C y[4][E];
    {
        gptr<const nv2<R>> p = cview<R>(S->buf[BUF_Y]) + t;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) y[q][m] = gload<C>(p, q * (long long)N + T * m);
    }
    __syncthreads();

    const R Ky = (R)S->kap[1], Kz = (R)S->kap[2], inv_n = (R)S->inv_n;
    const double dk = S->dk[0];
    const double dt = a.dt;
    const R h = (R)(-dt), h2 = (R)(-0.5 * dt), h3 = (R)(-dt / 3.0), h6 = (R)(-dt / 6.0);
    const int n_first = *a.step;

    // v = IFFT[-i H0 FFT(yi)]/N - i V(ts) (yi + psi_b(ts)); par selects the
    // broadcast buffer of this stage
    auto rhs = [&](const C (&yi)[4][E], C (&v)[4][E], double ts, int par) {
        for (int j = t; j < nterm; j += T) {
            const TermDev tm = a.terms[S->term0 + j];
            sh_coef[par][j] = (R)(tm.amp * profile_t(tm.ft_type, tm.c, tm.w, tm.k, tm.phi, ts));
        }
        if (t >= T - 4) {
            const int q = t - (T - 4);
            double sn, cs;
            sincos(-S->E * ts, &sn, &cs);
            const double wr = S->w[2 * q], wi = S->w[2 * q + 1];
            sh_wc[par][q] = cmake<C>((R)(wr * cs - wi * sn), (R)(wr * sn + wi * cs));
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) v[q][m] = yi[q][m];
        // the exchanges' barriers also publish sh_coef / sh_wc
        const int tf = t + opaque_zero();
        fft_line<C, N, T, -1, 4, CG, Lay, PL>(v, xch, tf, 0, tw);
#pragma unroll
        for (int m = 0; m < E; ++m)
            apply_h0(v[0][m], v[1][m], v[2][m], v[3][m], (R)(dk * kindex(tf + T * m, N)), Ky, Kz, inv_n);
        const int ti = t + opaque_zero();
        fft_line<C, N, T, +1, 4, CG, Lay, PL>(v, xch, ti, 0, tw);
        const C wc[4] = {sh_wc[par][0], sh_wc[par][1], sh_wc[par][2], sh_wc[par][3]};
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int i = ti + T * m;
            R A[4] = {(R)0, (R)0, (R)0, (R)0};
            for (int j = 0; j < nterm; ++j) {
                const R f = sh_coef[par][j] * fx[j * N + i];
                const int mu = sh_mu[j];
                A[0] += mu == 0 ? f : (R)0;
                A[1] += mu == 1 ? f : (R)0;
                A[2] += mu == 2 ? f : (R)0;
                A[3] += mu == 3 ? f : (R)0;
            }
            const C ph = phx[i];
            C sv[4], vs[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) sv[q] = cadd(yi[q][m], cmul(wc[q], ph));
            apply_pot(sv, vs, A[0], A[1], A[2], A[3]);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q][m] = cadd(v[q][m], cmul_mi(vs[q]));
        }
    };
    // this lane's RK4 sum slot of component q, point m
    auto acc = [&](int q, int m) -> C& { return accl[(q * E + m) * T + t]; };

#pragma unroll 1
    for (int n = 0; n < a.nsteps; ++n) {
        const double tn = a.t_out - (double)(n_first + n) * dt;
        C yi[4][E], k[4][E];
        // stage 1 at t_n
        rhs(y, k, tn, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) {
                acc(q, m) = cadd(y[q][m], cscale(k[q][m], h6));
                yi[q][m] = cadd(y[q][m], cscale(k[q][m], h2));
            }
        // stage 2 at t_n + h/2
        rhs(yi, k, tn - 0.5 * dt, 1);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) {
                acc(q, m) = cadd(acc(q, m), cscale(k[q][m], h3));
                yi[q][m] = cadd(y[q][m], cscale(k[q][m], h2));
            }
        // stage 3 at t_n + h/2
        rhs(yi, k, tn - 0.5 * dt, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) {
                acc(q, m) = cadd(acc(q, m), cscale(k[q][m], h3));
                yi[q][m] = cadd(y[q][m], cscale(k[q][m], h));
            }
        // stage 4 at t_n + h, then the absorber
        rhs(yi, k, tn - dt, 1);
        const int o = opaque_zero();
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const R mk = msk[t + T * m + o];
#pragma unroll
            for (int q = 0; q < 4; ++q) y[q][m] = cscale(cadd(acc(q, m), cscale(k[q][m], h6)), mk);
        }
    }
    {
        gptr<nv2<R>> p = wview<R>(S->buf[BUF_Y]) + t;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int m = 0; m < E; ++m) gstore<C>(p, q * (long long)N + T * m, y[q][m]);
    }
}

// Kernel table of one (precision, N) instantiation.
struct RowVariant { const void* stage[4]; const void* dp5[6]; int threads, rows; size_t lds; };   // RK4 / Dormand-Prince stages
struct CdVariant { const void* fn[2][2]; int threads, w; size_t lds; int pipe; };   // [axis - 1][accumulate]; pipe: persistent y pass
struct ColVariant { const void* fn[2][3]; int threads, w; size_t lds; };
struct SizeKernels {
    int nvar;                      // tile variants of the stepping passes
    RowVariant row[NVAR];          // the RK4 stage row pass, by variant
    CdVariant cd[NVAR];            // the stepping column passes, by variant
    const void* row_other[ROW_NMODES];  // whole-state row modes
    int row0_threads, row0_rows;
    size_t row0_lds;
    ColVariant col;                // whole-state column transforms
    const void* line[2];           // 1D whole-loop kernel, narrow / wide exchange rounds
                                   // (NULL where there is no 4-point plan)
    int line_threads;
    size_t line_lds[2];            // their dynamic LDS without the field-term profiles
};

template <class R, int N, int V>
RowVariant make_row_variant() {
    using VC = RdVar<R, N, V>;
    return RowVariant{{(const void*)row_d_kernel<R, N, V, 0>, (const void*)row_d_kernel<R, N, V, 1>,
                       (const void*)row_d_kernel<R, N, V, 2>, (const void*)row_d_kernel<R, N, V, 3>},
                      {(const void*)row_d_kernel<R, N, V, 4>, (const void*)row_d_kernel<R, N, V, 5>,
                       (const void*)row_d_kernel<R, N, V, 6>, (const void*)row_d_kernel<R, N, V, 7>,
                       (const void*)row_d_kernel<R, N, V, 8>, (const void*)row_d_kernel<R, N, V, 9>},
                      VC::THREADS, VC::ROWS, VC::BYTES};
}
template <class R, int N, int V>
CdVariant make_cd_variant() {
    using VC = CdVar<R, N, V>;
    CdVariant c;
    c.fn[0][0] = (const void*)col_d_kernel<R, N, V, 1, 0>;
    c.fn[0][1] = (const void*)col_d_kernel<R, N, V, 1, 1>;
    c.fn[1][0] = (const void*)col_d_kernel<R, N, V, 2, 0>;
    c.fn[1][1] = (const void*)col_d_kernel<R, N, V, 2, 1>;
    c.threads = VC::THREADS;
    c.w = VC::W;
    c.lds = VC::BYTES;
    c.pipe = VC::PIPE ? 1 : 0;
    return c;
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
    k.cd[0] = make_cd_variant<R, N, 0>();
    if constexpr (nvar<N>() > 1) {
        k.row[1] = make_row_variant<R, N, 1>();
        k.row[2] = make_row_variant<R, N, 2>();
        k.row[3] = make_row_variant<R, N, 3>();
        k.cd[1] = make_cd_variant<R, N, 1>();
        k.cd[2] = make_cd_variant<R, N, 2>();
        k.cd[3] = make_cd_variant<R, N, 3>();
    } else {
        for (int v = 1; v < NVAR; ++v) {
            k.row[v] = k.row[0];
            k.cd[v] = k.cd[0];
        }
    }
    // whole-state column transforms: the few-points plan where there is one
    k.col = make_col_variant<R, N, (nvar<N>() > 1 && has_small_plan<N>()) ? 2 : 0>();
    k.row_other[ROW_FWD] = (const void*)row_kernel<R, N, 0, ROW_FWD, 0>;
    k.row_other[ROW_STAGE] = nullptr;
    k.row_other[ROW_INV] = (const void*)row_kernel<R, N, 0, ROW_INV, 0>;
    k.row_other[ROW_RHS] = (const void*)row_kernel<R, N, 0, ROW_RHS, 0>;
    k.row_other[ROW_FWDPH] = (const void*)row_kernel<R, N, 0, ROW_FWDPH, 0>;
    k.row_other[ROW_SRC] = (const void*)row_kernel<R, N, 0, ROW_SRC, 0>;
    k.row0_threads = RowVar<R, N, 0>::THREADS;
    k.row0_rows = RowVar<R, N, 0>::ROWS;
    k.row0_lds = RowVar<R, N, 0>::BYTES;
    if constexpr (has_plan4<N>()) {
        k.line[0] = (const void*)line_kernel<R, N, false>;
        k.line[1] = (const void*)line_kernel<R, N, true>;
        k.line_threads = LineVar<R, N, false>::T;
        k.line_lds[0] = LineVar<R, N, false>::BASE_BYTES;
        k.line_lds[1] = LineVar<R, N, true>::BASE_BYTES;
    } else {
        k.line[0] = k.line[1] = nullptr;
        k.line_threads = 0;
        k.line_lds[0] = k.line_lds[1] = 0;
    }
    return k;
}

}  // namespace swf
