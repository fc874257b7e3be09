// Device-side data structures and FFT building blocks of the SWF solver.
//
// The scattered wave of one solve is stored "spinor of arrays": four complex
// planes [component][z][y][x] (x fastest), so every pass reads and writes
// contiguous, coalesced lines.  Spatial derivatives are spectral (section
// "Numerical approach" of arXiv 2512.16889): each RK stage transforms along
// every non-trivial axis, multiplies by -i H0(k), and transforms back.
//
// FFTs are register-resident Stockham transforms: a line of N points is held
// by T threads, E = N/T points each (thread t owns points t, t+T, t+2T, ...).
// A radix-R step is done in registers; between steps the points are exchanged
// through LDS.  The plan (list of radices) for each N is chosen so that every
// radix divides E and T divides N/R, which keeps the first step's input and the
// last step's output in natural order: loads and stores stay coalesced and no
// bit-reversal pass is needed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swf {

constexpr int MAX_TERMS = 8;

// ---------------------------------------------------------------- complex
template <class R> struct cpx_t;
template <> struct cpx_t<float> { using type = float2; };
template <> struct cpx_t<double> { using type = double2; };
template <class R> using cpx = typename cpx_t<R>::type;

template <class C> __device__ __forceinline__ C cmake(decltype(C::x) a, decltype(C::x) b) { C r; r.x = a; r.y = b; return r; }
template <class C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <class C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <class C> __device__ __forceinline__ C cmul(C a, C b) { return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
template <class C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <class C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return cmake<C>(a.x * s, a.y * s); }
template <class C> __device__ __forceinline__ C cmul_i(C a) { return cmake<C>(-a.y, a.x); }    // i a
template <class C> __device__ __forceinline__ C cmul_mi(C a) { return cmake<C>(a.y, -a.x); }   // -i a
// multiply by (dir * i): dir = -1 gives -i (forward transforms), +1 gives +i
template <int DIR, class C> __device__ __forceinline__ C cmul_di(C a) { return DIR < 0 ? cmul_mi(a) : cmul_i(a); }

// ---------------------------------------------------------------- descriptors
// One separable term of a field: A_mu += amp * ft(t) * fx(x) fy(y) fz(z).
struct TermDev {
    int mu;
    int ft_type;
    double amp, c, w, k, phi;   // time profile (evaluated in double on the device)
    long long tab;              // offset (reals) of the spatial tables: n0 + n1 + n2 entries
};

// Everything a kernel needs to know about one solve.
struct SolveDev {
    void* buf[8];         // state arrays: Y (psi_s), ACC (RK accumulator), YS (stage input), T (FFT work);
                          // A0, A1: transforms of the partial-integration BW route; with the
                          // Dormand-Prince stepper ACC, A0, A1, K3, K4 hold its stage slopes k_0..k_4
                          // (NULL where unused)
    int dim;
    int n[3];
    long long nsites;     // n0 * n1 * n2
    int nrows;            // n1 * n2 (x-lines)
    int kind;             // 0 = U_out, 1 = V_out
    double dk[3];         // 2 pi / L
    double kap[3];        // conserved momentum on trivial axes (axes >= dim)
    double w[8];          // background spinor (re, im) x 4
    double E;             // background energy: psi_b = w exp(-i E t + i K.x)
    double dV;
    double inv_n;         // 1 / nsites (normalisation of the inverse transform)
    int term0, nterm;     // field terms
    long long ph;         // offset (complex) of the background phase tables exp(i K_j x_j): n0 + n1 + n2 entries
    long long mask;       // offset (reals) of absorber mask tables, -1 if off
    long long tw[3];      // offset (complex) of the twiddle table of each axis' length
};

enum { BUF_Y = 0, BUF_ACC = 1, BUF_YS = 2, BUF_T = 3, BUF_A0 = 4, BUF_A1 = 5, BUF_K3 = 6, BUF_K4 = 7 };
constexpr int NBUF = 8;

// Dormand-Prince 5(4) tableau (Dormand and Prince 1980; the Dopri5 of the
// paper's listing), fixed step: stage nodes c_s and the coefficients a_ij of
// the stage inputs y_i = y + h sum_j a_ij k_j, with row 6 the fifth-order
// weights b (b_6 = 0: the last row's slope serves only the error estimate,
// which is not formed).  The slopes k_0..k_4 live in these state arrays.
__host__ __device__ constexpr double dp5_c(int s) {
    return s == 0 ? 0.0 : s == 1 ? 0.2 : s == 2 ? 0.3 : s == 3 ? 0.8 : s == 4 ? 8.0 / 9.0 : 1.0;
}
__host__ __device__ constexpr double dp5_a(int i, int j) {
    return i == 1 ? (j == 0 ? 0.2 : 0.0)
         : i == 2 ? (j == 0 ? 3.0 / 40 : j == 1 ? 9.0 / 40 : 0.0)
         : i == 3 ? (j == 0 ? 44.0 / 45 : j == 1 ? -56.0 / 15 : j == 2 ? 32.0 / 9 : 0.0)
         : i == 4 ? (j == 0 ? 19372.0 / 6561 : j == 1 ? -25360.0 / 2187 : j == 2 ? 64448.0 / 6561
                     : j == 3 ? -212.0 / 729 : 0.0)
         : i == 5 ? (j == 0 ? 9017.0 / 3168 : j == 1 ? -355.0 / 33 : j == 2 ? 46732.0 / 5247 : j == 3 ? 49.0 / 176
                     : j == 4 ? -5103.0 / 18656 : 0.0)
         : i == 6 ? (j == 0 ? 35.0 / 384 : j == 2 ? 500.0 / 1113 : j == 3 ? 125.0 / 192 : j == 4 ? -2187.0 / 6784
                     : j == 5 ? 11.0 / 84 : 0.0)
         : 0.0;
}
__host__ __device__ constexpr int dp5_kbuf(int j) {   // the array holding slope k_j
    return j == 0 ? BUF_ACC : j == 1 ? BUF_A0 : j == 2 ? BUF_A1 : j == 3 ? BUF_K3 : BUF_K4;
}

// ---------------------------------------------------------------- FFT plans
template <int N> struct FftPlan;
#define SWF_PLAN(N_, T_, ...)                                            \
    template <> struct FftPlan<N_> {                                     \
        static constexpr int T = T_;                                     \
        static constexpr int R[] = {__VA_ARGS__};                        \
        static constexpr int NR = sizeof(R) / sizeof(int);               \
    };
SWF_PLAN(16, 2, 8, 2)
SWF_PLAN(32, 4, 8, 4)
SWF_PLAN(64, 8, 8, 8)
SWF_PLAN(128, 16, 8, 8, 2)
SWF_PLAN(256, 32, 8, 8, 4)
SWF_PLAN(512, 64, 8, 8, 8)
SWF_PLAN(1024, 64, 8, 8, 8, 2)
SWF_PLAN(48, 4, 3, 4, 4)
SWF_PLAN(96, 8, 3, 4, 4, 2)
SWF_PLAN(192, 16, 3, 4, 4, 4)
SWF_PLAN(384, 32, 3, 4, 4, 4, 2)
SWF_PLAN(768, 64, 3, 4, 4, 4, 4)
SWF_PLAN(40, 2, 5, 4, 2)
SWF_PLAN(80, 4, 5, 4, 4)
SWF_PLAN(160, 8, 5, 4, 4, 2)
SWF_PLAN(320, 16, 5, 4, 4, 4)
#undef SWF_PLAN

// Plans with 4 points per thread (radix 4, a final radix 2 when log2 N is
// odd): twice the threads per line and half the registers of the default.
template <int N> struct Plan4;
#define SWF_PLAN4(N_, ...)                                               \
    template <> struct Plan4<N_> {                                       \
        static constexpr int T = N_ / 4;                                 \
        static constexpr int R[] = {__VA_ARGS__};                        \
        static constexpr int NR = sizeof(R) / sizeof(int);               \
    };
SWF_PLAN4(64, 4, 4, 4)
SWF_PLAN4(128, 4, 4, 4, 2)
SWF_PLAN4(256, 4, 4, 4, 4)
SWF_PLAN4(512, 4, 4, 4, 4, 2)
SWF_PLAN4(1024, 4, 4, 4, 4, 4)
#undef SWF_PLAN4
template <int N> constexpr bool has_plan4() { return N == 64 || N == 128 || N == 256 || N == 512 || N == 1024; }

// Plans with few points per thread for the mixed-radix lengths: a radix-6
// (3 * 2^a) or radix-10 (5 * 2^a) first step and radix-2 steps after it, so a
// thread holds 6 or 10 points instead of 12 or 20 (the default plans' radix-4
// steps need a multiple of 4 and of 3 or 5 per thread).
template <int N> struct PlanS;
#define SWF_PLANS(N_, E_, ...)                                           \
    template <> struct PlanS<N_> {                                       \
        static constexpr int T = N_ / E_;                                \
        static constexpr int R[] = {__VA_ARGS__};                        \
        static constexpr int NR = sizeof(R) / sizeof(int);               \
    };
SWF_PLANS(384, 6, 6, 2, 2, 2, 2, 2, 2)
SWF_PLANS(768, 6, 6, 2, 2, 2, 2, 2, 2, 2)
SWF_PLANS(320, 10, 10, 2, 2, 2, 2, 2)
#undef SWF_PLANS
template <int N> constexpr bool has_plans() { return N == 384 || N == 768 || N == 320; }

// The few-points-per-thread plan of a length (tile variants that use it).
template <int N, bool P4 = has_plan4<N>(), bool PS = has_plans<N>()> struct SmallPlan { using type = FftPlan<N>; };
template <int N, bool PS> struct SmallPlan<N, true, PS> { using type = Plan4<N>; };
template <int N> struct SmallPlan<N, false, true> { using type = PlanS<N>; };
template <int N> constexpr bool has_small_plan() { return has_plan4<N>() || has_plans<N>(); }

template <class P> constexpr int plan_stride(int j) {
    int s = 1;
    for (int i = 0; i < j; ++i) s *= P::R[i];
    return s;
}

// ---------------------------------------------------------------- small DFTs
// y[q] = sum_k a[k] exp(DIR * 2 pi i k q / R), in place.
template <int R, int DIR, class C> struct Dft;

template <int DIR, class C> struct Dft<2, DIR, C> {
    static __device__ __forceinline__ void run(C* a) {
        C t = a[1];
        a[1] = csub(a[0], t);
        a[0] = cadd(a[0], t);
    }
};

template <int DIR, class C> struct Dft<3, DIR, C> {
    static __device__ __forceinline__ void run(C* a) {
        using R = decltype(C::x);
        const R s = (R)0.86602540378443864676;   // sin(2 pi / 3)
        C t1 = cadd(a[1], a[2]);
        C t2 = csub(a[0], cscale(t1, (R)0.5));
        C t3 = cscale(csub(a[1], a[2]), s);
        a[0] = cadd(a[0], t1);
        a[1] = cadd(t2, cmul_di<DIR>(t3));
        a[2] = csub(t2, cmul_di<DIR>(t3));
    }
};

template <int DIR, class C> struct Dft<4, DIR, C> {
    static __device__ __forceinline__ void run(C* a) {
        C s02 = cadd(a[0], a[2]), d02 = csub(a[0], a[2]);
        C s13 = cadd(a[1], a[3]), d13 = cmul_di<DIR>(csub(a[1], a[3]));
        a[0] = cadd(s02, s13);
        a[2] = csub(s02, s13);
        a[1] = cadd(d02, d13);
        a[3] = csub(d02, d13);
    }
};

template <int DIR, class C> struct Dft<5, DIR, C> {
    static __device__ __forceinline__ void run(C* a) {
        using R = decltype(C::x);
        const R c1 = (R)0.30901699437494742410;   // cos(2 pi/5)
        const R c2 = (R)-0.80901699437494742410;  // cos(4 pi/5)
        const R s1 = (R)0.95105651629515357212;   // sin(2 pi/5)
        const R s2 = (R)0.58778525229247312917;   // sin(4 pi/5)
        C a1 = cadd(a[1], a[4]), b1 = csub(a[1], a[4]);
        C a2 = cadd(a[2], a[3]), b2 = csub(a[2], a[3]);
        C r1 = cadd(a[0], cadd(cscale(a1, c1), cscale(a2, c2)));
        C r2 = cadd(a[0], cadd(cscale(a1, c2), cscale(a2, c1)));
        C i1 = cmul_di<DIR>(cadd(cscale(b1, s1), cscale(b2, s2)));
        C i2 = cmul_di<DIR>(csub(cscale(b1, s2), cscale(b2, s1)));
        a[0] = cadd(a[0], cadd(a1, a2));
        a[1] = cadd(r1, i1);
        a[4] = csub(r1, i1);
        a[2] = cadd(r2, i2);
        a[3] = csub(r2, i2);
    }
};

template <int DIR, class C> struct Dft<8, DIR, C> {
    static __device__ __forceinline__ void run(C* a) {
        using R = decltype(C::x);
        const R h = (R)0.70710678118654752440;
        C e[4] = {a[0], a[2], a[4], a[6]};
        C o[4] = {a[1], a[3], a[5], a[7]};
        Dft<4, DIR, C>::run(e);
        Dft<4, DIR, C>::run(o);
        // o[q] *= exp(DIR 2 pi i q / 8)
        o[1] = cscale(cadd(o[1], cmul_di<DIR>(o[1])), h);
        o[2] = cmul_di<DIR>(o[2]);
        o[3] = cscale(csub(cmul_di<DIR>(o[3]), o[3]), h);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            a[q] = cadd(e[q], o[q]);
            a[q + 4] = csub(e[q], o[q]);
        }
    }
};

// radix 6 = 2 x 3: y[k] = E[k mod 3] + w^k O[k mod 3], w = exp(DIR 2 pi i / 6),
// E and O the 3-point transforms of the even and odd inputs (w^3 = -1)
template <int DIR, class C> struct Dft<6, DIR, C> {
    static __device__ __forceinline__ void run(C* a) {
        using R = decltype(C::x);
        const R h = (R)0.5, s = (R)(DIR * 0.86602540378443864676);   // w = h + i s, w^2 = -h + i s
        C e[3] = {a[0], a[2], a[4]};
        C o[3] = {a[1], a[3], a[5]};
        Dft<3, DIR, C>::run(e);
        Dft<3, DIR, C>::run(o);
        const C o1 = cmul(o[1], cmake<C>(h, s));
        const C o2 = cmul(o[2], cmake<C>(-h, s));
        a[0] = cadd(e[0], o[0]);
        a[3] = csub(e[0], o[0]);
        a[1] = cadd(e[1], o1);
        a[4] = csub(e[1], o1);
        a[2] = cadd(e[2], o2);
        a[5] = csub(e[2], o2);
    }
};

// radix 10 = 2 x 5, the same even/odd split around the 5-point transform
template <int DIR, class C> struct Dft<10, DIR, C> {
    static __device__ __forceinline__ void run(C* a) {
        using R = decltype(C::x);
        const R c1 = (R)0.80901699437494742410, s1 = (R)(DIR * 0.58778525229247312917);   // w^1 (36 degrees)
        const R c2 = (R)0.30901699437494742410, s2 = (R)(DIR * 0.95105651629515357212);   // w^2 (72)
        C e[5] = {a[0], a[2], a[4], a[6], a[8]};
        C o[5] = {a[1], a[3], a[5], a[7], a[9]};
        Dft<5, DIR, C>::run(e);
        Dft<5, DIR, C>::run(o);
        C ow[5];
        ow[0] = o[0];
        ow[1] = cmul(o[1], cmake<C>(c1, s1));
        ow[2] = cmul(o[2], cmake<C>(c2, s2));
        ow[3] = cmul(o[3], cmake<C>(-c2, s2));    // w^3 (108)
        ow[4] = cmul(o[4], cmake<C>(-c1, s1));    // w^4 (144)
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            a[k] = cadd(e[k], ow[k]);
            a[k + 5] = csub(e[k], ow[k]);
        }
    }
};

// ---------------------------------------------------------------- Stockham steps
// Registers: v[q][m] holds component q's point t + T*m (natural order) before
// the first step and after the last.  Step J (radix R, stride NS = product of the
// previous radices) runs butterflies b = t + T*c, c < E/R; input k of butterfly
// b is point b + k N/R (register c + (E/R) k), output k goes to position
// (b / NS) NS R + (b % NS) + k NS of the step's output.
template <class C, int N, int T, int J, int DIR, int NC, class P>
__device__ __forceinline__ void fft_step(C (&v)[NC][N / T], int t, const C* __restrict__ tw) {
    constexpr int R = P::R[J];
    constexpr int NS = plan_stride<P>(J);
    constexpr int E = N / T;
    constexpr int B = E / R;
#pragma unroll
    for (int c = 0; c < B; ++c) {
        C w[R];
        if constexpr (NS > 1) {
            const int r = (t + T * c) % NS;
#pragma unroll
            for (int k = 1; k < R; ++k) {
                C x = tw[r * k * (N / (NS * R))];
                w[k] = DIR < 0 ? x : cconj(x);
            }
        }
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            C a[R];
#pragma unroll
            for (int k = 0; k < R; ++k) a[k] = v[q][c + B * k];
            if constexpr (NS > 1) {
#pragma unroll
                for (int k = 1; k < R; ++k) a[k] = cmul(a[k], w[k]);
            }
            Dft<R, DIR, C>::run(a);
#pragma unroll
            for (int k = 0; k < R; ++k) v[q][c + B * k] = a[k];
        }
    }
}

// Exchange the outputs of step J-1 into the inputs of step J through LDS,
// CG components at a time.  Lay::addr(q, line, idx) is the LDS slot of point
// idx of component q (within the group) of this thread's line.
template <class C, int N, int T, int J, int NC, int CG, class Lay, class P>
__device__ __forceinline__ void fft_exchange(C (&v)[NC][N / T], C* lds, int t, int line) {
    constexpr int Rp = P::R[J - 1];
    constexpr int NSp = plan_stride<P>(J - 1);
    constexpr int R = P::R[J];
    constexpr int E = N / T;
    constexpr int Bp = E / Rp;
    constexpr int B = E / R;
#pragma unroll
    for (int g = 0; g < NC; g += CG) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CG; ++q) {
#pragma unroll
            for (int c = 0; c < Bp; ++c) {
                const int b = t + T * c;
                const int d = (b / NSp) * NSp * Rp + (b % NSp);
#pragma unroll
                for (int k = 0; k < Rp; ++k) lds[Lay::addr(q, line, d + k * NSp)] = v[g + q][c + Bp * k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < CG; ++q) {
#pragma unroll
            for (int c = 0; c < B; ++c) {
                const int b = t + T * c;
#pragma unroll
                for (int k = 0; k < R; ++k) v[g + q][c + B * k] = lds[Lay::addr(q, line, b + k * (N / R))];
            }
        }
    }
}

template <class C, int N, int T, int J, int DIR, int NC, int CG, class Lay, class P>
struct FftRun {
    static __device__ __forceinline__ void run(C (&v)[NC][N / T], C* lds, int t, int line, const C* tw) {
        if constexpr (J < P::NR) {
            if constexpr (J > 0) fft_exchange<C, N, T, J, NC, CG, Lay, P>(v, lds, t, line);
            fft_step<C, N, T, J, DIR, NC, P>(v, t, tw);
            FftRun<C, N, T, J + 1, DIR, NC, CG, Lay, P>::run(v, lds, t, line, tw);
        }
    }
};

// Unnormalised transform of NC components along one line, DIR = -1 forward
// (numpy sign), +1 inverse.  tw[m] = exp(-2 pi i m / N).  P gives the radix
// list; every radix must divide N/T and T must divide N/radix.
template <class C, int N, int T, int DIR, int NC, int CG, class Lay, class P = FftPlan<N>>
__device__ __forceinline__ void fft_line(C (&v)[NC][N / T], C* lds, int t, int line, const C* tw) {
    FftRun<C, N, T, 0, DIR, NC, CG, Lay, P>::run(v, lds, t, line, tw);
}

// LDS layouts.  Row passes: lanes run along the line (t fastest), one padded
// LDS row per line.  Column passes: lanes run across the W lines (x fastest),
// so points of equal index sit next to each other.
template <int N, int ROWS> struct RowLay {
    static constexpr int STRIDE = N + N / 16 + 1;
    static __device__ __forceinline__ int addr(int q, int line, int idx) {
        return (q * ROWS + line) * STRIDE + idx + (idx >> 4);
    }
};
template <int N, int W> struct ColLay {
    static __device__ __forceinline__ int addr(int q, int line, int idx) { return (q * N + idx) * W + line; }
};

// ---------------------------------------------------------------- physics helpers
// k of FFT index i on an n-point axis (numpy fftfreq order, Nyquist negative).
__device__ __forceinline__ int kindex(int i, int n) { return (2 * i < n) ? i : i - n; }

// out = -i s (alpha.K + beta) psi for one site (Dirac representation).
template <class C>
__device__ __forceinline__ void apply_h0(C& p0, C& p1, C& p2, C& p3, decltype(C::x) Kx, decltype(C::x) Ky,
                                         decltype(C::x) Kz, decltype(C::x) s) {
    using R = decltype(C::x);
    // sigma.K = [[Kz, Kx - i Ky], [Kx + i Ky, -Kz]]
    const C km = cmake<C>(Kx, -Ky), kp = cmake<C>(Kx, Ky);
    C t0 = cadd(p0, cadd(cscale(p2, Kz), cmul(km, p3)));
    C t1 = cadd(p1, csub(cmul(kp, p2), cscale(p3, Kz)));
    C t2 = csub(cadd(cscale(p0, Kz), cmul(km, p1)), p2);
    C t3 = csub(csub(cmul(kp, p0), cscale(p1, Kz)), p3);
    p0 = cscale(cmul_mi(t0), s);
    p1 = cscale(cmul_mi(t1), s);
    p2 = cscale(cmul_mi(t2), s);
    p3 = cscale(cmul_mi(t3), s);
    (void)sizeof(R);
}

// The free evolution over tau of one Fourier mode, times s:
// exp(-i H0(K) tau) = cos(E tau) - i sin(E tau) H0(K) / E with E = sqrt(1 + K^2)
// (H0^2 = E^2); E and the angle in double.
template <class C>
__device__ __forceinline__ void apply_expo(C& p0, C& p1, C& p2, C& p3, double Kx, double Ky, double Kz, double tau,
                                           double s) {
    using R = decltype(C::x);
    const double E = sqrt(1.0 + Kx * Kx + Ky * Ky + Kz * Kz);
    double sn, cs;
    sincos(E * tau, &sn, &cs);
    C q0 = p0, q1 = p1, q2 = p2, q3 = p3;
    apply_h0(q0, q1, q2, q3, (R)Kx, (R)Ky, (R)Kz, (R)(s * sn / E));
    const R c = (R)(s * cs);
    p0 = cadd(cscale(p0, c), q0);
    p1 = cadd(cscale(p1, c), q1);
    p2 = cadd(cscale(p2, c), q2);
    p3 = cadd(cscale(p3, c), q3);
}

// (A_0 + alpha^j A_j) s for one site; A1..A3 covariant components.
template <class C>
__device__ __forceinline__ void apply_pot(const C (&s)[4], C (&o)[4], decltype(C::x) A0, decltype(C::x) A1,
                                          decltype(C::x) A2, decltype(C::x) A3) {
    const C am = cmake<C>(A1, -A2), ap = cmake<C>(A1, A2);
    o[0] = cadd(cscale(s[0], A0), cadd(cscale(s[2], A3), cmul(am, s[3])));
    o[1] = cadd(cscale(s[1], A0), csub(cmul(ap, s[2]), cscale(s[3], A3)));
    o[2] = cadd(cscale(s[2], A0), cadd(cscale(s[0], A3), cmul(am, s[1])));
    o[3] = cadd(cscale(s[3], A0), csub(cmul(ap, s[0]), cscale(s[1], A3)));
}

// Time profile env((s - c)/w) cos(k s + phi), in double.
__device__ __forceinline__ double profile_t(int type, double c, double w, double k, double phi, double s) {
    double env = 1.0;
    if (type != 0) {
        const double u = (s - c) / w;
        if (type == 1) env = exp(-u * u);
        else if (type == 2) { const double ch = cosh(u); env = 1.0 / (ch * ch); }
        else if (type == 3) env = tanh(u);
        else env = u * exp(-u * u);
    }
    if (k != 0.0 || phi != 0.0) env *= cos(k * s + phi);
    return env;
}

}  // namespace swf
