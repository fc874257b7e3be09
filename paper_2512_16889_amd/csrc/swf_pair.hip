// Pair-amplitude matrix: the two inner products of eq. (Nmn) (arXiv
// 2512.16889) for every pair of an electron out-state U_m and a positron
// out-state V_n at t_in at once,
//     form 1: (U_b,m | V_s,n)  and  (U_s,m | Pi_+ | V_s,n),
//     form 2: (U_s,m | V_b,n)  and  (U_s,m | Pi_- | V_s,n).
// Each is a dense complex contraction over K = (lattice site, spinor
// component),
//     G[m][n] = sum_K conj(A_m[K]) B_n[K],
// so an M x N amplitude matrix reads each state once instead of once per
// pair.  An operand row is a state array (x space, or k space with the
// projector Pi applied, as (Pi A)^dag (Pi B) = A^dag Pi B), or a background
// plane-wave spinor w e^{i K.x} generated on the fly.
//
// The contraction runs on the FP64 matrix cores: a workgroup owns a 64 x 64
// output tile (four waves of 32 x 32, each 2 x 2 blocks of 16 x 16) and a
// range of sites, so a matrix up to 64 x 64 reads every state once; per site
// the four spinor components are the k = 4 block of v_mfma_f64_16x16x4, and a
// complex product is four real ones (re re + im im, re im - im re).  Operands
// are staged through LDS, 8 sites at a time, with coalesced loads along the
// sites.  Workgroups write partial tiles per site range; a second kernel adds
// them in a fixed order (no atomics: bitwise repeatable).
#include "swf_reduce.h"
#include "swf_dmath.h"

namespace swf {

constexpr int PG_THREADS = 256;
constexpr int PG_T = 64;                  // output tile edge (rows = cols); each wave owns 32 x 32
constexpr int PG_CS = 8;                  // sites per staged chunk
constexpr int PG_STR = 4 * PG_T + 1;      // LDS doubles per staged site (one pad)
constexpr int PG_ITEMS = 2 * PG_T * PG_CS / PG_THREADS;   // staged (side, row, site) items per thread

typedef double v4d __attribute__((ext_vector_type(4)));

static_assert(PG_ITEMS * PG_THREADS == 2 * PG_T * PG_CS, "whole staged items per thread");
static_assert(PG_ITEMS % 2 == 0, "half of a thread's items on each side");

// Global-address-space views (the arrays' pointers come from the solve
// descriptors, so the compiler cannot infer the address space and would emit
// flat loads, which also count against the LDS wait counter); complex
// numbers cross that address space as native clang vectors.
template <class T> using gp = T __attribute__((address_space(1)))*;
template <class R> using vc2 = R __attribute__((ext_vector_type(2)));
template <class R> __device__ __forceinline__ double2 gld(gp<const vc2<R>> p, long long i) {
    const vc2<R> v = p[i];
    return d2((double)v.x, (double)v.y);
}

// Staging.  Thread t stages, for each chunk of PG_CS consecutive sites, site
// t % PG_CS of the rows (t + PG_THREADS j) / PG_CS mod PG_T, j < PG_ROWS, on
// both sides.  The rows, and with them each row's source (the state array, or
// the background spinor w and its phase tables), are fixed for the whole
// kernel, so they are read once into the thread's slots before the site
// loop; in the loop a state row costs its four component loads, issued for
// the next chunk while this one is multiplied.  The chunk's sites are
// consecutive, so the thread's site follows from the chunk's first site (cx,
// cy, cz) by at most one carry (every lattice axis has at least 16 points).
constexpr int PG_ROWS = PG_ITEMS / 2;     // rows per thread and side
static_assert(PG_THREADS % PG_CS == 0, "a thread's site within the chunk is the same for all its rows");

template <class R, int SRC, bool PROJ>
struct PgSlot {
    bool ok;                  // the row exists
    gp<const vc2<R>> p;       // PG_STATE: the state array
    gp<const vc2<double>> ph; // PG_BKG, double tables: exp(i K_j x_j) per axis
    double w[8];              // PG_BKG: the free spinor (re, im per component)
    double K[3];              // PG_BKG, single-precision tables: its momentum on the lattice axes
    double kap1, kap2;        // PROJ: the solve's K on trivial axes y, z
};

template <class R, int SRC, bool PROJ>
__device__ __forceinline__ void pg_slot(const PairArgs& a, const PairSide& sd, int r, PgSlot<R, SRC, PROJ>& sl) {
    sl.ok = r < sd.n;
    if (!sl.ok) r = 0;   // (any valid descriptor: the slot's values are zero)
    const PairOp op = sd.ops[r];
    const SolveDev* S = a.solves + op.solve;
    if constexpr (SRC == PG_STATE) {
        sl.p = (gp<const vc2<R>>)S->buf[sd.role];
        if constexpr (PROJ) {
            sl.kap1 = S->kap[1];
            sl.kap2 = S->kap[2];
        }
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) sl.w[k] = S->w[k];
        if constexpr (sizeof(R) == 8) sl.ph = (gp<const vc2<double>>)a.ctab + S->ph;
        else
#pragma unroll
            for (int j = 0; j < 3; ++j) sl.K[j] = op.K[j];
    }
}

__device__ __forceinline__ void pg_site(int cx, int cy, int cz, int ls, int n0, int n1, int& x, int& y, int& z) {
    x = cx + ls;
    y = cy;
    z = cz;
    if (x >= n0) {
        x -= n0;
        if (++y >= n1) {
            y = 0;
            ++z;
        }
    }
}

template <class R, int SRC, bool PROJ>
__device__ __forceinline__ void pg_load(const PairArgs& a, const PgSlot<R, SRC, PROJ>& sl, long long site, bool in,
                                        double2 (&v)[4]) {
    if constexpr (SRC == PG_STATE) {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = sl.ok && in ? gld<R>(sl.p, q * a.ns + site) : d2(0, 0);
    }
}

// Finishes a staged value (the projector on a k-space state, or the generated
// plane wave) and writes it to re/im[site][component][row].
template <class R, int SRC, bool PROJ>
__device__ __forceinline__ void pg_put(const PairArgs& a, const PgSlot<R, SRC, PROJ>& sl, int row, int ls, bool in,
                                       int x, int y, int z, double2 (&v)[4], double* re, double* im) {
    if (sl.ok && in) {
        if constexpr (SRC == PG_STATE) {
            if constexpr (PROJ) {
                const double Kx = a.dk[0] * kindex(x, a.n0);
                const double Ky = a.dim >= 2 ? a.dk[1] * kindex(y, a.n1) : sl.kap1;
                const double Kz = a.dim >= 3 ? a.dk[2] * kindex(z, a.n2) : sl.kap2;
                const double sg = a.proj / sqrt(1.0 + Kx * Kx + Ky * Ky + Kz * Kz);
                double2 h[4];
                h0d(v, h, Kx, Ky, Kz);
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = dsc(dadd(v[q], dsc(h[q], sg)), 0.5);
            }
        } else {
            double2 e;
            if constexpr (sizeof(R) == 8) {
                // the solve's per-axis tables, formed in double at plan time
                e = dmul(dmul(gld<double>(sl.ph, x), gld<double>(sl.ph, a.n0 + y)), gld<double>(sl.ph, a.n0 + a.n1 + z));
            } else {
                // (single-precision contexts hold those tables in float: the phase is formed in double here)
                double p = sl.K[0] * (a.x0[0] + x * a.dx[0]);
                if (a.dim >= 2) p += sl.K[1] * (a.x0[1] + y * a.dx[1]);
                if (a.dim >= 3) p += sl.K[2] * (a.x0[2] + z * a.dx[2]);
                sincos(p, &e.y, &e.x);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = dmul(d2(sl.w[2 * q], sl.w[2 * q + 1]), e);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = d2(0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        re[ls * PG_STR + q * PG_T + row] = v[q].x;
        im[ls * PG_STR + q * PG_T + row] = v[q].y;
    }
}

// SA, SB: the sources of sides a and b; PROJ: Pi_{a.proj} between them, applied
// to side b alone ((Pi A)^dag (Pi B) = A^dag Pi B for the Hermitian idempotent Pi).
template <class R, int SA, int SB, bool PROJ>
__global__ void __launch_bounds__(PG_THREADS) pair_gemm_kernel(PairArgs a) {
    __shared__ double are[PG_CS * PG_STR], aim[PG_CS * PG_STR], bre[PG_CS * PG_STR], bim[PG_CS * PG_STR];
    const int ntile = a.tiles_m * a.tiles_n;
    const int tile = blockIdx.x % ntile, split = blockIdx.x / ntile;
    const int r0 = (tile / a.tiles_n) * PG_T, c0 = (tile % a.tiles_n) * PG_T;
    const long long sb = (long long)split * a.per;
    const long long se = sb + a.per < a.ns ? sb + a.per : a.ns;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int q = lane >> 4, i = lane & 15;
    // accumulators of the wave's 2 x 2 blocks of 16 x 16
    v4d cre[2][2], cim[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) {
            cre[bi][bj] = v4d{0, 0, 0, 0};
            cim[bi][bj] = v4d{0, 0, 0, 0};
        }
    const int ls = threadIdx.x % PG_CS;
    int row[PG_ROWS];
    PgSlot<R, SA, false> sa[PG_ROWS];
    PgSlot<R, SB, PROJ> sbl[PG_ROWS];
#pragma unroll
    for (int j = 0; j < PG_ROWS; ++j) {
        row[j] = ((threadIdx.x + PG_THREADS * j) % (PG_T * PG_CS)) / PG_CS;
        pg_slot(a, a.a, r0 + row[j], sa[j]);
        pg_slot(a, a.b, c0 + row[j], sbl[j]);
    }
    double2 va[PG_ROWS][4], vb[PG_ROWS][4];
#pragma unroll
    for (int j = 0; j < PG_ROWS; ++j) {
        pg_load(a, sa[j], sb + ls, sb + ls < se, va[j]);
        pg_load(a, sbl[j], sb + ls, sb + ls < se, vb[j]);
    }
    for (long long s0 = sb; s0 < se; s0 += PG_CS) {
        // this thread's site (a lattice has at most 2^30 sites)
        const unsigned u0 = (unsigned)s0, r1 = u0 / (unsigned)a.n0;
        int x, y, z;
        pg_site((int)(u0 - r1 * (unsigned)a.n0), (int)(r1 % (unsigned)a.n1), (int)(r1 / (unsigned)a.n1), ls, a.n0,
                a.n1, x, y, z);
        const bool in = s0 + ls < se;
        __syncthreads();   // the previous chunk's operands have been consumed
#pragma unroll
        for (int j = 0; j < PG_ROWS; ++j) {
            pg_put(a, sa[j], row[j], ls, in, x, y, z, va[j], are, aim);
            pg_put(a, sbl[j], row[j], ls, in, x, y, z, vb[j], bre, bim);
        }
        __syncthreads();
        // the next chunk's loads stay in flight during this chunk's products
        if (s0 + PG_CS < se) {
            const long long nx = s0 + PG_CS + ls;
#pragma unroll
            for (int j = 0; j < PG_ROWS; ++j) {
                pg_load(a, sa[j], nx, nx < se, va[j]);
                pg_load(a, sbl[j], nx, nx < se, vb[j]);
            }
        }
#pragma unroll 2
        for (int l = 0; l < PG_CS; ++l) {
            // lane (i, q) holds A[m = i][k = q] and B[k = q][n = i] of each 16 x 16 block
            const int o = l * PG_STR + q * PG_T;
            double ar[2], ai[2], br[2], bi_[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                ar[b] = are[o + wm + 16 * b + i];
                ai[b] = aim[o + wm + 16 * b + i];
                br[b] = bre[o + wn + 16 * b + i];
                bi_[b] = bim[o + wn + 16 * b + i];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    // conj(A) B = (ar br + ai bi) + i (ar bi - ai br)
                    cre[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[x], br[y], cre[x][y], 0, 0, 0);
                    cre[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[x], bi_[y], cre[x][y], 0, 0, 0);
                    cim[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[x], bi_[y], cim[x][y], 0, 0, 0);
                    cim[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[x], br[y], cim[x][y], 0, 0, 0);
                }
        }
    }
    // result element e of lane (i, q) in block (x, y): row q + 4 e, column i of
    // that block; partials are stored split-fastest for the reduction below
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int rr = r0 + wm + 16 * x + q + 4 * e, cc = c0 + wn + 16 * y + i;
                a.part[((long long)rr * a.np + cc) * a.splits + split] = d2(cre[x][y][e], cim[x][y][e]);
            }
}

// out[j] = sum over splits of part[j][split]: one wave per output, lanes
// strided over the splits, then a fixed butterfly across the lanes.
__global__ void __launch_bounds__(256) pair_reduce_kernel(const double2* part, int splits, long long count,
                                                          double2* out) {
    const long long j = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (j >= count) return;
    double re = 0.0, im = 0.0;
    for (int k = lane; k < splits; k += 64) {
        const double2 v = part[j * splits + k];
        re += v.x;
        im += v.y;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o);
        im += __shfl_xor(im, o);
    }
    if (lane == 0) out[j] = d2(re, im);
}

template <class R>
static hipError_t launch_pair_gemm_t(const PairArgs& a, hipStream_t st) {
    const dim3 g(a.tiles_m * a.tiles_n * a.splits), b(PG_THREADS);
    if (a.a.src == PG_STATE && a.b.src == PG_STATE) {
        if (a.proj) hipLaunchKernelGGL((pair_gemm_kernel<R, PG_STATE, PG_STATE, true>), g, b, 0, st, a);
        else hipLaunchKernelGGL((pair_gemm_kernel<R, PG_STATE, PG_STATE, false>), g, b, 0, st, a);
    } else if (a.proj == 0 && a.a.src == PG_BKG && a.b.src == PG_STATE) {
        hipLaunchKernelGGL((pair_gemm_kernel<R, PG_BKG, PG_STATE, false>), g, b, 0, st, a);
    } else if (a.proj == 0 && a.a.src == PG_STATE && a.b.src == PG_BKG) {
        hipLaunchKernelGGL((pair_gemm_kernel<R, PG_STATE, PG_BKG, false>), g, b, 0, st, a);
    } else {
        return hipErrorInvalidValue;   // (two background sides, or a projector beside one: not used)
    }
    return hipGetLastError();
}

hipError_t launch_pair_gemm(int fp64, const PairArgs& a, hipStream_t st) {
    hipError_t e = fp64 ? launch_pair_gemm_t<double>(a, st) : launch_pair_gemm_t<float>(a, st);
    if (e != hipSuccess) return e;
    const long long count = (long long)a.mp * a.np;
    hipLaunchKernelGGL(pair_reduce_kernel, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, st, a.part, a.splits,
                       count, a.part + (long long)a.splits * count);
    return hipGetLastError();
}

}  // namespace swf
