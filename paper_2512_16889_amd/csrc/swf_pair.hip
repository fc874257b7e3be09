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

// Staged item j of this thread: side j / (PG_ITEMS/2) (a, then b), row
// p / PG_CS and site p % PG_CS of that side's chunk, p = (tid + PG_THREADS j)
// modulo PG_T * PG_CS.  pg_load issues the global loads of a state row (kept
// in registers while the previous chunk is multiplied); pg_put finishes the
// item (projector, or the generated plane wave) and writes it to
// re/im[site][component][row].
__device__ __forceinline__ void pg_item(int j, int& row, int& ls) {
    const int p = (threadIdx.x + PG_THREADS * j) % (PG_T * PG_CS);
    row = p / PG_CS;
    ls = p % PG_CS;
}

template <class R>
__device__ __forceinline__ void pg_load(const PairArgs& a, const PairSide& sd, int r0, int row, int ls, long long s0,
                                        long long s1, double2 (&v)[4]) {
    using C = cpx<R>;
    const long long site = s0 + ls;
    const int r = r0 + row;
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = d2(0, 0);
    if (sd.src == PG_STATE && r < sd.n && site < s1) {
        const C* B = reinterpret_cast<const C*>(a.solves[sd.ops[r].solve].buf[sd.role]);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = todbl(B[q * a.ns + site]);
    }
}

__device__ __forceinline__ void pg_put(const PairArgs& a, const PairSide& sd, int r0, int row, int ls, long long s0,
                                       long long s1, double2 (&v)[4], double* re, double* im) {
    const long long site = s0 + ls;
    const int r = r0 + row;
    if (r < sd.n && site < s1) {
        const PairOp op = sd.ops[r];
        const SolveDev* S = a.solves + op.solve;
        int x, y, z;
        site_xyz(site, S, x, y, z);
        if (sd.src == PG_STATE) {
            if (a.proj != 0) {
                double Kx, Ky, Kz;
                site_k(S, x, y, z, Kx, Ky, Kz);
                const double sg = a.proj / sqrt(1.0 + Kx * Kx + Ky * Ky + Kz * Kz);
                double2 h[4];
                h0d(v, h, Kx, Ky, Kz);
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = dsc(dadd(v[q], dsc(h[q], sg)), 0.5);
            }
        } else {
            double ph = op.K[0] * (a.x0[0] + x * a.dx[0]);
            if (a.dim >= 2) ph += op.K[1] * (a.x0[1] + y * a.dx[1]);
            if (a.dim >= 3) ph += op.K[2] * (a.x0[2] + z * a.dx[2]);
            double sn, cs;
            sincos(ph, &sn, &cs);
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = dmul(d2(S->w[2 * q], S->w[2 * q + 1]), d2(cs, sn));
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        re[ls * PG_STR + q * PG_T + row] = v[q].x;
        im[ls * PG_STR + q * PG_T + row] = v[q].y;
    }
}

template <class R>
__global__ void __launch_bounds__(PG_THREADS) pair_gemm_kernel(PairArgs a) {
    __shared__ double are[PG_CS * PG_STR], aim[PG_CS * PG_STR], bre[PG_CS * PG_STR], bim[PG_CS * PG_STR];
    constexpr int HALF = PG_ITEMS / 2;
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
    int row[PG_ITEMS], ls[PG_ITEMS];
#pragma unroll
    for (int j = 0; j < PG_ITEMS; ++j) pg_item(j, row[j], ls[j]);
    double2 v[PG_ITEMS][4];
#pragma unroll
    for (int j = 0; j < PG_ITEMS; ++j) {
        if (j < HALF) pg_load<R>(a, a.a, r0, row[j], ls[j], sb, se, v[j]);
        else pg_load<R>(a, a.b, c0, row[j], ls[j], sb, se, v[j]);
    }
    for (long long s0 = sb; s0 < se; s0 += PG_CS) {
        __syncthreads();   // the previous chunk's operands have been consumed
#pragma unroll
        for (int j = 0; j < PG_ITEMS; ++j) {
            if (j < HALF) pg_put(a, a.a, r0, row[j], ls[j], s0, se, v[j], are, aim);
            else pg_put(a, a.b, c0, row[j], ls[j], s0, se, v[j], bre, bim);
        }
        __syncthreads();
        // the next chunk's loads stay in flight during this chunk's products
        if (s0 + PG_CS < se) {
#pragma unroll
            for (int j = 0; j < PG_ITEMS; ++j) {
                if (j < HALF) pg_load<R>(a, a.a, r0, row[j], ls[j], s0 + PG_CS, se, v[j]);
                else pg_load<R>(a, a.b, c0, row[j], ls[j], s0 + PG_CS, se, v[j]);
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

hipError_t launch_pair_gemm(int fp64, const PairArgs& a, hipStream_t st) {
    const dim3 g(a.tiles_m * a.tiles_n * a.splits), b(PG_THREADS);
    if (fp64) hipLaunchKernelGGL(pair_gemm_kernel<double>, g, b, 0, st, a);
    else hipLaunchKernelGGL(pair_gemm_kernel<float>, g, b, 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long count = (long long)a.mp * a.np;
    hipLaunchKernelGGL(pair_reduce_kernel, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, st, a.part, a.splits,
                       count, a.part + (long long)a.splits * count);
    return hipGetLastError();
}

}  // namespace swf
