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
// The contraction runs on the FP64 matrix cores: a workgroup owns a 32 x 32
// output tile (four waves of 16 x 16) and a range of sites; per site the four
// spinor components are the k = 4 block of v_mfma_f64_16x16x4, and a complex
// product is four real ones (re re + im im, re im - im re).  Operands are
// staged through LDS, 8 sites at a time, with coalesced loads along the
// sites.  Workgroups write partial tiles per site range; a second kernel adds
// them in a fixed order (no atomics: bitwise repeatable).
#include "swf_reduce.h"
#include "swf_dmath.h"

namespace swf {

constexpr int PG_THREADS = 256;
constexpr int PG_T = 32;                  // output tile edge (rows = cols)
constexpr int PG_CS = 8;                  // sites per staged chunk
constexpr int PG_STR = 4 * PG_T + 1;      // LDS doubles per staged site (one pad)

typedef double v4d __attribute__((ext_vector_type(4)));

static_assert(PG_T * PG_CS == PG_THREADS, "one staged (row, site) item per thread and side");

// This thread's staged item of a chunk: row r0 + p / PG_CS, site s0 + p % PG_CS.
// pg_load issues the global loads of a state row (kept in registers while the
// previous chunk is multiplied); pg_put finishes the item (projector, or the
// generated plane wave) and writes it to re/im[site][component][row].
template <class R>
__device__ __forceinline__ void pg_load(const PairArgs& a, const PairSide& sd, int r0, long long s0, long long s1,
                                        double2 (&v)[4]) {
    using C = cpx<R>;
    const int row = threadIdx.x / PG_CS, ls = threadIdx.x % PG_CS;
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

__device__ __forceinline__ void pg_put(const PairArgs& a, const PairSide& sd, int r0, long long s0, long long s1,
                                       double2 (&v)[4], double* re, double* im) {
    const int row = threadIdx.x / PG_CS, ls = threadIdx.x % PG_CS;
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
    const int ntile = a.tiles_m * a.tiles_n;
    const int tile = blockIdx.x % ntile, split = blockIdx.x / ntile;
    const int r0 = (tile / a.tiles_n) * PG_T, c0 = (tile % a.tiles_n) * PG_T;
    const long long sb = (long long)split * a.per;
    const long long se = sb + a.per < a.ns ? sb + a.per : a.ns;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = (wave >> 1) * 16, wn = (wave & 1) * 16;
    const int q = lane >> 4, i = lane & 15;
    v4d cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
    double2 va[4], vb[4];
    pg_load<R>(a, a.a, r0, sb, se, va);
    pg_load<R>(a, a.b, c0, sb, se, vb);
    for (long long s0 = sb; s0 < se; s0 += PG_CS) {
        __syncthreads();   // the previous chunk's operands have been consumed
        pg_put(a, a.a, r0, s0, se, va, are, aim);
        pg_put(a, a.b, c0, s0, se, vb, bre, bim);
        __syncthreads();
        // the next chunk's loads stay in flight during this chunk's products
        if (s0 + PG_CS < se) {
            pg_load<R>(a, a.a, r0, s0 + PG_CS, se, va);
            pg_load<R>(a, a.b, c0, s0 + PG_CS, se, vb);
        }
#pragma unroll 4
        for (int ls = 0; ls < PG_CS; ++ls) {
            // lane (i, q) holds A[m = i][k = q] and B[k = q][n = i]
            const double ar = are[ls * PG_STR + q * PG_T + wm + i], ai = aim[ls * PG_STR + q * PG_T + wm + i];
            const double br = bre[ls * PG_STR + q * PG_T + wn + i], bi = bim[ls * PG_STR + q * PG_T + wn + i];
            // conj(A) B = (ar br + ai bi) + i (ar bi - ai br)
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, cre, 0, 0, 0);
            cre = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, cim, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, br, cim, 0, 0, 0);
        }
    }
    // result element e of lane (i, q): row q + 4 e, column i of the wave's
    // sub-tile; partials are stored split-fastest for the reduction below
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = r0 + wm + q + 4 * e, col = c0 + wn + i;
        a.part[((long long)row * a.np + col) * a.splits + split] = d2(cre[e], cim[e]);
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
