// Host/device interface of the reduction kernels and the per-size kernel tables.
#pragma once
#include <hip/hip_runtime.h>

#include "swf_dev.h"

namespace swf {

enum { RED_KPROJ = 0, RED_KBWPAST = 1, RED_XFOURIER = 2, RED_XDIAG = 3 };

struct RedArgs {
    const SolveDev* solves;
    int sa, sb;          // solves
    int ra, rb;          // buffer roles
    int sign;            // projector sign (RED_KPROJ)
    double kv[3];        // photon momentum (RED_KBWPAST), kappa (RED_XFOURIER), K (RED_XDIAG)
    double k0;           // photon energy
    double eps[3];       // polarisation
    double t;            // time (RED_XDIAG)
    double x0[3], dx[3]; // lattice coordinates x_i = x0 + i dx
    double2* out;        // per-block partials
};

// One plane-wave component of a photon wave packet.
struct ModeDev {
    double k0;
    double c[2];         // weight (re, im)
    double eps[3];
    long long phk;       // complex offset of its exp(i k_j x_j) tables (n0 + n1 + n2 entries)
};
constexpr int MAX_MODES = 64;

struct VertexDev {
    int su, sv;
    int nmodes, mode0;   // wave packet: its modes (0: plane wave)
    double k0;
    double eps[3];
    long long phk;       // complex offset of exp(i k_j x_j) tables (n0 + n1 + n2 entries)
    // partial-integration route
    double k[3];         // photon 3-momentum
    double kbs[3];       // p - k: momentum of the (back, scat) term's Fourier coefficient
    double ksb[3];       // k - q: that of the (scat, back) term
    double p0, q0;       // electron and positron energies
    double x0[3], dx[3]; // lattice coordinates x_i = x0 + i dx
};

// Vertices reduced together at each RK4 stage: every state of the group's (at
// most 2) U and (at most 2) V solves is read once for all its vertices.
constexpr int BWG_SOLVES = 2;
constexpr int BWG_VERTS = 4;
struct VertexGroupDev {
    int nu, nv, nvx;
    int su[BWG_SOLVES], sv[BWG_SOLVES];   // the solves
    int vtx[BWG_VERTS];                   // the vertices
    int ui[BWG_VERTS], vi[BWG_VERTS];     // each vertex's U and V solve within su / sv
    double eps[3];                        // the photon's polarisation (real)
    double cu[BWG_SOLVES][8];             // u of each U solve (re, im per component)
    double cv[BWG_SOLVES][8];             // (alpha.eps) v of each V solve
    long long tk;                         // exp(i k.x) tables (complex offset, n0 + n1 + n2 entries)
    long long t1[BWG_SOLVES];             // conj(U background phase) exp(i k.x), per U solve
    long long t2[BWG_SOLVES];             // V background phase exp(i k.x), per V solve
};

struct BwArgs {
    const SolveDev* solves;
    const VertexDev* verts;
    const VertexGroupDev* groups;   // the first route's stage reduction, one group per blockIdx.y
    const ModeDev* modes;           // wave-packet components
    const int* packets;             // the wave-packet vertices, one per blockIdx.y of their reduction
    const void* ctab;
    const int* step;
    double t_out, dt;
    int stage;
    double cst;          // the stage's time node: t = t_out - (step + cst) dt
    int nst;             // stages per step (4 RK4, 6 Dormand-Prince)
    double wst[6];       // the stages' quadrature weights (sum 1)
    int nvert;
    double2* part;       // [vertex][stage][block][3]
    double2* M;          // [vertex][3] accumulated integrals (device, double)
    // partial-integration route
    int vtx;             // vertex of a per-vertex launch
    double2* part2;      // [vertex][stage][9][block]: k-space (s,s) sum, then 8 Fourier sums
    double2* M2;         // [vertex][3] accumulated integrals of that route
};

// Pair-amplitude matrix contraction G[m][n] = sum_K conj(A_m[K]) B_n[K].
enum { PG_STATE = 0, PG_BKG = 1 };
struct PairOp {
    int solve;
    int pad;
    double K[3];         // PG_BKG: plane-wave momentum on the lattice axes (w e^{i K.x})
};
struct PairSide {
    const PairOp* ops;   // one per row (side a) or column (side b)
    int n;
    int src;             // PG_STATE: the state array of buffer role `role`; PG_BKG: background
    int role;
};
struct PairArgs {
    const SolveDev* solves;
    PairSide a, b;
    int proj;            // 0, or +1 / -1: Pi_+ / Pi_- of k-space states on both sides
    long long ns;        // sites of the (common) lattice
    int dim;
    int n0, n1, n2;      // lattice points per axis (1 on trivial axes)
    double x0[3], dx[3]; // lattice coordinates x_i = x0 + i dx
    double dk[3];        // lattice wavenumber steps 2 pi / L_j
    const void* ctab;    // complex tables (the solves' background phase tables)
    int tiles_m, tiles_n, splits;
    long long per;       // sites per split (a multiple of the staging chunk)
    int mp, np;          // padded output dimensions (multiples of the 64-row tile)
    double2* part;       // [mp][np][splits] partial tiles, then [mp][np] the sum
};

// Pointwise combination of state arrays of a group's solves (the interaction
// picture's stage inputs and update): out_j = sum_i c[j][i] in_i over every
// site and component, optionally times the absorber mask.
struct ComboArgs {
    const SolveDev* solves;
    const int2* items;   // (solve, block of `rows` x-lines) per workgroup
    int rows;
    const void* rtab;    // real tables (the masks)
    int in[3];           // input roles (-1: unused)
    int out[2];          // output roles (-1: unused)
    double c[2][3];
    int mask;            // 1: output 0 is multiplied by the solve's absorber mask (if it has one)
};
hipError_t launch_combo(int fp64, const ComboArgs& a, int nitems, hipStream_t st);

hipError_t launch_reduction(int fp64, int kind, const RedArgs& a, int blocks, hipStream_t st);
hipError_t launch_pair_gemm(int fp64, const PairArgs& a, hipStream_t st);
// a.groups: ngroups consecutive groups, all of nu U and nv V solves (1 or 2 each)
hipError_t launch_bw_stage(int fp64, const BwArgs& a, int blocks, int nu, int nv, int ngroups, hipStream_t st);
hipError_t launch_bw_packet_stage(int fp64, const BwArgs& a, int blocks, int npackets, hipStream_t st);
hipError_t launch_bw_accum(const BwArgs& a, int nblk, hipStream_t st);
hipError_t launch_bw2_src(int fp64, const BwArgs& a, int blocks, hipStream_t st);
hipError_t launch_bw2_kss(int fp64, const BwArgs& a, int blocks, hipStream_t st);
hipError_t launch_bw2_accum(const BwArgs& a, int nblk, hipStream_t st);
hipError_t launch_tick(int* step, hipStream_t st);
hipError_t launch_advance(int* step, int n, hipStream_t st);
hipError_t launch_finite_check(int fp64, const SolveDev* solves, int nsolves, int step, unsigned long long* flag,
                               hipStream_t st);

struct SizeKernels;
// Kernel table of an FFT length for single (fp64 = 0) or double precision, NULL if unsupported.
const SizeKernels* size_kernels(int fp64, int n);

}  // namespace swf
