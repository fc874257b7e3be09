// Host side of the SWF C ABI: validation, planning, table construction,
// device memory layout, pass scheduling (eager, batched or per-instance, and
// hipGraph replay), and the host-side FP64 arithmetic of the amplitudes.
//
// Method: arXiv 2512.16889.  Scattered waves solve eq. (scatDirac) backward
// from t_out (out-states) or forward from t_in (in-states); at the end of the
// run (t_in or t_out) the pair amplitude (eq. (Nmn)), the marginals and, for
// out-states, the Breit-Wheeler amplitude (finite part eq. (Mabfinite) + past
// part eq. (MScatScatPast) and partners) are formed from FP64 reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <sstream>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/swf.h"
#include "swf_kernels.h"
#include "swf_reduce.h"

using swf::SolveDev;
using swf::TermDev;
using swf::VertexDev;
using cd = std::complex<double>;

namespace {

thread_local std::string g_init_error;

constexpr int RED_BLOCKS = 512;          // blocks of every reduction launch (fixed: deterministic sums)
constexpr int BW_BLOCKS = 256;           // blocks per vertex of the BW stage reduction
constexpr size_t LINE_STATIC_LDS = 1024;  // bound on the line kernel's static LDS
constexpr int NKIND = 6;                 // kernel-stats kinds (swf_kernel_stats)
constexpr int PROF_POOL = 2048;          // event pairs kept in flight when profiling

const double PI = 3.14159265358979323846;

// Device scratch of swf_pair_matrix_noalloc: row descriptors and partial
// tiles, in a static array instead of context-owned memory.  Each GPU holds
// its own copy at its own address (resolved once per device at swf_init);
// host code must use that address, never the array's name.
constexpr size_t NOALLOC_SCRATCH_BYTES = 32u << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static void* g_scratch_ptr[MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// Address of this device's scratch array (dev must be current).
static hipError_t scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

// ------------------------------------------------------------ host Dirac algebra
struct Spinor { cd c[4]; };

// sigma.p as 2x2
static void sigma_dot(const double* p, cd m[2][2]) {
    m[0][0] = p[2];
    m[0][1] = cd(p[0], -p[1]);
    m[1][0] = cd(p[0], p[1]);
    m[1][1] = -p[2];
}

// u_s(p) = (1 + pslash) R_s / sqrt(2 p0 (p0 - p^1)), v_s(p) = (1 - pslash) R_s / same
// (eq. (uv) with p_1 = -p^1; R_s = (1, s, s, 1)/2 from eq. (Reqs), Dirac representation).
static Spinor free_spinor(int kind, int s, const double* p) {
    const double E = std::sqrt(1.0 + p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
    const cd a[2] = {0.5, 0.5 * s}, b[2] = {0.5 * s, 0.5};
    cd sp[2][2];
    sigma_dot(p, sp);
    const double sg = kind == 0 ? 1.0 : -1.0;   // u: 1 + pslash, v: 1 - pslash
    // pslash = [[E, -sigma.p], [sigma.p, -E]]
    Spinor r;
    for (int i = 0; i < 2; ++i) {
        cd spb = sp[i][0] * b[0] + sp[i][1] * b[1];
        cd spa = sp[i][0] * a[0] + sp[i][1] * a[1];
        r.c[i] = a[i] + sg * (E * a[i] - spb);
        r.c[2 + i] = b[i] + sg * (spa - E * b[i]);
    }
    const double nrm = std::sqrt(2.0 * E * (E - p[0]));
    for (auto& x : r.c) x /= nrm;
    return r;
}

static Spinor h0_apply(const Spinor& p, const double* K) {
    cd s[2][2];
    sigma_dot(K, s);
    Spinor o;
    for (int i = 0; i < 2; ++i) {
        o.c[i] = p.c[i] + s[i][0] * p.c[2] + s[i][1] * p.c[3];
        o.c[2 + i] = s[i][0] * p.c[0] + s[i][1] * p.c[1] - p.c[2 + i];
    }
    return o;
}

static Spinor proj(const Spinor& p, const double* K, int sign) {
    const double E = std::sqrt(1.0 + K[0] * K[0] + K[1] * K[1] + K[2] * K[2]);
    Spinor h = h0_apply(p, K), o;
    for (int q = 0; q < 4; ++q) o.c[q] = 0.5 * (p.c[q] + (double)sign * h.c[q] / E);
    return o;
}

static Spinor gamma_eps(const Spinor& p, const double* e) {   // (alpha.eps) psi
    cd s[2][2];
    sigma_dot(e, s);
    Spinor o;
    for (int i = 0; i < 2; ++i) {
        o.c[i] = s[i][0] * p.c[2] + s[i][1] * p.c[3];
        o.c[2 + i] = s[i][0] * p.c[0] + s[i][1] * p.c[1];
    }
    return o;
}

static cd dot(const Spinor& a, const Spinor& b) {
    cd s = 0;
    for (int q = 0; q < 4; ++q) s += std::conj(a.c[q]) * b.c[q];
    return s;
}

static double profile_h(const swf_profile& p, double s) {
    double env = 1.0;
    if (p.type != SWF_PROF_CONST) {
        const double u = (s - p.c) / p.w;
        switch (p.type) {
            case SWF_PROF_GAUSS: env = std::exp(-u * u); break;
            case SWF_PROF_SECH2: { const double ch = std::cosh(u); env = 1.0 / (ch * ch); } break;
            case SWF_PROF_TANH: env = std::tanh(u); break;
            default: env = u * std::exp(-u * u); break;
        }
    }
    if (p.k != 0.0 || p.phi != 0.0) env *= std::cos(p.k * s + p.phi);
    return env;
}

static bool supported_n(int n) {
    switch (n) {
        case 16: case 32: case 64: case 128: case 256: case 512: case 1024:
        case 48: case 96: case 192: case 384: case 768:
        case 40: case 80: case 160: case 320: return true;
        default: return false;
    }
}

// ------------------------------------------------------------ plan
struct Group {
    int grid;
    std::vector<int> solves;
    const swf::SizeKernels* k[3] = {nullptr, nullptr, nullptr};
    // offsets (int2) into the item array and counts: the stepping passes per
    // tile variant, then the whole-state row and column kernels
    size_t it_row[swf::NVAR] = {}, it_coly[swf::NVAR] = {}, it_colz[swf::NVAR] = {};
    int n_row[swf::NVAR] = {}, n_coly[swf::NVAR] = {}, n_colz[swf::NVAR] = {};
    size_t it_orow = 0, it_ocy = 0, it_ocz = 0;
    int n_orow = 0, n_ocy = 0, n_ocz = 0;
    int vr = 0, vy = 0, vz = 0;   // tile variants of the stepping passes in use
};

struct Plan {
    int fp64 = 0;
    size_t csize = 8, rsize = 4;
    int steps = 0;
    std::vector<swf_grid> grids;
    std::vector<std::vector<swf_term>> fields;
    std::vector<swf_solve> solves;
    std::vector<swf_vertex> verts;
    swf_window win{};
    // direction of the time loop: out-states run from t_out back to t_in,
    // in-states from t_in forward to t_out.  The kernels take t_n = t0 - n sdt
    // and the step h = -sdt, so (t0, sdt) = (t_out, dt) or (t_in, -dt); the
    // observables are read at t_obs, the end of the run.
    bool forward = false;
    double t0 = 0, sdt = 0, t_obs = 0;
    // time stepper: classical RK4 (4 stages) or fixed-step Dormand-Prince 5(4) (6 stages)
    bool dp5 = false;
    bool ip = false;                    // interaction-picture stepper (Lawson's integrating-factor RK4)
    int nst = 4;
    double cst[6] = {}, wst[6] = {};   // stage nodes and quadrature weights
    std::vector<SolveDev> hs;           // buf pointers filled after allocation (offsets meanwhile)
    std::vector<TermDev> ht;
    std::vector<VertexDev> hv;
    std::vector<swf::VertexGroupDev> hg;  // vertex groups of the stage reduction
    std::vector<swf::ModeDev> hm;         // wave-packet components of every packet vertex
    std::vector<std::vector<std::array<double, 8>>> vmodes;   // their host copies, per vertex
    std::vector<int> packets;             // the wave-packet vertices
    std::vector<double> rtab;           // real tables (rounded to the state precision on upload)
    std::vector<cd> ctab;               // complex tables
    std::vector<Group> batched, single; // groups per grid / per solve
    std::vector<int2> items;
    size_t state_bytes = 0;             // all state arrays
    // arena layout (byte offsets)
    size_t off_state = 0, off_solves = 0, off_terms = 0, off_verts = 0, off_vgroups = 0, off_modes = 0, off_packets = 0,
           off_rtab = 0, off_ctab = 0,
           off_items = 0, off_step = 0, off_M = 0, off_part = 0, off_red = 0, off_M2 = 0, off_part2 = 0, total = 0;
    std::vector<size_t> solve_off;      // state offset of each solve (bytes from off_state)
    bool bw2 = false;                   // partial-integration BW route on
    std::vector<int> bw2_solves;        // solves of its vertices (they get the A0, A1 buffers)
    std::vector<char> aux;              // per solve: 1 if it has the A0, A1 buffers
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

#define FAIL(code, ...)                                              \
    do {                                                             \
        char _b[512];                                                \
        snprintf(_b, sizeof(_b), __VA_ARGS__);                       \
        err = _b;                                                    \
        return code;                                                 \
    } while (0)

// Workgroups are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).
// The G column tiles that share 128-byte lines (x-adjacent tiles) are placed 8
// blocks apart so they all land on the same XCD and its L2 serves all but the
// first of them.
static void xcd_group_order(std::vector<int2>& items, size_t first, int G) {
    if (G <= 1) return;
    const size_t n = items.size() - first, span = 8 * (size_t)G;
    std::vector<int2> tmp(items.begin() + first, items.end());
    for (size_t i = 0; i + span <= n; i += span)
        for (size_t j = 0; j < span; ++j) items[first + i + (j % G) * 8 + j / G] = tmp[i + j];
}

// Work items (solve, tile) of a row pass with `rows` lines per block, or of a
// column pass along `axis` with `w` columns per block; returns the offset.
static size_t row_items(Plan& P, const Group& g, int rows, int& count) {
    const swf_grid& G = P.grids[g.grid];
    const int n1 = G.dim >= 2 ? G.n[1] : 1, n2 = G.dim >= 3 ? G.n[2] : 1;
    const size_t first = P.items.size();
    for (int s : g.solves)
        for (int tile = 0; tile < (n1 * n2 + rows - 1) / rows; ++tile) P.items.push_back(make_int2(s, tile));
    count = (int)(P.items.size() - first);
    return first;
}
static size_t col_items(Plan& P, const Group& g, int axis, int w, int& count) {
    const swf_grid& G = P.grids[g.grid];
    const int n0 = G.n[0], other = axis == 1 ? (G.dim >= 3 ? G.n[2] : 1) : G.n[1];
    const size_t first = P.items.size();
    const int ntx = (n0 + w - 1) / w;
    for (int s : g.solves)
        for (int tile = 0; tile < ntx * other; ++tile) P.items.push_back(make_int2(s, tile));
    count = (int)(P.items.size() - first);
    xcd_group_order(P.items, first, std::max(1, 128 / (w * (int)P.csize)));
    return first;
}

static void add_items(Plan& P, Group& g, int fp64) {
    const swf_grid& G = P.grids[g.grid];
    g.k[0] = swf::size_kernels(fp64, G.n[0]);
    if (G.dim >= 2) g.k[1] = swf::size_kernels(fp64, G.n[1]);
    if (G.dim >= 3) g.k[2] = swf::size_kernels(fp64, G.n[2]);
    for (int v = 0; v < swf::NVAR; ++v) {
        g.it_row[v] = row_items(P, g, g.k[0]->row[v].rows, g.n_row[v]);
        if (G.dim >= 2) g.it_coly[v] = col_items(P, g, 1, g.k[1]->cd[v].w, g.n_coly[v]);
        if (G.dim >= 3) g.it_colz[v] = col_items(P, g, 2, g.k[2]->cd[v].w, g.n_colz[v]);
    }
    g.it_orow = row_items(P, g, g.k[0]->row0_rows, g.n_orow);
    if (G.dim >= 2) g.it_ocy = col_items(P, g, 1, g.k[1]->col.w, g.n_ocy);
    if (G.dim >= 3) g.it_ocz = col_items(P, g, 2, g.k[2]->col.w, g.n_ocz);
}

// State arrays of solve i: Y, ACC, YS, T; A0, A1 for the partial-integration
// BW route; all eight (the Dormand-Prince slopes) with that stepper.
static int nbufs(const Plan& P, size_t i) { return P.dp5 ? swf::NBUF : (P.aux[i] || P.ip ? 6 : 4); }

static int build_plan(Plan& P, std::string& err, const swf_grid* grids, int n_grids, const swf_term* terms,
                      const int* ffirst, int n_fields, const swf_solve* solves, int n_solves,
                      const swf_vertex* verts, int n_verts, const swf_window* win, const swf_options* opt) {
    if (!grids || n_grids <= 0 || !solves || n_solves <= 0 || !win || !opt) FAIL(SWF_E_ARG, "missing inputs");
    if (n_fields < 0 || (n_fields > 0 && (!ffirst || !terms))) FAIL(SWF_E_ARG, "bad field arrays");
    if (n_verts < 0 || (n_verts > 0 && !verts)) FAIL(SWF_E_ARG, "bad vertex array");
    if (opt->prec != SWF_FP64 && opt->prec != SWF_MIXED) FAIL(SWF_E_ARG, "unknown precision %d", opt->prec);
    P.fp64 = opt->prec == SWF_FP64;
    P.csize = P.fp64 ? 16 : 8;
    P.rsize = P.fp64 ? 8 : 4;
    // window
    P.win = *win;
    if (!(win->dt > 0) || !(win->t_out > win->t_in)) FAIL(SWF_E_ARG, "need dt > 0 and t_out > t_in");
    const double span = win->t_out - win->t_in;
    P.steps = (int)std::llround(span / win->dt);
    if (P.steps < 1 || std::fabs(P.steps * win->dt - span) > 1e-9 * span)
        FAIL(SWF_E_ARG, "(t_out - t_in)/dt = %.12g is not an integer step count", span / win->dt);
    P.forward = solves[0].kind >= 2;
    P.t0 = P.forward ? win->t_in : win->t_out;
    P.sdt = P.forward ? -win->dt : win->dt;
    P.t_obs = P.forward ? win->t_out : win->t_in;
    if (opt->stepper != SWF_RK4 && opt->stepper != SWF_DP5 && opt->stepper != SWF_IPRK4)
        FAIL(SWF_E_ARG, "stepper must be SWF_RK4, SWF_DP5 or SWF_IPRK4");
    P.dp5 = opt->stepper == SWF_DP5;
    P.ip = opt->stepper == SWF_IPRK4;
    if (P.dp5 && opt->bw_partial) FAIL(SWF_E_UNSUPPORTED, "the Dormand-Prince stepper does not combine with bw_partial");
    if (P.ip && opt->bw_partial) FAIL(SWF_E_UNSUPPORTED, "the interaction-picture stepper does not combine with bw_partial");
    P.nst = P.dp5 ? 6 : 4;
    for (int st = 0; st < P.nst; ++st) {
        P.cst[st] = P.dp5 ? swf::dp5_c(st) : (st == 0 ? 0.0 : st == 3 ? 1.0 : 0.5);
        P.wst[st] = P.dp5 ? swf::dp5_a(6, st) : (st == 0 || st == 3 ? 1.0 / 6.0 : 1.0 / 3.0);
    }
    // grids
    for (int g = 0; g < n_grids; ++g) {
        swf_grid G = grids[g];
        if (G.dim < 1 || G.dim > 3) FAIL(SWF_E_ARG, "grid %d: dim must be 1..3", g);
        for (int j = 0; j < 3; ++j) {
            if (j < G.dim) {
                if (!supported_n(G.n[j])) FAIL(SWF_E_UNSUPPORTED, "grid %d: no FFT plan for n[%d] = %d", g, j, G.n[j]);
                if (!(G.L[j] > 0)) FAIL(SWF_E_ARG, "grid %d: L[%d] must be > 0", g, j);
            } else {
                G.n[j] = 1;
                G.L[j] = 1.0;
            }
        }
        if (G.absorb_cells < 0 || (G.absorb_cells > 0 && (2 * G.absorb_cells >= G.n[0] ||
                                                          (G.dim >= 2 && 2 * G.absorb_cells >= G.n[1]) ||
                                                          (G.dim >= 3 && 2 * G.absorb_cells >= G.n[2]))))
            FAIL(SWF_E_ARG, "grid %d: absorb_cells out of range", g);
        if (G.absorb_cells > 0 && !(G.absorb_strength >= 0 && G.absorb_strength <= 1))
            FAIL(SWF_E_ARG, "grid %d: absorb_strength must be in [0,1]", g);
        P.grids.push_back(G);
    }
    // fields
    for (int f = 0; f < n_fields; ++f) {
        const int a = ffirst[f], b = ffirst[f + 1];
        if (a < 0 || b < a) FAIL(SWF_E_ARG, "field %d: bad term range", f);
        if (b - a > swf::MAX_TERMS) FAIL(SWF_E_UNSUPPORTED, "field %d: more than %d terms", f, swf::MAX_TERMS);
        std::vector<swf_term> tl;
        for (int i = a; i < b; ++i) {
            const swf_term& t = terms[i];
            if (t.mu < 0 || t.mu > 3) FAIL(SWF_E_ARG, "term %d: mu must be 0..3", i);
            const swf_profile* ps[4] = {&t.ft, &t.fx[0], &t.fx[1], &t.fx[2]};
            for (auto* p : ps) {
                if (p->type < 0 || p->type > 4) FAIL(SWF_E_ARG, "term %d: unknown profile type %d", i, p->type);
                if (p->type != SWF_PROF_CONST && !(p->w != 0)) FAIL(SWF_E_ARG, "term %d: profile width 0", i);
            }
            tl.push_back(t);
        }
        P.fields.push_back(tl);
    }
    // solves
    for (int i = 0; i < n_solves; ++i) {
        const swf_solve& s = solves[i];
        if (s.kind < 0 || s.kind > 3) FAIL(SWF_E_ARG, "solve %d: kind must be 0..3 (U_out, V_out, U_in, V_in)", i);
        if ((s.kind >= 2) != (solves[0].kind >= 2))
            FAIL(SWF_E_UNSUPPORTED, "solve %d: in- and out-states cannot share a context (opposite time directions)", i);
        if (s.spin != 1 && s.spin != -1) FAIL(SWF_E_ARG, "solve %d: spin must be +1 or -1", i);
        if (s.grid < 0 || s.grid >= n_grids) FAIL(SWF_E_ARG, "solve %d: bad grid index", i);
        if (s.field < 0 || s.field >= n_fields) FAIL(SWF_E_ARG, "solve %d: bad field index", i);
        const swf_grid& G = P.grids[s.grid];
        for (const auto& t : P.fields[s.field])
            for (int j = G.dim; j < 3; ++j)
                if (t.fx[j].type != SWF_PROF_CONST || t.fx[j].k != 0 || t.fx[j].phi != 0)
                    FAIL(SWF_E_ARG, "solve %d: its field depends on trivial axis %d", i, j);
        double emax2 = 1.0;
        for (int j = 0; j < 3; ++j) {
            if (!std::isfinite(s.p[j])) FAIL(SWF_E_ARG, "solve %d: non-finite momentum", i);
            if (j < G.dim) {
                const double kny = PI * G.n[j] / G.L[j];
                if (std::fabs(s.p[j]) >= kny) FAIL(SWF_E_ARG, "solve %d: |p[%d]| beyond the grid's Nyquist wavenumber %g", i, j, kny);
                emax2 += kny * kny;
            } else {
                emax2 += s.p[j] * s.p[j];
            }
        }
        if (win->dt * std::sqrt(emax2) >= 2.8)
            FAIL(SWF_E_ARG, "solve %d: dt * E_max = %g violates the RK4 stability bound 2.8", i, win->dt * std::sqrt(emax2));
        P.solves.push_back(s);
    }
    // vertices
    for (int v = 0; v < n_verts; ++v) {
        const swf_vertex& V = verts[v];
        if (V.u_solve < 0 || V.u_solve >= n_solves || V.v_solve < 0 || V.v_solve >= n_solves)
            FAIL(SWF_E_ARG, "vertex %d: bad solve index", v);
        const swf_solve &su = solves[V.u_solve], &sv = solves[V.v_solve];
        if (su.kind != 0 || sv.kind != 1) FAIL(SWF_E_ARG, "vertex %d: needs a U_out solve and a V_out solve", v);
        if (su.grid != sv.grid || su.field != sv.field) FAIL(SWF_E_ARG, "vertex %d: solves must share grid and field", v);
        const swf_grid& G = P.grids[su.grid];
        if (V.n_modes < 0 || V.n_modes > swf::MAX_MODES || (V.n_modes > 0 && !V.modes))
            FAIL(SWF_E_ARG, "vertex %d: n_modes must be 0..%d with a modes array", v, swf::MAX_MODES);
        if (V.n_modes > 0 && opt->bw_partial)
            FAIL(SWF_E_UNSUPPORTED, "vertex %d: wave packets do not combine with bw_partial", v);
        // the photon's plane-wave components: the vertex's own, or the packet's
        std::vector<std::array<double, 8>> ms;
        if (V.n_modes == 0) {
            ms.push_back({V.k[0], V.k[1], V.k[2], V.eps[0], V.eps[1], V.eps[2], 1.0, 0.0});
        } else {
            for (int m = 0; m < V.n_modes; ++m) {
                std::array<double, 8> r;
                for (int c = 0; c < 8; ++c) {
                    r[c] = V.modes[8 * m + c];
                    if (!std::isfinite(r[c])) FAIL(SWF_E_ARG, "vertex %d: mode %d is not finite", v, m);
                }
                ms.push_back(r);
            }
        }
        for (size_t m = 0; m < ms.size(); ++m) {
            const double* k = ms[m].data();
            if (!(std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]) > 0))
                FAIL(SWF_E_ARG, "vertex %d: photon momentum must be non-zero", v);
            for (int j = G.dim; j < 3; ++j)
                if (std::fabs(su.p[j] + sv.p[j] - k[j]) > 1e-9 * (1.0 + std::fabs(k[j])))
                    FAIL(SWF_E_ARG, "vertex %d: p + q != k on trivial axis %d", v, j);
        }
        P.verts.push_back(V);
        P.verts.back().modes = nullptr;   // the caller's array is not kept
        P.vmodes.push_back(V.n_modes > 0 ? ms : std::vector<std::array<double, 8>>());
        if (V.n_modes > 0) P.packets.push_back(v);
    }

    // ---- tables
    auto add_r = [&](const std::vector<double>& v) { size_t o = P.rtab.size(); P.rtab.insert(P.rtab.end(), v.begin(), v.end()); return o; };
    auto add_c = [&](const std::vector<cd>& v) { size_t o = P.ctab.size(); P.ctab.insert(P.ctab.end(), v.begin(), v.end()); return o; };
    auto xcoord = [&](const swf_grid& G, int j, int i) { return j < G.dim ? -0.5 * G.L[j] + i * (G.L[j] / G.n[j]) : 0.0; };
    // twiddles per length
    std::vector<std::pair<int, size_t>> twoff;
    auto tw_for = [&](int n) -> size_t {
        for (auto& p : twoff) if (p.first == n) return p.second;
        std::vector<cd> tw(n);
        for (int m = 0; m < n; ++m) tw[m] = std::polar(1.0, -2.0 * PI * m / n);
        size_t o = add_c(tw);
        twoff.push_back({n, o});
        return o;
    };
    // field tables per (grid, field)
    std::vector<std::pair<std::pair<int, int>, int>> combos;   // (grid, field) -> first TermDev
    for (int i = 0; i < n_solves; ++i) {
        const swf_solve& s = P.solves[i];
        const swf_grid& G = P.grids[s.grid];
        int first = -1;
        for (auto& c : combos) if (c.first.first == s.grid && c.first.second == s.field) first = c.second;
        if (first < 0) {
            first = (int)P.ht.size();
            for (const auto& t : P.fields[s.field]) {
                std::vector<double> tab;
                for (int j = 0; j < 3; ++j)
                    for (int k = 0; k < G.n[j]; ++k) tab.push_back(profile_h(t.fx[j], xcoord(G, j, k)));
                TermDev d;
                d.mu = t.mu;
                d.ft_type = t.ft.type;
                d.amp = t.amp;
                d.c = t.ft.c;
                d.w = t.ft.w;
                d.k = t.ft.k;
                d.phi = t.ft.phi;
                d.tab = (long long)add_r(tab);
                P.ht.push_back(d);
            }
            combos.push_back({{s.grid, s.field}, first});
        }
        SolveDev d;
        memset(&d, 0, sizeof(d));
        d.dim = G.dim;
        d.nsites = 1;
        for (int j = 0; j < 3; ++j) {
            d.n[j] = G.n[j];
            d.nsites *= G.n[j];
            d.dk[j] = 2.0 * PI / G.L[j];
        }
        d.nrows = G.n[1] * G.n[2];
        d.kind = s.kind % 2;                          // U or V (in- and out-states share the background)
        const double sgn = d.kind == 0 ? 1.0 : -1.0;   // K = p for U, -p for V
        for (int j = 0; j < 3; ++j) d.kap[j] = j >= G.dim ? sgn * s.p[j] : 0.0;
        Spinor w = free_spinor(d.kind, s.spin, s.p);
        for (int q = 0; q < 4; ++q) {
            d.w[2 * q] = w.c[q].real();
            d.w[2 * q + 1] = w.c[q].imag();
        }
        const double E = std::sqrt(1.0 + s.p[0] * s.p[0] + s.p[1] * s.p[1] + s.p[2] * s.p[2]);
        d.E = sgn * E;
        d.dV = 1.0;
        for (int j = 0; j < G.dim; ++j) d.dV *= G.L[j] / G.n[j];
        d.inv_n = 1.0 / (double)d.nsites;
        d.term0 = first;
        d.nterm = (int)P.fields[s.field].size();
        std::vector<cd> ph;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < G.n[j]; ++k) ph.push_back(j < G.dim ? std::polar(1.0, sgn * s.p[j] * xcoord(G, j, k)) : cd(1.0));
        d.ph = (long long)add_c(ph);
        d.mask = -1;
        if (G.absorb_cells > 0) {
            std::vector<double> m;
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < G.n[j]; ++k) {
                    double v = 1.0;
                    if (j < G.dim) {
                        const int dd = std::min(k, G.n[j] - 1 - k);
                        if (dd < G.absorb_cells) {
                            const double sn = std::sin(0.5 * PI * (G.absorb_cells - dd) / G.absorb_cells);
                            v = 1.0 - G.absorb_strength * sn * sn;
                        }
                    }
                    m.push_back(v);
                }
            d.mask = (long long)add_r(m);
        }
        for (int j = 0; j < 3; ++j) d.tw[j] = (long long)tw_for(G.n[j] > 1 ? G.n[j] : G.n[0]);
        P.hs.push_back(d);
    }
    for (int v = 0; v < n_verts; ++v) {
        const swf_vertex& V = P.verts[v];
        const swf_grid& G = P.grids[P.solves[V.u_solve].grid];
        VertexDev d;
        memset(&d, 0, sizeof(d));
        d.su = V.u_solve;
        d.sv = V.v_solve;
        d.k0 = std::sqrt(V.k[0] * V.k[0] + V.k[1] * V.k[1] + V.k[2] * V.k[2]);
        for (int j = 0; j < 3; ++j) d.eps[j] = V.eps[j];
        const double* pu = P.solves[V.u_solve].p;
        const double* qv = P.solves[V.v_solve].p;
        d.p0 = std::sqrt(1.0 + pu[0] * pu[0] + pu[1] * pu[1] + pu[2] * pu[2]);
        d.q0 = std::sqrt(1.0 + qv[0] * qv[0] + qv[1] * qv[1] + qv[2] * qv[2]);
        for (int j = 0; j < 3; ++j) {
            d.k[j] = V.k[j];
            d.kbs[j] = pu[j] - V.k[j];
            d.ksb[j] = V.k[j] - qv[j];
            d.x0[j] = xcoord(G, j, 0);
            d.dx[j] = j < G.dim ? G.L[j] / G.n[j] : 0.0;
        }
        std::vector<cd> ph;
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < G.n[j]; ++k) ph.push_back(j < G.dim ? std::polar(1.0, V.k[j] * xcoord(G, j, k)) : cd(1.0));
        d.phk = (long long)add_c(ph);
        d.nmodes = (int)P.vmodes[v].size();
        d.mode0 = (int)P.hm.size();
        for (const auto& r : P.vmodes[v]) {
            swf::ModeDev md;
            memset(&md, 0, sizeof(md));
            md.k0 = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            md.c[0] = r[6];
            md.c[1] = r[7];
            for (int j = 0; j < 3; ++j) md.eps[j] = r[3 + j];
            std::vector<cd> phm;
            for (int j = 0; j < 3; ++j)
                for (int k = 0; k < G.n[j]; ++k) phm.push_back(j < G.dim ? std::polar(1.0, r[j] * xcoord(G, j, k)) : cd(1.0));
            md.phk = (long long)add_c(phm);
            P.hm.push_back(md);
        }
        P.hv.push_back(d);
    }
    // vertices reduced together: greedily, at most 2 U and 2 V solves and 4
    // vertices of one grid and one photon per group, so a solve shared by
    // several vertices is read once per stage
    auto same_photon = [&](int v, int w) {
        for (int j = 0; j < 3; ++j)
            if (P.verts[v].k[j] != P.verts[w].k[j] || P.verts[v].eps[j] != P.verts[w].eps[j]) return false;
        return true;
    };
    for (int v = 0; v < n_verts; ++v) {
        if (P.verts[v].n_modes > 0) continue;   // wave packets have their own reduction
        const int su = P.verts[v].u_solve, sv = P.verts[v].v_solve;
        bool placed = false;
        for (auto& g : P.hg) {
            if (g.nvx >= swf::BWG_VERTS || P.solves[g.su[0]].grid != P.solves[su].grid || !same_photon(g.vtx[0], v))
                continue;
            int ui = -1, vi = -1;
            for (int k = 0; k < g.nu; ++k) if (g.su[k] == su) ui = k;
            for (int k = 0; k < g.nv; ++k) if (g.sv[k] == sv) vi = k;
            if ((ui < 0 && g.nu >= swf::BWG_SOLVES) || (vi < 0 && g.nv >= swf::BWG_SOLVES)) continue;
            if (ui < 0) { ui = g.nu; g.su[g.nu++] = su; }
            if (vi < 0) { vi = g.nv; g.sv[g.nv++] = sv; }
            g.vtx[g.nvx] = v;
            g.ui[g.nvx] = ui;
            g.vi[g.nvx] = vi;
            ++g.nvx;
            placed = true;
            break;
        }
        if (!placed) {
            swf::VertexGroupDev g;
            memset(&g, 0, sizeof(g));
            g.nu = g.nv = g.nvx = 1;
            g.su[0] = su;
            g.sv[0] = sv;
            g.vtx[0] = v;
            P.hg.push_back(g);
        }
    }
    std::stable_sort(P.hg.begin(), P.hg.end(), [](const swf::VertexGroupDev& a, const swf::VertexGroupDev& b) {
        return a.nu != b.nu ? a.nu < b.nu : a.nv < b.nv;
    });
    // per group: the constant spinors of the background terms and the spatial
    // phase tables of its three integrands, products formed in double once
    // (the time phases multiply the block sums)
    for (auto& g : P.hg) {
        const swf_vertex& V0 = P.verts[g.vtx[0]];
        const VertexDev& D0 = P.hv[g.vtx[0]];
        const swf_grid& G = P.grids[P.solves[g.su[0]].grid];
        const size_t nt = (size_t)G.n[0] + G.n[1] + G.n[2];
        for (int j = 0; j < 3; ++j) g.eps[j] = V0.eps[j];
        g.tk = D0.phk;
        for (int u = 0; u < g.nu; ++u) {
            const SolveDev& S = P.hs[g.su[u]];
            std::vector<cd> t(nt);
            for (size_t k = 0; k < nt; ++k) t[k] = std::conj(P.ctab[S.ph + k]) * P.ctab[D0.phk + k];
            g.t1[u] = (long long)add_c(t);
            for (int q = 0; q < 8; ++q) g.cu[u][q] = S.w[q];
        }
        for (int v = 0; v < g.nv; ++v) {
            const SolveDev& S = P.hs[g.sv[v]];
            std::vector<cd> t(nt);
            for (size_t k = 0; k < nt; ++k) t[k] = P.ctab[S.ph + k] * P.ctab[D0.phk + k];
            g.t2[v] = (long long)add_c(t);
            Spinor w;
            for (int q = 0; q < 4; ++q) w.c[q] = cd(S.w[2 * q], S.w[2 * q + 1]);
            const Spinor gw = gamma_eps(w, V0.eps);
            for (int q = 0; q < 4; ++q) {
                g.cv[v][2 * q] = gw.c[q].real();
                g.cv[v][2 * q + 1] = gw.c[q].imag();
            }
        }
    }
    // ---- groups and work items
    if (opt->chunk < 0) FAIL(SWF_E_ARG, "chunk must be >= 0");
    if (opt->check_every < 0) FAIL(SWF_E_ARG, "check_every must be >= 0");
    if (opt->graph_steps < 0) FAIL(SWF_E_ARG, "graph_steps must be >= 0");
    for (int g = 0; g < n_grids; ++g) {
        std::vector<int> all;
        for (int i = 0; i < n_solves; ++i) if (P.solves[i].grid == g) all.push_back(i);
        const size_t cs = opt->chunk > 0 ? (size_t)opt->chunk : std::max<size_t>(1, all.size());
        for (size_t a = 0; a < all.size(); a += cs) {
            Group gr;
            gr.grid = g;
            gr.solves.assign(all.begin() + a, all.begin() + std::min(all.size(), a + cs));
            add_items(P, gr, P.fp64);
            P.batched.push_back(gr);
        }
    }
    for (int i = 0; i < n_solves; ++i) {
        Group gr;
        gr.grid = P.solves[i].grid;
        gr.solves.push_back(i);
        add_items(P, gr, P.fp64);
        P.single.push_back(gr);
    }
    // ---- layout
    P.bw2 = opt->bw_partial != 0 && n_verts > 0;
    P.aux.assign(n_solves, 0);
    if (P.bw2) {
        for (const auto& V : P.verts) P.aux[V.u_solve] = P.aux[V.v_solve] = 1;
        for (int i = 0; i < n_solves; ++i)
            if (P.aux[i]) P.bw2_solves.push_back(i);
    }
    size_t off = 0;
    P.off_state = 0;
    for (int i = 0; i < n_solves; ++i) {
        P.solve_off.push_back(off);
        off += (size_t)nbufs(P, i) * align256(4 * (size_t)P.hs[i].nsites * P.csize);
    }
    P.state_bytes = off;
    P.off_solves = off = align256(off);
    off += sizeof(SolveDev) * n_solves;
    P.off_terms = off = align256(off);
    off += sizeof(TermDev) * std::max<size_t>(1, P.ht.size());
    P.off_verts = off = align256(off);
    off += sizeof(VertexDev) * std::max(1, n_verts);
    P.off_vgroups = off = align256(off);
    off += sizeof(swf::VertexGroupDev) * std::max<size_t>(1, P.hg.size());
    P.off_modes = off = align256(off);
    off += sizeof(swf::ModeDev) * std::max<size_t>(1, P.hm.size());
    P.off_packets = off = align256(off);
    off += sizeof(int) * std::max<size_t>(1, P.packets.size());
    P.off_rtab = off = align256(off);
    off += P.rsize * std::max<size_t>(1, P.rtab.size());
    P.off_ctab = off = align256(off);
    off += P.csize * std::max<size_t>(1, P.ctab.size());
    P.off_items = off = align256(off);
    off += sizeof(int2) * std::max<size_t>(1, P.items.size());
    P.off_step = off = align256(off);
    off += 256;
    P.off_M = off = align256(off);
    off += sizeof(double2) * 3 * std::max(1, n_verts);
    P.off_part = off = align256(off);
    off += sizeof(double2) * 3 * P.nst * (size_t)BW_BLOCKS * std::max(1, n_verts);
    P.off_red = off = align256(off);
    off += sizeof(double2) * 4 * (size_t)RED_BLOCKS;
    if (P.bw2) {
        P.off_M2 = off = align256(off);
        off += sizeof(double2) * 3 * n_verts;
        P.off_part2 = off = align256(off);
        off += sizeof(double2) * 4 * 9 * (size_t)BW_BLOCKS * n_verts;
    }
    P.total = align256(off);
    return SWF_OK;
}

}  // namespace

// ------------------------------------------------------------ context
struct PendingEv { hipEvent_t a, b; int kind; double bytes; };

struct swf_ctx {
    Plan P;
    swf_options opt{};
    hipStream_t user = nullptr, st = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    char* arena = nullptr;
    bool own_arena = false;
    int step = 0;
    size_t lds_max = 65536;       // dynamic LDS one workgroup may use on this device
    int ncu = 256;                // compute units of this device
    void* pm_buf = nullptr;       // pair-matrix scratch (grown on demand, freed by swf_free)
    size_t pm_bytes = 0;
    void* noalloc_scratch = nullptr;   // this device's static scratch array (swf_pair_matrix_noalloc)
    std::vector<char> kvalid;
    std::vector<int> bw_done;
    std::vector<cd> bw_cache;     // 3 terms finite + 3 past per vertex
    hipGraph_t graph = nullptr, graph_k = nullptr;   // one step; graph_steps steps
    hipGraphExec_t gexec = nullptr, gexec_k = nullptr;
    int graph_k_steps = 0;
    std::string err;
    std::string tune_path;
    std::string tune_report;
    // profiling
    std::vector<hipEvent_t> ev_free;
    std::vector<PendingEv> pending;
    long long st_launch[NKIND] = {};
    double st_ms[NKIND] = {};
    double st_bytes[NKIND] = {};

    SolveDev* d_solves() { return (SolveDev*)(arena + P.off_solves); }
    TermDev* d_terms() { return (TermDev*)(arena + P.off_terms); }
    VertexDev* d_verts() { return (VertexDev*)(arena + P.off_verts); }
    swf::VertexGroupDev* d_vgroups() { return (swf::VertexGroupDev*)(arena + P.off_vgroups); }
    swf::ModeDev* d_modes() { return (swf::ModeDev*)(arena + P.off_modes); }
    int* d_packets() { return (int*)(arena + P.off_packets); }
    void* d_rtab() { return arena + P.off_rtab; }
    void* d_ctab() { return arena + P.off_ctab; }
    int2* d_items() { return (int2*)(arena + P.off_items); }
    int* d_step() { return (int*)(arena + P.off_step); }
    // first (step, solve) of a non-finite value seen by the in-loop check, as ~key (0: none)
    unsigned long long* d_flag() { return (unsigned long long*)(arena + P.off_step + 64); }
    double2* d_M() { return (double2*)(arena + P.off_M); }
    double2* d_part() { return (double2*)(arena + P.off_part); }
    double2* d_red() { return (double2*)(arena + P.off_red); }
    double2* d_M2() { return (double2*)(arena + P.off_M2); }
    double2* d_part2() { return (double2*)(arena + P.off_part2); }
    void* buf(int s, int role) { return arena + P.off_state + P.solve_off[s] + role * align256(4 * (size_t)P.hs[s].nsites * P.csize); }
};

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) {                                                               \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(_e);                     \
            return SWF_E_HIP;                                                                 \
        }                                                                                     \
    } while (0)

namespace {

// Order the context's own stream after the caller's stream (on entry) and the
// caller's stream after the context's work (on exit).
static int enter(swf_ctx* ctx) {
    HIPCHK(hipEventRecord(ctx->ev_in, ctx->user));
    HIPCHK(hipStreamWaitEvent(ctx->st, ctx->ev_in, 0));
    return SWF_OK;
}
static int leave(swf_ctx* ctx) {
    HIPCHK(hipEventRecord(ctx->ev_out, ctx->st));
    HIPCHK(hipStreamWaitEvent(ctx->user, ctx->ev_out, 0));
    return SWF_OK;
}

static int drain_profile(swf_ctx* ctx) {
    for (auto& p : ctx->pending) {
        HIPCHK(hipEventSynchronize(p.b));
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
        ctx->st_launch[p.kind] += 1;
        ctx->st_ms[p.kind] += ms;
        ctx->st_bytes[p.kind] += p.bytes;
        ctx->ev_free.push_back(p.a);
        ctx->ev_free.push_back(p.b);
    }
    ctx->pending.clear();
    return SWF_OK;
}

static int get_event(swf_ctx* ctx, hipEvent_t* e) {
    if (ctx->ev_free.empty()) {
        if ((int)ctx->pending.size() >= PROF_POOL) {
            int r = drain_profile(ctx);
            if (r) return r;
        }
    }
    if (!ctx->ev_free.empty()) {
        *e = ctx->ev_free.back();
        ctx->ev_free.pop_back();
        return SWF_OK;
    }
    HIPCHK(hipEventCreate(e));
    return SWF_OK;
}

static swf::PassArgs pass_args(swf_ctx* ctx) {
    swf::PassArgs a;
    memset(&a, 0, sizeof(a));
    a.solves = ctx->d_solves();
    a.terms = ctx->d_terms();
    a.rtab = ctx->d_rtab();
    a.ctab = ctx->d_ctab();
    a.step = ctx->d_step();
    a.t_out = ctx->P.t0;
    a.dt = ctx->P.sdt;
    return a;
}

static double group_sites(swf_ctx* ctx, const Group& g) {
    double s = 0;
    for (int i : g.solves) s += (double)ctx->P.hs[i].nsites;
    return s;
}

// Launch one pass kernel over n items starting at item offset `it`.
// maxblocks > 0: a persistent kernel that loops over the items with the grid's
// stride, given at most that many workgroups per blockIdx.y.
static int launch(swf_ctx* ctx, const void* fn, int nitems, size_t it, int threads, size_t lds, swf::PassArgs a,
                  int kind, double bytes, int gy = 1, int maxblocks = 0) {
    if (nitems <= 0) return SWF_OK;
    a.items = ctx->d_items() + it;
    a.nitems = nitems;
    const int blocks = maxblocks > 0 ? std::min(nitems, maxblocks) : nitems;
    void* args[] = {&a};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = ctx->opt.profile && !ctx->gexec;
    if (prof) {
        int r = get_event(ctx, &e0);
        if (!r) r = get_event(ctx, &e1);
        if (r) return r;
        HIPCHK(hipEventRecord(e0, ctx->st));
    }
    HIPCHK(hipLaunchKernel(fn, dim3(blocks, gy), dim3(threads), args, lds, ctx->st));
    if (prof) {
        HIPCHK(hipEventRecord(e1, ctx->st));
        ctx->pending.push_back({e0, e1, kind, bytes});
    }
    return SWF_OK;
}

// x-axis pass of a group in the given mode (ROW_STAGE: the RK4 stage pass).
static int row_pass(swf_ctx* ctx, const Group& g, int mode, int stage, int src, int dst, double tex, long long ph2,
                    int kind = 4, int expo = 0, double tau = 0.0) {
    const auto* k = g.k[0];
    swf::PassArgs a = pass_args(ctx);
    a.stage = stage;
    a.src = src;
    a.dst = dst;
    a.t_explicit = tex;
    a.ph2 = ph2;
    a.h0row = ctx->P.grids[g.grid].dim == 1 ? 1 : 0;
    a.expo = expo;
    a.tau = tau;
    double trav = 2;
    if (mode == swf::ROW_STAGE) {
        // stage input, the G buffer (2D, 3D), the RK4 operand and outputs; for
        // Dormand-Prince also y and the earlier slopes read, the slope written
        static const double tr[4] = {2, 4, 3, 3};
        static const double tr5[6] = {3, 5, 6, 7, 8, 7};
        trav = (ctx->P.dp5 ? tr5[stage] : tr[stage]) + (ctx->P.grids[g.grid].dim >= 2 ? 1 : 0);
    } else if (mode == swf::ROW_RHS) {
        trav = 3;
    }
    const double bytes = trav * 4.0 * ctx->P.csize * group_sites(ctx, g);
    if (mode == swf::ROW_STAGE) {
        const auto& v = k->row[g.vr];
        return launch(ctx, ctx->P.dp5 ? v.dp5[stage] : v.stage[stage], g.n_row[g.vr], g.it_row[g.vr], v.threads,
                      v.lds, a, kind, bytes);
    }
    return launch(ctx, k->row_other[mode], g.n_orow, g.it_orow, k->row0_threads, k->row0_lds, a, kind, bytes);
}

// Whole-state column transform of a group along `axis` (in place on `role`).
static int col_pass(swf_ctx* ctx, const Group& g, int axis, int mode, int role, int kind = 4, int expo = 0,
                    double tau = 0.0) {
    const auto& cv = g.k[axis]->col;
    swf::PassArgs a = pass_args(ctx);
    a.dst = role;
    a.src = role;
    a.expo = expo;
    a.tau = tau;
    const int n = axis == 1 ? g.n_ocy : g.n_ocz;
    const size_t it = axis == 1 ? g.it_ocy : g.it_ocz;
    return launch(ctx, cv.fn[axis - 1][mode], n, it, cv.threads, cv.lds, a, kind,
                  2.0 * 4.0 * ctx->P.csize * group_sites(ctx, g));
}

// Stepping column pass along `axis` of the stage input `src`: alpha^j D_j of
// every component into the G buffer (written for y, added for z).
static int cd_pass(swf_ctx* ctx, const Group& g, int axis, int src, int kind) {
    const int v = axis == 1 ? g.vy : g.vz;
    const auto& cv = g.k[axis]->cd[v];
    const int accum = axis == 2 ? 1 : 0;
    swf::PassArgs a = pass_args(ctx);
    a.src = src;
    a.dst = swf::BUF_T;
    const int n = axis == 1 ? g.n_coly[v] : g.n_colz[v];
    const size_t it = axis == 1 ? g.it_coly[v] : g.it_colz[v];
    // persistent y passes: one workgroup per compute unit (all the LDS they leave room for)
    return launch(ctx, cv.fn[axis - 1][accum], n, it, cv.threads, cv.lds, a, kind,
                  (2.0 + accum) * 4.0 * ctx->P.csize * group_sites(ctx, g), 4, cv.pipe && !accum ? ctx->ncu : 0);
}

// The passes of one RK4 stage of a group: the column derivatives of the stage
// input, then the row pass.
static int stage_passes(swf_ctx* ctx, const Group& g, int s) {
    const int dim = ctx->P.grids[g.grid].dim;
    const int src = s == 0 ? swf::BUF_Y : swf::BUF_YS;
    int r = SWF_OK;
    if (dim >= 2) r = cd_pass(ctx, g, 1, src, 1);
    if (!r && dim >= 3) r = cd_pass(ctx, g, 2, src, 2);
    if (!r) r = row_pass(ctx, g, swf::ROW_STAGE, s, 0, 0, 0, 0, 0);
    return r;
}

// k-space kinetic term of a whole state that the forward x pass left in
// `role` (operator test hook): column transforms with -i H0 / N on the last axis.
static int kinetic_cols(swf_ctx* ctx, const Group& g, int role) {
    const int dim = ctx->P.grids[g.grid].dim;
    int r = SWF_OK;
    if (dim == 2) r = col_pass(ctx, g, 1, swf::COL_H0, role);
    if (dim == 3) {
        r = col_pass(ctx, g, 1, swf::COL_FWD, role);
        if (!r) r = col_pass(ctx, g, 2, swf::COL_H0, role);
        if (!r) r = col_pass(ctx, g, 1, swf::COL_INV, role);
    }
    return r;
}

static const std::vector<Group>& groups(swf_ctx* ctx) { return ctx->opt.batched ? ctx->P.batched : ctx->P.single; }

static int bw_stage(swf_ctx* ctx, int stage) {
    if (ctx->P.hv.empty()) return SWF_OK;
    swf::BwArgs b;
    memset(&b, 0, sizeof(b));
    b.solves = ctx->d_solves();
    b.verts = ctx->d_verts();
    b.ctab = ctx->d_ctab();
    b.step = ctx->d_step();
    b.t_out = ctx->P.win.t_out;
    b.dt = ctx->P.win.dt;
    b.stage = stage;
    b.cst = ctx->P.cst[stage];
    b.nst = ctx->P.nst;
    b.nvert = (int)ctx->P.hv.size();
    b.part = ctx->d_part();
    b.M = ctx->d_M();
    b.groups = ctx->d_vgroups();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool prof = ctx->opt.profile && !ctx->gexec;
    if (prof) {
        int r = get_event(ctx, &e0);
        if (!r) r = get_event(ctx, &e1);
        if (r) return r;
        HIPCHK(hipEventRecord(e0, ctx->st));
    }
    b.modes = ctx->d_modes();
    b.packets = ctx->d_packets();
    // one launch per group shape (the groups are sorted by shape)
    const auto& hg = ctx->P.hg;
    for (size_t g0 = 0; g0 < hg.size();) {
        size_t g1 = g0;
        while (g1 < hg.size() && hg[g1].nu == hg[g0].nu && hg[g1].nv == hg[g0].nv) ++g1;
        swf::BwArgs bg = b;
        bg.groups = ctx->d_vgroups() + g0;
        HIPCHK(swf::launch_bw_stage(ctx->P.fp64, bg, BW_BLOCKS, hg[g0].nu, hg[g0].nv, (int)(g1 - g0), ctx->st));
        g0 = g1;
    }
    if (!ctx->P.packets.empty())
        HIPCHK(swf::launch_bw_packet_stage(ctx->P.fp64, b, BW_BLOCKS, (int)ctx->P.packets.size(), ctx->st));
    if (prof) {
        // every state of a group's solves is read once; a packet reads its two
        double bytes = 0;
        for (auto& g : ctx->P.hg) bytes += (g.nu + g.nv) * 4.0 * ctx->P.csize * (double)ctx->P.hs[g.su[0]].nsites;
        for (int v : ctx->P.packets) bytes += 2.0 * 4.0 * ctx->P.csize * (double)ctx->P.hs[ctx->P.hv[v].su].nsites;
        HIPCHK(hipEventRecord(e1, ctx->st));
        ctx->pending.push_back({e0, e1, 3, bytes});
    }
    return SWF_OK;
}

static int bw_accum(swf_ctx* ctx) {
    if (ctx->P.hv.empty()) return SWF_OK;
    swf::BwArgs b;
    memset(&b, 0, sizeof(b));
    b.solves = ctx->d_solves();
    b.verts = ctx->d_verts();
    b.dt = ctx->P.win.dt;
    b.nst = ctx->P.nst;
    for (int st = 0; st < ctx->P.nst; ++st) b.wst[st] = ctx->P.wst[st];
    b.nvert = (int)ctx->P.hv.size();
    b.part = ctx->d_part();
    b.M = ctx->d_M();
    HIPCHK(swf::launch_bw_accum(b, BW_BLOCKS, ctx->st));
    return SWF_OK;
}

// Partial-integration BW route at one RK4 stage (see bw2_src_kernel): the
// source S of every vertex solve into its A1 buffer, the x-space Fourier sums
// of the (b,s) and (s,b) terms, then per vertex the full transforms
// U~ = FFT(U), S~_U = FFT(S_U), V~' = FFT(V e^{i k.x}), S~'_V = FFT(S_V e^{i k.x})
// into A0 / A1 and the k-space (s,s) sum.  A solve's transforms are reused by
// the next vertex that needs the same photon phase.
static int bw2_stage(swf_ctx* ctx, int stage) {
    const Plan& P = ctx->P;
    const int src = stage == 0 ? swf::BUF_Y : swf::BUF_YS;
    int r = SWF_OK;
    for (int i : P.bw2_solves) {
        r = row_pass(ctx, P.single[i], swf::ROW_SRC, stage, src, swf::BUF_A1, 0, 0);
        if (r) return r;
    }
    swf::BwArgs b;
    memset(&b, 0, sizeof(b));
    b.solves = ctx->d_solves();
    b.verts = ctx->d_verts();
    b.step = ctx->d_step();
    b.t_out = P.win.t_out;
    b.dt = P.win.dt;
    b.stage = stage;
    b.nvert = (int)P.hv.size();
    b.part2 = ctx->d_part2();
    b.M2 = ctx->d_M2();
    HIPCHK(swf::launch_bw2_src(P.fp64, b, BW_BLOCKS, ctx->st));
    // phase held by each solve's A0/A1: NONE = A1 still holds S in x space
    const long long NONE = -2;
    std::vector<long long> held(P.solves.size(), NONE);
    auto transform = [&](int i, long long ph) -> int {
        if (held[i] == ph) return SWF_OK;
        const Group& g = P.single[i];
        int rr = SWF_OK;
        if (held[i] != NONE) rr = row_pass(ctx, g, swf::ROW_SRC, stage, src, swf::BUF_A1, 0, 0);
        const int mode = ph < 0 ? swf::ROW_FWD : swf::ROW_FWDPH;
        const long long ph2 = ph < 0 ? 0 : ph;
        if (!rr) rr = row_pass(ctx, g, mode, 0, src, swf::BUF_A0, 0, ph2);
        if (!rr) rr = row_pass(ctx, g, mode, 0, swf::BUF_A1, swf::BUF_A1, 0, ph2);
        for (int ax = 1; !rr && ax < P.grids[g.grid].dim; ++ax) {
            rr = col_pass(ctx, g, ax, swf::COL_FWD, swf::BUF_A0);
            if (!rr) rr = col_pass(ctx, g, ax, swf::COL_FWD, swf::BUF_A1);
        }
        held[i] = ph;
        return rr;
    };
    for (int v = 0; v < (int)P.hv.size(); ++v) {
        r = transform(P.hv[v].su, -1);
        if (!r) r = transform(P.hv[v].sv, P.hv[v].phk);
        if (r) return r;
        b.vtx = v;
        HIPCHK(swf::launch_bw2_kss(P.fp64, b, BW_BLOCKS, ctx->st));
    }
    return SWF_OK;
}

static int bw2_accum(swf_ctx* ctx) {
    swf::BwArgs b;
    memset(&b, 0, sizeof(b));
    b.solves = ctx->d_solves();
    b.verts = ctx->d_verts();
    b.step = ctx->d_step();
    b.t_out = ctx->P.win.t_out;
    b.dt = ctx->P.win.dt;
    b.nvert = (int)ctx->P.hv.size();
    b.part2 = ctx->d_part2();
    b.M2 = ctx->d_M2();
    HIPCHK(swf::launch_bw2_accum(b, BW_BLOCKS, ctx->st));
    return SWF_OK;
}

// ---- interaction picture (Lawson's integrating-factor RK4)
// The free evolution exp(-i H0 tau) of a whole state, in place: the forward x
// transform into the work buffer T, the column transforms with the propagator
// applied on the last axis (in the inverse x transform for 1D), the inverse x
// transform back.
static int free_evolve(swf_ctx* ctx, const Group& g, int role, double tau) {
    const int dim = ctx->P.grids[g.grid].dim;
    int r = row_pass(ctx, g, swf::ROW_FWD, 0, role, swf::BUF_T, 0, 0);
    if (!r && dim == 2) r = col_pass(ctx, g, 1, swf::COL_H0, swf::BUF_T, 4, 1, tau);
    if (!r && dim == 3) {
        r = col_pass(ctx, g, 1, swf::COL_FWD, swf::BUF_T);
        if (!r) r = col_pass(ctx, g, 2, swf::COL_H0, swf::BUF_T, 4, 1, tau);
        if (!r) r = col_pass(ctx, g, 1, swf::COL_INV, swf::BUF_T);
    }
    if (!r) r = row_pass(ctx, g, swf::ROW_INV, 0, role, role, 0, 0, 4, 1, tau);
    return r;
}

// out_j = sum_i c[j][i] in_i over a group's states (roles; -1 unused).
static int combo(swf_ctx* ctx, const Group& g, const int (&in)[3], const int (&out)[2], const double (&c)[2][3],
                 int mask = 0) {
    swf::ComboArgs a;
    memset(&a, 0, sizeof(a));
    a.solves = ctx->d_solves();
    a.items = ctx->d_items() + g.it_orow;
    a.rows = g.k[0]->row0_rows;
    a.rtab = ctx->d_rtab();
    for (int i = 0; i < 3; ++i) {
        a.in[i] = in[i];
        a.c[0][i] = c[0][i];
        a.c[1][i] = c[1][i];
    }
    a.out[0] = out[0];
    a.out[1] = out[1];
    a.mask = mask;
    HIPCHK(swf::launch_combo(ctx->P.fp64, a, g.n_orow, ctx->st));
    return SWF_OK;
}

// One step: with h the signed step, E = exp(-i H0 h/2) and N(t, y) = -i V(t) (y + psi_b),
//   k1 = N(t, y),                a = E (y + h/2 k1),
//   k2 = N(t + h/2, a),          b = E y + h/2 k2,
//   k3 = N(t + h/2, b),          c = E (E y + h k3),
//   k4 = N(t + h, c),            y' = E (E (y + h/6 k1) + h/3 (k2 + k3)) + h/6 k4
// (= E^2 y + h/6 (E^2 k1 + 2 E k2 + 2 E k3 + k4)).  The stage inputs y, a, b, c
// pass through YS (y itself at stage 0) so that the BW reductions read them as
// for the classical stepper; ACC carries the update, A0 the sum k2 + k3, A1 the
// latest slope, T is the transforms' work buffer.
static int ip_step(swf_ctx* ctx) {
    using namespace swf;
    const double h = -ctx->P.sdt;
    auto each = [&](auto&& f) {
        for (const auto& g : groups(ctx)) {
            int r = f(g);
            if (r) return r;
        }
        return (int)SWF_OK;
    };
    int r = bw_stage(ctx, 0);
    if (!r) r = each([&](const Group& g) {
        int rr = row_pass(ctx, g, ROW_SRC, 0, BUF_Y, BUF_A1, 0, 0);
        if (!rr) rr = combo(ctx, g, {BUF_Y, BUF_A1, -1}, {BUF_YS, BUF_ACC}, {{1.0, 0.5 * h, 0.0}, {1.0, h / 6.0, 0.0}});
        if (!rr) rr = free_evolve(ctx, g, BUF_YS, 0.5 * h);   // a
        if (!rr) rr = free_evolve(ctx, g, BUF_Y, 0.5 * h);    // E y
        return rr;
    });
    if (!r) r = bw_stage(ctx, 1);
    if (!r) r = each([&](const Group& g) {
        int rr = row_pass(ctx, g, ROW_SRC, 1, BUF_YS, BUF_A1, 0, 0);
        if (!rr) rr = combo(ctx, g, {BUF_Y, BUF_A1, -1}, {BUF_YS, BUF_A0}, {{1.0, 0.5 * h, 0.0}, {0.0, 1.0, 0.0}});   // b, k2
        return rr;
    });
    if (!r) r = bw_stage(ctx, 2);
    if (!r) r = each([&](const Group& g) {
        int rr = row_pass(ctx, g, ROW_SRC, 2, BUF_YS, BUF_A1, 0, 0);
        if (!rr) rr = combo(ctx, g, {BUF_Y, BUF_A1, BUF_A0}, {BUF_YS, BUF_A0}, {{1.0, h, 0.0}, {0.0, 1.0, 1.0}});
        if (!rr) rr = free_evolve(ctx, g, BUF_YS, 0.5 * h);   // c
        if (!rr) rr = free_evolve(ctx, g, BUF_ACC, 0.5 * h);
        if (!rr) rr = combo(ctx, g, {BUF_ACC, BUF_A0, -1}, {BUF_ACC, -1}, {{1.0, h / 3.0, 0.0}, {0.0, 0.0, 0.0}});
        if (!rr) rr = free_evolve(ctx, g, BUF_ACC, 0.5 * h);
        return rr;
    });
    if (!r) r = bw_stage(ctx, 3);
    if (!r) r = each([&](const Group& g) {
        int rr = row_pass(ctx, g, ROW_SRC, 3, BUF_YS, BUF_A1, 0, 0);
        if (!rr) rr = combo(ctx, g, {BUF_ACC, BUF_A1, -1}, {BUF_Y, -1}, {{1.0, h / 6.0, 0.0}, {0.0, 0.0, 0.0}}, 1);
        return rr;
    });
    if (!r) r = bw_accum(ctx);
    if (r) return r;
    HIPCHK(swf::launch_tick(ctx->d_step(), ctx->st));
    return SWF_OK;
}

// Enqueue one full RK4 step of every solve.
static int enqueue_step(swf_ctx* ctx) {
    if (ctx->P.ip) return ip_step(ctx);
    if (ctx->opt.batched && ctx->opt.chunk > 0 && ctx->P.hv.empty()) {
        // chunk-major: all stages of one chunk before the next chunk
        for (const auto& g : groups(ctx))
            for (int s = 0; s < ctx->P.nst; ++s) {
                int r = stage_passes(ctx, g, s);
                if (r) return r;
            }
        HIPCHK(swf::launch_tick(ctx->d_step(), ctx->st));
        return SWF_OK;
    }
    for (int s = 0; s < ctx->P.nst; ++s) {
        int r = bw_stage(ctx, s);
        if (!r && ctx->P.bw2) r = bw2_stage(ctx, s);
        if (r) return r;
        for (const auto& g : groups(ctx)) {
            r = stage_passes(ctx, g, s);
            if (r) return r;
        }
    }
    int r = bw_accum(ctx);
    if (!r && ctx->P.bw2) r = bw2_accum(ctx);
    if (r) return r;
    HIPCHK(swf::launch_tick(ctx->d_step(), ctx->st));
    return SWF_OK;
}

// One-dimensional whole-loop path: every group is a 1D grid with a line
// kernel and no vertex couples two solves.
static size_t line_lds(const swf_ctx* ctx, const Group& g, int nterm_max, int wide) {
    return g.k[0]->line_lds[wide] + (size_t)nterm_max * ctx->P.grids[g.grid].n[0] * ctx->P.rsize;
}

static int max_terms(const swf_ctx* ctx, const Group& g) {
    int m = 0;
    for (int i : g.solves) m = std::max(m, ctx->P.hs[i].nterm);
    return m;
}

// The line kernel build a group runs: 1 wide exchange rounds, 0 narrow, -1
// none fits the LDS of one workgroup.
static int line_build(const swf_ctx* ctx, const Group& g) {
    if (ctx->P.grids[g.grid].dim != 1 || !g.k[0]->line[0]) return -1;
    const int nt = max_terms(ctx, g);
    for (int w = 1; w >= 0; --w)
        if (line_lds(ctx, g, nt, w) + LINE_STATIC_LDS <= ctx->lds_max) return w;
    return -1;
}

// One-dimensional whole-loop path: every group is a 1D grid with a line
// kernel whose LDS (with the group's field terms) fits, and no vertex couples
// two solves.
static bool line_path(swf_ctx* ctx) {
    if (!ctx->opt.persistent || !ctx->P.hv.empty() || ctx->P.dp5 || ctx->P.ip) return false;
    for (const auto& g : groups(ctx))
        if (line_build(ctx, g) < 0) return false;
    return true;
}

// n RK4 steps of every solve: launches of at most LINE_STEPS steps each, then
// the device step counter is advanced by the same count.
constexpr int LINE_STEPS = 1024;
static int line_steps(swf_ctx* ctx, int n) {
    for (int done = 0; done < n;) {
        const int c = std::min(LINE_STEPS, n - done);
        for (const auto& g : groups(ctx)) {
            swf::PassArgs a = pass_args(ctx);
            a.nsteps = c;
            const double bytes = 2.0 * 4.0 * ctx->P.csize * group_sites(ctx, g);
            const int w = line_build(ctx, g);
            int r = launch(ctx, g.k[0]->line[w], g.n_row[0], g.it_row[0], g.k[0]->line_threads,
                           line_lds(ctx, g, max_terms(ctx, g), w), a, 5, bytes);
            if (r) return r;
        }
        HIPCHK(swf::launch_advance(ctx->d_step(), c, ctx->st));
        done += c;
    }
    return SWF_OK;
}

// Capture `steps` consecutive time steps (every launch, the device step
// counter advanced by each) as one graph.
static int capture_steps(swf_ctx* ctx, int steps, hipGraph_t* graph, hipGraphExec_t* exec) {
    HIPCHK(hipStreamBeginCapture(ctx->st, hipStreamCaptureModeThreadLocal));
    int r = SWF_OK;
    for (int i = 0; i < steps && !r; ++i) r = enqueue_step(ctx);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->st, &g);
    if (r) {
        if (g) hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) {
        ctx->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
        return SWF_E_HIP;
    }
    *graph = g;
    HIPCHK(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
    return SWF_OK;
}

// The one-step graph, and with options.graph_steps > 1 a graph of that many
// steps, replayed while at least that many steps remain.
static int build_graph(swf_ctx* ctx) {
    int r = capture_steps(ctx, 1, &ctx->graph, &ctx->gexec);
    if (r || ctx->opt.graph_steps <= 1) return r;
    ctx->graph_k_steps = std::min(ctx->opt.graph_steps, ctx->P.steps);
    return capture_steps(ctx, ctx->graph_k_steps, &ctx->graph_k, &ctx->gexec_k);
}

// ------------------------------------------------------------ autotuner
// Times every tile variant of the three stepping passes of each group on the
// problem itself (zero state, stage 1), keeps the fastest, and caches the
// choice by (precision, grid, batch size) in a text file.
static std::string tune_key(swf_ctx* ctx, const Group& g) {
    const swf_grid& G = ctx->P.grids[g.grid];
    char b[160];
    snprintf(b, sizeof(b), "deriv%s %s d%d n%dx%dx%d b%zu", ctx->P.dp5 ? "-dp5" : "", ctx->P.fp64 ? "f64" : "f32", G.dim,
             G.n[0], G.n[1], G.n[2], g.solves.size());
    return b;
}

static int time_it(swf_ctx* ctx, const std::function<int()>& f, int reps, float* ms) {
    hipEvent_t a = nullptr, b = nullptr;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    int r = f();
    if (!r) {
        HIPCHK(hipEventRecord(a, ctx->st));
        for (int i = 0; i < reps && !r; ++i) r = f();
        HIPCHK(hipEventRecord(b, ctx->st));
        HIPCHK(hipEventSynchronize(b));
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, a, b));
        *ms = t / reps;
    }
    hipEventDestroy(a);
    hipEventDestroy(b);
    return r;
}

static int autotune(swf_ctx* ctx, std::vector<Group>& gl) {
    std::map<std::string, std::array<int, 3>> cache;
    if (!ctx->tune_path.empty()) {
        std::ifstream in(ctx->tune_path);
        std::string line;
        while (std::getline(in, line)) {
            const size_t bar = line.find('|');
            if (bar == std::string::npos) continue;
            std::istringstream vs(line.substr(bar + 1));
            std::array<int, 3> v{0, 0, 0};
            vs >> v[0] >> v[1] >> v[2];
            if (vs) cache[line.substr(0, bar)] = v;
        }
    }
    const int prof = ctx->opt.profile;
    ctx->opt.profile = 0;
    std::ostringstream rep;
    for (auto& g : gl) {
        const std::string key = tune_key(ctx, g);
        auto it = cache.find(key);
        const int dim = ctx->P.grids[g.grid].dim;
        if (it != cache.end()) {
            g.vr = std::min(it->second[0], g.k[0]->nvar - 1);
            g.vy = dim >= 2 ? std::min(it->second[1], g.k[1]->nvar - 1) : 0;
            g.vz = dim >= 3 ? std::min(it->second[2], g.k[2]->nvar - 1) : 0;
            rep << key << ": cached " << g.vr << " " << g.vy << " " << g.vz << "\n";
            continue;
        }
        const int reps = 4;
        float best = 1e30f;
        int bv = 0;
        for (int v = 0; v < g.k[0]->nvar; ++v) {
            g.vr = v;
            float ms = 0;
            const int st = ctx->P.dp5 ? 3 : 1;   // a middle stage of the stepper
            int r = time_it(ctx, [&] { return row_pass(ctx, g, swf::ROW_STAGE, st, 0, 0, 0, 0, 4); }, reps, &ms);
            if (r) { ctx->opt.profile = prof; return r; }
            rep << key << ": row v" << v << " " << ms << " ms\n";
            if (ms < best) { best = ms; bv = v; }
        }
        g.vr = bv;
        for (int axis = 1; axis < dim; ++axis) {
            best = 1e30f;
            bv = 0;
            for (int v = 0; v < g.k[axis]->nvar; ++v) {
                (axis == 1 ? g.vy : g.vz) = v;
                float ms = 0;
                int r = time_it(ctx, [&] { return cd_pass(ctx, g, axis, swf::BUF_YS, 4); }, reps, &ms);
                if (r) { ctx->opt.profile = prof; return r; }
                rep << key << ": col" << axis << " v" << v << " " << ms << " ms\n";
                if (ms < best) { best = ms; bv = v; }
            }
            (axis == 1 ? g.vy : g.vz) = bv;
        }
        cache[key] = {g.vr, g.vy, g.vz};
        if (!ctx->tune_path.empty()) {
            std::ofstream out(ctx->tune_path, std::ios::app);
            out << key << "|" << g.vr << " " << g.vy << " " << g.vz << "\n";
        }
    }
    ctx->opt.profile = prof;
    ctx->tune_report = rep.str();
    // the tuning launches stepped the state: start from psi_s(t_out) = 0 again
    HIPCHK(hipMemsetAsync(ctx->arena + ctx->P.off_state, 0, ctx->P.state_bytes, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    return SWF_OK;
}

// Host sum of per-block partials (fixed order).
static int reduce(swf_ctx* ctx, int kind, swf::RedArgs a, int nv, std::vector<cd>& out) {
    a.solves = ctx->d_solves();
    a.out = ctx->d_red();
    HIPCHK(swf::launch_reduction(ctx->P.fp64, kind, a, RED_BLOCKS, ctx->st));
    std::vector<double2> h((size_t)RED_BLOCKS * nv);
    HIPCHK(hipMemcpyAsync(h.data(), ctx->d_red(), h.size() * sizeof(double2), hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    out.assign(nv, cd(0));
    for (int b = 0; b < RED_BLOCKS; ++b)
        for (int v = 0; v < nv; ++v) out[v] += cd(h[(size_t)b * nv + v].x, h[(size_t)b * nv + v].y);
    return SWF_OK;
}

static void lattice_x(swf_ctx* ctx, int s, swf::RedArgs& a) {
    const swf_grid& G = ctx->P.grids[ctx->P.solves[s].grid];
    for (int j = 0; j < 3; ++j) {
        a.x0[j] = j < G.dim ? -0.5 * G.L[j] : 0.0;
        a.dx[j] = j < G.dim ? G.L[j] / G.n[j] : 0.0;
    }
}

// Full forward transform of psi_s of solve s into its T buffer.
static int kspace(swf_ctx* ctx, int s) {
    if (ctx->kvalid[s]) return SWF_OK;
    const Group& g = ctx->P.single[s];
    const int dim = ctx->P.grids[g.grid].dim;
    int r = row_pass(ctx, g, swf::ROW_FWD, 0, swf::BUF_Y, swf::BUF_T, 0, 0);
    if (!r && dim >= 2) r = col_pass(ctx, g, 1, swf::COL_FWD, swf::BUF_T);
    if (!r && dim >= 3) r = col_pass(ctx, g, 2, swf::COL_FWD, swf::BUF_T);
    if (r) return r;
    ctx->kvalid[s] = 1;
    return SWF_OK;
}

// F_q = dV sum_x psi_q(x) exp(-i kappa.x) of solve s's Y buffer.
static int fourier_coeff(swf_ctx* ctx, int s, const double* kappa, Spinor& F) {
    swf::RedArgs a;
    memset(&a, 0, sizeof(a));
    a.sa = s;
    a.ra = swf::BUF_Y;
    for (int j = 0; j < 3; ++j) a.kv[j] = kappa[j];
    lattice_x(ctx, s, a);
    std::vector<cd> o;
    int r = reduce(ctx, swf::RED_XFOURIER, a, 4, o);
    if (r) return r;
    for (int q = 0; q < 4; ++q) F.c[q] = o[q] * ctx->P.hs[s].dV;
    return SWF_OK;
}

static Spinor solve_spinor(swf_ctx* ctx, int s) {
    Spinor w;
    for (int q = 0; q < 4; ++q) w.c[q] = cd(ctx->P.hs[s].w[2 * q], ctx->P.hs[s].w[2 * q + 1]);
    return w;
}

static int projected(swf_ctx* ctx, int sa, int sb, int sign, cd& out) {
    int r = kspace(ctx, sa);
    if (!r && sb != sa) r = kspace(ctx, sb);
    if (r) return r;
    swf::RedArgs a;
    memset(&a, 0, sizeof(a));
    a.sa = sa;
    a.sb = sb;
    a.ra = a.rb = swf::BUF_T;
    a.sign = sign;
    std::vector<cd> o;
    r = reduce(ctx, swf::RED_KPROJ, a, 1, o);
    if (r) return r;
    out = o[0] * ctx->P.hs[sa].dV * ctx->P.hs[sa].inv_n;
    return SWF_OK;
}

static int check_pair(swf_ctx* ctx, int i, int j) {
    const auto& P = ctx->P;
    if (i < 0 || j < 0 || i >= (int)P.solves.size() || j >= (int)P.solves.size()) {
        ctx->err = "bad solve index";
        return SWF_E_ARG;
    }
    if (P.solves[i].kind % 2 != 0 || P.solves[j].kind % 2 != 1) {
        ctx->err = "pair amplitude needs a U solve (i) and a V solve (j)";
        return SWF_E_ARG;
    }
    if (P.solves[i].grid != P.solves[j].grid) {
        ctx->err = "pair amplitude needs both solves on one grid";
        return SWF_E_ARG;
    }
    for (int a = P.grids[P.solves[i].grid].dim; a < 3; ++a)
        if (std::fabs(P.solves[i].p[a] + P.solves[j].p[a]) > 1e-12) {
            ctx->err = "pair amplitude needs q_perp = -p_perp on trivial axes";
            return SWF_E_ARG;
        }
    return SWF_OK;
}

static int pair_amp(swf_ctx* ctx, int i, int j, int form, cd& out) {
    int r = check_pair(ctx, i, j);
    if (r) return r;
    const double tin = ctx->P.t_obs;   // t_in (out-states) or t_out (in-states)
    const auto& HU = ctx->P.hs[i];
    const auto& HV = ctx->P.hs[j];
    cd proj_term;
    r = projected(ctx, i, j, form == 1 ? +1 : -1, proj_term);
    if (r) return r;
    const swf_solve& su = ctx->P.solves[i];
    const swf_solve& sv = ctx->P.solves[j];
    cd direct;
    if (form == 1) {
        // (U_b|V_s) = dV e^{i E_U t} sum_q conj(u_q) F_V,q(p)
        Spinor F;
        r = fourier_coeff(ctx, j, su.p, F);
        if (r) return r;
        direct = std::polar(1.0, HU.E * tin) * dot(solve_spinor(ctx, i), F);
    } else {
        // (U_s|V_b) = dV e^{-i E_V t} sum_q v_q conj(F_U,q(-q))
        double kap[3] = {-sv.p[0], -sv.p[1], -sv.p[2]};
        Spinor F;
        r = fourier_coeff(ctx, i, kap, F);
        if (r) return r;
        direct = std::polar(1.0, -HV.E * tin) * dot(F, solve_spinor(ctx, j));
    }
    out = direct + proj_term;
    return SWF_OK;
}

// ------------------------------------------------------------ pair matrix
// G[m][n] = sum_K conj(A_m[K]) B_n[K] over sites and spinor components, every
// A_m from rows `ra` and B_n from `rb` (PG_STATE rows: the solves' buffer
// `role`; PG_BKG rows: their background plane-wave spinors), optionally with
// Pi_sign applied to k-space states.  Result: na x nb, row-major.
static int pair_gemm(swf_ctx* ctx, const std::vector<int>& ra, int asrc, int arole, const std::vector<int>& rb,
                     int bsrc, int brole, int proj, std::vector<cd>& out, void* ext = nullptr, size_t ext_bytes = 0) {
    const int s0 = ra[0];
    const swf_grid& G = ctx->P.grids[ctx->P.solves[s0].grid];
    const long long ns = ctx->P.hs[s0].nsites;
    const int na = (int)ra.size(), nb = (int)rb.size();
    swf::PairArgs a;
    memset(&a, 0, sizeof(a));
    a.tiles_m = (na + 63) / 64;       // 64 x 64 output tiles
    a.tiles_n = (nb + 63) / 64;
    a.mp = 64 * a.tiles_m;
    a.np = 64 * a.tiles_n;
    const long long chunks = (ns + 7) / 8;
    const long long want = std::max(1LL, 1024LL / (a.tiles_m * a.tiles_n));
    a.splits = (int)std::min(chunks, want);
    const size_t ops_bytes = align256(sizeof(swf::PairOp) * (na + nb));
    const size_t tile_bytes = sizeof(double2) * (size_t)a.mp * a.np;
    if (ext) {
        // a fixed scratch: as many splits as its partial tiles leave room for
        if (ops_bytes + 2 * tile_bytes > ext_bytes) {
            ctx->err = "pair matrix too large for the static scratch";
            return SWF_E_ARG;
        }
        a.splits = (int)std::min<long long>(a.splits, (long long)((ext_bytes - ops_bytes) / tile_bytes) - 1);
    }
    a.per = ((chunks + a.splits - 1) / a.splits) * 8;
    a.splits = (int)((ns + a.per - 1) / a.per);
    a.ns = ns;
    a.dim = G.dim;
    a.n0 = G.n[0];
    a.n1 = G.n[1];
    a.n2 = G.n[2];
    for (int j = 0; j < 3; ++j) {
        a.x0[j] = j < G.dim ? -0.5 * G.L[j] : 0.0;
        a.dx[j] = j < G.dim ? G.L[j] / G.n[j] : 0.0;
        a.dk[j] = ctx->P.hs[s0].dk[j];
    }
    a.ctab = ctx->d_ctab();
    a.proj = proj;
    // scratch: row descriptors, then the partial tiles and their sum
    const size_t part_bytes = tile_bytes * (size_t)(a.splits + 1);
    const size_t need = ops_bytes + part_bytes;
    void* buf = ext;
    if (!ext && need > ctx->pm_bytes) {
        HIPCHK(hipStreamSynchronize(ctx->st));
        if (ctx->pm_buf) HIPCHK(hipFree(ctx->pm_buf));
        ctx->pm_buf = nullptr;
        ctx->pm_bytes = 0;
        HIPCHK(hipMalloc(&ctx->pm_buf, need));
        ctx->pm_bytes = need;
    }
    if (!ext) buf = ctx->pm_buf;
    std::vector<swf::PairOp> ops(na + nb);
    auto fill = [&](const std::vector<int>& rows, swf::PairOp* o) {
        for (size_t r = 0; r < rows.size(); ++r) {
            const swf_solve& sv = ctx->P.solves[rows[r]];
            o[r].solve = rows[r];
            o[r].pad = 0;
            // background plane wave exp(i K.x): K = p for U, -q for V
            for (int j = 0; j < 3; ++j) o[r].K[j] = sv.kind % 2 == 0 ? sv.p[j] : -sv.p[j];
        }
    };
    fill(ra, ops.data());
    fill(rb, ops.data() + na);
    swf::PairOp* d_ops = (swf::PairOp*)buf;
    a.part = (double2*)((char*)buf + ops_bytes);
    a.solves = ctx->d_solves();
    a.a = swf::PairSide{d_ops, na, asrc, arole};
    a.b = swf::PairSide{d_ops + na, nb, bsrc, brole};
    HIPCHK(hipMemcpyAsync(d_ops, ops.data(), sizeof(swf::PairOp) * ops.size(), hipMemcpyHostToDevice, ctx->st));
    HIPCHK(swf::launch_pair_gemm(ctx->P.fp64, a, ctx->st));
    std::vector<double2> h((size_t)a.mp * a.np);
    HIPCHK(hipMemcpyAsync(h.data(), a.part + (size_t)a.splits * a.mp * a.np, sizeof(double2) * h.size(),
                          hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    out.resize((size_t)na * nb);
    for (int m = 0; m < na; ++m)
        for (int n = 0; n < nb; ++n) out[(size_t)m * nb + n] = cd(h[(size_t)m * a.np + n].x, h[(size_t)m * a.np + n].y);
    return SWF_OK;
}

// Omega(m, n) of eq. (Nmn) for every pair: the direct overlap with the
// background as one x-space contraction, the projected overlap as one
// k-space contraction, combined with the time phase and dV (dV/N for k space).
static int pair_matrix(swf_ctx* ctx, int form, const std::vector<int>& us, const std::vector<int>& vs,
                       std::vector<cd>& out, void* ext = nullptr, size_t ext_bytes = 0) {
    for (int u : us) {
        int r = check_pair(ctx, u, vs[0]);
        if (r) return r;
    }
    for (int v : vs) {
        int r = check_pair(ctx, us[0], v);
        if (r) return r;
    }
    for (int s : us) {
        int r = kspace(ctx, s);
        if (r) return r;
    }
    for (int s : vs) {
        int r = kspace(ctx, s);
        if (r) return r;
    }
    std::vector<cd> gk, gx;
    int r = pair_gemm(ctx, us, swf::PG_STATE, swf::BUF_T, vs, swf::PG_STATE, swf::BUF_T, form == 1 ? +1 : -1, gk,
                      ext, ext_bytes);
    if (r) return r;
    if (form == 1) r = pair_gemm(ctx, us, swf::PG_BKG, 0, vs, swf::PG_STATE, swf::BUF_Y, 0, gx, ext, ext_bytes);
    else r = pair_gemm(ctx, us, swf::PG_STATE, swf::BUF_Y, vs, swf::PG_BKG, 0, 0, gx, ext, ext_bytes);
    if (r) return r;
    const double tin = ctx->P.t_obs;   // t_in (out-states) or t_out (in-states)
    const double dV = ctx->P.hs[us[0]].dV, inv_n = ctx->P.hs[us[0]].inv_n;
    const size_t nu = us.size(), nv = vs.size();
    out.resize(nu * nv);
    for (size_t m = 0; m < nu; ++m)
        for (size_t n = 0; n < nv; ++n) {
            const cd ph = form == 1 ? std::polar(1.0, ctx->P.hs[us[m]].E * tin) : std::polar(1.0, -ctx->P.hs[vs[n]].E * tin);
            out[m * nv + n] = dV * ph * gx[m * nv + n] + dV * inv_n * gk[m * nv + n];
        }
    return SWF_OK;
}

// Breit-Wheeler amplitude terms of vertex v at t_in.
// Past terms of vertex v's solves for one plane-wave photon (k, eps; phk: its
// exp(i k.x) tables), added with weight w to out[0..2] = (scat,scat),
// (back,scat), (scat,back).
static int past_terms(swf_ctx* ctx, int v, const double* k, const double* eps, long long phk, cd w, cd* out) {
    const VertexDev& V = ctx->P.hv[v];
    const int su = V.su, sv = V.sv;
    const double tin = ctx->P.win.t_in;
    const double k0 = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    // (scat, scat) past term: FFT(U_s) and FFT(V_s e^{i k.x})
    int r = kspace(ctx, su);
    if (r) return r;
    {
        const Group& g = ctx->P.single[sv];
        const int dim = ctx->P.grids[g.grid].dim;
        r = row_pass(ctx, g, swf::ROW_FWDPH, 0, swf::BUF_Y, swf::BUF_ACC, 0, phk);
        if (!r && dim >= 2) r = col_pass(ctx, g, 1, swf::COL_FWD, swf::BUF_ACC);
        if (!r && dim >= 3) r = col_pass(ctx, g, 2, swf::COL_FWD, swf::BUF_ACC);
        if (r) return r;
    }
    swf::RedArgs a;
    memset(&a, 0, sizeof(a));
    a.sa = su;
    a.sb = sv;
    a.ra = swf::BUF_T;
    a.rb = swf::BUF_ACC;
    for (int j = 0; j < 3; ++j) {
        a.kv[j] = k[j];
        a.eps[j] = eps[j];
    }
    a.k0 = k0;
    std::vector<cd> o;
    r = reduce(ctx, swf::RED_KBWPAST, a, 1, o);
    if (r) return r;
    const auto& HU = ctx->P.hs[su];
    out[0] += w * std::polar(1.0, -k0 * tin) * o[0] * HU.dV * HU.inv_n;
    const swf_solve& SU = ctx->P.solves[su];
    const swf_solve& SV = ctx->P.solves[sv];
    // (back, scat): kappa = p - k
    {
        double kap[3];
        for (int j = 0; j < 3; ++j) kap[j] = SU.p[j] - k[j];
        Spinor Vc;
        r = fourier_coeff(ctx, sv, kap, Vc);
        if (r) return r;
        const double p0 = std::sqrt(1.0 + SU.p[0] * SU.p[0] + SU.p[1] * SU.p[1] + SU.p[2] * SU.p[2]);
        const double Ek = std::sqrt(1.0 + kap[0] * kap[0] + kap[1] * kap[1] + kap[2] * kap[2]);
        const Spinor u = solve_spinor(ctx, su);
        cd m = 0;
        for (int sp = -1; sp <= 1; sp += 2) {
            const Spinor PV = proj(Vc, kap, sp);
            m += dot(u, gamma_eps(PV, eps)) / cd(0.0, p0 - sp * Ek - k0);
        }
        out[1] += w * m * std::polar(1.0, (p0 - k0) * tin);
    }
    // (scat, back): kappa = k - q
    {
        double kap[3];
        for (int j = 0; j < 3; ++j) kap[j] = k[j] - SV.p[j];
        Spinor Uc;
        r = fourier_coeff(ctx, su, kap, Uc);
        if (r) return r;
        const double q0 = std::sqrt(1.0 + SV.p[0] * SV.p[0] + SV.p[1] * SV.p[1] + SV.p[2] * SV.p[2]);
        const double Ek = std::sqrt(1.0 + kap[0] * kap[0] + kap[1] * kap[1] + kap[2] * kap[2]);
        const Spinor vsp = solve_spinor(ctx, sv);
        const Spinor gv = gamma_eps(vsp, eps);
        cd m = 0;
        for (int sg = -1; sg <= 1; sg += 2) {
            const Spinor PU = proj(Uc, kap, sg);
            m += dot(PU, gv) / cd(0.0, sg * Ek + q0 - k0);
        }
        out[2] += w * m * std::polar(1.0, (q0 - k0) * tin);
    }
    return SWF_OK;
}

// Breit-Wheeler amplitude terms of vertex v at t_in: the finite parts from the
// integrated Mdot, the past parts of its photon (for a wave packet, summed over
// its modes with their weights).
static int bw_terms(swf_ctx* ctx, int v) {
    if (ctx->bw_done[v]) return SWF_OK;
    const VertexDev& V = ctx->P.hv[v];
    const swf_vertex& VX = ctx->P.verts[v];
    // finite parts: M(t_in) accumulated from t_out, M_finite = -M(t_in)
    double2 M[3];
    HIPCHK(hipMemcpyAsync(M, ctx->d_M() + 3 * v, sizeof(M), hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    for (int t = 0; t < 3; ++t) ctx->bw_cache[6 * v + t] = -cd(M[t].x, M[t].y);
    cd past[3] = {0, 0, 0};
    int r = SWF_OK;
    if (V.nmodes == 0 || ctx->P.vmodes[v].empty()) {
        r = past_terms(ctx, v, VX.k, VX.eps, V.phk, cd(1.0), past);
    } else {
        for (int m = 0; m < V.nmodes && !r; ++m) {
            const auto& md = ctx->P.vmodes[v][m];
            r = past_terms(ctx, v, md.data(), md.data() + 3, ctx->P.hm[V.mode0 + m].phk, cd(md[6], md[7]), past);
        }
    }
    if (r) return r;
    for (int t = 0; t < 3; ++t) ctx->bw_cache[6 * v + 3 + t] = past[t];
    ctx->bw_done[v] = 1;
    return SWF_OK;
}

static swf_ctx* g_dummy = nullptr;

}  // namespace

// ============================================================ C ABI
extern "C" {

int swf_supported_n(int n) { return supported_n(n) ? 1 : 0; }

swf_status swf_workspace_size(const swf_grid* grids, int n_grids, const swf_term* terms, const int* ffirst,
                              int n_fields, const swf_solve* solves, int n_solves, const swf_vertex* vertices,
                              int n_vertices, const swf_window* window, const swf_options* opt, size_t* bytes) {
    Plan P;
    std::string err;
    int r = build_plan(P, err, grids, n_grids, terms, ffirst, n_fields, solves, n_solves, vertices, n_vertices, window, opt);
    if (r) {
        g_init_error = err;
        return (swf_status)r;
    }
    if (bytes) *bytes = P.total;
    return SWF_OK;
}

swf_status swf_init(const swf_grid* grids, int n_grids, const swf_term* terms, const int* ffirst, int n_fields,
                    const swf_solve* solves, int n_solves, const swf_vertex* vertices, int n_vertices,
                    const swf_window* window, const swf_options* opt, swf_ctx** out) {
    if (out) *out = nullptr;
    if (!out) {
        g_init_error = "out is NULL";
        return SWF_E_ARG;
    }
    swf_ctx* ctx = new swf_ctx();
    std::string err;
    int r = build_plan(ctx->P, err, grids, n_grids, terms, ffirst, n_fields, solves, n_solves, vertices, n_vertices, window, opt);
    if (r) {
        g_init_error = err;
        delete ctx;
        return (swf_status)r;
    }
    ctx->opt = *opt;
    if (opt->tune_cache) ctx->tune_path = opt->tune_cache;
    ctx->opt.tune_cache = nullptr;
    ctx->user = (hipStream_t)opt->stream;
    auto fail = [&](int code) {
        g_init_error = ctx->err;
        swf_free(ctx);
        return (swf_status)code;
    };
#define INITCHK(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) {                                                         \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(_e);               \
            return fail(SWF_E_HIP);                                                     \
        }                                                                               \
    } while (0)
    INITCHK(hipStreamCreateWithFlags(&ctx->st, hipStreamNonBlocking));
    INITCHK(hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming));
    INITCHK(hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming));
    Plan& P = ctx->P;
    if (opt->workspace) {
        if (opt->workspace_bytes < P.total) {
            char b[256];
            snprintf(b, sizeof(b), "workspace of %zu bytes is smaller than the %zu needed", opt->workspace_bytes, P.total);
            ctx->err = b;
            return fail(SWF_E_NOMEM);
        }
        if (((uintptr_t)opt->workspace) & 255) {
            ctx->err = "workspace must be 256-byte aligned";
            return fail(SWF_E_ARG);
        }
        ctx->arena = (char*)opt->workspace;
    } else {
        hipError_t e = hipMalloc((void**)&ctx->arena, P.total);
        if (e != hipSuccess) {
            ctx->arena = nullptr;
            ctx->err = std::string("hipMalloc of the arena failed: ") + hipGetErrorString(e);
            return fail(SWF_E_NOMEM);
        }
        ctx->own_arena = true;
    }
    // fill buffer pointers and upload descriptors / tables
    for (size_t i = 0; i < P.hs.size(); ++i)
        for (int role = 0; role < swf::NBUF; ++role) P.hs[i].buf[role] = role < nbufs(P, i) ? ctx->buf((int)i, role) : nullptr;
    INITCHK(hipMemsetAsync(ctx->arena + P.off_state, 0, P.state_bytes, ctx->st));
    INITCHK(hipMemcpyAsync(ctx->d_solves(), P.hs.data(), sizeof(SolveDev) * P.hs.size(), hipMemcpyHostToDevice, ctx->st));
    if (!P.ht.empty())
        INITCHK(hipMemcpyAsync(ctx->d_terms(), P.ht.data(), sizeof(TermDev) * P.ht.size(), hipMemcpyHostToDevice, ctx->st));
    if (!P.hv.empty())
        INITCHK(hipMemcpyAsync(ctx->d_verts(), P.hv.data(), sizeof(VertexDev) * P.hv.size(), hipMemcpyHostToDevice, ctx->st));
    if (!P.hg.empty())
        INITCHK(hipMemcpyAsync(ctx->d_vgroups(), P.hg.data(), sizeof(swf::VertexGroupDev) * P.hg.size(),
                               hipMemcpyHostToDevice, ctx->st));
    if (!P.hm.empty())
        INITCHK(hipMemcpyAsync(ctx->d_modes(), P.hm.data(), sizeof(swf::ModeDev) * P.hm.size(), hipMemcpyHostToDevice,
                               ctx->st));
    if (!P.packets.empty())
        INITCHK(hipMemcpyAsync(ctx->d_packets(), P.packets.data(), sizeof(int) * P.packets.size(),
                               hipMemcpyHostToDevice, ctx->st));
    std::vector<char> rt(P.rsize * std::max<size_t>(1, P.rtab.size())), ct(P.csize * std::max<size_t>(1, P.ctab.size()));
    for (size_t i = 0; i < P.rtab.size(); ++i) {
        if (P.fp64) ((double*)rt.data())[i] = P.rtab[i];
        else ((float*)rt.data())[i] = (float)P.rtab[i];
    }
    for (size_t i = 0; i < P.ctab.size(); ++i) {
        if (P.fp64) {
            ((double*)ct.data())[2 * i] = P.ctab[i].real();
            ((double*)ct.data())[2 * i + 1] = P.ctab[i].imag();
        } else {
            ((float*)ct.data())[2 * i] = (float)P.ctab[i].real();
            ((float*)ct.data())[2 * i + 1] = (float)P.ctab[i].imag();
        }
    }
    INITCHK(hipMemcpyAsync(ctx->d_rtab(), rt.data(), rt.size(), hipMemcpyHostToDevice, ctx->st));
    INITCHK(hipMemcpyAsync(ctx->d_ctab(), ct.data(), ct.size(), hipMemcpyHostToDevice, ctx->st));
    INITCHK(hipMemcpyAsync(ctx->d_items(), P.items.data(), sizeof(int2) * P.items.size(), hipMemcpyHostToDevice, ctx->st));
    INITCHK(hipMemsetAsync(ctx->d_step(), 0, 256, ctx->st));
    INITCHK(hipMemsetAsync(ctx->d_M(), 0, sizeof(double2) * 3 * std::max<size_t>(1, P.hv.size()), ctx->st));
    if (P.bw2) INITCHK(hipMemsetAsync(ctx->d_M2(), 0, sizeof(double2) * 3 * P.hv.size(), ctx->st));
    INITCHK(hipStreamSynchronize(ctx->st));
    {
        int dev = 0, lds = 0;
        INITCHK(hipGetDevice(&dev));
        INITCHK(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        ctx->lds_max = (size_t)lds;
        INITCHK(hipDeviceGetAttribute(&ctx->ncu, hipDeviceAttributeMultiprocessorCount, dev));
        // this device's copy of the static scratch (swf_pair_matrix_noalloc)
        INITCHK(scratch_address(dev, &ctx->noalloc_scratch));
    }
    // allow the dynamic LDS every pass kernel of these sizes asks for
    for (const auto* gl : {&P.batched, &P.single})
        for (const auto& g : *gl)
            for (int ax = 0; ax < 3; ++ax) {
                const auto* k = g.k[ax];
                if (!k) continue;
                for (int m = 0; m < swf::ROW_NMODES; ++m)
                    if (k->row_other[m])
                        INITCHK(hipFuncSetAttribute(k->row_other[m], hipFuncAttributeMaxDynamicSharedMemorySize, (int)k->row0_lds));
                for (int a = 0; a < 2; ++a)
                    for (int m = 0; m < 3; ++m)
                        INITCHK(hipFuncSetAttribute(k->col.fn[a][m], hipFuncAttributeMaxDynamicSharedMemorySize, (int)k->col.lds));
                if (k->line[0] && ax == 0)
                    for (int w = 0; w < 2; ++w)
                        INITCHK(hipFuncSetAttribute(k->line[w], hipFuncAttributeMaxDynamicSharedMemorySize,
                                                    (int)std::min(ctx->lds_max - LINE_STATIC_LDS,
                                                                  line_lds(ctx, g, swf::MAX_TERMS, w))));
                for (int v = 0; v < swf::NVAR; ++v) {
                    for (int st = 0; st < 4; ++st)
                        INITCHK(hipFuncSetAttribute(k->row[v].stage[st], hipFuncAttributeMaxDynamicSharedMemorySize, (int)k->row[v].lds));
                    for (int st = 0; st < 6; ++st)
                        INITCHK(hipFuncSetAttribute(k->row[v].dp5[st], hipFuncAttributeMaxDynamicSharedMemorySize, (int)k->row[v].lds));
                    for (int a = 0; a < 2; ++a)
                        for (int m = 0; m < 2; ++m)
                            INITCHK(hipFuncSetAttribute(k->cd[v].fn[a][m], hipFuncAttributeMaxDynamicSharedMemorySize, (int)k->cd[v].lds));
                }
            }
    ctx->kvalid.assign(P.solves.size(), 0);
    ctx->bw_done.assign(P.hv.size(), 0);
    ctx->bw_cache.assign(6 * P.hv.size(), cd(0));
    if (opt->force_variant > 0) {
        const int v = opt->force_variant - 1;
        for (auto* gl : {&P.batched, &P.single})
            for (auto& g : *gl) {
                g.vr = std::min(v, g.k[0]->nvar - 1);
                g.vy = g.k[1] ? std::min(v, g.k[1]->nvar - 1) : 0;
                g.vz = g.k[2] ? std::min(v, g.k[2]->nvar - 1) : 0;
            }
    } else if (opt->tune && !line_path(ctx) && !ctx->P.ip) {   // (the interaction picture runs no stage pass)
        int rr = autotune(ctx, ctx->opt.batched ? ctx->P.batched : ctx->P.single);
        if (rr) return fail(rr);
    }
    if (opt->use_graph && !opt->profile) {
        int rr = build_graph(ctx);
        if (rr) return fail(rr);
    }
    *out = ctx;
    return SWF_OK;
#undef INITCHK
}

swf_status swf_step(swf_ctx* ctx, int n_steps, int* steps_left) {
    if (!ctx) return SWF_E_ARG;
    if (n_steps < 0) {
        ctx->err = "n_steps must be >= 0";
        return SWF_E_ARG;
    }
    if (ctx->step + n_steps > ctx->P.steps) {
        ctx->err = "swf_step past the end of the window";
        return SWF_E_ORDER;
    }
    int r = enter(ctx);
    if (r) return (swf_status)r;
    const int K = ctx->opt.check_every;
    unsigned long long* flag = ctx->d_flag();
    bool checked = false;
    // the in-loop finite check after step index `at` (a multiple of K)
    auto check = [&](int at) -> int {
        HIPCHK(swf::launch_finite_check(ctx->P.fp64, ctx->d_solves(), (int)ctx->P.solves.size(), at, flag, ctx->st));
        checked = true;
        return SWF_OK;
    };
    if (line_path(ctx)) {
        for (int done = 0; done < n_steps;) {
            int c = n_steps - done;
            if (K > 0) c = std::min(c, K - (ctx->step + done) % K);
            r = line_steps(ctx, c);
            if (r) return (swf_status)r;
            done += c;
            if (K > 0 && (ctx->step + done) % K == 0 && (r = check(ctx->step + done))) return (swf_status)r;
        }
    } else {
        for (int i = 0; i < n_steps;) {
            if (ctx->gexec_k && K == 0 && n_steps - i >= ctx->graph_k_steps) {
                HIPCHK(hipGraphLaunch(ctx->gexec_k, ctx->st));
                i += ctx->graph_k_steps;
                continue;
            }
            ++i;
            if (ctx->gexec) {
                HIPCHK(hipGraphLaunch(ctx->gexec, ctx->st));
            } else {
                r = enqueue_step(ctx);
                if (r) return (swf_status)r;
            }
            if (K > 0 && (ctx->step + i) % K == 0 && (r = check(ctx->step + i))) return (swf_status)r;
        }
    }
    if (n_steps > 0) {
        ctx->step += n_steps;
        std::fill(ctx->kvalid.begin(), ctx->kvalid.end(), 0);
        std::fill(ctx->bw_done.begin(), ctx->bw_done.end(), 0);
    }
    r = leave(ctx);
    if (r) return (swf_status)r;
    if (steps_left) *steps_left = ctx->P.steps - ctx->step;
    if (checked) {
        unsigned long long key = 0;
        HIPCHK(hipMemcpyAsync(&key, flag, sizeof(key), hipMemcpyDeviceToHost, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
        if (key) {
            key = ~key;
            char b[160];
            snprintf(b, sizeof(b), "non-finite value in solve %u, first seen at the check after step %llu",
                     (unsigned)(key & 0xffffffffu), key >> 32);
            ctx->err = b;
            return SWF_E_NONFINITE;
        }
    }
    return SWF_OK;
}

swf_status swf_reset(swf_ctx* ctx) {
    if (!ctx) return SWF_E_ARG;
    int r = enter(ctx);
    if (r) return (swf_status)r;
    HIPCHK(hipMemsetAsync(ctx->arena + ctx->P.off_state, 0, ctx->P.state_bytes, ctx->st));
    HIPCHK(hipMemsetAsync(ctx->d_step(), 0, 256, ctx->st));
    HIPCHK(hipMemsetAsync(ctx->d_M(), 0, sizeof(double2) * 3 * std::max<size_t>(1, ctx->P.hv.size()), ctx->st));
    if (ctx->P.bw2) HIPCHK(hipMemsetAsync(ctx->d_M2(), 0, sizeof(double2) * 3 * ctx->P.hv.size(), ctx->st));
    ctx->step = 0;
    std::fill(ctx->kvalid.begin(), ctx->kvalid.end(), 0);
    std::fill(ctx->bw_done.begin(), ctx->bw_done.end(), 0);
    r = leave(ctx);
    return (swf_status)r;
}

swf_status swf_sync(swf_ctx* ctx) {
    if (!ctx) return SWF_E_ARG;
    HIPCHK(hipStreamSynchronize(ctx->st));
    int r = drain_profile(ctx);
    return (swf_status)r;
}

swf_status swf_amplitude(swf_ctx* ctx, int which, int i, int j, double out[2]) {
    if (!ctx || !out) return SWF_E_ARG;
    if (ctx->step != ctx->P.steps) {
        ctx->err = "amplitudes are defined at the end of the window: step to the end first";
        return SWF_E_ORDER;
    }
    int r = enter(ctx);
    if (r) return (swf_status)r;
    cd val;
    if (which == SWF_AMP_PAIR1 || which == SWF_AMP_PAIR2) {
        r = pair_amp(ctx, i, j, which == SWF_AMP_PAIR1 ? 1 : 2, val);
    } else if (which == SWF_AMP_BW_PARTIAL) {
        if (i < 0 || i >= (int)ctx->P.hv.size() || j < -1 || j > 2) {
            ctx->err = "bad vertex or term index";
            return SWF_E_ARG;
        }
        if (!ctx->P.bw2) {
            ctx->err = "the partial-integration route needs options.bw_partial at init";
            return SWF_E_ARG;
        }
        // M2(t_in) accumulated from t_out: the terms are -M2 (no past part)
        double2 M[3];
        HIPCHK(hipMemcpyAsync(M, ctx->d_M2() + 3 * i, sizeof(M), hipMemcpyDeviceToHost, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
        val = 0;
        for (int t = 0; t < 3; ++t)
            if (j < 0 || j == t) val -= cd(M[t].x, M[t].y);
    } else if (which == SWF_AMP_BW) {
        if (i < 0 || i >= (int)ctx->P.hv.size() || j < -1 || j > 2) {
            ctx->err = "bad vertex or term index";
            return SWF_E_ARG;
        }
        r = bw_terms(ctx, i);
        if (!r) {
            if (j < 0) {
                val = 0;
                for (int t = 0; t < 6; ++t) val += ctx->bw_cache[6 * i + t];
            } else {
                val = ctx->bw_cache[6 * i + j] + ctx->bw_cache[6 * i + 3 + j];
            }
        }
    } else {
        ctx->err = "unknown amplitude kind";
        return SWF_E_ARG;
    }
    if (r) return (swf_status)r;
    r = leave(ctx);
    if (r) return (swf_status)r;
    out[0] = val.real();
    out[1] = val.imag();
    return std::isfinite(out[0]) && std::isfinite(out[1]) ? SWF_OK : SWF_E_NONFINITE;
}

static swf_status pair_matrix_abi(swf_ctx* ctx, int form, const int* u_solves, int nu, const int* v_solves, int nv,
                                  double* out, void* ext, size_t ext_bytes) {
    if (!ctx || !out || !u_solves || !v_solves || nu <= 0 || nv <= 0) return SWF_E_ARG;
    if (form != 1 && form != 2) {
        ctx->err = "form must be 1 or 2";
        return SWF_E_ARG;
    }
    if (ctx->step != ctx->P.steps) {
        ctx->err = "amplitudes are defined at the end of the window: step to the end first";
        return SWF_E_ORDER;
    }
    int r = enter(ctx);
    if (r) return (swf_status)r;
    std::vector<int> us(u_solves, u_solves + nu), vs(v_solves, v_solves + nv);
    std::vector<cd> res;
    r = pair_matrix(ctx, form, us, vs, res, ext, ext_bytes);
    if (r) return (swf_status)r;
    r = leave(ctx);
    if (r) return (swf_status)r;
    bool finite = true;
    for (size_t k = 0; k < res.size(); ++k) {
        out[2 * k] = res[k].real();
        out[2 * k + 1] = res[k].imag();
        finite = finite && std::isfinite(out[2 * k]) && std::isfinite(out[2 * k + 1]);
    }
    return finite ? SWF_OK : SWF_E_NONFINITE;
}

swf_status swf_pair_matrix(swf_ctx* ctx, int form, const int* u_solves, int nu, const int* v_solves, int nv,
                           double* out) {
    return pair_matrix_abi(ctx, form, u_solves, nu, v_solves, nv, out, nullptr, 0);
}

swf_status swf_pair_matrix_noalloc(swf_ctx* ctx, int form, const int* u_solves, int nu, const int* v_solves, int nv,
                                   double* out) {
    if (!ctx) return SWF_E_ARG;
    if (!ctx->noalloc_scratch) {
        ctx->err = "the static scratch of this device was not resolved at swf_init";
        return SWF_E_HIP;
    }
    if (nu > 0 && nv > 0) {
        // the row descriptors and at least two padded output tiles (one split and the sum) must fit
        const size_t mp = 64 * (((size_t)nu + 63) / 64), np = 64 * (((size_t)nv + 63) / 64);
        const size_t need = align256(sizeof(swf::PairOp) * ((size_t)nu + nv)) + 2 * sizeof(double2) * mp * np;
        if (need > NOALLOC_SCRATCH_BYTES) {
            char b[200];
            snprintf(b, sizeof(b), "a %d x %d pair matrix needs %zu bytes of scratch, more than the static %zu",
                     nu, nv, need, NOALLOC_SCRATCH_BYTES);
            ctx->err = b;
            return SWF_E_ARG;
        }
    }
    return pair_matrix_abi(ctx, form, u_solves, nu, v_solves, nv, out, ctx->noalloc_scratch, NOALLOC_SCRATCH_BYTES);
}

size_t swf_noalloc_scratch_bytes(void) { return NOALLOC_SCRATCH_BYTES; }

swf_status swf_probability(swf_ctx* ctx, int which, int i, int j, double* out) {
    if (!ctx || !out) return SWF_E_ARG;
    if (ctx->step != ctx->P.steps) {
        ctx->err = "probabilities are defined at the end of the window: step to the end first";
        return SWF_E_ORDER;
    }
    if (which == SWF_P_MARGINAL_E || which == SWF_P_MARGINAL_POS) {
        if (i < 0 || i >= (int)ctx->P.solves.size()) {
            ctx->err = "bad solve index";
            return SWF_E_ARG;
        }
        const int want = which == SWF_P_MARGINAL_E ? 0 : 1;
        if (ctx->P.solves[i].kind % 2 != want) {
            ctx->err = which == SWF_P_MARGINAL_E ? "electron marginal needs a U solve" : "positron marginal needs a V solve";
            return SWF_E_ARG;
        }
        int r = enter(ctx);
        if (r) return (swf_status)r;
        cd v;
        r = projected(ctx, i, i, want == 0 ? -1 : +1, v);
        if (r) return (swf_status)r;
        r = leave(ctx);
        if (r) return (swf_status)r;
        *out = v.real();
    } else if (which == SWF_P_PAIR || which == SWF_P_BW) {
        double a[2];
        swf_status r = swf_amplitude(ctx, which == SWF_P_PAIR ? SWF_AMP_PAIR1 : SWF_AMP_BW, i, which == SWF_P_PAIR ? j : -1, a);
        if (r) return r;
        *out = a[0] * a[0] + a[1] * a[1];
    } else {
        ctx->err = "unknown probability kind";
        return SWF_E_ARG;
    }
    return std::isfinite(*out) ? SWF_OK : SWF_E_NONFINITE;
}

swf_status swf_diagnostics(swf_ctx* ctx, int i, double out[4]) {
    if (!ctx || !out) return SWF_E_ARG;
    if (i < 0 || i >= (int)ctx->P.solves.size()) {
        ctx->err = "bad solve index";
        return SWF_E_ARG;
    }
    int r = enter(ctx);
    if (r) return (swf_status)r;
    swf::RedArgs a;
    memset(&a, 0, sizeof(a));
    a.sa = i;
    a.ra = swf::BUF_Y;
    const swf_solve& s = ctx->P.solves[i];
    const double sgn = s.kind % 2 == 0 ? 1.0 : -1.0;
    for (int j = 0; j < 3; ++j) a.kv[j] = sgn * s.p[j];
    a.t = ctx->P.t0 - (double)ctx->step * ctx->P.sdt;
    lattice_x(ctx, i, a);
    a.solves = ctx->d_solves();
    a.out = ctx->d_red();
    HIPCHK(swf::launch_reduction(ctx->P.fp64, swf::RED_XDIAG, a, RED_BLOCKS, ctx->st));
    std::vector<double2> h((size_t)RED_BLOCKS * 3);
    HIPCHK(hipMemcpyAsync(h.data(), ctx->d_red(), h.size() * sizeof(double2), hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    double ss = 0, mx = 0, bad = 0;
    cd bs = 0;
    for (int b = 0; b < RED_BLOCKS; ++b) {
        ss += h[3 * b].x;
        bs += cd(h[3 * b + 1].x, h[3 * b + 1].y);
        mx = std::max(mx, h[3 * b + 2].x);
        bad += h[3 * b + 2].y;
    }
    const double dV = ctx->P.hs[i].dV;
    out[0] = ss * dV;
    out[1] = 2.0 * (bs * dV).real();
    out[2] = mx;
    out[3] = bad == 0 ? 1.0 : 0.0;
    r = leave(ctx);
    if (r) return (swf_status)r;
    if (bad != 0) {
        ctx->err = "non-finite values in the state";
        return SWF_E_NONFINITE;
    }
    return SWF_OK;
}

static swf_status copy_state(swf_ctx* ctx, int i, int role, double* host, bool to_host) {
    const size_t n = 4 * (size_t)ctx->P.hs[i].nsites;
    void* d = ctx->buf(i, role);
    if (ctx->P.fp64) {
        if (to_host) HIPCHK(hipMemcpyAsync(host, d, n * 16, hipMemcpyDeviceToHost, ctx->st));
        else HIPCHK(hipMemcpyAsync(d, host, n * 16, hipMemcpyHostToDevice, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
    } else {
        std::vector<float> tmp(2 * n);
        if (to_host) {
            HIPCHK(hipMemcpyAsync(tmp.data(), d, n * 8, hipMemcpyDeviceToHost, ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
            for (size_t k = 0; k < 2 * n; ++k) host[k] = tmp[k];
        } else {
            for (size_t k = 0; k < 2 * n; ++k) tmp[k] = (float)host[k];
            HIPCHK(hipMemcpyAsync(d, tmp.data(), n * 8, hipMemcpyHostToDevice, ctx->st));
            HIPCHK(hipStreamSynchronize(ctx->st));
        }
    }
    return SWF_OK;
}

swf_status swf_get_psi(swf_ctx* ctx, int i, double* host) {
    if (!ctx || !host || i < 0 || i >= (int)ctx->P.solves.size()) return SWF_E_ARG;
    int r = enter(ctx);
    if (r) return (swf_status)r;
    return copy_state(ctx, i, swf::BUF_Y, host, true);
}

swf_status swf_set_psi(swf_ctx* ctx, int i, const double* host, int step_index) {
    if (!ctx || !host || i < 0 || i >= (int)ctx->P.solves.size()) return SWF_E_ARG;
    if (step_index < 0 || step_index > ctx->P.steps) {
        ctx->err = "step_index out of range";
        return SWF_E_ARG;
    }
    int r = enter(ctx);
    if (r) return (swf_status)r;
    swf_status s = copy_state(ctx, i, swf::BUF_Y, const_cast<double*>(host), false);
    if (s) return s;
    ctx->step = step_index;
    HIPCHK(hipMemcpyAsync(ctx->d_step(), &step_index, sizeof(int), hipMemcpyHostToDevice, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    std::fill(ctx->kvalid.begin(), ctx->kvalid.end(), 0);
    std::fill(ctx->bw_done.begin(), ctx->bw_done.end(), 0);
    return SWF_OK;
}

// Vertex i's integrals: 0 <= i < nv the first route, nv <= i < 2 nv the
// partial-integration route (with options.bw_partial).
static double2* bw_state_ptr(swf_ctx* ctx, int i) {
    const int nv = (int)ctx->P.hv.size();
    if (i >= 0 && i < nv) return ctx->d_M() + 3 * i;
    if (ctx->P.bw2 && i >= nv && i < 2 * nv) return ctx->d_M2() + 3 * (i - nv);
    return nullptr;
}

swf_status swf_get_bw_state(swf_ctx* ctx, int i, double out[6]) {
    if (!ctx || !out || !bw_state_ptr(ctx, i)) return SWF_E_ARG;
    int r = enter(ctx);
    if (r) return (swf_status)r;
    HIPCHK(hipMemcpyAsync(out, bw_state_ptr(ctx, i), 6 * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    return SWF_OK;
}

swf_status swf_set_bw_state(swf_ctx* ctx, int i, const double in[6]) {
    if (!ctx || !in || !bw_state_ptr(ctx, i)) return SWF_E_ARG;
    int r = enter(ctx);
    if (r) return (swf_status)r;
    HIPCHK(hipMemcpyAsync(bw_state_ptr(ctx, i), in, 6 * sizeof(double), hipMemcpyHostToDevice, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    ctx->bw_done[i % (int)ctx->P.hv.size()] = 0;
    return SWF_OK;
}

swf_status swf_apply_op(swf_ctx* ctx, int op, int i, double t, const double* in, double* out) {
    if (!ctx || !in || !out || i < 0 || i >= (int)ctx->P.solves.size() || op < 0 || op > 2) return SWF_E_ARG;
    if (ctx->step != 0 && ctx->step != ctx->P.steps) {
        ctx->err = "swf_apply_op is only valid before stepping or at the end of the window";
        return SWF_E_ORDER;
    }
    int r = enter(ctx);
    if (r) return (swf_status)r;
    swf_status s = copy_state(ctx, i, swf::BUF_YS, const_cast<double*>(in), false);
    if (s) return s;
    const Group& g = ctx->P.single[i];
    const int dim = ctx->P.grids[g.grid].dim;
    r = row_pass(ctx, g, swf::ROW_FWD, 0, swf::BUF_YS, swf::BUF_T, 0, 0);
    if (r) return (swf_status)r;
    int role_out = swf::BUF_T;
    if (op == 0) {
        if (dim >= 2) r = col_pass(ctx, g, 1, swf::COL_FWD, swf::BUF_T);
        if (!r && dim >= 3) r = col_pass(ctx, g, 2, swf::COL_FWD, swf::BUF_T);
    } else {
        r = kinetic_cols(ctx, g, swf::BUF_T);
        if (!r) r = row_pass(ctx, g, op == 1 ? swf::ROW_INV : swf::ROW_RHS, 0, swf::BUF_YS, swf::BUF_ACC, t, 0);
        role_out = swf::BUF_ACC;
    }
    if (r) return (swf_status)r;
    ctx->kvalid[i] = 0;
    std::fill(ctx->bw_done.begin(), ctx->bw_done.end(), 0);
    return copy_state(ctx, i, role_out, out, true);
}

swf_status swf_kernel_stats(swf_ctx* ctx, int kind, long long* launches, double* ms, double* bytes) {
    if (!ctx || kind < 0 || kind >= NKIND) return SWF_E_ARG;
    int r = drain_profile(ctx);
    if (r) return (swf_status)r;
    if (launches) *launches = ctx->st_launch[kind];
    if (ms) *ms = ctx->st_ms[kind];
    if (bytes) *bytes = ctx->st_bytes[kind];
    return SWF_OK;
}

swf_status swf_reset_stats(swf_ctx* ctx) {
    if (!ctx) return SWF_E_ARG;
    int r = drain_profile(ctx);
    if (r) return (swf_status)r;
    for (int k = 0; k < NKIND; ++k) {
        ctx->st_launch[k] = 0;
        ctx->st_ms[k] = 0;
        ctx->st_bytes[k] = 0;
    }
    return SWF_OK;
}

swf_status swf_steps(swf_ctx* ctx, int* total, int* done) {
    if (!ctx) return SWF_E_ARG;
    if (total) *total = ctx->P.steps;
    if (done) *done = ctx->step;
    return SWF_OK;
}

const char* swf_tune_report(const swf_ctx* ctx) { return ctx ? ctx->tune_report.c_str() : ""; }

const char* swf_last_error(const swf_ctx* ctx) { return ctx ? ctx->err.c_str() : g_init_error.c_str(); }

void swf_free(swf_ctx* ctx) {
    if (!ctx) return;
    if (ctx->st) hipStreamSynchronize(ctx->st);
    for (auto& p : ctx->pending) {
        hipEventDestroy(p.a);
        hipEventDestroy(p.b);
    }
    for (auto e : ctx->ev_free) hipEventDestroy(e);
    if (ctx->gexec) hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) hipGraphDestroy(ctx->graph);
    if (ctx->gexec_k) hipGraphExecDestroy(ctx->gexec_k);
    if (ctx->graph_k) hipGraphDestroy(ctx->graph_k);
    if (ctx->own_arena && ctx->arena) hipFree(ctx->arena);
    if (ctx->pm_buf) hipFree(ctx->pm_buf);
    if (ctx->ev_in) hipEventDestroy(ctx->ev_in);
    if (ctx->ev_out) hipEventDestroy(ctx->ev_out);
    if (ctx->st) hipStreamDestroy(ctx->st);
    (void)g_dummy;
    delete ctx;
}

}  // extern "C"
