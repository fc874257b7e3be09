/*
 * swf.h -- C ABI of the MI355X scattered-wave-function (SWF) solver.
 *
 * Method: arXiv 2512.16889 (G. Torgrimsson), "Solving the Dirac equation on a
 * GPU for strong-field processes in multidimensional background fields".
 *
 *   - The scattered wave psi_s of an out-state U_out(s,p) or V_out(s,p) solves
 *     the inhomogeneous Dirac equation (i Dslash - 1) psi_s = Aslash psi_back,
 *     eq. (scatDirac), with psi_s(t_out) = 0, where D_mu = d_mu + i A_mu and
 *     psi_back = u_s(p) e^{-ipx} or v_s(p) e^{ipx} (section "Scattered wave
 *     functions"; spinors of eq. (uv) with R_s of eq. (Reqs)).  The
 *     in-states U_in(s,p), V_in(s,p) of the same section have the same
 *     backgrounds and psi_s(t_in) = 0.
 *   - Space is discretised pseudo-spectrally on a periodic grid (section
 *     "Numerical approach"); time is stepped with classical RK4, h = -dt
 *     from t_out back to t_in for out-states, h = +dt from t_in forward to
 *     t_out for in-states (one direction per context).
 *   - At the end of the run (t_in for out-states, t_out for in-states) the
 *     library forms the inner products of eq. (Nmn) (pair amplitude and
 *     marginals) and, for out-states, the Breit-Wheeler vertex amplitude
 *     M = M_finite + M_past of the section "Nonlinear Breit-Wheeler pair
 *     production" (eqs. (Mabfinite), (MScatScatPast) and partners).
 *
 * Units: m = c = hbar = 1, the charge absorbed into A.  Metric (+,-,-,-).
 * All host scalars are double; a complex number is double[2] = {re, im}.
 *
 * Threading: a context is not thread-safe; distinct contexts are independent.
 * Errors: every call returns a status; nothing is thrown across the ABI.
 * swf_last_error(ctx) returns the message of the context's last failure
 * (swf_last_error(NULL) that of the last failed swf_init on this thread).
 */
#ifndef SWF_H
#define SWF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct swf_ctx swf_ctx; /* opaque; owned by the library */

typedef enum {
    SWF_OK = 0,
    SWF_E_ARG = 1,         /* invalid argument (see each call)                      */
    SWF_E_NOMEM = 2,       /* device allocation failed or workspace too small       */
    SWF_E_HIP = 3,         /* a HIP runtime call failed                              */
    SWF_E_ORDER = 4,       /* call out of order (e.g. amplitude before t_in)         */
    SWF_E_UNSUPPORTED = 5, /* grid size / option the library does not support       */
    SWF_E_NONFINITE = 6    /* a NaN or Inf was detected in the state                 */
} swf_status;

typedef enum {
    SWF_FP64 = 0,  /* state, FFTs and stepping in complex double                      */
    SWF_MIXED = 1  /* state, FFTs and stepping in complex float; plane-wave phases,
                      times, field time factors and every reduction in double       */
} swf_precision;

typedef enum { SWF_U_OUT = 0, SWF_V_OUT = 1, SWF_U_IN = 2, SWF_V_IN = 3 } swf_kind;

/* Profile shapes: f(s) = env((s - c)/w) * cos(k s + phi). */
enum {
    SWF_PROF_CONST = 0,  /* env = 1 (c and w ignored)  */
    SWF_PROF_GAUSS = 1,  /* env = exp(-u^2)            */
    SWF_PROF_SECH2 = 2,  /* env = sech(u)^2            */
    SWF_PROF_TANH = 3,   /* env = tanh(u)              */
    SWF_PROF_UGAUSS = 4  /* env = u exp(-u^2)          */
};

typedef struct { int type; double c, w, k, phi; } swf_profile;

/* One separable term of a background potential (section "Numerical examples"
 * writes its fields this way): covariant A_mu(t,x,y,z) += amp * ft(t) *
 * fx[0](x) * fx[1](y) * fx[2](z).  mu = 0 is the scalar potential, A_j = -A^j.
 * fx[j] must be SWF_PROF_CONST (with k = phi = 0) on trivial axes j >= dim. */
typedef struct { int mu; double amp; swf_profile ft; swf_profile fx[3]; } swf_term;

/* Periodic grid of the pseudo-spectral discretisation (array (g, n_x, n_y, n_z)
 * of section "Numerical approach", g = 4).  dim = number of non-trivial axes
 * (x; x,y; x,y,z).  Axis j has n[j] points x_i = -L[j]/2 + i L[j]/n[j].
 * Supported n: 16..1024 of the forms 2^a, 3*2^a, 5*2^a (see swf_supported_n).
 * absorb_cells > 0 enables a boundary mask applied to psi_s after every step:
 * m = 1 - absorb_strength * sin^2(pi/2 (cells - d)/cells) within `cells` of an
 * edge (d = distance in cells).  The mask is not part of the paper's method. */
typedef struct { int dim; int n[3]; double L[3]; int absorb_cells; double absorb_strength; } swf_grid;

/* Time window shared by every solve of a context: steps = round((t_out - t_in)/dt).
 * The field must be negligible before t_in and after t_out (eq. (Nmn) text). */
typedef struct { double t_in, t_out, dt; } swf_window;

/* One solve: U_out(spin, p) (kind 0), V_out(spin, p) (kind 1), U_in(spin, p)
 * (kind 2) or V_in(spin, p) (kind 3) of the section "Scattered wave
 * functions"; p is the contravariant 3-momentum; spin = +1 or -1 labels R_s of
 * eq. (Reqs).  grid/field index the arrays given to swf_init.  The solves of a
 * context are all out-states or all in-states (SWF_E_UNSUPPORTED otherwise):
 * the two run in opposite time directions. */
typedef struct { int kind; int spin; double p[3]; int grid; int field; } swf_solve;

/* Breit-Wheeler vertex: photon with 3-momentum k (k^0 = |k|) and polarisation
 * eps (epsilon_mu = (0, eps), eq. (epsParaPerp) gives the usual basis).
 * u_solve must be a U solve and v_solve a V solve on the same grid and field;
 * on trivial axes p + q = k must hold.
 * Photon wave packet (the BW section's numerical approach): with n_modes > 0
 * the photon is f_mu(x) = sum_m c_m eps_m,mu exp(-i k_m x) instead, f taking
 * the place of eps_mu e^{-ikx} in the finite-time integrand of eq. (Mabfinite)
 * and the past terms (eq. (MScatScatPast) and partners) evaluated for every
 * k_m and summed with the weights c_m; k and eps are then unused.  modes:
 * n_modes records of 8 doubles {k[3], eps[3], Re c, Im c}, caller-owned and
 * copied by swf_init; every k_m must be non-zero and satisfy p + q = k_m on the
 * trivial axes; at most SWF_MAX_MODES modes (SWF_E_ARG otherwise).  Packets do
 * not combine with options.bw_partial (SWF_E_UNSUPPORTED). */
#define SWF_MAX_MODES 64
typedef struct { int u_solve, v_solve; double k[3]; double eps[3]; int n_modes; const double* modes; } swf_vertex;

typedef struct {
    int prec;               /* swf_precision                                          */
    void* stream;           /* hipStream_t the work is ordered with (NULL = null stream) */
    void* workspace;        /* optional caller-owned device memory for every buffer     */
    size_t workspace_bytes; /* its size; must be >= swf_workspace_size()                */
    int use_graph;          /* 1: replay each time step as a captured hipGraph          */
    int batched;            /* 1: one launch per pass for all solves of a grid size;
                               0: separate launches per solve ("per-instance")          */
    int profile;            /* 1: time every pass with HIP events (see swf_kernel_stats) */
    int tune;               /* 1: autotune tile shapes at init (results cached)         */
    const char* tune_cache; /* path of the tune cache file, or NULL                     */
    int chunk;              /* batched mode: at most this many solves per launch group
                               (0 = all solves of a grid size).  Without BW vertices a
                               time step then runs all passes of one chunk before the
                               next, so a chunk's arrays can stay in the on-die cache  */
    int force_variant;      /* > 0: use tile variant force_variant - 1 (0..3) for every pass
                               (testing); 0: the autotuned or the default variant       */
    int persistent;         /* 1: when every grid is one-dimensional with a power-of-two
                               length 64..1024, the field's profile tables fit in LDS
                               next to the state (FP64, 1024 points: up to 4 terms) and
                               there are no BW vertices, each swf_step call runs all its
                               time steps in one kernel per launch group (at most 1024
                               steps per launch), one workgroup per solve, with the state
                               held on chip; otherwise, and with 0, one launch per pass
                               and RK4 stage                                            */
    int bw_partial;         /* 1: also integrate every BW vertex by the partial-integration
                               route of the paper's BW section (eq. (MScatScat2) and its
                               (back,scat), (scat,back) partners), read back with
                               SWF_AMP_BW_PARTIAL.  Each vertex solve gets two more
                               state-sized buffers, and every RK4 stage adds, per vertex,
                               the source term in x space, four full forward transforms
                               and two reductions; 0: off                              */
    int check_every;        /* > 0: after every check_every-th step (by step index) swf_step
                               reads every psi_s once on the device and records the first
                               step and solve holding a NaN or an Inf; a swf_step call that
                               queued a check then waits for its work and returns
                               SWF_E_NONFINITE if one was seen (the steps are still taken;
                               swf_last_error names the step and solve).  0: no check   */
    int stepper;            /* swf_stepper: SWF_RK4 (classical RK4, four stages, four
                               state arrays per solve) or SWF_DP5: the Dormand-Prince
                               5(4) tableau of the paper's Dopri5 solver (section
                               "Numerical approach") with the fixed step dt, its
                               fifth-order solution (six stages per step; eight state
                               arrays per solve; no embedded error estimate or step
                               control).  BW integrals take the tableau's weights over
                               the stages.  SWF_DP5 does not combine with bw_partial or
                               the persistent 1D kernel (the pass path runs instead).
                               SWF_IPRK4: the interaction picture, Lawson's
                               integrating-factor RK4 (J. D. Lawson, SIAM J. Numer.
                               Anal. 4 (1967) 372): the free evolution exp(-i H0(k) h/2)
                               exact in Fourier space, the field terms -i V (psi_s +
                               psi_b) by the classical tableau; five free-evolution
                               transforms of a whole state per step, six state arrays
                               per solve, BW integrals with the RK4 weights over its
                               stage inputs; not with bw_partial or the persistent 1D
                               kernel                                                   */
    int graph_steps;        /* with use_graph: > 1 also captures that many consecutive
                               time steps as one graph, replayed while at least that
                               many steps remain (the one-step graph takes the rest,
                               and every step when check_every > 0); 0 or 1: one step
                               per graph                                                */
} swf_options;

typedef enum { SWF_RK4 = 0, SWF_DP5 = 1, SWF_IPRK4 = 2 } swf_stepper;

/* Device bytes swf_init needs for these inputs (tables, states, scratch). */
swf_status swf_workspace_size(const swf_grid* grids, int n_grids, const swf_term* terms,
                              const int* field_first_term, int n_fields, const swf_solve* solves,
                              int n_solves, const swf_vertex* vertices, int n_vertices,
                              const swf_window* window, const swf_options* opt, size_t* bytes);

/* Validate, plan, allocate and upload.  Field f is terms[field_first_term[f] ..
 * field_first_term[f+1]) (field_first_term has n_fields + 1 entries).  Inputs are
 * deep-copied; all-or-nothing (on failure *out = NULL).
 * SWF_E_ARG: bad sizes/indices, momentum beyond the grid's Nyquist wavenumber on a
 * non-trivial axis, dt * E_max >= 2.8 (RK4 stability on the imaginary axis is
 * 2 sqrt 2), a field depending on a trivial axis, an invalid vertex.
 * SWF_E_UNSUPPORTED: a grid size without an FFT plan. */
swf_status swf_init(const swf_grid* grids, int n_grids, const swf_term* terms,
                    const int* field_first_term, int n_fields, const swf_solve* solves,
                    int n_solves, const swf_vertex* vertices, int n_vertices,
                    const swf_window* window, const swf_options* opt, swf_ctx** out);

/* Enqueue n_steps RK4 steps of every solve (and of the BW vertex integrals)
 * toward the end of the window (t_in for out-states, t_out for in-states) on
 * the context's stream.  One step is classical RK4 with h = -dt (out-states)
 * or h = +dt (in-states) of eq. (scatDirac) multiplied by gamma^0 (section "Numerical
 * approach": spatial derivatives through FFTs, the vector of spinors stepped
 * in time), each BW vertex's finite-time integral, eq. (Mabfinite), carried
 * along as an extra component of the stepped state.  Asynchronous: returns
 * after enqueueing, unless options.check_every > 0 and a check fell in the
 * call (then it waits for the call's work).  *steps_left (optional) receives
 * the remaining step count.  SWF_E_ORDER if n_steps exceeds the steps left;
 * SWF_E_ARG if n_steps < 0; SWF_E_NONFINITE if the in-loop check saw a NaN or
 * an Inf. */
swf_status swf_step(swf_ctx* ctx, int n_steps, int* steps_left);

/* Return every solve to psi_s = 0 at step 0 and clear the BW integrals,
 * keeping the plan, tables and captured graph (to run the same job again). */
swf_status swf_reset(swf_ctx* ctx);

/* Wait for the context's queued work.  SWF_E_HIP on a device error. */
swf_status swf_sync(swf_ctx* ctx);

enum {
    SWF_AMP_PAIR1 = 0, /* Omega(m,n), form 1 of eq. (Nmn): (U_b|V_s) + (U_s|Pi_+|V_s); i = U solve, j = V solve */
    SWF_AMP_PAIR2 = 1, /* form 2: (U_s|V_b) + (U_s|Pi_-|V_s) (= -form 1 by orthogonality)                     */
    SWF_AMP_BW = 2,    /* BW amplitude of vertex i; j = -1 total, j = 0/1/2 the (s,s)/(b,s)/(s,b) term          */
    SWF_AMP_BW_PARTIAL = 3 /* the same amplitude by partial integration in t (needs options.bw_partial,
                              else SWF_E_ARG): each term is an integral over [t_in, t_out] of the
                              energy-projected overlaps with the source -i V (psi_s + psi_b), so there
                              is no asymptotic-past part.  Equal to SWF_AMP_BW up to the time and lattice
                              discretisation (exactly so on the lattice when p, q and k are lattice
                              momenta); an independent check of it                                 */
};
/* Amplitudes at the end of the window (requires steps_left == 0, else
 * SWF_E_ORDER): at t_in from out-states; from in-states the two PAIR forms are
 * read at t_out, where they give (U_in|Pi_+|V_in) = -(U_in|Pi_-|V_in), the
 * time-reversed counterpart of Omega (-Omega at first order in the field).
 * BW: out-states only (a vertex needs a U_out and a V_out solve).
 * PAIR: coefficient of (2 pi)^(3-d) delta(p_perp + q_perp), d = dim; requires
 * q_perp = -p_perp on trivial axes (else SWF_E_ARG).  BW: M per
 * (2 pi)^(3-d) delta_perp(p + q - k), no phase-space or e^2 factors (Fig. 7). */
swf_status swf_amplitude(swf_ctx* ctx, int which, int i, int j, double out[2]);

/* Pair-amplitude matrix, eq. (Nmn) for every pair at once: out[2*(m*nv + n)],
 * out[2*(m*nv + n) + 1] = re, im of Omega(u_solves[m], v_solves[n]) in form 1
 * or 2, the same value swf_amplitude(SWF_AMP_PAIR1/2) returns for that pair.
 * Both inner products are evaluated as dense complex contractions over all
 * sites and spinor components (the background overlap in x space, the
 * projected one in k space), so every state is read once for the whole
 * matrix instead of once per pair; they run on the FP64 matrix cores with
 * FP64 accumulation in either precision.
 * Requirements: at the end of the window (SWF_E_ORDER otherwise); every u_solves[m] a U solve
 * and every v_solves[n] a V solve, all on one grid, and p_perp + q_perp = 0 on
 * the trivial axes for every pair (SWF_E_ARG otherwise).  out: caller-owned,
 * 2 * nu * nv doubles.  The first call (or a larger matrix) allocates device
 * scratch owned by the context.  Overwrites the solves' FFT buffers (like
 * swf_amplitude), not their states. */
swf_status swf_pair_matrix(swf_ctx* ctx, int form, const int* u_solves, int nu, const int* v_solves, int nv,
                           double* out);

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * matrix as swf_pair_matrix, with its device scratch (row descriptors and
 * partial output tiles) in a static device array of swf_noalloc_scratch_bytes()
 * bytes (32 MiB) instead of context memory allocated on the first call.  The
 * call allocates no device memory.  Each GPU the library runs on holds its own
 * copy of the array until the process ends (its address is resolved once per
 * device by swf_init).  Limit: align256(32 (nu + nv)) + 32 mp np bytes must fit
 * the array, with mp = 64 ceil(nu/64) and np = 64 ceil(nv/64) (every nu, nv up
 * to 960 x 1024); larger matrices give SWF_E_ARG before any work is queued.
 * The sums are split over fewer site ranges than swf_pair_matrix uses when the
 * array is short, so the two agree to rounding, not bitwise.  Every call on a
 * GPU shares that GPU's array and its contents are overwritten: calls that
 * overlap on one GPU (from two threads, or on two streams) race, so the caller
 * must serialise them.  Requirements, outputs and other errors as
 * swf_pair_matrix. */
swf_status swf_pair_matrix_noalloc(swf_ctx* ctx, int form, const int* u_solves, int nu, const int* v_solves,
                                   int nv, double* out);
size_t swf_noalloc_scratch_bytes(void);

enum {
    SWF_P_MARGINAL_E = 0,   /* electron marginal (U_s|Pi_-|U_s) of U solve i           */
    SWF_P_MARGINAL_POS = 1, /* positron marginal (V_s|Pi_+|V_s) of V solve i           */
    SWF_P_PAIR = 2,         /* |Omega_1(i,j)|^2                                        */
    SWF_P_BW = 3            /* |M|^2 of vertex i                                       */
};
/* Probabilities at the end of the window (SWF_E_ORDER before it; for
 * in-states the same projections at t_out).  PAIR: the pair number
 * N = |Omega|^2 of eq. (Nmn) (form 1).  MARGINAL_E / MARGINAL_POS: the sum of
 * eq. (Nmn)'s N over every partner state, which the completeness of the free
 * states turns into the energy-projected norm of the scattered wave at t_in
 * (same inner products as eq. (Nmn)).  BW: |M|^2 of the vertex amplitude of the
 * Breit-Wheeler section (eqs. (Mabfinite), (MScatScatPast) and partners).
 * Marginals are densities in d^d p/(2 pi)^d per unit transverse volume. */
swf_status swf_probability(swf_ctx* ctx, int which, int i, int j, double* out);

/* Diagnostics of solve i at the current time t = t_out - step*dt (out-states)
 * or t_in + step*dt (in-states), accumulated in
 * double: out[0] = (psi_s|psi_s), out[1] = 2 Re(psi_b|psi_s) with the inner
 * product (psi|phi) = int d^3x psi^dagger phi of eq. (Nmn)'s text.  The full
 * psi = psi_b + psi_s solves the Dirac equation (eq. (scatDirac) with
 * psi_s(t_out) = 0), which keeps its norm, so for a momentum on the lattice
 * out[0] + out[1] stays 0.  out[2] = max |psi_s component|, out[3] = 1 if every
 * value is finite else 0.  Returns SWF_E_NONFINITE if out[3] == 0. */
swf_status swf_diagnostics(swf_ctx* ctx, int i, double out[4]);

/* Copy the scattered wave of solve i to / from host memory as complex double,
 * layout [component 0..3][z][y][x] (x fastest), 8 * n_sites doubles.  set_psi
 * also sets the step index (0 <= step_index <= steps) and, for BW vertices that
 * use the solve, leaves their accumulated M unchanged (use swf_set_bw_state).
 * Both synchronise the context's stream. */
swf_status swf_get_psi(swf_ctx* ctx, int i, double* host);
swf_status swf_set_psi(swf_ctx* ctx, int i, const double* host, int step_index);

/* Accumulated finite-time BW integrals of vertex i at the current step
 * (3 complex: (s,s), (b,s), (s,b) of int_{t_out}^{t} dt' Mdot): get / set, for
 * checkpoint and resume.  With options.bw_partial, i = n_vertices + v addresses
 * vertex v's integrals of the partial-integration route. */
swf_status swf_get_bw_state(swf_ctx* ctx, int i, double out[6]);
swf_status swf_set_bw_state(swf_ctx* ctx, int i, const double in[6]);

/* Test hook: apply one spatial operator to solve i's layout.  op 0: out = FFT of
 * in over the non-trivial axes (unnormalised, numpy sign); op 1: out = the
 * kinetic term IFFT(-i H0(k) FFT(in)) of the stepper; op 2: out = the full
 * right-hand side F(t, in) at time t (kinetic + source).  in/out as swf_get_psi.
 * Uses the solve's ACC/YS/T buffers: only valid before stepping or at the end
 * of the window (SWF_E_ORDER otherwise). */
swf_status swf_apply_op(swf_ctx* ctx, int op, int i, double t, const double* in, double* out);

/* Pass timing collected when options.profile = 1.  kind: 0 row pass (x axis,
 * with the stage epilogue), 1 column pass (y axis), 2 column pass (z axis),
 * 3 BW vertex reduction, 4 other, 5 one-dimensional whole-loop kernel
 * (options.persistent).  Returns launches, summed device milliseconds and the
 * algorithmic HBM bytes those launches move (state reads + writes). */
swf_status swf_kernel_stats(swf_ctx* ctx, int kind, long long* launches, double* ms, double* bytes);
swf_status swf_reset_stats(swf_ctx* ctx);

/* 1 if the library has an FFT plan for length n. */
int swf_supported_n(int n);

/* Total steps of the context's window; current step index. */
swf_status swf_steps(swf_ctx* ctx, int* total, int* done);

/* Text report of the autotuner run at init (variant timings per group), or "". */
const char* swf_tune_report(const swf_ctx* ctx);

const char* swf_last_error(const swf_ctx* ctx);
void swf_free(swf_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* SWF_H */
