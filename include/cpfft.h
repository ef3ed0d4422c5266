/*
 * cpfft -- Green-operator FFT solver for voxelized periodic polycrystals
 * with the regularized Meric-Cailletaud crystal-plasticity law, on one
 * AMD Instinct MI355X (gfx950).
 *
 * The problem follows the paper's statement (abstract; Section 5 opening):
 * a grain-label voxel grid with one crystal orientation per label, an
 * anisotropic crystal stiffness, a set of slip and twinning pseudo-slip
 * systems (Table 1), the law parameters (Section 3, equations 1-6, with
 * the viscous-hardening regularization of Section 4, equation "regu"),
 * and a macroscopic loading path whose steps prescribe, per component,
 * either the mean strain or the mean stress.  The solver returns effective
 * (mean) stress-strain histories and the local fields.
 *
 * Units: MPa, seconds; strains dimensionless.  Symmetric tensors cross the
 * ABI as 6 tensor components in the order 11, 22, 33, 23, 13, 12.
 *
 * Memory: the library never allocates device memory.  The caller obtains
 * the size with cpf_solver_workspace_size(), allocates one device buffer
 * (e.g. a torch uint8 tensor) and hands it over with cpf_solver_bind();
 * it must stay alive and untouched until cpf_solver_destroy().  All device
 * work is ordered on the bound HIP stream.  Host arrays passed in are
 * copied; the caller keeps ownership.
 *
 * Errors: every call returns CPF_OK (0) or a negative CPF_E_* code and
 * never throws or aborts across the ABI.  cpf_last_error_message() gives a
 * thread-local description of the last failure on the calling thread.
 */
#ifndef CPFFT_H
#define CPFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CPF_VERSION 10000

#define CPF_OK 0
#define CPF_E_INVALID_ARG (-1)
#define CPF_E_WORKSPACE (-2)
#define CPF_E_HIP (-3)
#define CPF_E_NOT_CONVERGED (-4)
#define CPF_E_NAN (-5)          /* a non-finite stress or residual during the
                                   step, or a non-finite component of the
                                   converged strain or state (not committed) */
#define CPF_E_UNSUPPORTED_SIZE (-6)
#define CPF_E_BAD_STATE (-7)

#define CPF_FAMILY_SLIP 0
#define CPF_FAMILY_TWIN 1

/* Twin rate law (Section 3, equation 6).
 * NORTON: same regularized Norton rate as slip, one-sided (>= 0).
 * PAPER : rate prefactor gamma_T * K_c * (f_m - sum_beta f_beta). */
#define CPF_TWIN_NORTON 0
#define CPF_TWIN_PAPER 1

#define CPF_PREC_FP64 0
#define CPF_PREC_FP32 1 /* FP32 fields and law, FP64 reductions and means */

#define CPF_FIELD_STRESS 0         /* 6 components                     */
#define CPF_FIELD_STRAIN 1         /* 6 components                     */
#define CPF_FIELD_PLASTIC_STRAIN 2 /* 6 components                     */
#define CPF_FIELD_ACC_SLIP 3       /* n_sys components (v)             */
#define CPF_FIELD_BACK_STRAIN 4    /* n_sys components (alpha)         */
#define CPF_FIELD_SUBSTEPS 5       /* 1 component: RK4 substeps of the current load step */

#define CPF_MAX_SYSTEMS 32

/* Per-family hardening and viscosity parameters (Section 3, equations 4
 * and 5): r = tau0 + Q sum_t q_st (1 - exp(-b v_t)) within the family,
 * with q_st = q_self on the diagonal and q_latent elsewhere; Norton
 * viscosity K (MPa s^(1/n)) and exponent n.  Kinematic hardening
 * x = c*alpha, dalpha/dt = gdot - d |gdot| alpha (c = 0: the paper's law). */
typedef struct cpf_law {
    double Q, b, c, d, K, n, q_self, q_latent;
} cpf_law;

typedef struct cpf_problem_desc {
    int nx, ny, nz;           /* grid; each 2^a 3^b, 2 <= n <= 256             */
    const int32_t *labels;    /* host [nz][ny][nx], x fastest, in [0,n_labels) */
    int n_labels;
    const double *euler;      /* host [n_labels][3] Bunge (phi1, Phi, phi2),
                                 radians: Q = Rz(phi1) Rx(Phi) Rz(phi2),
                                 v_lab = Q v_crystal                           */
    double C_crystal[36];     /* Voigt 6x6 (engineering shear), MPa            */
    int n_sys;                /* 1 .. CPF_MAX_SYSTEMS                          */
    const double *n_miller;   /* host [n_sys][3] plane normals (normalized
                                 internally)                                  */
    const double *l_miller;   /* host [n_sys][3] slip directions               */
    const int32_t *family;    /* host [n_sys] CPF_FAMILY_*                     */
    const double *tau0;       /* host [n_sys] initial resistance, MPa          */
    cpf_law law[2];           /* [CPF_FAMILY_SLIP], [CPF_FAMILY_TWIN]          */
    int twin_mode;            /* CPF_TWIN_*                                    */
    double K_c, f_m, gamma_T; /* twin-fraction law (PAPER mode); f = v/gamma_T */
    double eta;               /* regularization r' = r + eta |gdot|, MPa s     */
} cpf_problem_desc;

typedef struct cpf_options {
    int precision;     /* CPF_PREC_*                                         */
    double tol;        /* convergence: err_eq <= tol and err_bc <= tol       */
    int max_iter;      /* iterations per load step before NOT_CONVERGED      */
    double h_max;      /* RK4 substeps per step: ceil(dt/h_max)              */
    int rk4_M;         /* > 0: fixed substep count (overrides h_max)         */
    double lam0, mu0;  /* > 0: reference medium override (MPa)               */
    double stag_tol;   /* FP32: accept a stalled residual below this (0: off)*/
    int check_every;   /* iterations queued per host convergence poll (0: auto) */
    int green;         /* CPF_GREEN_*: which Green operator (Section 3)      */
    double rk_tol;     /* > 0: frozen error-controlled substep counts, below */
    int aa_depth;      /* > 0: Anderson-accelerated fixed point, below       */
    int nyquist_mode;  /* CPF_NYQUIST_*: Nyquist frequencies, below          */
    int cutback;       /* > 0: a load step that ends CPF_E_NOT_CONVERGED or
                          CPF_E_NAN is retried as two half steps (times and
                          targets halved from the committed state of the
                          first RVE), recursively up to this many halvings */
    int reg_mode;      /* CPF_REG_*: when eta |gdot| enters the resistance,
                          below                                           */
} cpf_options;

/* Regularization of the yield stress (Section 4, equation "regu": the
 * resistance is raised by eta |gdot|, instantaneously; Section 4 also
 * remarks that without regularization elastoplastic and purely elastic
 * steps alternate).
 * CPF_REG_IMPLICIT (default): the rate solves gdot = A <(|tau - x| -
 *   r - eta |gdot|)/K>^n for itself at every rate evaluation (a scalar
 *   Newton solve per active system).
 * CPF_REG_LAGGED: eta times each system's mean slip rate over the previous
 *   load step, (v_n - v_{n-1}) eta / dt (zero in the first step after
 *   creation or reset), raises the resistance for the whole step, and the
 *   rate is the plain Norton law A <(|tau - x| - r - raise)/K>^n.  With
 *   eta much larger than K the steps then alternate between no slip and
 *   slip.  The raise [S][N] per RVE is part of the saved state and takes
 *   S N words of workspace.  Needs rk_tol = 0 and aa_depth = 0; the adjoint
 *   entry points and cpf_op_constitutive reject it. */
#define CPF_REG_IMPLICIT 0
#define CPF_REG_LAGGED 1

/* Anderson acceleration of the fixed point (an option; the paper's scheme
 * is the basic one; Walker and Ni, 2011).  With aa_depth = m in 1..8, the
 * iterate after x_k is x_k + f_k - sum_s gamma_s (dX_s + dF_s) instead of
 * the basic x_k + f_k, where f_j = -Gamma0 * sigma(x_j) + dE_j is the basic
 * step, dX, dF are the differences of the last (up to) m iterates and
 * steps of the load step, and gamma solves (G + lam I) gamma = dF^T f_k,
 * G = dF^T dF (Frobenius products over the voxels, FP64), lam = 1e-14
 * trace(G) / m_k (a degenerate system falls back to the basic step); the
 * mean strain is mixed with the same coefficients.  Converged results are
 * those of the basic scheme to the tolerance; iterations are fewer.  Costs
 * (2 m + 2) strain fields of workspace per RVE and a pass over them per
 * iteration.  The adjoint entry points need aa_depth = 0, and it excludes
 * rk_tol > 0. */

/* Error-controlled substeps (an option; the paper integrates each load
 * step with a fixed number of RK4 substeps).  With rk_tol > 0, at the first
 * fixed-point iteration of every load step each voxel takes the least count
 * M 2^j, j = 0 .. CPF_RK_MAX_DOUBLINGS, whose RK4 result agrees with that
 * of twice the count within Richardson's bound: the larger of the squared
 * Frobenius norm of the plastic strain difference and the squared
 * differences of each v and alpha is at most (15 rk_tol)^2 (j = the maximum
 * when none does).  The voxel keeps the result of that count, and the count
 * stays for the rest of the load step, so the stress stays a smooth
 * function of the strain iterate and the fixed point converges as with a
 * fixed count.  The adjoint entry points need rk_tol = 0.  The counts of
 * the current step are exported as CPF_FIELD_SUBSTEPS. */
#define CPF_RK_MAX_DOUBLINGS 4

/* Green operator of the fixed point (Section 3 names only "the Green
 * operator" of the reference medium).
 * CPF_GREEN_CONTINUOUS: the continuous isotropic operator at the unit
 *   frequency direction; zero at the zero frequency and at every frequency
 *   with a Nyquist component.
 * CPF_GREEN_ROTATED: its discrete variant of the rotated finite-difference
 *   scheme (Willot, 2015): the same formula at the unit vector of
 *   s_j = sin(q_j/2) prod_{l != j} cos(q_l/2), q_j = 2 pi m_j / N_j; zero
 *   only at the zero frequency and where two or more components are at
 *   Nyquist.  The solver then also stores and transforms the kx = nx/2
 *   column of the spectrum.  The equilibrium residual uses the same
 *   directions. */
#define CPF_GREEN_CONTINUOUS 0
#define CPF_GREEN_ROTATED 1

/* Nyquist frequencies of the continuous operator (even grid sizes; the
 * paper does not say how they are treated).
 * CPF_NYQUIST_ZERO (default): Gamma0 = 0 at every frequency with a
 *   component m_j = N_j/2, and those frequencies are left out of the
 *   residual; the kx = nx/2 column is then neither stored nor transformed.
 * CPF_NYQUIST_FORMULA: the formula at every nonzero frequency, with
 *   m_j = +N_j/2 at Nyquist, and the real part of the inverse transform
 *   (the formula there is not Hermitian-symmetric: the partner index -k has
 *   the same +N_j/2, so the applied operator is the average of the formula
 *   at m and at m with its Nyquist components negated); the residual sums
 *   |sigma_hat . xi_hat|^2 over every nonzero frequency of the full
 *   spectrum.  The averaged operator is not a projector where a Nyquist
 *   component meets another nonzero one, and the fixed point contracts
 *   far more slowly there (5-20 times the iterations of CPF_NYQUIST_ZERO on
 *   small even grids).  Needs CPF_GREEN_CONTINUOUS. */
#define CPF_NYQUIST_ZERO 0
#define CPF_NYQUIST_FORMULA 1

/* Loading path: n_steps increments; t has n_steps+1 times (s).  For step
 * n, strain_ctrl[n][i] = 1 prescribes the mean strain component i to
 * target[n][i] at the end of the step; 0 prescribes the mean stress. */
typedef struct cpf_path {
    int n_steps;
    const double *t;
    const uint8_t *strain_ctrl;
    const double *target;
} cpf_path;

/* Per-step results (Section 5 measures): mean stress and strain, von Mises
 * of the mean stress, mean of the local von Mises stress, mean accumulated
 * slip over slip systems, mean twin fraction over twin systems. */
typedef struct cpf_step_out {
    double Sigma[6], E[6];
    double sig_eq_of_mean, mean_sig_eq, mean_v, mean_f;
    double err_eq, err_bc;
    double n_active;  /* work counters over the step's iterations: system  */
    double n_newton;  /* rate evaluations above yield, Newton iterations   */
    int iters;        /* constitutive evaluations (fixed-point iterations) */
    int status;       /* CPF_OK, CPF_E_NOT_CONVERGED or CPF_E_NAN          */
    int stagnated;    /* 1: ended by the stalled-residual acceptance
                         (stag_tol), with err above tol                    */
    int host_syncs;   /* host waits on the device during the step (polls of
                         the step status; the same for every member)       */
    long long n_symptom; /* voxels whose stress moved by more than E0 |dE|:
                         |sigma_{n+1} - sigma_n|_F > E0 |E_{n+1} - E_n|_F
                         (Frobenius norms of tensor components, E0 the
                         Young's modulus of the reference medium), the
                         local condition under which Section 4 reports
                         that equilibrium stops being enforced; summed
                         over the sub-steps of a cut-back step             */
    int cutbacks;     /* failed attempts of the step that were retried as
                         two half steps (options.cutback)                  */
} cpf_step_out;

typedef struct cpf_problem cpf_problem;
typedef struct cpf_solver cpf_solver;

int cpf_version(void);
const char *cpf_error_string(int code);
const char *cpf_last_error_message(void);
void cpf_options_default(cpf_options *opt);

/* Validate and copy a problem (host only, no device work). */
int cpf_problem_create(const cpf_problem_desc *desc, cpf_problem **out);
void cpf_problem_destroy(cpf_problem *p);
/* Isotropic reference medium chosen for the problem's crystal stiffness:
 * k0 = (1/9) 1:C:1, mu0 = mean of the extreme deviatoric shear moduli,
 * lam0 = k0 - 2 mu0/3. */
int cpf_problem_reference_medium(const cpf_problem *p, double *lam0, double *mu0);

/* Solver: creation is host only; bind uploads the problem to the caller's
 * workspace on the caller's stream (hipStream_t, NULL = default). */
int cpf_solver_create(const cpf_problem *p, const cpf_options *opt, cpf_solver **out);
int cpf_solver_workspace_size(const cpf_solver *s, size_t *bytes);
int cpf_solver_bind(cpf_solver *s, void *dev_workspace, size_t bytes, void *hip_stream);
/* Return to the undeformed, stress-free state at t = 0. */
int cpf_solver_reset(cpf_solver *s);
/* Run load step n of the path from the committed state (the caller runs
 * steps in order); fills *out.  Synchronous. */
int cpf_solver_step(cpf_solver *s, const cpf_path *path, int n, cpf_step_out *out);
/* All steps of the path from the current state; out has n_steps entries. */
int cpf_solver_run(cpf_solver *s, const cpf_path *path, cpf_step_out *out);
/* Copy a committed local field into dev_out, [ncomp][nz][ny][nx] in the
 * solver's precision (float or double). */
int cpf_solver_field(cpf_solver *s, int field, void *dev_out);
void cpf_solver_destroy(cpf_solver *s);

/* Batches (many RVEs in one solve).  All members share the crystal
 * stiffness, the systems and the law; each has its own grid, labels and
 * orientations (the paper's realizations, Section 2.3).  Every kernel of an
 * iteration covers all members in one launch, each member keeps its own
 * convergence flag on the device, and the load step ends when all members
 * have converged.  cpf_solver_* calls act on member 0 where a single RVE is
 * meant (fields, component operators); cpf_solver_step/run need n = 1. */
int cpf_batch_create(int n, const cpf_problem *const *probs, const cpf_options *opt, cpf_solver **out);
int cpf_batch_size(const cpf_solver *s, int *n);
/* Load step n for every member; outs has one entry per member. */
int cpf_batch_step(cpf_solver *s, const cpf_path *path, int n, cpf_step_out *outs);
int cpf_batch_field(cpf_solver *s, int rve, int field, void *dev_out);
/* Launch iterations as captured HIP graphs (all members, device-side early
 * exit: the kernels of iterations after the step has ended return at
 * once).  iters_per_launch = G > 0: graphs of G iterations, replayed until
 * the step ends (one host poll per replay).  CPF_GRAPH_ADAPTIVE: each load
 * step replays a graph of the least power-of-two length (8 .. 1024)
 * covering 1.25 times the previous step's largest iteration count plus 2,
 * so that a step is normally one replay and one host poll; graphs are
 * captured per length on first use and kept.  0 returns to direct launches
 * (chunks of the previous step's iteration count between polls).  Kernel
 * timing does not see inside graphs. */
#define CPF_GRAPH_ADAPTIVE (-1)
int cpf_solver_set_graph(cpf_solver *s, int iters_per_launch);
/* Pick the y and z pass tile widths (kx columns per block) of every
 * member's grid size by timing the candidates on the bound workspace
 * (results are cached per grid and precision for the process).  Resets the
 * committed state.  *n_timed receives the number of timed configurations. */
int cpf_solver_autotune(cpf_solver *s, int *n_timed);
int cpf_solver_tiles(const cpf_solver *s, int rve, int *ty, int *tz);
/* Set the y and z pass tile widths of RVE `rve` by hand (for timing
 * studies; results do not depend on the tiles).  CPF_E_INVALID_ARG if
 * the tiles exceed the kx columns, the kernels' elements per thread or
 * their LDS.  Synchronizes the bound stream; drops captured graphs. */
int cpf_solver_set_tiles(cpf_solver *s, int rve, int ty, int tz);

/* Kernel timing (profiling aid).  While enabled, each kernel launch of the
 * iteration is bracketed by HIP events on the bound stream and its device
 * time is accumulated per kernel class: 0 x pass (local law and x
 * transforms), 1 forward y pass, 2 z pass with the Green operator, 3
 * inverse y pass, 4 boundary update.  Enabling clears the counters.
 * Launches that return at once after the step has ended are included.
 * `enable`: CPF_TIMING_OFF, CPF_TIMING_ALL (every kernel class) or
 * CPF_TIMING_XPASS (class 0 only: two events per iteration instead of
 * ten, for timing the dominant kernel with the least disturbance of the
 * rest; the other classes then stay at zero).  Other values:
 * CPF_E_INVALID_ARG.  The events are timing markers only (no system-scope
 * release).  Synchronizes the bound stream. */
#define CPF_NKERNELS 5
#define CPF_TIMING_OFF 0
#define CPF_TIMING_ALL 1
#define CPF_TIMING_XPASS 2
int cpf_solver_set_timing(cpf_solver *s, int enable);
int cpf_solver_get_timing(const cpf_solver *s, double *ms /*[5]*/, long long *launches /*[5]*/);

/* Component operators on the bound solver, for parity checks of single
 * steps of the iteration.  Device arrays in the solver's precision.
 * fields [c][nz][ny][nx]; spectra complex [nz][ny][nx/2+1][c] (re, im):
 * the six components of a frequency adjacent, as the solver stores its
 * own spectrum. */
/* Forward 3D DFT (unnormalized) of 6 real fields: spec = F[field]. */
int cpf_op_forward_fft(cpf_solver *s, const void *dev_field, void *dev_spec);
/* One Green-operator application: out = F^-1[Gamma0(xi) : spec](x), with
 * Gamma0 = 0 at xi = 0 and at frequencies with a Nyquist component, plus
 * *err2 = sum over controlled frequencies of |spec(xi).xi_hat|^2.  The
 * input spectrum is consumed (overwritten). */
int cpf_op_green(cpf_solver *s, void *dev_spec, void *dev_out, double *err2);
/* Local law over one increment for every voxel: total strain linear in
 * time from eps0 to eps1, internal variables state0 -> state1 by RK4 with
 * M substeps.  state = [6 + 2 n_sys][nvox]: plastic strain (lab frame,
 * tensor components), accumulated slip v[n_sys], back strain alpha[n_sys].
 * sig1 = C_lab:(eps1 - eps_p). */
int cpf_op_constitutive(cpf_solver *s, const void *dev_eps0, const void *dev_eps1,
                        const void *dev_state0, void *dev_state1, void *dev_sig1,
                        double dt, int M);

/* Discrete adjoint of the load-stepped solve.  The paper identifies the
 * plastic parameters of its law (Section 3, the paragraph on their values)
 * from effective stress responses; this is the gradient such an
 * identification, or any training through the solver, needs: the exact
 * derivative of a loss of the effective stress history with respect to
 * the law parameters of equations 2-6 (the paper itself prints no
 * gradient; the computation follows from differentiating the discrete
 * scheme of Sections 3-4 step by step).  Loss
 *   L = sum_n (Sigma_11(t_n+1) - target_xx[n])^2
 * over the path's steps, and its exact gradient with respect to the 14
 * parameters theta[f][k], f = 0 slip / 1 twin family, k = r0 (initial
 * critical resolved shear stress of every system of the family), Q, b, c, d,
 * K, n.  Single-RVE solvers only; the solver must be bound.
 *
 * Forward: the whole path is solved on the device, and the committed
 * (strain, state) pair is copied to the adjoint workspace every
 * checkpoint_every steps and at the end.  Reverse: segment by segment, from
 * the last, the segment's steps but its last are recomputed from its
 * checkpoint keeping every step's start state (checkpoint_every = 1
 * recomputes nothing), then for each step (last to first) one launch per voxel recomputes
 * the RK4 stage states (kept in the workspace) and sweeps them backwards for
 * the tangent d sigma / d eps and the load vector; the transposed-tangent
 * equilibrium is solved with the forward FFT and Green-operator passes to
 * adj_tol (residuals normalized by the load vector's norm); a last sweep
 * gives the cotangents carried to the previous step and the step's
 * parameter gradient (FP64 block partials, summed on the host in a fixed
 * order).
 *
 * dev_ws: device buffer of at least cpf_adjoint_workspace_size() bytes,
 *   256-byte aligned, owned by the caller, used only during the call.
 * target_xx[n_steps], grad[14] (row-major [2][7]), *loss: host, written by
 *   the call.  sigma_xx[n_steps] (host, may be NULL) receives the forward
 *   Sigma_11 per step.
 * The solver is reset to the undeformed state on return (also on errors
 * raised after the forward solve started).  Errors: CPF_E_WORKSPACE for a
 * short or misaligned buffer, CPF_E_NOT_CONVERGED / CPF_E_NAN from the
 * forward steps or an adjoint equilibrium, CPF_E_INVALID_ARG for batches,
 * checkpoint_every < 1, adj_tol <= 0 or a bad path.  The graph mode is not
 * used inside the call. */
int cpf_adjoint_workspace_size(const cpf_solver *s, const cpf_path *path, int checkpoint_every,
                               size_t *bytes);
int cpf_adjoint_gradient(cpf_solver *s, const cpf_path *path, const double *target_xx,
                         int checkpoint_every, double adj_tol, void *dev_ws, size_t bytes,
                         double *loss, double *grad /*[2][7]*/, double *sigma_xx);
/* Vector-Jacobian product of the effective stress history with respect to
 * the 14 law parameters (the general form of cpf_adjoint_gradient, for any
 * loss of the mean stresses): sigma_bar[n_steps][6] (host) is the cotangent
 * dJ/dSigma_n of each step's mean stress, tensor components
 * (11,22,33,23,13,12); grad[14] (host, [2][7] as above) receives
 * dJ/dtheta of J = sum_n sigma_bar_n . Sigma_n; sigma[n_steps][6] (host,
 * may be NULL) receives the forward mean stresses.  The forward steps are
 * solved again inside the call (with checkpoints); workspace, errors and
 * the final solver state as for cpf_adjoint_gradient, plus
 * CPF_E_INVALID_ARG for a non-finite sigma_bar. */
int cpf_adjoint_vjp(cpf_solver *s, const cpf_path *path, const double *sigma_bar, int checkpoint_every,
                    double adj_tol, void *dev_ws, size_t bytes, double *grad /*[2][7]*/, double *sigma);

/* Distribution of the local von Mises stress of the committed state (the
 * statistic of Section 5's probability density of sigma_eq, taken over all
 * voxels of all realizations): counts[nbins + 2] (host, written) of
 * sigma_eq = sqrt(3/2 dev(sigma):dev(sigma)), sigma = C:(eps - eps_p) per
 * voxel, over RVE `rve` of the batch, or all RVEs for rve = -1.  Bin
 * edges e_k = lo + k w, w = (hi - lo) / nbins (k = 0..nbins, FP64):
 * counts[0]: sigma_eq < e_0; counts[1 + k]: e_k <= sigma_eq < e_k+1;
 * counts[nbins + 1]: sigma_eq >= e_nbins or not finite.  The decision
 * compares squares in FP64, sigma_eq^2 from the stress in the solver's
 * precision by a fixed order of single correctly rounded operations (no
 * fused multiply-add),
 *   m = ((s11 + s22) + s33) / 3, d_i = s_ii - m,
 *   sigma_eq^2 = 1.5 (((d1 d1 + d2 d2) + d3 d3)
 *                     + 2 ((s23 s23 + s13 s13) + s12 s12)),
 * against e_k e_k (edges <= 0 lie below every value), so the counts are
 * reproducible bit for bit from the exported stress field.
 * 1 <= nbins <= CPF_MAX_HIST_BINS, finite lo < hi.  Synchronizes the bound
 * stream. */
#define CPF_MAX_HIST_BINS 4096
int cpf_seq_histogram(cpf_solver *s, int rve, int nbins, double lo, double hi, unsigned long long *counts);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the histogram of
 * cpf_seq_histogram, with the same bins and the same decision rule, of a
 * stress field the caller holds, without a solver or a workspace.  The
 * call allocates nothing: its device counts and squared edges live in one
 * fixed array of CPF_HIST_SCRATCH_BYTES per GPU (held by the library until
 * the process ends), hence the limit nbins <= CPF_MAX_HIST_BINS.
 *
 * dev_sig: device [6][nvox] stress components (11,22,33,23,13,12), double
 *   for precision CPF_PREC_FP64, float for CPF_PREC_FP32, caller-owned
 *   (read only); nvox >= 0 (0 gives all-zero counts).
 * counts[nbins + 2]: host, written as for cpf_seq_histogram.
 * hip_stream: a stream of the current device (NULL = default); the work is
 *   ordered on it and the call synchronizes it before returning.
 * Every call on one GPU uses that GPU's array, which keeps the last call's
 * contents (each call clears the counts first): calls that overlap on one
 * GPU (other host threads, other streams) race and must be serialized by
 * the caller.  Errors: CPF_E_INVALID_ARG for a null pointer, a bad
 * precision, nvox < 0, nbins outside 1..CPF_MAX_HIST_BINS, or not
 * (finite lo < hi); CPF_E_HIP for runtime failures. */
#define CPF_HIST_SCRATCH_BYTES 66048
int cpf_seq_histogram_field(const void *dev_sig, int precision, long long nvox, int nbins, double lo, double hi,
                            unsigned long long *counts, void *hip_stream);

/* Committed state of every RVE (strain, plastic strain, accumulated slip,
 * back strain, the step's mean stress and strain, and with CPF_REG_LAGGED
 * the resistance raises of the next step), for checkpoints
 * and restarts along a path.  dev_buf: device memory of at least
 * cpf_state_size() bytes, 256-byte aligned, caller-owned.  Save copies the
 * committed state into it; restore makes it the committed state again (the
 * same solver, or one created from the same problems and options).  Both
 * synchronize the bound stream.  Errors: CPF_E_BAD_STATE if not bound,
 * CPF_E_WORKSPACE for a misaligned buffer, CPF_E_INVALID_ARG if restore
 * finds no saved state in the buffer, or one saved under the other
 * reg_mode (whose buffer has another size); it then copies nothing. */
int cpf_state_size(const cpf_solver *s, size_t *bytes);
int cpf_state_save(cpf_solver *s, void *dev_buf);
int cpf_state_restore(cpf_solver *s, const void *dev_buf);

/* Work of the last cpf_adjoint_gradient or cpf_adjoint_vjp call on this
 * solver: fixed-point iterations of the forward steps (the first pass and
 * the recomputed steps), iterations of the adjoint equilibria, and the
 * number of recomputed steps (n_steps - ceil(n_steps / checkpoint_every)
 * per call). */
int cpf_adjoint_last_stats(const cpf_solver *s, long long *fwd_iters, long long *adj_iters,
                           int *recomputed_steps);

#ifdef __cplusplus
}
#endif
#endif /* CPFFT_H */
