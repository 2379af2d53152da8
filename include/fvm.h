/*
 * fvm.h -- C ABI of the MI355X (gfx950) solver for the single-fluid
 * four-equation model with the All-Mach THINC-TDU scheme
 * (Jiao, Schmidt, Adams, arXiv:2304.00140).
 *
 * The library advances the conserved state q = (rho, rho u_1..rho u_D,
 * rho E, rho xi) of eq. (2-1) with the right-hand side of Algorithm 1 (one
 * Runge-Kutta stage: reconstruction with limiters / THINC / fourth-order
 * central switching of Section 3.3 and Appendix D, the All-Mach Riemann solver
 * of Section 3.2, the thermodynamic dependent update of eq. (3-5) and
 * Appendix B, the CSF surface-tension source of Section 3.5) and the explicit
 * four-stage low-storage Runge-Kutta scheme named in the abstract.  xi is the
 * mass fraction of component 1 ("G"); component 0 ("L") is the liquid or
 * ambient fluid.  Each component follows a stiffened-gas law (eq. A.1.1) or
 * the Peng-Robinson law (eq. A.2.1); a cell is in pressure and temperature
 * equilibrium (Appendix A, Table A.1).
 *
 * Conventions for every call:
 *  - all calls return 0 (FVM_OK) on success or a negative FVM_E* code; no call
 *    throws or aborts; fvm_last_error() gives a message for the last failure
 *    on that context;
 *  - host arrays are caller-owned and only read/written during the call;
 *  - device pointers are caller-owned device memory (e.g. a torch tensor's
 *    data pointer) on the context's device; they are used on the context's
 *    stream and only during the call;
 *  - field layout of every state array: SoA, [field][cell], interior cells
 *    only, cell = i + n0 * (j + n1 * k), x fastest, FP64;
 *  - the context owns its device buffers and its stream is borrowed
 *    (a hipStream_t, NULL = default stream); the context is not thread-safe.
 */
#ifndef FVM_H
#define FVM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FVM_VERSION 4

enum {
  FVM_OK = 0,
  FVM_EINVAL = -1,    /* bad argument or descriptor */
  FVM_EHIP = -2,      /* HIP runtime error (message kept) */
  FVM_ENOMEM = -3,    /* device allocation failed */
  FVM_ENONPHYS = -4,  /* a cell failed the closure: rho <= 0, T <= 0 or no equilibrium state */
  FVM_ENAN = -5,      /* NaN or Inf in the state */
  FVM_ESTATE = -6     /* call out of order (e.g. stepping before a state was set) */
};

enum { FVM_FP64 = 0,      /* FP64 storage and arithmetic */
       FVM_MIXED = 1 };   /* FP32 storage, reconstruction, fluxes and update;
                             FP64 closure inversion, time step and totals */

enum { FVM_BC_PERIODIC = 0, FVM_BC_WALL = 1, FVM_BC_ZEROGRAD = 2, FVM_BC_INFLOW = 3, FVM_BC_FARFIELD = 4 };
enum { FVM_EOS_SG = 0, FVM_EOS_PR = 1 };
enum { FVM_MODEL_FOUR_EQ = 0, FVM_MODEL_BAROTROPIC = 1 };
enum { FVM_LIM_MINMOD = 0, FVM_LIM_KOREN = 1, FVM_LIM_VANALBADA = 2, FVM_LIM_VANLEER = 3,
       FVM_LIM_CHAKRAVARTHY = 4, FVM_LIM_MC = 5, FVM_LIM_SUPERBEE = 6, FVM_LIM_NONE = 7 };

#define FVM_MAXSPEC 4

/* Grid of one case: uniform Cartesian, 2 ghost layers (the four-cell stencil
 * of Fig. 3.1) generated inside the kernels from the boundary kinds.
 * n[d] >= 2 for d < dim, n[d] = 1 otherwise.  bc[d][0] / bc[d][1] apply at
 * the min / max side of direction d.  FVM_BC_INFLOW is allowed only at the
 * x-min side: inside the disk |(x_2, x_3) - in_center| < in_radius (2D: the
 * slot |x_2 - in_center[0]| < in_radius; 1D: everywhere) the ghost cells hold
 * the state (in_p, in_T, alpha_G = in_alpha, u = (in_u, 0, 0) + noise) with
 * noise_c = in_noise * in_u * (2 h - 1), h a SplitMix64 hash of
 * (in_seed, step, j, k, c); outside the disk the plane is a slip wall.
 * FVM_BC_FARFIELD (any side): the ghost cells hold the fixed state at rest
 * (ff_p, ff_T, alpha_G = ff_alpha), a reservoir standing in for non-reflective
 * far-field boundaries; a ghost cell beyond any far-field side takes it. */
typedef struct fvm_grid_desc {
  int dim;
  int n[3];
  double dx[3];
  int bc[3][2];
  double in_p, in_T, in_alpha, in_u, in_radius, in_center[2], in_noise;
  uint64_t in_seed;
  double ff_p, ff_T, ff_alpha;
} fvm_grid_desc;

/* Closure of the two components (Appendix A).
 * Stiffened gas: p = (gamma - 1) rho (e - q) - gamma pinf with e = cv T + pinf v + q.
 * Peng-Robinson (kind FVM_EOS_PR): fixed-composition pseudo-mixture of pr_ns
 * species (mole fractions pr_X, critical temperature/pressure/molar volume/
 * compressibility, acentric factor, molar mass [kg/mol], binary interaction
 * pr_kij) with the mixing rules of A.2.1; its ideal-gas part has constant cv and
 * reference energy q.  gamma and pinf are ignored for a PR component.
 * p_ref, T_ref: reference state of the FP32 storage shifts (FVM_MIXED only):
 * the partial density of each stiffened gas with pinf > 0 and the energy of
 * both components are stored relative to their values at (p_ref, T_ref), which
 * keeps FP32 storage accurate in stiff liquids; T_ref = 0 disables the shifts.
 * FVM_FP64 stores the conserved variables unshifted.
 * mu [Pa s], kc [W/(m K)]: dynamic viscosity and thermal conductivity of each
 * component for the stress part of the flux of eq. (2-2); a cell mixes them by
 * its gas volume fraction, (1 - alpha_G) value_0 + alpha_G value_1 (eq. 2-8
 * with one gas and no vapour).  All zero: inviscid and adiabatic (the stress
 * terms are skipped).  Negative or non-finite values are FVM_EINVAL.
 * ncomp: 2 (0 means 2) or 3.  With three components (Table A.1, eqs.
 * A.1.2-A.1.5: a liquid and two gases, the second gas species of eq. 2-1)
 * every component is a stiffened gas and components 1 and 2 are ideal gases
 * (pinf = 0); the state gains rho xi_2 (N_q = D + 4: rho, rho u, rho E,
 * rho xi_1, rho xi_2), the primitive input gains alpha_2 after u, the
 * primitive output gains xi_2 and alpha_2 (11 rows), and the mixing above is
 * (1 - alpha_1 - alpha_2) value_0 + alpha_1 value_1 + alpha_2 value_2.  Three
 * components run in 1D, 2D and 3D; in 3D in FP64 the 8x8x8 tile does not fit
 * the LDS of a workgroup (fvm_set_tile returns FVM_EINVAL for it).
 * model: FVM_MODEL_FOUR_EQ (0, everything above) or FVM_MODEL_BAROTROPIC, the
 * barotropic equilibrium model of Section 2.2 (eqs. 2-3 .. 2-7), which
 * replaces the components above (kind, gamma, pinf, cv, q, PR data and T_ref
 * are ignored; kc must be 0; ncomp 0 or 2: one gas, 3: two gases): a liquid with
 * rho = bt_rho_sat + (p - bt_p_sat) / bt_c_liq^2 at p >= bt_p_sat that is a
 * liquid-vapour mixture below it (the same law with c_M^2 = p_sat / rho_sat),
 * and one isothermal ideal gas rho_G = p / bt_RT (bt_RT = R_Gas T_ref); with
 * ncomp = 3 a second one, rho_G2 = p / bt_RT2 (eqs. 2-5, 2-6 with Gas1 and
 * Gas2), whose mass fraction xi_2 is transported like xi.
 * There is no energy equation: N_q = D + 2 (rho, rho u, rho xi; two gases:
 * D + 3 with rho xi_2 last); p follows from (rho, xi[, xi_2]); the T row of the primitive input and in_T, ff_T of the grid
 * are ignored (a far-field or inflow state needs p > 0 instead); the primitive
 * output has 12 rows (the 11 above with T = xi_2 = alpha_2 = 0, then the
 * vapour volume fraction of eq. 2-7, at most 0.995).  Where the upwind cell
 * of a face is a liquid-vapour interface cell (eps < alpha_V < 1 - eps, and
 * alpha_V and rho monotone through it) the face density is the THINC value
 * of rho (eqs. 3-7, 3-8, Remarks 1-2), elsewhere rho(p*, xi_face).  FP32
 * storage (FVM_MIXED) keeps the liquid's partial density relative to its
 * density at p_ref.  Viscous stress (no heat conduction, no energy): mu[0]
 * (liquid), mu[1] (gas), mu[2] (second gas) and bt_mu_vap (vapour) enter the
 * mixture viscosity of eq. 2-8, (1 - alpha_G - alpha_G2)[(1 - a_v)(1 + 5/2 a_v)
 * mu_liq + a_v mu_vap] + alpha_G mu_gas + alpha_G2 mu_gas2, a_v = alpha_V /
 * (1 - alpha_G - alpha_G2) the vapour share of the liquid-vapour part; all
 * zero: inviscid.  The primitive input of two gases has alpha_G2 after u; the
 * output keeps 12 rows with xi_2 and alpha_G2 in rows 9 and 10.  Requires bt_rho_sat > 0,
 * bt_p_sat > 0, bt_c_liq > 0, 0 <= bt_rho_vap < bt_rho_sat, bt_RT > 0 (and
 * bt_RT2 > 0 with two gases), finite viscosities >= 0; 1D, 2D and 3D. */
typedef struct fvm_eos_desc {
  int kind[3];
  double gamma[3], pinf[3], cv[3], q[3];
  int pr_ns[2];
  double pr_X[2][FVM_MAXSPEC], pr_Tc[2][FVM_MAXSPEC], pr_pc[2][FVM_MAXSPEC];
  double pr_omega[2][FVM_MAXSPEC], pr_M[2][FVM_MAXSPEC];
  double pr_Zc[2][FVM_MAXSPEC], pr_vc[2][FVM_MAXSPEC];
  double pr_kij[2][FVM_MAXSPEC][FVM_MAXSPEC];
  double p_ref, T_ref;
  double mu[3], kc[3];
  int ncomp;
  int model;
  double bt_rho_sat, bt_p_sat, bt_c_liq, bt_rho_vap, bt_RT;
  double bt_mu_vap;
  double bt_RT2;
} fvm_eos_desc;

/* Scheme parameters (Section 3.3, Appendix D; defaults in brackets):
 * switching: 0 = discontinuous branch at every face (Section 3), 1 = sensor
 * switching of eq. (D.3)/(D.4) with the Ducros and gas-volume-fraction sensors
 * (barotropic model: also the vapour-volume-fraction sensor, threshold theta_gas);
 * lim_u / lim_s: limiter for velocities [Koren] / for p, T, xi [Minmod];
 * thinc: THINC for xi at interface cells [1]; beta [1.6], thinc_gamma [1e-20],
 * eps_interface [1e-4] (eligibility eps < xi < 1 - eps and monotone);
 * theta_ducros [0.95], theta_gas [0.4], eps_ducros [1e-20];
 * kappa3 [1/4]: scale of the third-difference pressure term of eq. (D.5);
 * rk[4] [1/4, 1/3, 1/2, 1]: q^(k) = q^n + rk[k-1] dt R(q^(k-1));
 * cfl [0.5]: dt = cfl / max_cells [sum_d (|u_d| + c) / dx_d + 2 nu sum_d 1/dx_d^2],
 *   nu = max(mu, kc / cv) / rho of the cell (cv mixed by mass fraction; the
 *   second term only with viscous or conducting fluids);
 * sigma [0]: surface tension (CSF on when > 0); eps_normal [1e-12];
 * gravity[3] [0]: body-force acceleration g [m/s^2] of eq. (2-2): the source
 *   rho g on the momentum and rho u.g on the energy;
 * thermal [0]: the thermal variable reconstructed at a face (Appendix B): 0
 *   the temperature, rho_f and e_f from the closure at (p*, T_f, xi_f); 1 the
 *   specific internal energy, reconstructed as T would be, rho_f from the
 *   closure at (p*, xi_f, e_f).  thermal = 1 takes the two-component
 *   stiffened-gas closure in 1D and 2D (FVM_EINVAL otherwise). */
typedef struct fvm_scheme_desc {
  int switching, lim_u, lim_s, thinc;
  double beta, thinc_gamma, eps_interface;
  double theta_ducros, theta_gas, eps_ducros;
  double kappa3;
  double rk[4];
  double cfl;
  double sigma;
  double eps_normal;
  double gravity[3];
  int thermal;
} fvm_scheme_desc;

typedef struct fvm_ctx fvm_ctx;

/* Create a context for one case.  precision: FVM_FP64 or FVM_MIXED.
 * stream: hipStream_t to launch on (borrowed).  Allocates the state buffers
 * (3 x N_q x ncell words of the storage type) on the current device; in 3D
 * also the primitive rows of the closure kernel (9 or 11 x ncell words) and,
 * for the four-equation closure + face tiles, 32 bytes per 256 cells and one
 * byte per tile for the surface-tension marks (tables of the tile set by
 * fvm_set_tile, reallocated with it). */
int fvm_create(fvm_ctx** out, const fvm_grid_desc* g, const fvm_eos_desc* e,
               const fvm_scheme_desc* s, int precision, void* stream);
void fvm_destroy(fvm_ctx* ctx);

/* Set the state from primitives on the host: prim[(3 + D) x ncell] =
 * (p, T, alpha_G, u_1..u_D) (three components: [(4 + D) x ncell], alpha_2
 * last); xi follows from alpha_G at the cell's (p, T) (barotropic model: at p).
 * Resets t and the step counter to 0.  FVM_ENONPHYS if a cell has no state. */
int fvm_init_primitive(fvm_ctx* ctx, const double* prim_host);
/* Set / read the conserved state (host or device arrays, [N_q x ncell] FP64).
 * set_state resets t and the step counter to 0. */
int fvm_set_state(fvm_ctx* ctx, const double* q_host);
int fvm_set_state_device(fvm_ctx* ctx, const double* q_dev);
int fvm_get_state(fvm_ctx* ctx, double* q_host);
int fvm_get_state_device(fvm_ctx* ctx, double* q_dev);
/* Primitives of the current state [9 x ncell] FP64 on the host:
 * rho, u_1, u_2, u_3, p, T, xi, c, alpha_G (unused velocity rows are 0);
 * three components: [11 x ncell], with xi_2 and alpha_2 appended;
 * barotropic model: [12 x ncell], T = xi_2 = alpha_2 = 0, alpha_V last. */
int fvm_get_primitive(fvm_ctx* ctx, double* w_host);

/* One right-hand side R(q) of Algorithm 1 without time update:
 * q_dev_in and r_dev_out are device arrays [N_q x ncell] FP64 (caller-owned).
 * The inflow noise uses step number `step`.  The context's own state is not
 * touched. */
int fvm_rhs(fvm_ctx* ctx, const double* q_dev_in, double* r_dev_out, int64_t step);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): fvm_rhs without a
 * context.  One right-hand side R(q) of the FP64 path for the case described
 * by g, e, s (validated as by fvm_create; the FP64 path stores q unshifted, so
 * e->p_ref / e->T_ref do not matter), q_dev_in and r_dev_out device arrays
 * [N_q x ncell] FP64 owned by the caller, inflow noise of step `step`,
 * launched on `stream` (a hipStream_t, NULL = default stream) of the current
 * device; returns after the launches without waiting (the result is ready
 * when the stream reaches them).  It allocates nothing: its tables and the
 * storage copy of q (3D also the primitive rows) live in one static device
 * array of FVM_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends.  A
 * case that needs more (about 40 bytes per cell in 2D, 120 in 3D) is
 * FVM_EINVAL with a message (fvm_last_error(NULL)).  All calls on one GPU
 * share that array and it keeps the last call's contents: calls that overlap
 * on one GPU (other streams or threads) race and must be ordered by the
 * caller.  The default tile shape of the dimension is used. */
#define FVM_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
int fvm_rhs_noalloc(const fvm_grid_desc* g, const fvm_eos_desc* e, const fvm_scheme_desc* s,
                    const double* q_dev_in, double* r_dev_out, int64_t step, void* stream);

/* Advance by one step (4 stages).  dt_out / t_out may be NULL.  Synchronises. */
int fvm_step(fvm_ctx* ctx, double* dt_out, double* t_out);
/* Advance by n steps entirely on the device (dt from the stage-4 reduction of
 * the previous step, no host round trip; launched as captured HIP graphs).
 * t_end > 0 shortens the step that reaches t_end and makes later steps
 * empty.  Synchronises once at the end and reports the first failure. */
int fvm_n_steps(fvm_ctx* ctx, int n, double t_end, double* t_out);
/* Time, dt of the last step and number of steps taken. */
int fvm_clock(fvm_ctx* ctx, double* t, double* dt, int64_t* steps);
/* Conserved totals sum_cells q * cell volume [N_q], FP64, deterministic order. */
int fvm_totals(fvm_ctx* ctx, double* out);
/* First failure recorded by the kernels: code (FVM_ENONPHYS / FVM_ENAN or 0),
 * cell index and step. */
int fvm_error_info(fvm_ctx* ctx, int* code, int64_t* cell, int64_t* step);

/* Launch configuration: tile shape index of the fused stage kernel for this
 * context's dimension (0 .. fvm_tile_count(dim) - 1) and its extent.  In 3D,
 * indices 0-4 and, after the z-marching kernel's, the last five are the
 * closure + face kernel pair (the last five with one thread per face of the
 * direction with the most faces); the z-marching tiles take only the
 * two-component inviscid closures with the default limiters.
 * fvm_set_tile / fvm_batch_set_tile return FVM_EINVAL (state unchanged) for an
 * index out of range or a tile whose kernels do not fit this closure and
 * precision (3D in FP64 with three components or with two gases in the
 * barotropic model: the 8x8x8 tiles). */
int fvm_tile_count(int dim);
int fvm_tile_shape(int dim, int tile, int* tx, int* ty, int* threads);
/* Kernels one stage of a tile index launches: FVM_TK_STAGE (the fused 1D/2D
 * stage kernel), FVM_TK_PAIR (3D: closure kernel, then the LDS-tiled face
 * kernel), FVM_TK_MARCH (3D: the z-marching kernel with the closure in it),
 * FVM_TK_PRIM_MARCH (3D: closure kernel, then the z-marching kernel);
 * FVM_EINVAL for no such tile. */
enum { FVM_TK_STAGE = 0, FVM_TK_PAIR = 1, FVM_TK_MARCH = 2, FVM_TK_PRIM_MARCH = 3 };
int fvm_tile_kernels(int dim, int tile);
int fvm_set_tile(fvm_ctx* ctx, int tile);
/* Mean duration [ms] of each of the four stage kernels over `steps` steps,
 * measured with HIP events on the context's stream around every stage
 * launch (the state advances). */
int fvm_time_stages(fvm_ctx* ctx, int steps, double* ms_per_stage);

/* ---- batches: many independent cases of uneven size advanced together ----
 * All cases share the scheme and the precision; every launch covers the tiles
 * of all cases (one entry per tile in a device table), each case keeps its own
 * dt, t and step counter. */
typedef struct fvm_batch fvm_batch;
int fvm_batch_create(fvm_batch** out, int ncases, const fvm_grid_desc* grids,
                     const fvm_eos_desc* eos, const fvm_scheme_desc* s, int precision,
                     void* stream);
void fvm_batch_destroy(fvm_batch* b);
int fvm_batch_init_primitive(fvm_batch* b, int icase, const double* prim_host);
int fvm_batch_set_state(fvm_batch* b, int icase, const double* q_host);
int fvm_batch_get_state(fvm_batch* b, int icase, double* q_host);
int fvm_batch_n_steps(fvm_batch* b, int n, double* t_out /* [ncases] or NULL */);
int fvm_batch_totals(fvm_batch* b, int icase, double* out);
int fvm_batch_error_info(fvm_batch* b, int* code, int* icase, int64_t* cell, int64_t* step);
int fvm_batch_time_stages(fvm_batch* b, int steps, double* ms_per_stage);
int fvm_batch_set_tile(fvm_batch* b, int tile);
int64_t fvm_batch_cells(fvm_batch* b);

const char* fvm_last_error(const fvm_ctx* ctx);
const char* fvm_batch_last_error(const fvm_batch* b);
int fvm_version(void);

#ifdef __cplusplus
}
#endif
#endif
