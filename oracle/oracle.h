/*
 * oracle.h -- plain CPU FP64 oracle of the All-Mach THINC-TDU four-equation
 * finite-volume right-hand side and its four-stage low-storage Runge-Kutta
 * step (Jiao, Schmidt, Adams, arXiv:2304.00140).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library under
 * paper_2304_00140_amd/; neither includes the other.
 *
 * Every routine follows the paper's steps in its own order and notation, one
 * plain loop per step, no blocking and no fusion.  Where the paper is silent or
 * garbled the reading taken is stated at the routine (the DESIGN notes list
 * them all).
 *
 * State layout: SoA, q[f * ncell + cell], cell = i + n0 * (j + n1 * k), interior
 * cells only, x fastest.  Fields f: rho, rho*u_1 .. rho*u_D, rho*E, rho*xi
 * (N_q = D + 3), xi = mass fraction of component 2 ("G"); with a second gas
 * rho*xi_2 follows (N_q = D + 4).  The barotropic model (Section 2.2) has no
 * energy equation: rho, rho*u_1 .. rho*u_D, rho*xi (N_q = D + 2).
 */
#ifndef ORACLE_H
#define ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OG_BC_PERIODIC = 0, OG_BC_WALL = 1, OG_BC_ZEROGRAD = 2, OG_BC_INFLOW = 3, OG_BC_FARFIELD = 4 };
enum { OG_EOS_SG = 0, OG_EOS_PR = 1 };
enum { OG_MODEL_FOUR_EQ = 0, OG_MODEL_BAROTROPIC = 1 };
enum {
  OG_LIM_MINMOD = 0, OG_LIM_KOREN = 1, OG_LIM_VANALBADA = 2, OG_LIM_VANLEER = 3,
  OG_LIM_CHAKRAVARTHY = 4, OG_LIM_MC = 5, OG_LIM_SUPERBEE = 6, OG_LIM_NONE = 7
};

#define OG_MAXSPEC 4

typedef struct {
  int dim;              /* 1, 2 or 3 */
  int n[3];             /* interior cells per direction (unused = 1) */
  double dx[3];         /* cell sizes [m] */
  int bc[3][2];         /* boundary kind per direction and side (0 = min) */
  /* inflow on the x-min side (only there): inside the disk of radius
   * in_radius about (in_center[0], in_center[1]) in the (x_1, x_2) plane the
   * ghost state is (in_p, in_T, in_alpha, in_u + noise); outside it the
   * ghost is a slip wall. */
  double in_p, in_T, in_alpha, in_u, in_radius, in_center[2];
  double in_noise;      /* noise amplitude as a fraction of in_u */
  uint64_t in_seed;
  /* far-field sides: ghost cells hold the fixed state (ff_p, ff_T, ff_alpha, u = 0) */
  double ff_p, ff_T, ff_alpha;
} og_grid;

#define OG_MAXCOMP 3

typedef struct {
  /* components: 0 (liquid or ambient fluid), 1 and, with ncomp = 3, 2 (gases,
   * transported mass fractions xi_1, xi_2).  ncomp = 0 means 2. */
  int kind[OG_MAXCOMP];   /* OG_EOS_SG or OG_EOS_PR per component */
  /* stiffened gas: p = (gamma-1) rho (e - q) - gamma p_inf, e = cv T + p_inf v + q */
  double gamma[OG_MAXCOMP], pinf[OG_MAXCOMP], cv[OG_MAXCOMP], q[OG_MAXCOMP];
  /* Peng-Robinson pseudo-mixture (kind == OG_EOS_PR, components 0 and 1 of a
   * two-component closure only): ns species with mole fractions X, critical
   * data, acentric factors, molar masses [kg/mol] and binary interaction
   * parameters; ideal-gas part with a constant specific cv (cv[k]) and
   * reference energy q[k]. */
  int pr_ns[2];
  double pr_X[2][OG_MAXSPEC], pr_Tc[2][OG_MAXSPEC], pr_pc[2][OG_MAXSPEC];
  double pr_omega[2][OG_MAXSPEC], pr_M[2][OG_MAXSPEC];
  double pr_Zc[2][OG_MAXSPEC], pr_vc[2][OG_MAXSPEC];
  double pr_kij[2][OG_MAXSPEC][OG_MAXSPEC];
  /* transport (eq. 2-2): dynamic viscosity [Pa s] and thermal conductivity
   * [W/(m K)] per component; the cell values mix them by volume fraction
   * (eq. 2-8 with one gas and no vapour).  All zero: inviscid, adiabatic. */
  double mu[OG_MAXCOMP], kc[OG_MAXCOMP];
  /* 2 (default when 0) or 3; with 3 components every component is a
   * stiffened gas and the gases (1, 2) are ideal (p_inf = 0), the form of
   * Appendix A's Table A.1 and eqs. (A.1.2)-(A.1.5) */
  int ncomp;
  /* model = OG_MODEL_BAROTROPIC: the barotropic equilibrium model of
   * Section 2.2 (eqs. 2-3 .. 2-7) replaces the components above: a liquid
   * (saturated density bt_rho_sat at bt_p_sat, speed of sound bt_c_liq)
   * that becomes a liquid-vapour mixture below bt_p_sat (c_M^2 = p_sat /
   * rho_sat; saturated vapour density bt_rho_vap for the vapour fraction),
   * and one isothermal ideal gas with rho_G = p / bt_RT (bt_RT = R_Gas T_ref).
   * Its viscosities: mu[0] liquid, mu[1] gas, bt_mu_vap vapour (eq. 2-8). */
  int model;
  double bt_rho_sat, bt_p_sat, bt_c_liq, bt_rho_vap, bt_RT;
  double bt_mu_vap;
  /* ncomp = 3 in the barotropic model: a second isothermal ideal gas with
   * rho_G2 = p / bt_RT2 (viscosity mu[2]) */
  double bt_RT2;
} og_eos;

typedef struct {
  int switching;        /* 0: discontinuous branch everywhere (f = 1); 1: App. D sensor switching */
  int lim_u, lim_s;     /* limiter for velocities / for p, T, xi */
  int thinc;            /* 1: THINC for xi at eligible cells */
  double beta, thinc_gamma, eps_interface;
  double theta_ducros, theta_gas, eps_ducros;
  double kappa3;        /* scale of the third-difference pressure term (D.5) */
  double rk[4];         /* low-storage RK stage coefficients */
  double cfl;
  double sigma;         /* surface tension [N/m]; 0 disables the CSF source */
  double eps_normal;    /* interface-normal regularisation, times 1/dx */
  double gravity[3];    /* body-force acceleration g [m/s^2] (eq. 2-2, source Q) */
  /* thermal variable reconstructed at a face (Appendix B): 0 the temperature,
   * with rho_f, e_f from the closure at (p*, T_f, xi_f); 1 the specific
   * internal energy, reconstructed as T would be, with rho_f from the closure
   * at (p*, xi_f, e_f) (two stiffened-gas components only) */
  int thermal;
} og_scheme;

/* primitive vector of one cell.  Y2, A2: second gas (0 with two components);
 * AV: vapour volume fraction (barotropic model; 0 otherwise); E: specific
 * internal energy; T and E are 0 in the barotropic model */
enum { OW_RHO = 0, OW_U = 1, OW_V = 2, OW_W = 3, OW_P = 4, OW_T = 5, OW_Y = 6, OW_C = 7, OW_A = 8,
       OW_Y2 = 9, OW_A2 = 10, OW_AV = 11, OW_E = 12, OW_N = 13 };

/* ---- thermodynamics (Appendix A) ---- */
/* number of components (2 or 3) and of conserved fields */
int og_ncomp(const og_eos* e);
int og_nq(const og_grid* g, const og_eos* e);
/* two components: Y is the mass fraction of component 1 */
int og_eos_forward(const og_eos* e, double p, double T, double Y, double* rho, double* ein);
/* (p, e, xi) -> (rho, T) for two stiffened-gas components in p-T equilibrium;
 * -1 for other closures or a state with no positive T */
int og_eos_forward_e(const og_eos* e, double p, double ein, double Y, double* rho, double* T);
int og_eos_inverse(const og_eos* e, double rho, double ein, double Y, double Tguess,
                   double* p, double* T);
/* any number of components: Y1, Y2 the gas mass fractions (Y2 = 0 with two) */
int og_eos_forward2(const og_eos* e, double p, double T, double Y1, double Y2, double* rho, double* ein);
int og_eos_inverse2(const og_eos* e, double rho, double ein, double Y1, double Y2, double Tguess,
                    double* p, double* T);
double og_sound(const og_eos* e, int k, double p, double T);
/* mass fraction clipped into [0, 1] for the inverse closure (NaN unchanged) */
double og_clip_fraction(double Y);
/* three components: the gas fractions as the closure takes them, Yk = (liquid, gas 1, gas 2) */
void og_clip_fractions3(double Y1, double Y2, double Yk[3]);
double og_mix_sound(const og_eos* e, double p, double T, double Y);
double og_mix_sound2(const og_eos* e, double p, double T, double Y1, double Y2);
double og_spec_volume(const og_eos* e, int k, double p, double T);
double og_spec_energy(const og_eos* e, int k, double p, double T);
int og_pr_coeffs(const og_eos* e, int k, double T, double* a, double* dadT, double* d2adT2,
                 double* b, double* M);
double og_pr_pressure(const og_eos* e, int k, double T, double vmass);
double og_pr_energy_tv(const og_eos* e, int k, double T, double vmass);

/* ---- barotropic model (Section 2.2) ---- */
int og_is_barotropic(const og_eos* e);
double og_baro_liquid_density(const og_eos* e, double p);
double og_baro_density(const og_eos* e, double p, double Y);
int og_baro_pressure(const og_eos* e, double rho, double Y, double* p);
double og_baro_sound(const og_eos* e, double p);
void og_baro_fractions(const og_eos* e, double rho, double Y, double p, double* alpha_G, double* alpha_V);
/* mixture viscosity of eq. 2-8 (one gas) from the cell's alpha_G and alpha_V */
double og_baro_viscosity(const og_eos* e, double alpha_G, double alpha_V);
/* the same with two gases (ncomp = 3): xi_2 / alpha_G2 of the second gas */
double og_baro_density2(const og_eos* e, double p, double Y, double Y2);
int og_baro_pressure2(const og_eos* e, double rho, double Y, double Y2, double* p);
void og_baro_fractions2(const og_eos* e, double rho, double Y, double Y2, double p, double* alpha_G,
                        double* alpha_G2, double* alpha_V);
double og_baro_viscosity2(const og_eos* e, double alpha_G, double alpha_G2, double alpha_V);

/* ---- reconstruction (Section 3.3, Table 4.2, Appendix D) ---- */
double og_limiter_table(int kind, double r);
double og_slope(int kind, double dfar, double dnear);
double og_thinc_left(double a, double b, double c, double beta, double gam);
double og_thinc_right(double a, double b, double c, double beta, double gam);
double og_central4(double a, double b, double c, double d);

/* one face flux from the primitives of the four cells i-1, i, i+1, i+2 along
 * direction dir.  f = 1 selects the discontinuous branch; s_left / s_right are
 * the THINC eligibilities of cells i and i+1 along dir (bit 0: xi_1, bit 1:
 * xi_2). */
int og_face_flux(const og_eos* e, const og_scheme* s, int dim, int dir,
                 const double W[4][OW_N], int f, int s_left, int s_right,
                 double* F, double* ustar, double* pstar);
/* the same for the barotropic model (bit 0: xi, bit 1: the vapour fraction) */
int og_face_flux_baro(const og_eos* e, const og_scheme* s, int dim, int dir,
                      const double W[4][OW_N], int f, int s_left, int s_right,
                      double* F, double* ustar, double* pstar);

/* ---- whole-field operations ---- */
int og_cons_from_prim(const og_grid* g, const og_eos* e, const double* prim, double* q);
int og_prim_from_cons(const og_grid* g, const og_eos* e, const double* q, double* W);
int og_rhs(const og_grid* g, const og_eos* e, const og_scheme* s, const double* q,
           int64_t step, double* r);
int og_curvature(const og_grid* g, const og_eos* e, const og_scheme* s, const double* q,
                 double* kappa);
int og_sensor_flags(const og_grid* g, const og_eos* e, const og_scheme* s, const double* q,
                    unsigned char* flags);
double og_dt(const og_grid* g, const og_eos* e, const og_scheme* s, const double* q);
int og_step(const og_grid* g, const og_eos* e, const og_scheme* s, double* q,
            int64_t step, double* t, double t_end, double* dt_out);
int og_run(const og_grid* g, const og_eos* e, const og_scheme* s, double* q,
           int64_t step0, int nsteps, double* t, double t_end);
void og_totals(const og_grid* g, const og_eos* e, const double* q, double* out);

/* low-storage RK combination with a caller-supplied right-hand side */
typedef void (*og_rhs_fn)(const double* q, double* r, int n, void* user);
void og_lsrk(const og_scheme* s, double* q, int n, double dt, og_rhs_fn f, void* user);

/* counter-based noise for the inflow: SplitMix64 chained over the keys */
uint64_t og_splitmix64(uint64_t x);
double og_noise01(uint64_t seed, uint64_t step, uint64_t j, uint64_t k, uint64_t comp);

int og_nthreads(void);
/* threads of the OpenMP loops from now on (n > 0) */
void og_set_nthreads(int n);
const char* og_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
