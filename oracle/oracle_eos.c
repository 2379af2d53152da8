/*
 * oracle_eos.c -- thermodynamic closure of the oracle (test infrastructure).
 *
 * Appendix A of the paper: each component follows a stiffened-gas law
 * (eq. A.1.1) or the Peng-Robinson law (eq. A.2.1); the mixture quantities
 * follow Table A.1 (volume- and mass-fraction weighted density and internal
 * energy).  The tables of the paper list one temperature per case for both
 * components, so the closure is read as pressure AND temperature equilibrium
 * inside a cell.
 *
 * Stiffened gas with a temperature (A.1.1 with rho_k = (p + p_inf) / ((gamma-1) cv T)):
 *   v_k(p,T) = (gamma_k - 1) cv_k T / (p + pinf_k)
 *   e_k(p,T) = cv_k T + pinf_k v_k + q_k
 *   c_k(T)^2 = gamma_k (p + pinf_k) v_k = gamma_k (gamma_k - 1) cv_k T
 * Peng-Robinson (A.2.1) on a molar basis, V = M v:
 *   p = R T / (V - b) - a(T) / (V^2 + 2 b V - b^2)
 *   e = cv T + q + (a - T a') / (2 sqrt2 b M) ln((V + (1-sqrt2) b) / (V + (1+sqrt2) b))
 * The energy is the ideal-gas part (constant cv; the NASA polynomial data the
 * paper cites are not used) plus the departure integral of T dp/dT - p over V.
 */
#include <math.h>
#include <float.h>
#include "oracle.h"
#include "oracle_internal.h"

static const double R_U = 8.314462618;          /* J / (mol K) */
static const double SQRT2 = 1.41421356237309505;

/* ---------------- Peng-Robinson pieces (A.2.1) ---------------- */

/* a(T), a'(T), a''(T) and b of the van der Waals one-fluid mixing rules of
 * A.2.1 with the combining rules for the critical data printed there. */
int og_pr_coeffs(const og_eos* e, int k, double T, double* a, double* dadT, double* d2adT2,
                 double* b, double* M)
{
  int ns = e->pr_ns[k];
  double A = 0, A1 = 0, A2 = 0, B = 0, MM = 0;
  if (ns < 1 || ns > OG_MAXSPEC || !(T > 0)) return -1;
  for (int al = 0; al < ns; ++al) {
    B += e->pr_X[k][al] * 0.077796 * R_U * e->pr_Tc[k][al] / e->pr_pc[k][al];
    MM += e->pr_X[k][al] * e->pr_M[k][al];
  }
  for (int al = 0; al < ns; ++al) {
    for (int be = 0; be < ns; ++be) {
      double Tc = sqrt(e->pr_Tc[k][al] * e->pr_Tc[k][be]) * (1.0 - e->pr_kij[k][al][be]);
      double cv3 = 0.5 * (cbrt(e->pr_vc[k][al]) + cbrt(e->pr_vc[k][be]));
      double vc = cv3 * cv3 * cv3;
      double Zc = 0.5 * (e->pr_Zc[k][al] + e->pr_Zc[k][be]);
      double pc = Zc * R_U * Tc / vc;
      double w = 0.5 * (e->pr_omega[k][al] + e->pr_omega[k][be]);
      double cc = 0.37464 + 1.5422 * w - 0.26992 * w * w;
      double a0 = 0.457236 * (R_U * Tc) * (R_U * Tc) / pc;
      double s = sqrt(T / Tc);
      double g = 1.0 + cc * (1.0 - s);
      double aab = a0 * g * g;
      double da = -a0 * cc * g / (Tc * s);
      double d2a = a0 * cc / (2.0 * Tc * Tc) * (cc / (s * s) + g / (s * s * s));
      double XX = e->pr_X[k][al] * e->pr_X[k][be];
      A += XX * aab;
      A1 += XX * da;
      A2 += XX * d2a;
    }
  }
  *a = A; *dadT = A1; *d2adT2 = A2; *b = B; *M = MM;
  return 0;
}

double og_pr_pressure(const og_eos* e, int k, double T, double vmass)
{
  double a, a1, a2, b, M;
  if (og_pr_coeffs(e, k, T, &a, &a1, &a2, &b, &M)) return NAN;
  double V = M * vmass;
  return R_U * T / (V - b) - a / (V * V + 2.0 * b * V - b * b);
}

static double pr_logterm(double V, double b)
{
  return log((V + (1.0 - SQRT2) * b) / (V + (1.0 + SQRT2) * b));
}

double og_pr_energy_tv(const og_eos* e, int k, double T, double vmass)
{
  double a, a1, a2, b, M;
  if (og_pr_coeffs(e, k, T, &a, &a1, &a2, &b, &M)) return NAN;
  double V = M * vmass;
  return e->cv[k] * T + e->q[k] + (a - T * a1) / (2.0 * SQRT2 * b * M) * pr_logterm(V, b);
}

/* molar volume of the Peng-Robinson fluid at (p, T): the largest real root of
 * the compressibility cubic, by Newton iteration from Z = 1 + B, which bounds
 * every root with V > b from above. */
static double pr_molar_volume(double p, double T, double a, double b)
{
  double Ad = a * p / (R_U * T * R_U * T);
  double Bd = b * p / (R_U * T);
  double c2 = Bd - 1.0;
  double c1 = Ad - 3.0 * Bd * Bd - 2.0 * Bd;
  double c0 = Bd * Bd * Bd + Bd * Bd - Ad * Bd;
  double Z = 1.0 + Bd;
  for (int it = 0; it < 100; ++it) {
    double f = ((Z + c2) * Z + c1) * Z + c0;
    double fp = (3.0 * Z + 2.0 * c2) * Z + c1;
    double dZ = f / fp;
    Z -= dZ;
    if (fabs(dZ) <= 1e-15 * fabs(Z)) break;
  }
  return Z * R_U * T / p;
}

/* mass-specific volume and energy of component k at (p, T) together with the
 * partial derivatives used by the Newton solves. */
typedef struct { double v, e, dv_dp, dv_dT, de_dp, de_dT; } og_state_pt;

static int comp_state(const og_eos* e, int k, double p, double T, og_state_pt* s)
{
  if (e->kind[k] == OG_EOS_SG) {
    double den = p + e->pinf[k];
    double v = (e->gamma[k] - 1.0) * e->cv[k] * T / den;
    s->v = v;
    s->e = e->cv[k] * T + e->pinf[k] * v + e->q[k];
    s->dv_dp = -v / den;
    s->dv_dT = v / T;
    s->de_dp = e->pinf[k] * s->dv_dp;
    s->de_dT = e->cv[k] + e->pinf[k] * s->dv_dT;
    return 0;
  }
  double a, a1, a2, b, M;
  if (og_pr_coeffs(e, k, T, &a, &a1, &a2, &b, &M)) return -1;
  double V = pr_molar_volume(p, T, a, b);
  double D = V * V + 2.0 * b * V - b * b;
  double dpdV = -R_U * T / ((V - b) * (V - b)) + a * (2.0 * V + 2.0 * b) / (D * D);
  double dpdT = R_U / (V - b) - a1 / D;
  double L = pr_logterm(V, b);
  double cvm = M * e->cv[k] - T * a2 / (2.0 * SQRT2 * b) * L;   /* molar cv */
  double dedV = T * dpdT - (R_U * T / (V - b) - a / D);          /* (de/dV)_T molar */
  double dVdp = 1.0 / dpdV;
  double dVdT = -dpdT / dpdV;
  s->v = V / M;
  s->e = e->cv[k] * T + e->q[k] + (a - T * a1) / (2.0 * SQRT2 * b * M) * L;
  s->dv_dp = dVdp / M;
  s->dv_dT = dVdT / M;
  s->de_dp = dedV * dVdp / M;
  s->de_dT = (cvm + dedV * dVdT) / M;
  return 0;
}

double og_spec_volume(const og_eos* e, int k, double p, double T)
{
  og_state_pt s;
  if (comp_state(e, k, p, T, &s)) return NAN;
  return s.v;
}

double og_spec_energy(const og_eos* e, int k, double p, double T)
{
  og_state_pt s;
  if (comp_state(e, k, p, T, &s)) return NAN;
  return s.e;
}

/* speed of sound of component k alone at (p, T) */
double og_sound(const og_eos* e, int k, double p, double T)
{
  if (e->kind[k] == OG_EOS_SG) return sqrt(e->gamma[k] * (e->gamma[k] - 1.0) * e->cv[k] * T);
  double a, a1, a2, b, M;
  if (og_pr_coeffs(e, k, T, &a, &a1, &a2, &b, &M)) return NAN;
  double V = pr_molar_volume(p, T, a, b);
  double D = V * V + 2.0 * b * V - b * b;
  double dpdV = -R_U * T / ((V - b) * (V - b)) + a * (2.0 * V + 2.0 * b) / (D * D);
  double dpdT = R_U / (V - b) - a1 / D;
  double cvm = M * e->cv[k] - T * a2 / (2.0 * SQRT2 * b) * pr_logterm(V, b);
  double c2 = -(V * V / M) * (dpdV - T * dpdT * dpdT / cvm);
  return sqrt(c2);
}

double og_clip_fraction(double Y)
{
  return Y < 0.0 ? 0.0 : (Y > 1.0 ? 1.0 : Y);   /* NaN passes through */
}

/* Impedances and the CFL condition use one speed of sound per cell: the largest
 * of the components' speeds at the cell's (p, T); with a liquid present that is
 * the liquid's (Appendix D asks for the maximum liquid speed of sound).  A
 * stiffened gas enters whether present or not (its c depends on T alone); a
 * Peng-Robinson component enters only where present, since at p < 0 (a pure
 * liquid in tension) its cubic need not have a root with V > b. */
double og_mix_sound(const og_eos* e, double p, double T, double Y)
{
  double Yc = og_clip_fraction(Y);
  double Yk[2] = {1.0 - Yc, Yc}, c = 0.0;
  for (int k = 0; k < 2; ++k) {
    if (e->kind[k] == OG_EOS_PR && Yk[k] == 0.0) continue;
    double ck = og_sound(e, k, p, T);
    if (!(ck <= c)) c = ck;     /* NaN propagates */
  }
  return c;
}

/* forward closure: (p, T, xi) -> (rho, e), Table A.1:
 * 1/rho = sum_k xi_k v_k(p,T), e = sum_k xi_k e_k(p,T) */
int og_eos_forward(const og_eos* e, double p, double T, double Y, double* rho, double* ein)
{
  double Yk[2] = {1.0 - Y, Y};
  double v = 0.0, en = 0.0;
  for (int k = 0; k < 2; ++k) {
    if (Yk[k] == 0.0) continue;
    og_state_pt s;
    if (comp_state(e, k, p, T, &s)) return -1;
    v += Yk[k] * s.v;
    en += Yk[k] * s.e;
  }
  *rho = 1.0 / v;
  *ein = en;
  return 0;
}

/* (p, e, xi) -> (rho, T), two stiffened-gas components (Appendix B's face
 * closure rho* = f(p*, xi*, e*)).  At fixed p each component's volume
 * v_k = (g_k - 1) cv_k T / (p + pinf_k) (A.1.2) and energy
 * e_k = cv_k T + pinf_k v_k + q_k (A.1.1, A.1.3) are linear in T, so the
 * mixture energy sum_k xi_k e_k = e fixes T directly. */
int og_eos_forward_e(const og_eos* e, double p, double ein, double Y, double* rho, double* T)
{
  if (og_ncomp(e) != 2 || e->kind[0] != OG_EOS_SG || e->kind[1] != OG_EOS_SG) return -1;
  double Yk[2] = {1.0 - Y, Y};
  double slope = 0.0, offset = 0.0;
  for (int k = 0; k < 2; ++k) {
    if (Yk[k] == 0.0) continue;
    double vT = (e->gamma[k] - 1.0) * e->cv[k] / (p + e->pinf[k]);   /* v_k / T */
    slope += Yk[k] * (e->cv[k] + e->pinf[k] * vT);
    offset += Yk[k] * e->q[k];
  }
  double t = (ein - offset) / slope;
  if (!(t > 0.0)) return -1;
  double v = 0.0;
  for (int k = 0; k < 2; ++k)
    if (Yk[k] != 0.0) v += Yk[k] * (e->gamma[k] - 1.0) * e->cv[k] * t / (p + e->pinf[k]);
  *rho = 1.0 / v;
  *T = t;
  return 0;
}

/* inverse of one stiffened-gas component alone (A.1.1 solved for p) */
static void sg_pure(const og_eos* e, int k, double rho, double ein, double* p, double* T)
{
  double v = 1.0 / rho;
  *p = (e->gamma[k] - 1.0) * rho * (ein - e->q[k]) - e->gamma[k] * e->pinf[k];
  *T = (ein - e->q[k] - e->pinf[k] * v) / e->cv[k];
}

/* The quadratic below for groups 0 and 1 of stiffened-gas terms sharing
 * p_inf = P0 and P1 (derivation in the next comment); its larger root. */
static void sg_quadratic(double v, double A0, double A1, double Cv, double Cp, double eh, double P0,
                         double P1, double* p, double* T)
{
  double qa = v * Cv;
  double qb = v * (Cp * (P0 + P1) - A0 * P1 - A1 * P0) - eh * (A0 + A1);
  double qc = v * Cp * P0 * P1 - eh * (A0 * P1 + A1 * P0);
  double disc = qb * qb - 4.0 * qa * qc;
  double sq = sqrt(disc);
  double pp = (qb < 0.0) ? (-qb + sq) / (2.0 * qa) : 2.0 * qc / (-qb - sq);
  *p = pp;
  *T = (eh + pp * v) / Cp;
}

/* Two stiffened-gas components in p-T equilibrium.  With A_k = xi_k (g_k-1) cv_k,
 * Cv = sum xi_k cv_k, Cp = sum xi_k g_k cv_k and eh = e - sum xi_k q_k the two
 * equilibrium conditions reduce to T = (eh + p v) / Cp and the quadratic
 *   (v Cv) p^2 + [v (Cp (P0+P1) - A0 P1 - A1 P0) - eh (A0+A1)] p
 *     + [v Cp P0 P1 - eh (A0 P1 + A1 P0)] = 0,
 * whose larger root is the physical one.  gam/pinf/cv/q are passed so that the
 * same routine serves as the ideal-gas starting guess of the Peng-Robinson solve. */
static void sg_pair(const double gam[2], const double pinf[2], const double cv[2], const double q[2],
                    double rho, double ein, double Y, double* p, double* T)
{
  double Yk[2] = {1.0 - Y, Y};
  double v = 1.0 / rho;
  double A0 = Yk[0] * (gam[0] - 1.0) * cv[0], A1 = Yk[1] * (gam[1] - 1.0) * cv[1];
  double Cv = Yk[0] * cv[0] + Yk[1] * cv[1];
  double Cp = Yk[0] * gam[0] * cv[0] + Yk[1] * gam[1] * cv[1];
  double eh = ein - Yk[0] * q[0] - Yk[1] * q[1];
  sg_quadratic(v, A0, A1, Cv, Cp, eh, pinf[0], pinf[1], p, T);
}

/* Three stiffened-gas components whose gases (1 and 2) are ideal: the two gas
 * terms of sum_k xi_k (g_k-1) cv_k T / (p + P_k) = v share P = 0 and add up,
 * so the same quadratic holds with A0 = xi_0 (g_0-1) cv_0,
 * A1 = sum_{k=1,2} xi_k (g_k-1) cv_k and the sums Cv, Cp, eh over all three
 * (eqs. A.1.2-A.1.3 of Table A.1 in p-T equilibrium). */
static void sg_three(const og_eos* e, const double Yk[3], double rho, double ein, double* p, double* T)
{
  double v = 1.0 / rho;
  double A0 = Yk[0] * (e->gamma[0] - 1.0) * e->cv[0];
  double A1 = Yk[1] * (e->gamma[1] - 1.0) * e->cv[1] + Yk[2] * (e->gamma[2] - 1.0) * e->cv[2];
  double Cv = Yk[0] * e->cv[0] + Yk[1] * e->cv[1] + Yk[2] * e->cv[2];
  double Cp = Yk[0] * e->gamma[0] * e->cv[0] + Yk[1] * e->gamma[1] * e->cv[1] + Yk[2] * e->gamma[2] * e->cv[2];
  double eh = ein - Yk[0] * e->q[0] - Yk[1] * e->q[1] - Yk[2] * e->q[2];
  sg_quadratic(v, A0, A1, Cv, Cp, eh, e->pinf[0], 0.0, p, T);
}

/* Peng-Robinson component alone: T from e at fixed v by Newton (the paper's
 * Appendix B), then p from (A.2.1). */
static int pr_pure(const og_eos* e, int k, double rho, double ein, double Tg, double* p, double* T)
{
  double vm = 1.0 / rho;
  double Tn = (Tg > 0.0) ? Tg : (ein - e->q[k]) / e->cv[k];
  if (!(Tn > 0.0)) Tn = 100.0;
  int ok = 0;
  for (int it = 0; it < 100; ++it) {
    double a, a1, a2, b, M;
    if (og_pr_coeffs(e, k, Tn, &a, &a1, &a2, &b, &M)) return -1;
    double V = M * vm;
    double L = pr_logterm(V, b);
    double f = e->cv[k] * Tn + e->q[k] + (a - Tn * a1) / (2.0 * SQRT2 * b * M) * L - ein;
    double fp = e->cv[k] - Tn * a2 / (2.0 * SQRT2 * b * M) * L;
    double dT = f / fp;
    double Tnew = Tn - dT;
    if (Tnew <= 0.0) Tnew = 0.5 * Tn;
    Tn = Tnew;
    if (fabs(dT) <= 1e-13 * Tn) { ok = 1; break; }
  }
  *T = Tn;
  *p = og_pr_pressure(e, k, Tn, vm);
  return ok ? 0 : -2;
}

/* Mixed cell with a Peng-Robinson component: Newton on the two equilibrium
 * conditions sum xi_k v_k(p,T) = 1/rho and sum xi_k e_k(p,T) = e.  Start: the
 * same cell with every Peng-Robinson component replaced by the ideal gas of
 * equal molar mass and cv (closed form above). */
static int pr_mixed(const og_eos* e, double rho, double ein, double Y, double* p, double* T)
{
  double Yk[2] = {1.0 - Y, Y};
  double gam[2], pinf[2], cv[2], q[2];
  for (int k = 0; k < 2; ++k) {
    cv[k] = e->cv[k];
    q[k] = e->q[k];
    if (e->kind[k] == OG_EOS_SG) { gam[k] = e->gamma[k]; pinf[k] = e->pinf[k]; }
    else {
      double M = 0.0;
      for (int al = 0; al < e->pr_ns[k]; ++al) M += e->pr_X[k][al] * e->pr_M[k][al];
      gam[k] = 1.0 + R_U / (M * e->cv[k]);
      pinf[k] = 0.0;
    }
  }
  double pp, TT;
  sg_pair(gam, pinf, cv, q, rho, ein, Y, &pp, &TT);
  double v = 1.0 / rho;
  /* pressure is resolved to rounding relative to p + p_inf of a stiff component */
  double pscale = 1.0;
  for (int k = 0; k < 2; ++k)
    if (e->kind[k] == OG_EOS_SG && e->pinf[k] > pscale) pscale = e->pinf[k];
  int ok = 0;
  for (int it = 0; it < 100; ++it) {
    double F1 = -v, F2 = -ein, J11 = 0, J12 = 0, J21 = 0, J22 = 0;
    for (int k = 0; k < 2; ++k) {
      if (Yk[k] == 0.0) continue;
      og_state_pt s;
      if (comp_state(e, k, pp, TT, &s)) return -1;
      F1 += Yk[k] * s.v;  F2 += Yk[k] * s.e;
      J11 += Yk[k] * s.dv_dp;  J12 += Yk[k] * s.dv_dT;
      J21 += Yk[k] * s.de_dp;  J22 += Yk[k] * s.de_dT;
    }
    double det = J11 * J22 - J12 * J21;
    double dp = (F1 * J22 - F2 * J12) / det;
    double dT = (J11 * F2 - J21 * F1) / det;
    double pn = pp - dp, Tn = TT - dT;
    if (Tn <= 0.0) Tn = 0.5 * TT;
    pp = pn; TT = Tn;
    if (fabs(dT) <= 1e-12 * TT && fabs(dp) <= 1e-12 * (fabs(pp) + pscale)) { ok = 1; break; }
  }
  *p = pp; *T = TT;
  return ok ? 0 : -2;
}

/* inverse closure: (rho, e, xi) -> (p, T) in p-T equilibrium */
int og_eos_inverse(const og_eos* e, double rho, double ein, double Y, double Tguess,
                   double* p, double* T)
{
  if (!(rho > 0.0)) return -1;
  /* a mass fraction a little outside [0, 1] (central reconstruction is not
   * bounded) is taken at the nearer pure component; the conserved rho xi keeps
   * its value, so conservation is untouched */
  Y = og_clip_fraction(Y);
  if (Y == 0.0 || Y == 1.0) {
    int k = (Y == 0.0) ? 0 : 1;
    if (e->kind[k] == OG_EOS_SG) { sg_pure(e, k, rho, ein, p, T); return 0; }
    return pr_pure(e, k, rho, ein, Tguess, p, T);
  }
  if (e->kind[0] == OG_EOS_SG && e->kind[1] == OG_EOS_SG) {
    sg_pair(e->gamma, e->pinf, e->cv, e->q, rho, ein, Y, p, T);
    return 0;
  }
  return pr_mixed(e, rho, ein, Y, p, T);
}

int og_ncomp(const og_eos* e)
{
  return e->ncomp == 3 ? 3 : 2;
}

/* three components: every component a stiffened gas, the gases ideal */
static int three_ok(const og_eos* e)
{
  for (int k = 0; k < 3; ++k)
    if (e->kind[k] != OG_EOS_SG) return 0;
  return e->pinf[1] == 0.0 && e->pinf[2] == 0.0;
}

int og_eos_forward2(const og_eos* e, double p, double T, double Y1, double Y2, double* rho, double* ein)
{
  if (og_ncomp(e) == 2) return og_eos_forward(e, p, T, Y1, rho, ein);
  if (!three_ok(e)) return -1;
  double Yk[3] = {1.0 - Y1 - Y2, Y1, Y2};
  double v = 0.0, en = 0.0;
  for (int k = 0; k < 3; ++k) {
    if (Yk[k] == 0.0) continue;
    og_state_pt s;
    if (comp_state(e, k, p, T, &s)) return -1;
    v += Yk[k] * s.v;
    en += Yk[k] * s.e;
  }
  *rho = 1.0 / v;
  *ein = en;
  return 0;
}

/* gas mass fractions of a cell as the closure takes them: each clipped into
 * [0, 1] (as with two components) and, if they then sum above 1, scaled to
 * sum to 1; the liquid gets the rest */
void og_clip_fractions3(double Y1, double Y2, double Yk[3])
{
  double a = og_clip_fraction(Y1), b = og_clip_fraction(Y2);
  double s = a + b;
  if (s > 1.0) { a /= s; b /= s; }
  double l = 1.0 - a - b;
  Yk[0] = l > 0.0 ? l : 0.0;
  Yk[1] = a;
  Yk[2] = b;
}

int og_eos_inverse2(const og_eos* e, double rho, double ein, double Y1, double Y2, double Tguess,
                    double* p, double* T)
{
  if (og_ncomp(e) == 2) return og_eos_inverse(e, rho, ein, Y1, Tguess, p, T);
  if (!three_ok(e) || !(rho > 0.0)) return -1;
  double Yk[3];
  og_clip_fractions3(Y1, Y2, Yk);
  int present = 0, only = 0;
  for (int k = 0; k < 3; ++k)
    if (Yk[k] > 0.0) { ++present; only = k; }
  if (present == 1) { sg_pure(e, only, rho, ein, p, T); return 0; }
  sg_three(e, Yk, rho, ein, p, T);
  return 0;
}

double og_mix_sound2(const og_eos* e, double p, double T, double Y1, double Y2)
{
  if (og_ncomp(e) == 2) return og_mix_sound(e, p, T, Y1);
  (void)Y2;
  double c = 0.0;
  for (int k = 0; k < 3; ++k) {   /* stiffened gases: c_k depends on T alone */
    double ck = og_sound(e, k, p, T);
    if (!(ck <= c)) c = ck;
  }
  return c;
}
