// fvm_device.hpp -- device-side data and point functions of the gfx950 solver.
//
// Thermodynamic closure (Appendix A: stiffened gas eq. A.1.1, Peng-Robinson
// eq. A.2.1, pressure-temperature equilibrium of the two components),
// reconstruction (Section 3.3, Table 4.2, Appendix D), All-Mach Riemann solver
// (Section 3.2, eq. D.5/D.6), thermodynamic dependent update (eq. 3-5,
// Appendix B) and the face flux of eq. (2-2).
//
// Storage ("internal") variables of a cell, N_q = D + 3 (D + 4 with a second
// gas species):
//   0: rho_L - rref_L   partial density of component 0 minus a reference
//   1: rho_G - rref_G   partial density of component 1 minus a reference
//   2..1+D: rho u
//   2+D: E' = rho E - sum_k rho_k Q_k   (energy in a shifted gauge)
//   3+D: rho_G2 - rref_G2 (second gas species only)
// The shifts are linear in the conserved variables, so fluxes telescope and
// conservation is unchanged; they keep FP32 storage accurate in stiff liquids
// (near the reference state the stored numbers are small).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fvm {

constexpr int MAXSPEC = 4;
constexpr int MAXPAIR = MAXSPEC * (MAXSPEC + 1) / 2;
constexpr double R_UNIV = 8.314462618;
constexpr double SQRT2 = 1.41421356237309505;

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_ZEROGRAD = 2, BC_INFLOW = 3, BC_FARFIELD = 4 };
enum { LIM_MINMOD = 0, LIM_KOREN = 1, LIM_VANALBADA = 2, LIM_VANLEER = 3,
       LIM_CHAKRAVARTHY = 4, LIM_MC = 5, LIM_SUPERBEE = 6, LIM_NONE = 7 };
enum { ERR_NONPHYS = -4, ERR_NAN = -5 };

// one component of the closure
struct Comp {
  int kind;            // 0 stiffened gas, 1 Peng-Robinson
  double gamma, pinf, cv;
  double qs;           // energy constant in the storage gauge: q - Q
  double A;            // (gamma - 1) cv
  double Cp;           // gamma cv
  double c2T;          // gamma (gamma - 1) cv : c^2 / T
  // Peng-Robinson pseudo-mixture: a(T) = sum_pairs w a0 (1 + cc (1 - sqrt(T) rs))^2
  int npair;
  double pw[MAXPAIR], pa0[MAXPAIR], pcc[MAXPAIR], prs[MAXPAIR];
  double b, M;         // covolume [m^3/mol], molar mass [kg/mol]
  // a(T) summed over the pairs is a quadratic in s = sqrt(T):
  //   a = pa_0 - pa_1 s + pa_2 s^2,  a - T a' = pa_0 - pa_1 s / 2,  T^2 a'' = pa_1 s / 4
  double pa_0, pa_1, pa_2;
  double iM;           // 1 / M
  double ikb;          // 1 / (2 sqrt(2) b M): energy departure per unit (a - T a') log(...)
  double gam_ig;       // 1 + R / (M cv): ideal-gas stand-in used as Newton start
  double mu, kc;       // dynamic viscosity [Pa s], thermal conductivity [W/(m K)]
};

struct CaseC {
  int dim, n[3];
  long long off, ncell;
  double dx[3], idx[3];
  int bc[3][2];
  double in_p, in_T, in_alpha, in_u, in_radius, in_c0, in_c1, in_noise;
  unsigned long long in_seed;
  double ff_p, ff_T, ff_alpha;   // far-field reservoir state (at rest)
  int any_ff;                    // some side is a far-field reservoir
  Comp comp[3];        // component 2: second gas (three-component closure only)
  int ncomp;           // 2 or 3
  double rref[3];      // partial-density shifts (FP32-exact for FP32 storage)
  double Q[3];         // energy gauge: E' = rho E - sum_k rho_k Q_k
  int tile0, tiles[3];
  int xslab;           // 3D tile table: tiles per x slab (the table runs slab by slab, x fastest in each)
  int diff;            // some component is viscous or conducting
  double sdx2;         // sum_d 1 / dx_d^2 over the used directions
  // barotropic model (Section 2.2; model = 1): saturated liquid density and
  // pressure, c_L^2, c_M^2 = p_sat / rho_sat, saturated vapour density, R T of
  // the gas, and the sound speed of impedances and CFL at p >= p_sat / below
  int model;
  double bt_rs, bt_ps, bt_cl2, bt_cm2, bt_rv, bt_RT, bt_c_hi, bt_c_lo;
  double bt_mu_l, bt_mu_g, bt_mu_v;   // barotropic model: liquid, gas, vapour viscosity (eq. 2-8)
  double bt_RT2, bt_mu_g2;            // barotropic model, second gas: R T and viscosity
};

// per-case scalars that live on the device across steps; slot s = step & 1
// holds the values of q^n, slot s ^ 1 those of q^(n+1)
constexpr int NSLOT = 32;   // CFL partial maxima are spread over slots to avoid one contended atomic

struct CaseDyn {
  // bits of max_cells sum (|u| + c)/dx, spread over NSLOT slots (workgroup b
  // writes slot b % NSLOT; non-negative doubles order as their integer bits)
  unsigned long long dtmax[2][NSLOT];
  double t[2];                   // time at the start of the step
  double dt_last;                // dt of the last step taken
  long long base;                // steps completed before the current launch chunk
  int err, pad;
  long long err_cell, err_step;
};

struct SchemeC {
  int switching, lim_u, lim_s, thinc;
  double beta, thinc_gamma, eps_int, th_d, th_g, eps_d, k3, sigma, eps_n, cfl;
  double tanh_b, icosh_b, itanh_b;
  double t_end;
  double grav[3];      // body-force acceleration
  int has_grav;
  int recon_e;         // 1: the face reconstructs e (not T); rho_f from (p*, xi_f, e_f)
};

// ------------------------------------------------------------------ math
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// reciprocal: hardware estimate refined by two Newton steps (relative error near
// one ulp; not correctly rounded)
__device__ inline double frcp(double x)
{
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ inline double fdiv(double a, double b) { return a * frcp(b); }
__device__ inline float fexp(float x) { return __expf(x); }
__device__ inline double fexp(double x) { return exp(x); }

// SplitMix64 (Steele, Lea, Flood 2014): Weyl increment then two xor-shift-multiply rounds
__device__ inline unsigned long long splitmix64(unsigned long long x)
{
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline double noise01(unsigned long long seed, unsigned long long step,
                                 unsigned long long j, unsigned long long k, unsigned long long c)
{
  unsigned long long h = splitmix64(seed);
  h = splitmix64(h ^ step);
  h = splitmix64(h ^ j);
  h = splitmix64(h ^ k);
  h = splitmix64(h ^ c);
  return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

// ------------------------------------------------------------------ Peng-Robinson (A.2.1)
struct PRab { double a, a1, a2; };

// a(T), a'(T), a''(T) of the pair sum  sum_q w_q a0_q (1 + c_q (1 - sqrt(T / Tc_q)))^2
// written as the quadratic in s = sqrt(T) it is (coefficients pa_* from the host)
__device__ inline PRab pr_a(const Comp& c, double T)
{
  double s = sqrt(T), is = frcp(s);
  PRab r;
  r.a = fma(c.pa_2, T, c.pa_0 - c.pa_1 * s);
  r.a1 = c.pa_2 - 0.5 * c.pa_1 * is;
  r.a2 = 0.25 * c.pa_1 * is * is * is;
  return r;
}

__device__ inline double pr_log(double V, double b)
{
  return log((V + (1.0 - SQRT2) * b) * frcp(V + (1.0 + SQRT2) * b));
}

// molar volume at (p, T): the largest root of the compressibility cubic
//   Z^3 + (B - 1) Z^2 + (A - 3 B^2 - 2 B) Z + (B^3 + B^2 - A B) = 0
// by Newton.  From Z = 1 + B (an upper bound of every root with V > b) the
// iterates fall monotonically onto it.  A start Z0 > B (e.g. the upwind cell's
// own compressibility) is tried first; its limit is kept only if it lies right
// of the inflection point with a positive slope, which makes it the largest
// root.  Newton stops once a correction falls below 1e-9 Z: the error left is
// then of order Z 1e-18.
__device__ inline double pr_cubic_newton(double Z, double c2, double c1, double c0, int& ok, double tol = 1e-9)
{
  ok = 0;
  for (int it = 0; it < 60; ++it) {
    double f = ((Z + c2) * Z + c1) * Z + c0;
    double fp = (3.0 * Z + 2.0 * c2) * Z + c1;
    double dZ = f * frcp(fp);
    Z -= dZ;
    if (fabs(dZ) <= tol * fabs(Z)) { ok = 1; break; }
  }
  return Z;
}

// tol: the relative correction at which Newton stops (1e-9: the error left is
// of order 1e-18; 1e-6, for face states rounded to FP32: of order 1e-12)
__device__ inline double pr_volume(double p, double T, double a, double b, double Z0 = 0.0, double tol = 1e-9)
{
  double RT = R_UNIV * T, iRT = frcp(RT);
  double Bd = b * p * iRT, Ad = a * p * iRT * iRT;
  double c2 = Bd - 1.0, c1 = Ad - 3.0 * Bd * Bd - 2.0 * Bd, c0 = Bd * Bd * Bd + Bd * Bd - Ad * Bd;
  int ok = 0;
  double Z = 0.0;
  if (Z0 > Bd && Z0 < 1e300) {
    Z = pr_cubic_newton(Z0, c2, c1, c0, ok, tol);
    ok = ok && Z > -c2 * (1.0 / 3.0) && (3.0 * Z + 2.0 * c2) * Z + c1 > 0.0;
  }
  if (!ok) Z = pr_cubic_newton(1.0 + Bd, c2, c1, c0, ok, tol);
  return Z * RT * frcp(p);
}

// mass-specific volume / energy of a component at (p, T) with derivatives
struct VE { double v, e, dvdp, dvdT, dedp, dedT; };

__device__ inline VE comp_ve(const Comp& c, double p, double T)
{
  VE r;
  if (c.kind == 0) {
    double den = frcp(p + c.pinf);
    double v = c.A * T * den;
    r.v = v;
    r.e = c.cv * T + c.pinf * v + c.qs;
    r.dvdp = -v * den;
    r.dvdT = c.A * den;
    r.dedp = c.pinf * r.dvdp;
    r.dedT = c.cv + c.pinf * r.dvdT;
    return r;
  }
  PRab A = pr_a(c, T);
  double b = c.b, M = c.M;
  double V = pr_volume(p, T, A.a, b);
  double D = V * V + 2.0 * b * V - b * b;
  double iD = frcp(D), iVb = frcp(V - b);
  double dpdV = -R_UNIV * T * iVb * iVb + A.a * (2.0 * V + 2.0 * b) * iD * iD;
  double dpdT = R_UNIV * iVb - A.a1 * iD;
  double L = pr_log(V, b);
  double cvm = M * c.cv - T * A.a2 * c.ikb * M * L;
  double dedV = T * dpdT - (R_UNIV * T * iVb - A.a * iD);
  double dVdp = frcp(dpdV), dVdT = -dpdT * dVdp;
  double iM = c.iM;
  r.v = V * iM;
  r.e = c.cv * T + c.qs + (A.a - T * A.a1) * c.ikb * L;
  r.dvdp = dVdp * iM;
  r.dvdT = dVdT * iM;
  r.dedp = dedV * dVdp * iM;
  r.dedT = (cvm + dedV * dVdT) * iM;
  return r;
}

// speed of sound of a Peng-Robinson component at molar volume V and T, with
// its a(T) terms A and L = log((V + (1 - sqrt 2) b) / (V + (1 + sqrt 2) b))
__device__ inline double pr_sound_VL(const Comp& c, double V, double T, const PRab& A, double L)
{
  double b = c.b, M = c.M;
  double D = V * V + 2.0 * b * V - b * b;
  double iD = frcp(D), iVb = frcp(V - b);
  double dpdV = -R_UNIV * T * iVb * iVb + A.a * (2.0 * V + 2.0 * b) * iD * iD;
  double dpdT = R_UNIV * iVb - A.a1 * iD;
  double cvm = M * c.cv - T * A.a2 * c.ikb * M * L;
  return sqrt(-(V * V * c.iM) * (dpdV - T * dpdT * dpdT * frcp(cvm)));
}

// ------------------------------------------------------------------ closure inversion
struct PT { double p, T, c, alpha, alpha2; int ok; };   // alpha2: second gas (0 with two components)

// the larger root of the quadratic below for groups 0 and 1 of stiffened-gas
// terms (A_k = sum of xi (g-1) cv over the group, sharing p_inf = P_k)
__device__ inline void sg_quad(double v, double A0, double A1, double Cv, double Cp, double eh, double P0,
                               double P1, double& p, double& T)
{
  double qa = v * Cv;
  double qb = v * (Cp * (P0 + P1) - A0 * P1 - A1 * P0) - eh * (A0 + A1);
  double qc = v * Cp * P0 * P1 - eh * (A0 * P1 + A1 * P0);
  double sq = sqrt(qb * qb - 4.0 * qa * qc);
  p = (qb < 0.0) ? (-qb + sq) * frcp(2.0 * qa) : 2.0 * qc * frcp(-qb - sq);
  T = (eh + p * v) * frcp(Cp);
}

// stiffened-gas pair in p-T equilibrium: T = (eh + p v) / Cp and the larger
// root of  (v Cv) p^2 + [v (Cp (P0+P1) - A0 P1 - A1 P0) - eh (A0+A1)] p
//          + [v Cp P0 P1 - eh (A0 P1 + A1 P0)] = 0
__device__ inline void sg_pair(double g0, double P0, double cv0, double q0,
                               double g1, double P1, double cv1, double q1,
                               double v, double e, double Y, double& p, double& T)
{
  double Y0 = 1.0 - Y;
  double A0 = Y0 * (g0 - 1.0) * cv0, A1 = Y * (g1 - 1.0) * cv1;
  double Cv = Y0 * cv0 + Y * cv1;
  double Cp = Y0 * g0 * cv0 + Y * g1 * cv1;
  double eh = e - Y0 * q0 - Y * q1;
  sg_quad(v, A0, A1, Cv, Cp, eh, P0, P1, p, T);
}

// gas fractions of a three-component cell as the closure takes them: each
// clipped into [0, 1], rescaled if they sum above one; the liquid the rest
__device__ inline void clip_fractions3(double Y1, double Y2, double& y0, double& y1, double& y2)
{
  double a = (Y1 < 0.0) ? 0.0 : ((Y1 > 1.0) ? 1.0 : Y1);
  double b = (Y2 < 0.0) ? 0.0 : ((Y2 > 1.0) ? 1.0 : Y2);
  double s = a + b;
  if (s > 1.0) { double is = 1.0 / s; a *= is; b *= is; }
  double l = 1.0 - a - b;
  y0 = l > 0.0 ? l : 0.0;
  y1 = a;
  y2 = b;
}

// Three stiffened-gas components whose gases (1, 2) are ideal (Table A.1,
// eqs. A.1.2-A.1.5): the gas terms share p_inf = 0 and add up, so the
// two-group quadratic holds; c is the largest of the three sound speeds.
__device__ inline PT closure3(const CaseC& C, double rho, double Y1, double Y2, double e)
{
  const Comp& c0 = C.comp[0];
  const Comp& c1 = C.comp[1];
  const Comp& c2 = C.comp[2];
  PT r;
  r.ok = 1;
  double y0, y1, y2;
  clip_fractions3(Y1, Y2, y0, y1, y2);
  double v = frcp(rho);
  double p, T;
  int present = (y0 > 0.0) + (y1 > 0.0) + (y2 > 0.0);
  if (present == 1) {
    const Comp& c = (y0 > 0.0) ? c0 : ((y1 > 0.0) ? c1 : c2);
    p = (c.gamma - 1.0) * rho * (e - c.qs) - c.gamma * c.pinf;
    T = (e - c.qs - c.pinf * v) / c.cv;
  } else {
    double A0 = y0 * (c0.gamma - 1.0) * c0.cv;
    double A1 = y1 * (c1.gamma - 1.0) * c1.cv + y2 * (c2.gamma - 1.0) * c2.cv;
    double Cv = y0 * c0.cv + y1 * c1.cv + y2 * c2.cv;
    double Cp = y0 * c0.gamma * c0.cv + y1 * c1.gamma * c1.cv + y2 * c2.gamma * c2.cv;
    double eh = e - y0 * c0.qs - y1 * c1.qs - y2 * c2.qs;
    sg_quad(v, A0, A1, Cv, Cp, eh, c0.pinf, 0.0, p, T);
  }
  r.p = p;
  r.T = T;
  r.c = sqrt(fmax(fmax(c0.c2T * T, c1.c2T * T), c2.c2T * T));
  r.alpha = (y1 == 0.0) ? 0.0 : y1 * rho * c1.A * T * frcp(p);
  r.alpha2 = (y2 == 0.0) ? 0.0 : y2 * rho * c2.A * T * frcp(p);
  return r;
}

// (rho, xi, e) -> (p, T), c = max of the components' sound speeds, alpha_G.
// e is the specific internal energy in the storage gauge.  PRK: component 1
// may be a Peng-Robinson fluid; its Newton iterations start from (pw, Tw)
// when given (Tw > 0: the cell's state of the previous stage, Appendix B) and
// from the ideal-gas stand-in otherwise or if that start does not converge.
template <bool PRK>
__device__ inline PT closure(const CaseC& C, double rho, double Y, double e, double Tw = 0.0, double pw = 0.0)
{
  const Comp& c0 = C.comp[0];
  const Comp& c1 = C.comp[1];
  PT r;
  r.ok = 1;
  r.alpha2 = 0.0;
  // a mass fraction a little outside [0, 1] (the central reconstruction is not
  // bounded) is closed as the nearer pure component; NaN passes through
  Y = (Y < 0.0) ? 0.0 : ((Y > 1.0) ? 1.0 : Y);
  double v = frcp(rho);
  double p, T;
  if (!PRK || c1.kind == 0) {
    if (Y == 0.0) {
      p = (c0.gamma - 1.0) * rho * (e - c0.qs) - c0.gamma * c0.pinf;
      T = (e - c0.qs - c0.pinf * v) / c0.cv;
    } else if (Y == 1.0) {
      p = (c1.gamma - 1.0) * rho * (e - c1.qs) - c1.gamma * c1.pinf;
      T = (e - c1.qs - c1.pinf * v) / c1.cv;
    } else {
      sg_pair(c0.gamma, c0.pinf, c0.cv, c0.qs, c1.gamma, c1.pinf, c1.cv, c1.qs, v, e, Y, p, T);
    }
    r.p = p;
    r.T = T;
    double cc0 = c0.c2T * T, cc1 = c1.c2T * T;
    r.c = sqrt(fmax(cc0, cc1));
    r.alpha = (Y == 0.0) ? 0.0 : Y * rho * c1.A * T * frcp(p + c1.pinf);
    return r;
  }
  if constexpr (PRK) {
    if (Y == 0.0) {
      p = (c0.gamma - 1.0) * rho * (e - c0.qs) - c0.gamma * c0.pinf;
      T = (e - c0.qs - c0.pinf * v) / c0.cv;
      // the absent Peng-Robinson gas does not enter c: at p < 0 (liquid in
      // tension) its cubic need not have a root with V > b
      r.p = p;
      r.T = T;
      r.c = sqrt(c0.c2T * T);
      r.alpha = 0.0;
      return r;
    }
    if (Y == 1.0) {
      // pure Peng-Robinson at this cell's fixed V: e(T) = cv T + q + (a - T a') k
      // with a - T a' = pa_0 - pa_1 sqrt(T) / 2 is a quadratic in s = sqrt(T),
      //   cv s^2 - beta s - gam = 0,  beta = pa_1 k / 2,  gam = e - q - pa_0 k,
      // whose positive root is taken in the form without cancellation (Appendix
      // B solves the same equation by Newton; this is its exact solution); p
      // then follows from (A.2.1)
      double V = c1.M * v;
      double L = pr_log(V, c1.b);
      double k = L * c1.ikb;
      double beta = 0.5 * c1.pa_1 * k, gam = e - c1.qs - c1.pa_0 * k;
      double D = fma(beta, beta, 4.0 * c1.cv * gam);
      double sD = sqrt(fmax(D, 0.0));
      double sT = beta >= 0.0 ? 0.5 * (beta + sD) * frcp(c1.cv) : 2.0 * gam * frcp(sD - beta);
      double Tn = sT * sT;
      int conv = gam > 0.0 && D >= 0.0 && sT > 0.0;
      PRab A = pr_a(c1, Tn);
      r.T = Tn;
      r.p = R_UNIV * Tn * frcp(V - c1.b) - A.a * frcp(V * V + 2.0 * c1.b * V - c1.b * c1.b);
      r.c = fmax(sqrt(c0.c2T * Tn), pr_sound_VL(c1, V, Tn, A, L));
      r.alpha = 1.0;
      r.ok = conv;
      return r;
    }
    // mixed cell: Newton on sum xi_k v_k = v, sum xi_k e_k = e from the
    // previous stage's (p, T) or the ideal-gas stand-in
    double Y0 = 1.0 - Y;
    // pressure is resolved to rounding relative to p + p_inf of the stiff component
    const double pscale = fmax(c0.pinf, 1.0);
    int conv = 0;
    const bool warm = Tw > 0.0 && Tw < 1e300 && fabs(pw) < 1e300;
    for (int start = warm ? 0 : 1; start < 2 && !conv; ++start) {
      if (start == 0) {
        p = pw;
        T = Tw;
      } else {
        sg_pair(c0.gamma, c0.pinf, c0.cv, c0.qs, c1.gam_ig, 0.0, c1.cv, c1.qs, v, e, Y, p, T);
      }
      for (int it = 0; it < 60; ++it) {
        VE a = comp_ve(c0, p, T), b = comp_ve(c1, p, T);
        double F1 = Y0 * a.v + Y * b.v - v, F2 = Y0 * a.e + Y * b.e - e;
        double J11 = Y0 * a.dvdp + Y * b.dvdp, J12 = Y0 * a.dvdT + Y * b.dvdT;
        double J21 = Y0 * a.dedp + Y * b.dedp, J22 = Y0 * a.dedT + Y * b.dedT;
        double idet = frcp(J11 * J22 - J12 * J21);
        double dp = (F1 * J22 - F2 * J12) * idet;
        double dT = (J11 * F2 - J21 * F1) * idet;
        double Tn = T - dT;
        if (Tn <= 0.0) Tn = 0.5 * T;
        p -= dp;
        T = Tn;
        if (fabs(dT) <= 1e-12 * T && fabs(dp) <= 1e-12 * (fabs(p) + pscale)) { conv = 1; break; }
      }
    }
    r.p = p;
    r.T = T;
    PRab Ag = pr_a(c1, T);
    double Vg = pr_volume(p, T, Ag.a, c1.b);
    r.c = fmax(sqrt(c0.c2T * T), pr_sound_VL(c1, Vg, T, Ag, pr_log(Vg, c1.b)));
    r.alpha = Y * rho * Vg / c1.M;
    r.ok = conv;
    return r;
  }
  return r;
}

// forward closure of three stiffened-gas components at (p, T, xi_1, xi_2) in
// precision R: 1 / rho and e (storage gauge); zero fractions are skipped
template <class R>
__device__ inline void tdu3(const CaseC& C, R ps, R Tf, R Y1, R Y2, R& rf, R& ef)
{
  R Yk[3] = {R(1) - Y1 - Y2, Y1, Y2};
  R vs = R(0), es = R(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (Yk[k] == R(0)) continue;
    const Comp& c = C.comp[k];
    R vk = R(c.A) * Tf * frcp(ps + R(c.pinf));
    vs += Yk[k] * vk;
    es += Yk[k] * (R(c.cv) * Tf + R(c.pinf) * vk + R(c.qs));
  }
  rf = frcp(vs);
  ef = es;
}

// forward closure at (p, T, xi) in FP64: 1 / rho and e (storage gauge).  Z0:
// a start for the Peng-Robinson compressibility (0: none).  F32: the result
// is rounded to FP32 (face states of the FP32-storage path), so the
// Peng-Robinson compressibility stops at a relative correction of 1e-6, and
// sqrt(T) and the departure energy's logarithm are taken in FP32; the cubic
// itself stays in FP64
template <bool PRK, bool F32 = false>
__device__ inline void closure_fwd(const CaseC& C, double p, double T, double Y, double& vmix, double& e,
                                   double Z0 = 0.0)
{
  double Yk[2] = {1.0 - Y, Y};
  vmix = 0.0;
  e = 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (Yk[k] == 0.0) continue;
    const Comp& c = C.comp[k];
    double vk, ek;
    if (!PRK || c.kind == 0) {
      vk = c.A * T * frcp(p + c.pinf);
      ek = c.cv * T + c.pinf * vk + c.qs;
    } else {
      // a - T a' = pa_0 - pa_1 sqrt(T) / 2 (with F32, T is an FP32 face value
      // and its square root is taken in FP32)
      double sT = F32 ? (double)sqrtf((float)T) : sqrt(T);
      double a = fma(c.pa_2, T, c.pa_0 - c.pa_1 * sT);
      double V = pr_volume(p, T, a, c.b, Z0, F32 ? 1e-6 : 1e-9);
      vk = V * c.iM;
      double L;
      if constexpr (F32) L = (double)logf((float)((V + (1.0 - SQRT2) * c.b) * frcp(V + (1.0 + SQRT2) * c.b)));
      else L = pr_log(V, c.b);
      ek = c.cv * T + c.qs + (c.pa_0 - 0.5 * c.pa_1 * sT) * c.ikb * L;
    }
    vmix += Yk[k] * vk;
    e += Yk[k] * ek;
  }
}

// ------------------------------------------------------------------ reconstruction
// limited slope: f(r) of Table 4.2 times the far-side difference, written
// without the division (r = near / far); zero at extrema
template <class R>
__device__ inline R slope(int kind, R far, R near)
{
  R a = fabs(far), b = fabs(near);
  R g;
  switch (kind) {
    case LIM_MINMOD: g = fmin(a, b); break;
    case LIM_KOREN: g = fmin(fmin(R(2) * a, R(2) * b), (a + R(2) * b) * R(1.0 / 3.0)); break;
    case LIM_VANALBADA: g = fdiv(a * b * (a + b), a * a + b * b); break;
    case LIM_VANLEER: g = fdiv(R(2) * a * b, a + b); break;
    case LIM_CHAKRAVARTHY: g = fmin(a, R(4) * b); break;
    case LIM_MC: g = fmin(fmin(R(2) * a, R(2) * b), R(0.5) * (a + b)); break;
    case LIM_SUPERBEE: g = fmax(fmin(a, R(2) * b), fmin(R(2) * a, b)); break;
    default: g = R(0);
  }
  return (far * near > R(0)) ? copysign(g, near) : R(0);
}

// THINC eligibility of the middle cell (Appendix D): eps < xi < 1 - eps and
// xi monotone through the cell
template <class R>
__device__ inline bool eligible(R a, R b, R c, R eps)
{
  return b > eps && b < R(1) - eps && (b - a) * (c - b) > R(0);
}

// upwind-biased left/right face values from cells i-1, i, i+1, i+2 (Section 3.3)
template <class R>
__device__ inline void recon(int kind, R a, R b, R c, R d, R& L, R& Rr)
{
  R dn = c - b;
  L = b + R(0.5) * slope<R>(kind, b - a, dn);
  Rr = c - R(0.5) * slope<R>(kind, d - c, dn);
}

// ------------------------------------------------------------------ face flux
// primitive stencil of one face: cells i-1, i, i+1, i+2 along the face normal
template <class R, int D>
struct Stencil {
  R u[D][4];
  R p[4], T[4], Y[4];
  R Y2[4];             // second gas fraction (three components only)
  R rho1, rho2, c1, c2;
};

// THINC face value of the upwind cell b between neighbours a, c
// (eqs. 3-3/3-4 with the range denominator): left = value at the cell's
// right face, else at its left face
template <class R>
__device__ inline R thinc_value(const SchemeC& S, bool left, R a, R b, R c)
{
  R mn = fmin(a, c), mx = fmax(a, c);
  R th = (c >= a) ? R(1) : R(-1);
  R Fv = fdiv(b - mn + R(S.thinc_gamma), mx - mn + R(S.thinc_gamma));
  R tb = R(S.tanh_b);
  R E = (fexp(th * R(S.beta) * (R(2) * Fv - R(1))) * R(S.icosh_b) - R(1)) * R(S.itanh_b);
  R prof = left ? fdiv(tb + E, R(1) + E * tb) : E;
  return mn + R(0.5) * (mx - mn) * (R(1) + th * prof);
}

// Thermodynamic dependent update at (p*, T_f, xi_f) in precision R for a
// stiffened-gas pair: 1 / rho_f and e_f (storage gauge)
template <class R>
__device__ inline void tdu_sg(const CaseC& C, R ps, R Tf, R Yf, R& rf, R& ef)
{
  const Comp& c0 = C.comp[0];
  const Comp& c1 = C.comp[1];
  R Y0 = R(1) - Yf;
  R P0 = R(c0.pinf), P1 = R(c1.pinf);
  R v0 = R(c0.A) * Tf * frcp(ps + P0);
  R v1 = R(c1.A) * Tf * frcp(ps + P1);
  R vs = (Y0 != R(0) ? Y0 * v0 : R(0)) + (Yf != R(0) ? Yf * v1 : R(0));
  rf = frcp(vs);
  ef = (Y0 != R(0) ? Y0 * (R(c0.cv) * Tf + P0 * v0 + R(c0.qs)) : R(0)) +
       (Yf != R(0) ? Yf * (R(c1.cv) * Tf + P1 * v1 + R(c1.qs)) : R(0));
}

// Face closure from the internal energy (Appendix B, rho* = f(p*, xi*, e*))
// for a stiffened-gas pair in precision R: at fixed p each component's volume
// v_k = A_k T / (p + pinf_k) and energy e_k = cv_k T + pinf_k v_k + q_k are
// linear in T, so sum_k xi_k e_k = e gives T, then 1 / rho_f.  ef_in is the
// face energy in the unshifted gauge; ef is returned in the storage gauge
// (minus sum_k xi_k Q_k)
template <class R>
__device__ inline void tdu_sg_e(const CaseC& C, R ps, R ef_in, R Yf, R& rf, R& ef)
{
  const Comp& c0 = C.comp[0];
  const Comp& c1 = C.comp[1];
  R Y0 = R(1) - Yf;
  R P0 = R(c0.pinf), P1 = R(c1.pinf);
  R w0 = R(c0.A) * frcp(ps + P0), w1 = R(c1.A) * frcp(ps + P1);   // v_k / T
  R slope = (Y0 != R(0) ? Y0 * (R(c0.cv) + P0 * w0) : R(0)) + (Yf != R(0) ? Yf * (R(c1.cv) + P1 * w1) : R(0));
  R off = (Y0 != R(0) ? Y0 * R(c0.qs + C.Q[0]) : R(0)) + (Yf != R(0) ? Yf * R(c1.qs + C.Q[1]) : R(0));
  R Tf = (ef_in - off) * frcp(slope);
  R vs = (Y0 != R(0) ? Y0 * w0 : R(0)) + (Yf != R(0) ? Yf * w1 : R(0));
  rf = frcp(vs * Tf);
  ef = ef_in - ((Y0 != R(0) ? Y0 * R(C.Q[0]) : R(0)) + (Yf != R(0) ? Yf * R(C.Q[1]) : R(0)));
}

// One face (Section 3.2/3.3, Appendix D):
//  impedances I_L = (3 rho_i + rho_{i+1}) c_m / 4, I_R = (rho_i + 3 rho_{i+1}) c_m / 4;
//  discontinuous branch: limited upwind-biased states, p* = (p_L + p_R)/2,
//   u* = (I_L u_L + I_R u_R + p_L - p_R) / (I_L + I_R), face state from the
//   upwind side of u* (ties to the left), xi by THINC when the upwind cell is
//   an interface cell;
//  smooth branch: fourth-order central u, p; second-order central T, xi;
//   u* = u_C + k3 (p_{i+2} - 3 p_{i+1} + 3 p_i - p_{i-1}) / (I_L + I_R);
//  TDU: rho_f, e_f from the closure at (p*, T_f, xi_f) (S.recon_e, in the
//   run-time limiter instantiations: the stencil's T rows hold e and rho_f
//   follows from the closure at (p*, xi_f, e_f));
//  flux (storage variables): (m xi_L, m xi_G, m u_f + p* n, m (e_f + |u_f|^2/2) + p* u*).
// LIM = 1 fixes the default limiters (Koren for velocities, Minmod for p, T,
// xi) at compile time; LIM = 0 takes the scheme's limiters at run time.
template <class R, int D, int DIR, bool PRK, bool G2 = false, int LIM = 0>
__device__ inline void face_flux(const SchemeC& S, const CaseC& C, const Stencil<R, D>& s,
                                 bool disc, bool sl, bool sr, R* F, bool sl2 = false, bool sr2 = false)
{
  const int lu = LIM ? int(LIM_KOREN) : S.lim_u;
  const int ls = LIM ? int(LIM_MINMOD) : S.lim_s;
  R cm = fmax(s.c1, s.c2);
  R rsum = s.rho1 + s.rho2;
  R IL = (R(3) * s.rho1 + s.rho2) * cm * R(0.25);
  R IR = (s.rho1 + R(3) * s.rho2) * cm * R(0.25);
  R iI = frcp(rsum * cm);
  R uf[D];
  R us, ps, Tf, Yf, Y2f = R(0);
  if (disc) {
    R uL[D], uR[D];
#pragma unroll
    for (int d = 0; d < D; ++d) recon<R>(lu, s.u[d][0], s.u[d][1], s.u[d][2], s.u[d][3], uL[d], uR[d]);
    R pL, pR, TL, TR, YL, YR;
    recon<R>(ls, s.p[0], s.p[1], s.p[2], s.p[3], pL, pR);
    recon<R>(ls, s.T[0], s.T[1], s.T[2], s.T[3], TL, TR);
    recon<R>(ls, s.Y[0], s.Y[1], s.Y[2], s.Y[3], YL, YR);
    ps = R(0.5) * (pL + pR);
    us = (IL * uL[DIR] + IR * uR[DIR] + pL - pR) * iI;
    bool left = us >= R(0);
#pragma unroll
    for (int d = 0; d < D; ++d) uf[d] = left ? uL[d] : uR[d];
    Tf = left ? TL : TR;
    Yf = left ? YL : YR;
    if (S.thinc && (left ? sl : sr))
      Yf = thinc_value<R>(S, left, left ? s.Y[0] : s.Y[1], left ? s.Y[1] : s.Y[2], left ? s.Y[2] : s.Y[3]);
    if constexpr (G2) {
      R Y2L, Y2R;
      recon<R>(ls, s.Y2[0], s.Y2[1], s.Y2[2], s.Y2[3], Y2L, Y2R);
      Y2f = left ? Y2L : Y2R;
      if (S.thinc && (left ? sl2 : sr2))
        Y2f = thinc_value<R>(S, left, left ? s.Y2[0] : s.Y2[1], left ? s.Y2[1] : s.Y2[2],
                             left ? s.Y2[2] : s.Y2[3]);
    }
  } else {
    const R c12 = R(1.0 / 12.0);
#pragma unroll
    for (int d = 0; d < D; ++d)
      uf[d] = (R(7) * (s.u[d][1] + s.u[d][2]) - s.u[d][0] - s.u[d][3]) * c12;
    ps = (R(7) * (s.p[1] + s.p[2]) - s.p[0] - s.p[3]) * c12;
    R d3p = s.p[3] - R(3) * s.p[2] + R(3) * s.p[1] - s.p[0];
    us = uf[DIR] + R(S.k3) * d3p * iI;
    Tf = R(0.5) * (s.T[1] + s.T[2]);
    Yf = R(0.5) * (s.Y[1] + s.Y[2]);
    if constexpr (G2) Y2f = R(0.5) * (s.Y2[1] + s.Y2[2]);
  }
  R rf, ef;
  if (LIM == 0 && !G2 && S.recon_e) {
    tdu_sg_e<R>(C, ps, Tf, Yf, rf, ef);
  } else if constexpr (G2) {
    // independently reconstructed gas fractions summing above one are
    // rescaled (no liquid mass may leave through a pure-gas face)
    R sum = Yf + Y2f;
    if (sum > R(1)) {
      R is = frcp(sum);
      Yf *= is;
      Y2f *= is;
    }
    tdu3<R>(C, ps, Tf, Yf, Y2f, rf, ef);
  } else if (!PRK || C.comp[1].kind == 0 || Yf == R(0)) {
    tdu_sg<R>(C, ps, Tf, Yf, rf, ef);
  } else {
    // a pure-gas face whose upwind cell is pure gas starts the compressibility
    // from that cell's own, p* M / (rho R T_f) (close: same fluid, nearby state)
    double Z0 = 0.0;
    const bool left = us >= R(0);
    if (Yf == R(1) && (left ? s.Y[1] : s.Y[2]) == R(1)) {
      double rup = (double)(left ? s.rho1 : s.rho2);
      Z0 = (double)ps * C.comp[1].M * frcp(rup * R_UNIV * (double)Tf);
    }
    double vm, em;
    closure_fwd<PRK, sizeof(R) == 4>(C, (double)ps, (double)Tf, (double)Yf, vm, em, Z0);
    rf = R(frcp(vm));
    ef = R(em);
  }
  R m = rf * us;
  R ke = R(0);
#pragma unroll
  for (int d = 0; d < D; ++d) ke += uf[d] * uf[d];
  F[0] = m * (R(1) - Yf - Y2f);
  F[1] = m * Yf;
#pragma unroll
  for (int d = 0; d < D; ++d) F[2 + d] = m * uf[d] + (d == DIR ? ps : R(0));
  F[2 + D] = m * (ef + R(0.5) * ke) + ps * us;
  if constexpr (G2) F[3 + D] = m * Y2f;
}

}  // namespace fvm
