/*
 * oracle_baro.c -- barotropic equilibrium model of the oracle (test
 * infrastructure): a liquid that turns into a liquid-vapour mixture below its
 * saturation pressure and one isothermal ideal gas (Section 2.2,
 * eqs. 2-3 .. 2-7), and its face flux with the liquid-vapour density THINC of
 * Section 3.4 (eqs. 3-7, 3-8, Remarks 1 and 2).
 *
 * No energy equation: the conserved fields are rho, rho u_1 .. rho u_D and
 * rho xi (xi the gas mass fraction); p = f(rho, xi).  With ncomp = 3 there
 * are two isothermal ideal gases (eqs. 2-5, 2-6 with Gas1 and Gas2; R T of
 * the second is bt_RT2) and rho xi_2 follows as the last conserved field.
 */
#include <math.h>
#include "oracle.h"
#include "oracle_internal.h"

int og_is_barotropic(const og_eos* e)
{
  return e->model == OG_MODEL_BAROTROPIC;
}

/* liquid (p >= p_sat, eq. 2-3) or liquid-vapour mixture (p < p_sat, eq. 2-4)
 * density at pressure p; the mixture's speed of sound is c_M^2 = p_sat / rho_sat */
double og_baro_liquid_density(const og_eos* e, double p)
{
  double c2 = (p >= e->bt_p_sat) ? e->bt_c_liq * e->bt_c_liq : e->bt_p_sat / e->bt_rho_sat;
  return e->bt_rho_sat + (p - e->bt_p_sat) / c2;
}

/* forward closure: density of the mixture at (p, xi_1, xi_2) from the
 * volume fractions (1/rho = sum_i xi_i / rho_Gi + (1 - sum_i xi_i) / rho_L/M,
 * rho_Gi = p / (R_i T_i), eq. 2-5, 2-6) */
double og_baro_density2(const og_eos* e, double p, double Y, double Y2)
{
  double v = 0.0, l = 1.0 - Y - Y2;
  if (Y != 0.0) v += Y * e->bt_RT / p;
  if (Y2 != 0.0) v += Y2 * e->bt_RT2 / p;
  if (l != 0.0) v += l / og_baro_liquid_density(e, p);
  return 1.0 / v;
}

double og_baro_density(const og_eos* e, double p, double Y)
{
  return og_baro_density2(e, p, Y, 0.0);
}

/* inverse closure p = f(rho, xi): the one-fluid equation of Section 2.2,
 *   (1 - rho xi R T / p) rho_L/M(p) = (1 - xi) rho,
 * multiplied by p.  With a = rho xi R T and b = (1 - xi) rho it reads
 *   (p - a) rho_L/M(p) - b p = 0,
 * a quadratic in p on each branch of rho_L/M.  Both branches agree at
 * p = p_sat, so the sign of the left-hand side there picks the branch
 * (<= 0: the root lies at p >= p_sat, liquid).  The root taken is the
 * positive (larger) one, evaluated without cancellation. */
int og_baro_pressure2(const og_eos* e, double rho, double Y, double Y2, double* p)
{
  /* with two gases a = rho (xi_1 R_1 T_1 + xi_2 R_2 T_2) and b = (1 - xi_1 - xi_2) rho:
   * the same quadratic (the fractions clipped as in the four-equation model) */
  double Yk[3];
  og_clip_fractions3(Y, Y2, Yk);
  double a = rho * (Yk[1] * e->bt_RT + Yk[2] * e->bt_RT2), b = Yk[0] * rho;
  double ps = e->bt_p_sat, rs = e->bt_rho_sat;
  double g = (ps - a) * rs - b * ps;
  double c2 = (g <= 0.0) ? e->bt_c_liq * e->bt_c_liq : ps / rs;
  /* rho_L/M(p) = rs + (p - ps) / c2 = (K + p) / c2 with K = rs c2 - ps:
   * (p - a)(K + p) - b c2 p = 0  ->  p^2 + B p + C = 0 */
  double K = rs * c2 - ps;
  double B = K - a - b * c2, Cc = -a * K;
  double disc = B * B - 4.0 * Cc;
  if (!(disc >= 0.0) || !(rho > 0.0)) { *p = NAN; return -1; }
  double s = sqrt(disc);
  *p = (B <= 0.0) ? 0.5 * (-B + s) : (-2.0 * Cc) / (B + s);
  return 0;
}

int og_baro_pressure(const og_eos* e, double rho, double Y, double* p)
{
  return og_baro_pressure2(e, rho, Y, 0.0, p);
}

/* speed of sound used by the impedances and the time step: the largest of
 * the components' speeds (the liquid's c_L, or c_M below p_sat, and the
 * isothermal gas's sqrt(R T)), as in the four-equation model */
double og_baro_sound(const og_eos* e, double p)
{
  double cl = (p >= e->bt_p_sat) ? e->bt_c_liq : sqrt(e->bt_p_sat / e->bt_rho_sat);
  double cg = sqrt(e->bt_RT);
  if (og_ncomp(e) == 3 && sqrt(e->bt_RT2) > cg) cg = sqrt(e->bt_RT2);
  return cl > cg ? cl : cg;
}

/* gas volume fraction alpha_G = rho xi R T / p (eq. 2-6) and vapour volume
 * fraction (eq. 2-7): (1 - alpha_G)(rho_sat - rho_M)/(rho_sat - rho_vap)
 * where the liquid is a mixture (rho_M < rho_sat), 0 otherwise, at most
 * 0.995 */
void og_baro_fractions2(const og_eos* e, double rho, double Y, double Y2, double p, double* alpha_G,
                        double* alpha_G2, double* alpha_V)
{
  double Yk[3];
  og_clip_fractions3(Y, Y2, Yk);
  double aG = (Yk[1] == 0.0) ? 0.0 : rho * Yk[1] * e->bt_RT / p;
  double aG2 = (Yk[2] == 0.0) ? 0.0 : rho * Yk[2] * e->bt_RT2 / p;
  double rM = og_baro_liquid_density(e, p);
  double aV = 0.0;
  if (rM < e->bt_rho_sat) aV = (1.0 - aG - aG2) * (e->bt_rho_sat - rM) / (e->bt_rho_sat - e->bt_rho_vap);
  if (aV > 0.995) aV = 0.995;
  if (aV < 0.0) aV = 0.0;
  *alpha_G = aG;
  *alpha_G2 = aG2;
  *alpha_V = aV;
}

void og_baro_fractions(const og_eos* e, double rho, double Y, double p, double* alpha_G, double* alpha_V)
{
  double aG2;
  og_baro_fractions2(e, rho, Y, 0.0, p, alpha_G, &aG2, alpha_V);
}

/* mixture viscosity of eq. 2-8 with one gas:
 *   (1 - alpha_G)[(1 - a_v)(1 + 5/2 a_v) mu_liq + a_v mu_vap] + alpha_G mu_gas.
 * The bracket is the viscosity of the liquid-vapour part and (1 - alpha_G)
 * its volume share, so a_v there is the vapour share of that part,
 * a_v = alpha_V / (1 - alpha_G) with alpha_V of eq. 2-7 (a share of the whole
 * cell); 0 where there is no liquid-vapour part. */
double og_baro_viscosity2(const og_eos* e, double alpha_G, double alpha_G2, double alpha_V)
{
  double aG = alpha_G < 0.0 ? 0.0 : (alpha_G > 1.0 ? 1.0 : alpha_G);
  double aG2 = alpha_G2 < 0.0 ? 0.0 : (alpha_G2 > 1.0 ? 1.0 : alpha_G2);
  double sum = aG + aG2;
  if (sum > 1.0) { aG /= sum; aG2 /= sum; }
  double m = 1.0 - aG - aG2;
  if (m < 0.0) m = 0.0;
  double av = (m > 0.0) ? alpha_V / m : 0.0;
  if (av > 1.0) av = 1.0;
  if (av < 0.0) av = 0.0;
  return m * ((1.0 - av) * (1.0 + 2.5 * av) * e->mu[0] + av * e->bt_mu_vap) + aG * e->mu[1] + aG2 * e->mu[2];
}

double og_baro_viscosity(const og_eos* e, double alpha_G, double alpha_V)
{
  return og_baro_viscosity2(e, alpha_G, 0.0, alpha_V);
}

static void upwind_pair(int lim, double a, double b, double c, double d, double* L, double* R)
{
  *L = b + 0.5 * og_slope(lim, b - a, c - b);
  *R = c - 0.5 * og_slope(lim, d - c, c - b);
}

/*
 * One face of the barotropic model between cells i (W[1]) and i+1 (W[2]):
 *  - impedances and p*, u* as in the four-equation model (eq. 3-1, 3-2, D.5,
 *    D.6), from reconstructed u and p;
 *  - xi: limited upwind-biased, THINC where the upwind cell is a gas
 *    interface cell (bit 0 of s_left / s_right; bit 2 for xi_2 with two
 *    gases), second-order central in the smooth branch;
 *  - TDU (eq. 3-5): rho_f = f(p*, xi_f);
 *  - Remark 1 and 2: where the upwind cell is a liquid-vapour interface cell
 *    (bit 1: eps < alpha_V < 1 - eps, alpha_V monotone through it) the face
 *    density is the THINC value of rho (eq. 3-7 / 3-8) instead;
 *  - flux: m = rho_f u*; (m, m u_f + p* n, m xi_f).
 */
int og_face_flux_baro(const og_eos* e, const og_scheme* s, int dim, int dir,
                      const double W[4][OW_N], int f, int s_left, int s_right,
                      double* F, double* ustar, double* pstar)
{
  double cm = fmax(W[1][OW_C], W[2][OW_C]);
  double IL = (3.0 * W[1][OW_RHO] + W[2][OW_RHO]) * cm / 4.0;
  double IR = (W[1][OW_RHO] + 3.0 * W[2][OW_RHO]) * cm / 4.0;
  double uf[3] = {0.0, 0.0, 0.0};
  double us, ps, Yf, Yf2 = 0.0, rf;
  int lv = 0, left = 1;
  const int two = og_ncomp(e) == 3;

  if (f) {
    double uL[3] = {0, 0, 0}, uR[3] = {0, 0, 0}, pL, pR, YL, YR, Y2L = 0.0, Y2R = 0.0;
    for (int d = 0; d < dim; ++d)
      upwind_pair(s->lim_u, W[0][OW_U + d], W[1][OW_U + d], W[2][OW_U + d], W[3][OW_U + d], &uL[d], &uR[d]);
    upwind_pair(s->lim_s, W[0][OW_P], W[1][OW_P], W[2][OW_P], W[3][OW_P], &pL, &pR);
    upwind_pair(s->lim_s, W[0][OW_Y], W[1][OW_Y], W[2][OW_Y], W[3][OW_Y], &YL, &YR);
    if (two) upwind_pair(s->lim_s, W[0][OW_Y2], W[1][OW_Y2], W[2][OW_Y2], W[3][OW_Y2], &Y2L, &Y2R);
    ps = 0.5 * (pL + pR);
    us = (IL * uL[dir] + IR * uR[dir] + pL - pR) / (IL + IR);
    left = us >= 0.0;
    int sb = left ? s_left : s_right;
    for (int d = 0; d < dim; ++d) uf[d] = left ? uL[d] : uR[d];
    Yf = left ? YL : YR;
    if (s->thinc && (sb & 1))
      Yf = left ? og_thinc_left(W[0][OW_Y], W[1][OW_Y], W[2][OW_Y], s->beta, s->thinc_gamma)
                : og_thinc_right(W[1][OW_Y], W[2][OW_Y], W[3][OW_Y], s->beta, s->thinc_gamma);
    if (two) {
      /* the second gas fraction on its own, THINC where the upwind cell is
       * one of its interface cells (bit 2) */
      Yf2 = left ? Y2L : Y2R;
      if (s->thinc && (sb & 4))
        Yf2 = left ? og_thinc_left(W[0][OW_Y2], W[1][OW_Y2], W[2][OW_Y2], s->beta, s->thinc_gamma)
                   : og_thinc_right(W[1][OW_Y2], W[2][OW_Y2], W[3][OW_Y2], s->beta, s->thinc_gamma);
    }
    lv = s->thinc && (sb & 2);
  } else {
    for (int d = 0; d < dim; ++d)
      uf[d] = og_central4(W[0][OW_U + d], W[1][OW_U + d], W[2][OW_U + d], W[3][OW_U + d]);
    ps = og_central4(W[0][OW_P], W[1][OW_P], W[2][OW_P], W[3][OW_P]);
    double d3p = W[3][OW_P] - 3.0 * W[2][OW_P] + 3.0 * W[1][OW_P] - W[0][OW_P];
    us = uf[dir] + s->kappa3 * d3p / (IL + IR);
    Yf = 0.5 * (W[1][OW_Y] + W[2][OW_Y]);
    if (two) Yf2 = 0.5 * (W[1][OW_Y2] + W[2][OW_Y2]);
  }
  /* the face gas fractions are taken in [0, 1] (cell values may overshoot by
   * round-off-sized amounts), two of them rescaled where they sum above one */
  if (two) {
    double Yk[3];
    og_clip_fractions3(Yf, Yf2, Yk);
    Yf = Yk[1];
    Yf2 = Yk[2];
  } else {
    Yf = og_clip_fraction(Yf);
  }
  if (!(ps > 0.0)) return -1;   /* no density of gas or mixture at p <= 0 */
  if (lv)
    rf = left ? og_thinc_left(W[0][OW_RHO], W[1][OW_RHO], W[2][OW_RHO], s->beta, s->thinc_gamma)
              : og_thinc_right(W[1][OW_RHO], W[2][OW_RHO], W[3][OW_RHO], s->beta, s->thinc_gamma);
  else
    rf = og_baro_density2(e, ps, Yf, Yf2);
  double m = rf * us;
  F[0] = m;
  for (int d = 0; d < dim; ++d) F[1 + d] = m * uf[d] + (d == dir ? ps : 0.0);
  F[1 + dim] = m * Yf;
  if (two) F[2 + dim] = m * Yf2;
  if (ustar) *ustar = us;
  if (pstar) *pstar = ps;
  return 0;
}
