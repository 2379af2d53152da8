/*
 * oracle_scheme.c -- face reconstruction, Riemann solver, thermodynamic
 * dependent update and face flux of the oracle (test infrastructure).
 *
 * Section 3.2 (eq. 3-1, 3-2), Section 3.3 (eq. 3-3 .. 3-5, the limiter
 * formulas), Table 4.2, Appendix B (reconstructed temperature, TDU of density
 * and energy) and Appendix D (eq. D.1 .. D.6).
 */
#include <math.h>
#include "oracle.h"
#include "oracle_internal.h"

/* Table 4.2.  r is the ratio of the near-face difference to the difference
 * that the limiter multiplies: the printed slope formulas of Section 3.3
 * multiply the far-side difference, and with that orientation the Koren
 * limiter is the third-order one its name promises (exact face values for
 * cell averages of a quadratic).  The printed "Minmod" of Section 3.3 is the
 * Superbee formula; Minmod is taken from Table 4.2 and Superbee kept as its
 * own entry. */
double og_limiter_table(int kind, double r)
{
  switch (kind) {
    case OG_LIM_MINMOD:       return fmax(0.0, fmin(1.0, r));
    case OG_LIM_KOREN:        return fmax(0.0, fmin(2.0, fmin(2.0 * r, (1.0 + 2.0 * r) / 3.0)));
    case OG_LIM_VANALBADA:    return (r + r * r) / (1.0 + r * r);
    case OG_LIM_VANLEER:      return (r + fabs(r)) / (1.0 + fabs(r));
    case OG_LIM_CHAKRAVARTHY: return fmax(0.0, fmin(1.0, 4.0 * r));
    case OG_LIM_MC:           return fmax(0.0, fmin(2.0, fmin(2.0 * r, 0.5 * (1.0 + r))));
    case OG_LIM_SUPERBEE:     return fmax(0.0, fmax(fmin(1.0, 2.0 * r), fmin(r, 2.0)));
    default:                  return 0.0;
  }
}

/* limited slope: f(r) times the far-side difference, zero at extrema (TVD) */
double og_slope(int kind, double dfar, double dnear)
{
  if (!(dfar * dnear > 0.0)) return 0.0;
  return dfar * og_limiter_table(kind, dnear / dfar);
}

/* THINC, eq. (3-3): left value at the face between cells 2 and 3 from cells
 * (1, 2, 3) = (a, b, c).  F is the normalised cell average; its denominator is
 * the range max - min (+gamma) of the neighbours: for min = 0 this is the
 * printed max + gamma, and only the range makes the face values those of the
 * tanh profile whose cell average F is. */
double og_thinc_left(double a, double b, double c, double beta, double gam)
{
  double mn = fmin(a, c), mx = fmax(a, c);
  double th = (c >= a) ? 1.0 : -1.0;
  double F = (b - mn + gam) / (mx - mn + gam);
  double tb = tanh(beta);
  double E = (exp(th * beta * (2.0 * F - 1.0)) / cosh(beta) - 1.0) / tb;
  return mn + 0.5 * (mx - mn) * (1.0 + th * (tb + E) / (1.0 + E * tb));
}

/* THINC, eq. (3-4): right value at the face between cells 2 and 3 from cells
 * (2, 3, 4) = (a, b, c). */
double og_thinc_right(double a, double b, double c, double beta, double gam)
{
  double mn = fmin(a, c), mx = fmax(a, c);
  double th = (c >= a) ? 1.0 : -1.0;
  double F = (b - mn + gam) / (mx - mn + gam);
  double tb = tanh(beta);
  double E = (exp(th * beta * (2.0 * F - 1.0)) / cosh(beta) - 1.0) / tb;
  return mn + 0.5 * (mx - mn) * (1.0 + th * E);
}

/* eq. (D.1): fourth-order central face value from cells i-1, i, i+1, i+2 */
double og_central4(double a, double b, double c, double d)
{
  return (7.0 * (b + c) - a - d) / 12.0;
}

static void upwind_pair(int lim, double a, double b, double c, double d, double* L, double* R)
{
  /* Section 3.3: L from cell i (= b) with the far difference b - a,
   * R from cell i+1 (= c) with the far difference d - c; near difference c - b */
  *L = b + 0.5 * og_slope(lim, b - a, c - b);
  *R = c - 0.5 * og_slope(lim, d - c, c - b);
}

/*
 * One face between cells i (W[1]) and i+1 (W[2]) along dir.
 *  - impedances of Appendix D (D.5): I_L = (3 rho_i + rho_{i+1}) c_m / 4,
 *    I_R = (rho_i + 3 rho_{i+1}) c_m / 4, c_m = max(c_i, c_{i+1});
 *  - f = 1 (discontinuous branch, also the whole of Section 3): upwind-biased
 *    limited states; p* and u* of eq. (3-1), (3-2) with the impedances above;
 *    the face state is the upwind side of u* (u* = 0 takes the left side);
 *    xi from THINC when the upwind cell is an interface cell, else limited;
 *  - f = 0 (smooth branch, Appendix D): fourth-order central u and p (D.1),
 *    second-order central T and xi, p* = p^C, u* = u^C + k3 * d3p / (I_L + I_R)
 *    with d3p = p_{i+2} - 3 p_{i+1} + 3 p_i - p_{i-1}; with k3 = 1/4 the added
 *    term equals p_L - p_R of unlimited upwind-biased states, i.e. the
 *    pressure term of eq. (3-2), which fixes its sign as dissipative;
 *  - TDU (eq. 3-5, Appendix B): the face temperature is reconstructed and
 *    rho_f, e_f follow from the closure at (p*, T_f, xi_f); with
 *    s->thermal = 1 the specific internal energy is reconstructed in its
 *    place (same limiter, upwind side, central average) and rho_f follows
 *    from the closure at (p*, xi_f, e_f);
 *  - flux of eq. (2-2): m = rho_f u*; (m, m u_f + p* n, m (e_f + |u_f|^2/2) + p* u*, m xi_f).
 * With three components the second gas fraction xi_2 is reconstructed like
 * xi_1 (limited, THINC where eligible, central) and TDU takes both
 * (Section 3.4: the TDU of rho_f with the gas fractions of Remark 2).
 */
int og_face_flux(const og_eos* e, const og_scheme* s, int dim, int dir,
                 const double W[4][OW_N], int f, int s_left, int s_right,
                 double* F, double* ustar, double* pstar)
{
  double cm = fmax(W[1][OW_C], W[2][OW_C]);
  double IL = (3.0 * W[1][OW_RHO] + W[2][OW_RHO]) * cm / 4.0;
  double IR = (W[1][OW_RHO] + 3.0 * W[2][OW_RHO]) * cm / 4.0;
  double uf[3] = {0.0, 0.0, 0.0};
  double us, ps, Tf, Yf, Y2f = 0.0;
  const int three = og_ncomp(e) == 3;
  const int th = s->thermal ? OW_E : OW_T;   /* the reconstructed thermal row */

  if (f) {
    double uL[3] = {0, 0, 0}, uR[3] = {0, 0, 0}, pL, pR, TL, TR, YL, YR, Y2L = 0.0, Y2R = 0.0;
    for (int d = 0; d < dim; ++d)
      upwind_pair(s->lim_u, W[0][OW_U + d], W[1][OW_U + d], W[2][OW_U + d], W[3][OW_U + d], &uL[d], &uR[d]);
    upwind_pair(s->lim_s, W[0][OW_P], W[1][OW_P], W[2][OW_P], W[3][OW_P], &pL, &pR);
    upwind_pair(s->lim_s, W[0][th], W[1][th], W[2][th], W[3][th], &TL, &TR);
    upwind_pair(s->lim_s, W[0][OW_Y], W[1][OW_Y], W[2][OW_Y], W[3][OW_Y], &YL, &YR);
    if (three) upwind_pair(s->lim_s, W[0][OW_Y2], W[1][OW_Y2], W[2][OW_Y2], W[3][OW_Y2], &Y2L, &Y2R);
    ps = 0.5 * (pL + pR);
    us = (IL * uL[dir] + IR * uR[dir] + pL - pR) / (IL + IR);
    if (us >= 0.0) {
      for (int d = 0; d < dim; ++d) uf[d] = uL[d];
      Tf = TL;
      Yf = (s->thinc && (s_left & 1))
               ? og_thinc_left(W[0][OW_Y], W[1][OW_Y], W[2][OW_Y], s->beta, s->thinc_gamma)
               : YL;
      if (three)
        Y2f = (s->thinc && (s_left & 2))
                  ? og_thinc_left(W[0][OW_Y2], W[1][OW_Y2], W[2][OW_Y2], s->beta, s->thinc_gamma)
                  : Y2L;
    } else {
      for (int d = 0; d < dim; ++d) uf[d] = uR[d];
      Tf = TR;
      Yf = (s->thinc && (s_right & 1))
               ? og_thinc_right(W[1][OW_Y], W[2][OW_Y], W[3][OW_Y], s->beta, s->thinc_gamma)
               : YR;
      if (three)
        Y2f = (s->thinc && (s_right & 2))
                  ? og_thinc_right(W[1][OW_Y2], W[2][OW_Y2], W[3][OW_Y2], s->beta, s->thinc_gamma)
                  : Y2R;
    }
  } else {
    for (int d = 0; d < dim; ++d)
      uf[d] = og_central4(W[0][OW_U + d], W[1][OW_U + d], W[2][OW_U + d], W[3][OW_U + d]);
    ps = og_central4(W[0][OW_P], W[1][OW_P], W[2][OW_P], W[3][OW_P]);
    double d3p = W[3][OW_P] - 3.0 * W[2][OW_P] + 3.0 * W[1][OW_P] - W[0][OW_P];
    us = uf[dir] + s->kappa3 * d3p / (IL + IR);
    Tf = 0.5 * (W[1][th] + W[2][th]);
    Yf = 0.5 * (W[1][OW_Y] + W[2][OW_Y]);
    if (three) Y2f = 0.5 * (W[1][OW_Y2] + W[2][OW_Y2]);
  }

  /* the two gas fractions are reconstructed independently; a face state
   * whose gas fractions sum above one (a negative liquid fraction, which
   * would move liquid mass into pure-gas cells) is rescaled to sum to one */
  if (three && Yf + Y2f > 1.0) {
    double sum = Yf + Y2f;
    Yf /= sum;
    Y2f /= sum;
  }
  double rf, ef;
  if (s->thermal) {
    double Tt;
    if (three || og_eos_forward_e(e, ps, Tf, Yf, &rf, &Tt)) return -1;
    ef = Tf;
  } else if (og_eos_forward2(e, ps, Tf, Yf, Y2f, &rf, &ef)) {
    return -1;
  }
  double m = rf * us;
  double ke = 0.0;
  for (int d = 0; d < dim; ++d) ke += uf[d] * uf[d];
  F[0] = m;
  for (int d = 0; d < dim; ++d) F[1 + d] = m * uf[d] + (d == dir ? ps : 0.0);
  F[1 + dim] = m * (ef + 0.5 * ke) + ps * us;
  F[2 + dim] = m * Yf;
  if (three) F[3 + dim] = m * Y2f;
  if (ustar) *ustar = us;
  if (pstar) *pstar = ps;
  return 0;
}
