/*
 * oracle_field.c -- whole-grid steps of one Runge-Kutta stage (Algorithm 1)
 * and the time step of the oracle (test infrastructure).
 *
 * Algorithm 1 lists, per stage: Riemann solver, reconstruction, sharpening,
 * surface tension, optional central switching (Appendix D), fluxes, update of
 * the conserved variables, primitives from the closure, boundary conditions.
 * The Riemann solver needs reconstructed states, so the oracle runs the steps
 * in the order in which their inputs exist:
 *   ghosts -> primitives -> sensors -> faces (reconstruction, THINC, Riemann,
 *   TDU, flux) -> divergence -> CSF source -> stage update.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "oracle.h"
#include "oracle_internal.h"

static __thread char g_err[256];
void og_set_error(const char* msg) { snprintf(g_err, sizeof g_err, "%s", msg); }
const char* og_last_error(void) { return g_err; }

int og_nthreads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void og_set_nthreads(int n)
{
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

void og_pad_init(og_pad* pd, const og_grid* g)
{
  pd->dim = g->dim;
  pd->ncell = 1;
  pd->npad = 1;
  for (int d = 0; d < 3; ++d) {
    pd->n[d] = (d < g->dim) ? g->n[d] : 1;
    pd->o[d] = (d < g->dim) ? 2 : 0;
    pd->P[d] = pd->n[d] + 2 * pd->o[d];
    pd->ncell *= (size_t)pd->n[d];
    pd->npad *= (size_t)pd->P[d];
  }
}

/* ---------------- counter-based inflow noise ---------------- */

/* SplitMix64 output function (Steele, Lea, Flood 2014): one increment of the
 * golden-ratio Weyl sequence followed by the two xor-shift-multiply rounds. */
uint64_t og_splitmix64(uint64_t x)
{
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* uniform number in [0, 1) keyed on (seed, step, j, k, component) */
double og_noise01(uint64_t seed, uint64_t step, uint64_t j, uint64_t k, uint64_t comp)
{
  uint64_t h = og_splitmix64(seed);
  h = og_splitmix64(h ^ step);
  h = og_splitmix64(h ^ j);
  h = og_splitmix64(h ^ k);
  h = og_splitmix64(h ^ comp);
  return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* ---------------- primitives <-> conserved ---------------- */

/* conserved state of one cell from (p, T, alpha_G, u): the volume fraction
 * alpha_G fixes xi = alpha_G rho_G / rho at the cell's (p, T) (Table A.1). */
static int cons_from_prim_cell(const og_eos* e, int dim, double p, double T, double al, double al2,
                               const double* u, double* qc)
{
  double rho, Y, Y2 = 0.0, r2, ein;
  if (og_is_barotropic(e)) {
    /* Section 2.2: rho = alpha_G rho_G(p) + (1 - alpha_G) rho_L/M(p) with
     * rho_G = p / (R T) (eq. 2-5), rho xi = alpha_G rho_G; T is not used */
    if (!(p > 0.0)) return -1;
    double rG = p / e->bt_RT, rL = og_baro_liquid_density(e, p);
    double rG2 = og_ncomp(e) == 3 ? p / e->bt_RT2 : 0.0;
    rho = al * rG + al2 * rG2 + (1.0 - al - al2) * rL;
    qc[0] = rho;
    for (int d = 0; d < dim; ++d) qc[1 + d] = rho * u[d];
    qc[1 + dim] = al * rG;
    if (og_ncomp(e) == 3) qc[2 + dim] = al2 * rG2;
    return rho > 0.0 ? 0 : -1;
  }
  if (og_ncomp(e) == 2) {
    double rL, eL, rG, eG;
    if (og_eos_forward(e, p, T, 0.0, &rL, &eL)) return -1;
    if (og_eos_forward(e, p, T, 1.0, &rG, &eG)) return -1;
    rho = al * rG + (1.0 - al) * rL;
    Y = al * rG / rho;
    if (og_eos_forward(e, p, T, Y, &r2, &ein)) return -1;
  } else {
    /* Table A.1: rho = sum_k alpha_k rho_k, xi_k = alpha_k rho_k / rho */
    double r[3];
    for (int k = 0; k < 3; ++k) r[k] = 1.0 / og_spec_volume(e, k, p, T);
    rho = (1.0 - al - al2) * r[0] + al * r[1] + al2 * r[2];
    Y = al * r[1] / rho;
    Y2 = al2 * r[2] / rho;
    if (og_eos_forward2(e, p, T, Y, Y2, &r2, &ein)) return -1;
  }
  double ke = 0.0;
  for (int d = 0; d < dim; ++d) ke += u[d] * u[d];
  qc[0] = rho;
  for (int d = 0; d < dim; ++d) qc[1 + d] = rho * u[d];
  qc[1 + dim] = rho * (ein + 0.5 * ke);
  qc[2 + dim] = rho * Y;
  if (og_ncomp(e) == 3) qc[3 + dim] = rho * Y2;
  return 0;
}

/* prim layout: [p, T, alpha_G, u_1 .. u_D][ncell], with three components
 * followed by alpha of the second gas */
int og_cons_from_prim(const og_grid* g, const og_eos* e, const double* prim, double* q)
{
  og_pad pd;
  og_pad_init(&pd, g);
  size_t nc = pd.ncell;
  int dim = g->dim, nq = og_nq(g, e), bad = 0;
  for (size_t c = 0; c < nc; ++c) {
    double u[3] = {0, 0, 0}, qc[7];
    for (int d = 0; d < dim; ++d) u[d] = prim[(3 + d) * nc + c];
    double al2 = og_ncomp(e) == 3 ? prim[(3 + dim) * nc + c] : 0.0;
    if (cons_from_prim_cell(e, dim, prim[c], prim[nc + c], prim[2 * nc + c], al2, u, qc)) bad = 1;
    for (int f = 0; f < nq; ++f) q[f * nc + c] = qc[f];
  }
  return bad ? -1 : 0;
}

/* primitives of one cell (Algorithm 1, "update primitive variables"):
 * u = rho u / rho, e = E - |u|^2/2, xi_k = rho xi_k / rho, (p, T) from the
 * closure, alpha_k = xi_k rho v_k(p, T) of each gas (with the fractions as the
 * closure takes them), c from og_mix_sound2. */
static int prim_cell(const og_eos* e, int dim, const double* qc, double* W)
{
  double rho = qc[0];
  double u[3] = {0, 0, 0}, ke = 0.0;
  for (int d = 0; d < dim; ++d) { u[d] = qc[1 + d] / rho; ke += u[d] * u[d]; }
  if (og_is_barotropic(e)) {
    /* p = f(rho, xi) (Section 2.2), alpha_G (eq. 2-6), alpha_V (eq. 2-7) */
    double Y = qc[1 + dim] / rho, p;
    double Y2 = og_ncomp(e) == 3 ? qc[2 + dim] / rho : 0.0;
    int rc = og_baro_pressure2(e, rho, Y, Y2, &p);
    W[OW_RHO] = rho;
    W[OW_U] = u[0]; W[OW_V] = u[1]; W[OW_W] = u[2];
    W[OW_P] = p; W[OW_T] = 0.0; W[OW_Y] = Y; W[OW_Y2] = Y2; W[OW_E] = 0.0;
    W[OW_C] = og_baro_sound(e, p);
    og_baro_fractions2(e, rho, Y, Y2, p, &W[OW_A], &W[OW_A2], &W[OW_AV]);
    if (rc || !(rho > 0.0) || !(p > 0.0) || !isfinite(p)) return -1;
    return 0;
  }
  double ein = qc[1 + dim] / rho - 0.5 * ke;
  double Y = qc[2 + dim] / rho;
  int three = og_ncomp(e) == 3;
  double Y2 = three ? qc[3 + dim] / rho : 0.0;
  double p, T;
  int rc = og_eos_inverse2(e, rho, ein, Y, Y2, 0.0, &p, &T);
  W[OW_RHO] = rho;
  W[OW_U] = u[0]; W[OW_V] = u[1]; W[OW_W] = u[2];
  W[OW_P] = p; W[OW_T] = T; W[OW_Y] = Y; W[OW_Y2] = Y2; W[OW_E] = ein;
  W[OW_C] = og_mix_sound2(e, p, T, Y, Y2);
  W[OW_AV] = 0.0;
  if (!three) {
    double Yc = og_clip_fraction(Y);
    W[OW_A] = (Yc == 0.0) ? 0.0 : Yc * rho * og_spec_volume(e, 1, p, T);
    W[OW_A2] = 0.0;
  } else {
    double Yk[3];
    og_clip_fractions3(Y, Y2, Yk);
    W[OW_A] = (Yk[1] == 0.0) ? 0.0 : Yk[1] * rho * og_spec_volume(e, 1, p, T);
    W[OW_A2] = (Yk[2] == 0.0) ? 0.0 : Yk[2] * rho * og_spec_volume(e, 2, p, T);
  }
  if (rc || !(rho > 0.0) || !(T > 0.0) || !isfinite(p) || !isfinite(W[OW_C])) return -1;
  return 0;
}

int og_prim_from_cons(const og_grid* g, const og_eos* e, const double* q, double* W)
{
  og_pad pd;
  og_pad_init(&pd, g);
  size_t nc = pd.ncell;
  int dim = g->dim, nq = og_nq(g, e), bad = 0;
  for (size_t c = 0; c < nc; ++c) {
    double qc[7], w[OW_N];
    for (int f = 0; f < nq; ++f) qc[f] = q[f * nc + c];
    if (prim_cell(e, dim, qc, w)) bad = 1;
    for (int f = 0; f < OW_N; ++f) W[f * nc + c] = w[f];
  }
  return bad ? -1 : 0;
}

/* ---------------- ghost cells (Algorithm 1, "update boundary conditions") ---------------- */

/* qp: padded conserved fields [nq][npad].  Two layers per side, filled
 * direction by direction (x, then y over the x-extended rows, then z), so that
 * edge and corner ghosts combine the two boundary kinds. */
static int fill_ghosts(const og_grid* g, const og_eos* e, const og_pad* pd, double* qp, int64_t step)
{
  int dim = g->dim, nq = og_nq(g, e);
  for (int d = 0; d < dim; ++d) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      /* directions already filled are swept over their ghosts too */
      lo[a] = (a < d) ? -pd->o[a] : 0;
      hi[a] = (a < d) ? pd->n[a] + pd->o[a] : pd->n[a];
    }
    lo[d] = 0; hi[d] = 1;   /* one pass over the transverse plane */
    int nd = pd->n[d];
    for (int k = lo[2]; k < hi[2]; ++k)
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int i = lo[0]; i < hi[0]; ++i) {
          int base[3] = {i, j, k};
          for (int side = 0; side < 2; ++side) {
            int bc = g->bc[d][side];
            for (int m = 0; m < 2; ++m) {
              int gc[3] = {base[0], base[1], base[2]};
              int sc[3] = {base[0], base[1], base[2]};
              int ghost = side == 0 ? -1 - m : nd + m;
              gc[d] = ghost;
              size_t gi = og_pidx(pd, gc[0], gc[1], gc[2]);
              if (bc == OG_BC_INFLOW && d == 0 && side == 0) {
                double y = 0.0, z = 0.0, r;
                if (dim > 1) y = (j + 0.5) * g->dx[1] - g->in_center[0];
                if (dim > 2) z = (k + 0.5) * g->dx[2] - g->in_center[1];
                r = sqrt(y * y + z * z);
                if (dim == 1 || r < g->in_radius) {
                  double u[3] = {g->in_u, 0.0, 0.0}, qc[7];
                  uint64_t jj = (uint64_t)(int64_t)j, kk = (uint64_t)(int64_t)k;
                  for (int c = 0; c < dim; ++c)
                    u[c] += g->in_noise * g->in_u *
                            (2.0 * og_noise01(g->in_seed, (uint64_t)step, jj, kk, (uint64_t)c) - 1.0);
                  if (cons_from_prim_cell(e, dim, g->in_p, g->in_T, g->in_alpha, 0.0, u, qc)) return -1;
                  for (int f = 0; f < nq; ++f) qp[f * pd->npad + gi] = qc[f];
                  continue;
                }
                bc = OG_BC_WALL;   /* outside the jet the inlet plane is a slip wall */
              }
              if (bc == OG_BC_FARFIELD) {
                /* a far-field reservoir at rest (stands in for the paper's
                 * non-reflective boundaries around a collapsing bubble) */
                double u[3] = {0.0, 0.0, 0.0}, qc[7];
                if (cons_from_prim_cell(e, dim, g->ff_p, g->ff_T, g->ff_alpha, 0.0, u, qc)) return -1;
                for (int f = 0; f < nq; ++f) qp[f * pd->npad + gi] = qc[f];
                continue;
              }
              int flip = 0;
              switch (bc) {
                case OG_BC_PERIODIC: sc[d] = side == 0 ? nd - 1 - m : m; break;
                case OG_BC_WALL:     sc[d] = side == 0 ? m : nd - 1 - m; flip = 1; break;
                case OG_BC_ZEROGRAD: sc[d] = side == 0 ? 0 : nd - 1; break;
                default: og_set_error("bad boundary kind"); return -1;
              }
              size_t si = og_pidx(pd, sc[0], sc[1], sc[2]);
              for (int f = 0; f < nq; ++f) {
                double v = qp[f * pd->npad + si];
                if (flip && f == 1 + d) v = -v;
                qp[f * pd->npad + gi] = v;
              }
            }
          }
        }
  }
  return 0;
}

/* ---------------- sensors (Appendix D) ---------------- */

/* per padded cell with one neighbour on each side: bit 0 = f (discontinuous
 * branch), bit 1+d = THINC eligibility along d */
static void sensors(const og_grid* g, const og_eos* e, const og_scheme* s, const og_pad* pd,
                    const double* W, unsigned short* flag)
{
  int dim = g->dim;
  size_t np = pd->npad;
  int lo[3], hi[3];
  for (int a = 0; a < 3; ++a) { lo[a] = (a < dim) ? -1 : 0; hi[a] = (a < dim) ? pd->n[a] + 1 : 1; }
#pragma omp parallel for collapse(2) schedule(static)
  for (int k = lo[2]; k < hi[2]; ++k)
    for (int j = lo[1]; j < hi[1]; ++j)
      for (int i = lo[0]; i < hi[0]; ++i) {
        size_t c = og_pidx(pd, i, j, k);
        size_t st[3] = {1, (size_t)pd->P[0], (size_t)pd->P[0] * pd->P[1]};
        unsigned short fl = 0;
        /* THINC eligibility: eps < xi_i < 1 - eps and xi monotone through i along d;
         * bits 1+d for xi_1, 4+d for xi_2 or, in the barotropic model, for the
         * vapour fraction alpha_V (liquid-vapour interface, Remark 1), and 7+d
         * for xi_2 of the barotropic model with two gases */
        const int nsets = (og_is_barotropic(e) && og_ncomp(e) == 3) ? 3 : 2;
        for (int g2 = 0; g2 < nsets; ++g2) {
          int f = g2 == 2 ? OW_Y2 : (g2 ? (og_is_barotropic(e) ? OW_AV : OW_Y2) : OW_Y);
          double Y = W[f * np + c];
          for (int d = 0; d < dim; ++d) {
            double Ym = W[f * np + c - st[d]], Yp = W[f * np + c + st[d]];
            int ok = Y > s->eps_interface && Y < 1.0 - s->eps_interface && (Y - Ym) * (Yp - Y) > 0.0;
            if (f == OW_AV) {
              /* the density that THINC then sharpens must be monotone too (with
               * gas present alpha_V alone does not make it so, and THINC of a
               * value outside its neighbours' range is unbounded) */
              double r0 = W[OW_RHO * np + c];
              ok = ok && (r0 - W[OW_RHO * np + c - st[d]]) * (W[OW_RHO * np + c + st[d]] - r0) > 0.0;
            }
            if (ok) fl |= (unsigned short)((g2 == 2 ? 128u : (g2 ? 16u : 2u)) << d);
          }
        }
        if (!s->switching) {
          fl |= 1u;
        } else {
          /* Ducros: (div u)^2 / ((div u)^2 + |curl u|^2 + eps), second-order central */
          double grad[3][3] = {{0}};
          for (int a = 0; a < dim; ++a)
            for (int d = 0; d < dim; ++d)
              grad[a][d] = (W[(OW_U + a) * np + c + st[d]] - W[(OW_U + a) * np + c - st[d]]) /
                           (2.0 * g->dx[d]);
          double div = 0.0;
          for (int d = 0; d < dim; ++d) div += grad[d][d];
          double w0 = grad[2][1] - grad[1][2];
          double w1 = grad[0][2] - grad[2][0];
          double w2 = grad[1][0] - grad[0][1];
          double curl2 = w0 * w0 + w1 * w1 + w2 * w2;
          double thD = div * div / (div * div + curl2 + s->eps_ducros);
          /* gas-volume-fraction variation over all directions (both gases together) */
          double thG = 0.0;
          double a0 = W[OW_A * np + c] + W[OW_A2 * np + c];
          for (int d = 0; d < dim; ++d) {
            double am = W[OW_A * np + c - st[d]] + W[OW_A2 * np + c - st[d]];
            double ap = W[OW_A * np + c + st[d]] + W[OW_A2 * np + c + st[d]];
            thG += fabs(a0 - am) + fabs(ap - a0);
          }
          /* the vapour-fraction detector theta^alpha, same expression and
           * (not given separately) the same threshold as theta^Gas */
          double thV = 0.0;
          for (int d = 0; d < dim; ++d)
            thV += fabs(W[OW_AV * np + c] - W[OW_AV * np + c - st[d]]) +
                   fabs(W[OW_AV * np + c + st[d]] - W[OW_AV * np + c]);
          if (thD > s->theta_ducros || thV > s->theta_gas || thG > s->theta_gas) fl |= 1u;   /* eq. (D.4) */
        }
        flag[c] = fl;
      }
}

/* ---------------- surface tension (Section 3.5) ---------------- */

/* Curvature of every interior cell from the mass fraction xi: one pass of the
 * binomial Gaussian kernel of eq. (3-9) (1-2-1 in each direction, /4 per
 * direction: /16 in 2D, /64 in 3D), gradients at the cell vertices from the
 * 2^D surrounding smoothed cells, unit normals n = g / (|g| + eps/dx), and
 * kappa = -div n over the cell from the vertex normals (the mean of the normals
 * on each face of the cell).  The minus sign together with grad(alpha_G) in
 * the force points the force towards the side of higher pressure for both a
 * drop and a bubble. */
static void curvature_field(const og_grid* g, const og_scheme* s, const og_pad* pd,
                            const double* W, double* kap)
{
  int dim = g->dim;
  size_t np = pd->npad;
  size_t st[3] = {1, (size_t)pd->P[0], (size_t)pd->P[0] * pd->P[1]};
  double* Hs = (double*)calloc(np, sizeof(double));
  double* nv = (double*)calloc(3 * np, sizeof(double));
  int lo[3], hi[3];
  /* smoothed indicator on the interior plus one ghost layer */
  for (int a = 0; a < 3; ++a) { lo[a] = (a < dim) ? -1 : 0; hi[a] = (a < dim) ? pd->n[a] + 1 : 1; }
  for (int k = lo[2]; k < hi[2]; ++k)
    for (int j = lo[1]; j < hi[1]; ++j)
      for (int i = lo[0]; i < hi[0]; ++i) {
        size_t c = og_pidx(pd, i, j, k);
        double acc = 0.0, wsum = 0.0;
        int r1 = dim > 0 ? 1 : 0, r2 = dim > 1 ? 1 : 0, r3 = dim > 2 ? 1 : 0;
        for (int dk = -r3; dk <= r3; ++dk)
          for (int dj = -r2; dj <= r2; ++dj)
            for (int di = -r1; di <= r1; ++di) {
              double w = (di == 0 ? 2.0 : 1.0) * (dim > 1 ? (dj == 0 ? 2.0 : 1.0) : 1.0) *
                         (dim > 2 ? (dk == 0 ? 2.0 : 1.0) : 1.0);
              size_t cc = c + di * st[0] + dj * st[1] + dk * st[2];
              acc += w * (W[OW_Y * np + cc] + W[OW_Y2 * np + cc]);
              wsum += w;
            }
        Hs[c] = acc / wsum;
      }
  /* vertex normals: vertex (i, j, k) sits at the upper corner of cell (i, j, k);
   * needed for i in [-1, n-1] in every used direction */
  double epsn = s->eps_normal / g->dx[0];
  for (int a = 0; a < 3; ++a) { lo[a] = (a < dim) ? -1 : 0; hi[a] = (a < dim) ? pd->n[a] : 1; }
  for (int k = lo[2]; k < hi[2]; ++k)
    for (int j = lo[1]; j < hi[1]; ++j)
      for (int i = lo[0]; i < hi[0]; ++i) {
        size_t c = og_pidx(pd, i, j, k);
        double gv[3] = {0, 0, 0};
        int nt = 1 << (dim - 1);
        for (int d = 0; d < dim; ++d) {
          /* sum over the 2^(D-1) cell pairs straddling the vertex along d */
          double acc = 0.0;
          for (int t = 0; t < nt; ++t) {
            size_t off = 0;
            int bit = 0;
            for (int a = 0; a < dim; ++a) {
              if (a == d) continue;
              if ((t >> bit) & 1) off += st[a];
              ++bit;
            }
            acc += Hs[c + off + st[d]] - Hs[c + off];
          }
          gv[d] = acc / (nt * g->dx[d]);
        }
        double mag = sqrt(gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2]);
        for (int d = 0; d < dim; ++d) nv[d * np + c] = gv[d] / (mag + epsn);
      }
  /* kappa = -sum_d (mean n_d on the +d face - mean n_d on the -d face) / dx_d */
  for (int k = 0; k < pd->n[2]; ++k)
    for (int j = 0; j < pd->n[1]; ++j)
      for (int i = 0; i < pd->n[0]; ++i) {
        size_t c = og_pidx(pd, i, j, k);
        int nt = 1 << (dim - 1);
        double kv = 0.0;
        for (int d = 0; d < dim; ++d) {
          double plus = 0.0, minus = 0.0;
          for (int t = 0; t < nt; ++t) {
            /* vertices of the +d face: offset 0 along d, 0 or -1 transversally;
             * vertices of the -d face: offset -1 along d */
            size_t off = 0;
            int bit = 0;
            for (int a = 0; a < dim; ++a) {
              if (a == d) continue;
              if ((t >> bit) & 1) off += st[a];
              ++bit;
            }
            /* off selects the vertex at -1 along the chosen transverse axes */
            plus += nv[d * np + c - off];
            minus += nv[d * np + c - off - st[d]];
          }
          kv += (plus - minus) / (nt * g->dx[d]);
        }
        kap[og_cidx(pd, i, j, k)] = -kv;
      }
  free(Hs);
  free(nv);
}

int og_nq(const og_grid* g, const og_eos* e)
{
  if (og_is_barotropic(e)) return g->dim + 2 + (og_ncomp(e) == 3 ? 1 : 0);
  return g->dim + og_ncomp(e) + 1;
}

/* ---------------- viscous stress and heat conduction (eq. 2-2) ---------------- */

static int has_diffusion(const og_eos* e)
{
  if (og_is_barotropic(e)) return e->mu[0] > 0.0 || e->mu[1] > 0.0 || e->mu[2] > 0.0 || e->bt_mu_vap > 0.0;
  for (int k = 0; k < og_ncomp(e); ++k)
    if (e->mu[k] > 0.0 || e->kc[k] > 0.0) return 1;
  return 0;
}

static double mix_alpha(const double* v, int ncomp, double a, double a2);

/* viscosity of a padded cell: eq. (2-8), with the vapour term in the
 * barotropic model */
static double cell_viscosity(const og_eos* e, const double* W, size_t np, size_t c)
{
  if (og_is_barotropic(e)) return og_baro_viscosity2(e, W[OW_A * np + c], W[OW_A2 * np + c], W[OW_AV * np + c]);
  return mix_alpha(e->mu, og_ncomp(e), W[OW_A * np + c], W[OW_A2 * np + c]);
}

/* a transport coefficient of a cell from its gas volume fractions: eq. (2-8)
 * without vapour, (1 - alpha_1 - alpha_2) value_L + alpha_1 value_1 +
 * alpha_2 value_2 (alpha_2 = 0 with two components) */
static double mix_alpha(const double* v, int ncomp, double a, double a2)
{
  double ac = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
  if (ncomp == 2) return (1.0 - ac) * v[0] + ac * v[1];
  double bc = a2 < 0.0 ? 0.0 : (a2 > 1.0 ? 1.0 : a2);
  double sum = ac + bc;
  if (sum > 1.0) { ac /= sum; bc /= sum; }
  return (1.0 - ac - bc) * v[0] + ac * v[1] + bc * v[2];
}

/* Stress part S(q) of the flux of eq. (2-2) through the face between the
 * padded cells c and c + st[d], second-order central: normal derivatives from
 * the two cells, transverse ones as the mean of the two cells' central
 * differences, face coefficients and face velocity as the two cells' mean.
 *   tau = mu (grad u + grad u^T - 2/3 div u I),
 *   F_rho u = -tau . n,   F_rho E = -u . tau . n - kc dT/dn. */
static void viscous_flux(const og_grid* g, const og_eos* e, const og_pad* pd, const double* W,
                         size_t c, int d, double* Fv)
{
  int dim = g->dim;
  size_t np = pd->npad;
  size_t st[3] = {1, (size_t)pd->P[0], (size_t)pd->P[0] * pd->P[1]};
  size_t R = c + st[d];
  double grad[3][3] = {{0.0}};
  for (int a = 0; a < dim; ++a) {
    const double* u = W + (size_t)(OW_U + a) * np;
    for (int b = 0; b < dim; ++b) {
      if (b == d) grad[a][b] = (u[R] - u[c]) / g->dx[d];
      else grad[a][b] = (u[c + st[b]] - u[c - st[b]] + u[R + st[b]] - u[R - st[b]]) / (4.0 * g->dx[b]);
    }
  }
  double div = 0.0;
  for (int b = 0; b < dim; ++b) div += grad[b][b];
  int nc = og_ncomp(e);
  double aL = W[OW_A * np + c], aR = W[OW_A * np + R];
  double bL = W[OW_A2 * np + c], bR = W[OW_A2 * np + R];
  double mu = 0.5 * (cell_viscosity(e, W, np, c) + cell_viscosity(e, W, np, R));
  double work = 0.0;
  for (int v = 0; v < 7; ++v) Fv[v] = 0.0;
  for (int a = 0; a < dim; ++a) {
    double tau = mu * (grad[a][d] + grad[d][a]);
    if (a == d) tau -= 2.0 / 3.0 * mu * div;
    Fv[1 + a] = -tau;
    work += 0.5 * (W[(OW_U + a) * np + c] + W[(OW_U + a) * np + R]) * tau;
  }
  /* the barotropic model has no energy equation: the stress acts on the
   * momentum only (row 1 + dim is rho xi there) */
  if (!og_is_barotropic(e)) {
    double kc = 0.5 * (mix_alpha(e->kc, nc, aL, bL) + mix_alpha(e->kc, nc, aR, bR));
    Fv[1 + dim] = -work - kc * (W[OW_T * np + R] - W[OW_T * np + c]) / g->dx[d];
  }
}

/* ---------------- right-hand side ---------------- */

typedef struct {
  og_pad pd;
  double* qp;            /* padded conserved [nq][npad] */
  double* W;             /* padded primitives [OW_N][npad] */
  unsigned short* flag;  /* padded sensor bits */
} og_work;

static int work_setup(og_work* w, const og_grid* g, const og_eos* e, const double* q, int64_t step)
{
  og_pad_init(&w->pd, g);
  int dim = g->dim, nq = og_nq(g, e);
  size_t np = w->pd.npad, nc = w->pd.ncell;
  w->qp = (double*)calloc((size_t)nq * np, sizeof(double));
  w->W = (double*)calloc((size_t)OW_N * np, sizeof(double));
  w->flag = (unsigned short*)calloc(np, sizeof(unsigned short));
  if (!w->qp || !w->W || !w->flag) { og_set_error("out of memory"); return -1; }
  for (int k = 0; k < w->pd.n[2]; ++k)
    for (int j = 0; j < w->pd.n[1]; ++j)
      for (int i = 0; i < w->pd.n[0]; ++i) {
        size_t pi = og_pidx(&w->pd, i, j, k), ci = og_cidx(&w->pd, i, j, k);
        for (int f = 0; f < nq; ++f) w->qp[f * np + pi] = q[f * nc + ci];
      }
  if (fill_ghosts(g, e, &w->pd, w->qp, step)) return -1;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (long long c = 0; c < (long long)np; ++c) {
    double qc[7], wc[OW_N];
    int anyq = 0;
    for (int f = 0; f < nq; ++f) { qc[f] = w->qp[f * np + c]; anyq |= (qc[f] != 0.0); }
    if (!anyq) { for (int f = 0; f < OW_N; ++f) w->W[f * np + c] = 0.0; continue; } /* unused corner */
    if (prim_cell(e, dim, qc, wc)) bad = 1;
    for (int f = 0; f < OW_N; ++f) w->W[f * np + c] = wc[f];
  }
  if (bad) { og_set_error("non-physical state in a cell or ghost"); return -2; }
  return 0;
}

static void work_free(og_work* w)
{
  free(w->qp); free(w->W); free(w->flag);
}

int og_rhs(const og_grid* g, const og_eos* e, const og_scheme* s, const double* q,
           int64_t step, double* r)
{
  og_work w;
  int rc = work_setup(&w, g, e, q, step);
  if (rc) { work_free(&w); return rc; }
  int dim = g->dim, nq = og_nq(g, e);
  og_pad* pd = &w.pd;
  size_t np = pd->npad, nc = pd->ncell;
  size_t st[3] = {1, (size_t)pd->P[0], (size_t)pd->P[0] * pd->P[1]};
  sensors(g, e, s, pd, w.W, w.flag);
  memset(r, 0, sizeof(double) * (size_t)nq * nc);
  int bad = 0;
  const int diffusive = has_diffusion(e);
  const int baro = og_is_barotropic(e);
  if (baro && (e->kc[0] != 0.0 || e->kc[1] != 0.0 || e->kc[2] != 0.0)) {
    work_free(&w);
    og_set_error("the barotropic model has no energy equation: no heat conduction");
    return -4;
  }
  for (int d = 0; d < dim; ++d) {
    /* faces i-1/2 for i = 0 .. n_d along d; transverse interior */
    int hi[3] = {pd->n[0], pd->n[1], pd->n[2]};
    hi[d] += 1;
    double* Fd = (double*)malloc(sizeof(double) * (size_t)nq * hi[0] * hi[1] * hi[2]);
#pragma omp parallel for collapse(2) schedule(static) reduction(| : bad)
    for (int k = 0; k < hi[2]; ++k)
      for (int j = 0; j < hi[1]; ++j)
        for (int i = 0; i < hi[0]; ++i) {
          int cc[3] = {i, j, k};
          cc[d] -= 1;   /* cell on the left of face i-1/2 */
          size_t c = og_pidx(pd, cc[0], cc[1], cc[2]);
          double Wl[4][OW_N];
          for (int m = 0; m < 4; ++m)
            for (int f = 0; f < OW_N; ++f) Wl[m][f] = w.W[f * np + c + (m - 1) * st[d]];
          int f = (w.flag[c] | w.flag[c + st[d]]) & 1;
          /* THINC eligibility of cells i and i+1 along d: bit 0 xi_1, bit 1 xi_2 */
          int fl = w.flag[c], fr = w.flag[c + st[d]];
          int sl = ((fl >> (1 + d)) & 1) | (((fl >> (4 + d)) & 1) << 1) | (((fl >> (7 + d)) & 1) << 2);
          int sr = ((fr >> (1 + d)) & 1) | (((fr >> (4 + d)) & 1) << 1) | (((fr >> (7 + d)) & 1) << 2);
          double F[7];
          if (baro ? og_face_flux_baro(e, s, dim, d, Wl, f, sl, sr, F, NULL, NULL)
                   : og_face_flux(e, s, dim, d, Wl, f, sl, sr, F, NULL, NULL))
            bad = 1;
          if (diffusive) {
            double Fv[7];
            viscous_flux(g, e, pd, w.W, c, d, Fv);
            for (int v = 0; v < nq; ++v) F[v] += Fv[v];
          }
          size_t fi = (size_t)i + (size_t)hi[0] * ((size_t)j + (size_t)hi[1] * k);
          size_t nf = (size_t)hi[0] * hi[1] * hi[2];
          for (int v = 0; v < nq; ++v) Fd[v * nf + fi] = F[v];
        }
    size_t nf = (size_t)hi[0] * hi[1] * hi[2];
    size_t fs[3] = {1, (size_t)hi[0], (size_t)hi[0] * hi[1]};
    for (int k = 0; k < pd->n[2]; ++k)
      for (int j = 0; j < pd->n[1]; ++j)
        for (int i = 0; i < pd->n[0]; ++i) {
          size_t fi = (size_t)i + (size_t)hi[0] * ((size_t)j + (size_t)hi[1] * k);
          size_t ci = og_cidx(pd, i, j, k);
          for (int v = 0; v < nq; ++v)
            r[v * nc + ci] -= (Fd[v * nf + fi + fs[d]] - Fd[v * nf + fi]) / g->dx[d];
        }
    free(Fd);
  }
  if (s->sigma > 0.0) {
    /* CSF source (eq. 2-2 with f = sigma kappa grad H): S = sigma kappa grad(alpha_G)
     * with the central gradient, S_E = u . S */
    double* kap = (double*)malloc(sizeof(double) * nc);
    curvature_field(g, s, pd, w.W, kap);
    for (int k = 0; k < pd->n[2]; ++k)
      for (int j = 0; j < pd->n[1]; ++j)
        for (int i = 0; i < pd->n[0]; ++i) {
          size_t c = og_pidx(pd, i, j, k), ci = og_cidx(pd, i, j, k);
          double se = 0.0;
          for (int d = 0; d < dim; ++d) {
            size_t cp = c + st[d], cm = c - st[d];
            double gH = (w.W[OW_A * np + cp] + w.W[OW_A2 * np + cp] - (w.W[OW_A * np + cm] + w.W[OW_A2 * np + cm])) /
                        (2.0 * g->dx[d]);
            double S = s->sigma * kap[ci] * gH;
            r[(1 + d) * nc + ci] += S;
            se += w.W[(OW_U + d) * np + c] * S;
          }
          if (!baro) r[(1 + dim) * nc + ci] += se;
        }
    free(kap);
  }
  if (s->gravity[0] != 0.0 || s->gravity[1] != 0.0 || s->gravity[2] != 0.0) {
    /* body force (eq. 2-2, source Q): rho g on the momentum, rho u . g on the energy */
    for (int k = 0; k < pd->n[2]; ++k)
      for (int j = 0; j < pd->n[1]; ++j)
        for (int i = 0; i < pd->n[0]; ++i) {
          size_t c = og_pidx(pd, i, j, k), ci = og_cidx(pd, i, j, k);
          double rho = w.W[OW_RHO * np + c], pw = 0.0;
          for (int d = 0; d < dim; ++d) {
            r[(1 + d) * nc + ci] += rho * s->gravity[d];
            pw += w.W[(OW_U + d) * np + c] * s->gravity[d];
          }
          if (!baro) r[(1 + dim) * nc + ci] += rho * pw;
        }
  }
  work_free(&w);
  if (bad) { og_set_error("face closure failed"); return -3; }
  return 0;
}

/* sensor bits of the interior cells (bit 0: discontinuous branch, bit 1+d:
 * THINC eligibility along d) */
int og_sensor_flags(const og_grid* g, const og_eos* e, const og_scheme* s, const double* q,
                    unsigned char* flags)
{
  og_work w;
  int rc = work_setup(&w, g, e, q, 0);
  if (!rc) {
    sensors(g, e, s, &w.pd, w.W, w.flag);
    for (int k = 0; k < w.pd.n[2]; ++k)
      for (int j = 0; j < w.pd.n[1]; ++j)
        for (int i = 0; i < w.pd.n[0]; ++i)
          flags[og_cidx(&w.pd, i, j, k)] = (unsigned char)(w.flag[og_pidx(&w.pd, i, j, k)] & 0xffu);
  }
  work_free(&w);
  return rc;
}

int og_curvature(const og_grid* g, const og_eos* e, const og_scheme* s, const double* q, double* kappa)
{
  og_work w;
  int rc = work_setup(&w, g, e, q, 0);
  if (!rc) curvature_field(g, s, &w.pd, w.W, kappa);
  work_free(&w);
  return rc;
}

/* ---------------- time step ---------------- */

/* dt = CFL / max over cells of [sum_d (|u_d| + c) / dx_d + 2 nu sum_d 1/dx_d^2]
 * (the paper gives no formula): the usual convective limit with the cell's
 * speed of sound, plus the explicit diffusion limit with
 * nu = max(mu, kc / cv) / rho (cv mixed by mass fraction) when the fluids
 * are viscous or conducting (barotropic model: nu = mu / rho with the mixture
 * viscosity of eq. 2-8) */
double og_dt(const og_grid* g, const og_eos* e, const og_scheme* s, const double* q)
{
  og_pad pd;
  og_pad_init(&pd, g);
  size_t nc = pd.ncell;
  int dim = g->dim, nq = og_nq(g, e);
  int diffusive = has_diffusion(e);
  double sdx2 = 0.0;
  for (int d = 0; d < dim; ++d) sdx2 += 1.0 / (g->dx[d] * g->dx[d]);
  double lam = 0.0;
  for (size_t c = 0; c < nc; ++c) {
    double qc[7], w[OW_N];
    for (int f = 0; f < nq; ++f) qc[f] = q[f * nc + c];
    if (prim_cell(e, dim, qc, w)) return NAN;
    double l = 0.0;
    for (int d = 0; d < dim; ++d) l += (fabs(w[OW_U + d]) + w[OW_C]) / g->dx[d];
    if (diffusive && og_is_barotropic(e)) {
      /* viscous limit with the mixture viscosity of eq. (2-8) */
      l += 2.0 * og_baro_viscosity2(e, w[OW_A], w[OW_A2], w[OW_AV]) / w[OW_RHO] * sdx2;
    } else if (diffusive) {
      int ncomp = og_ncomp(e);
      double cvm;
      if (ncomp == 2) {
        double Yc = og_clip_fraction(w[OW_Y]);
        cvm = (1.0 - Yc) * e->cv[0] + Yc * e->cv[1];
      } else {
        double Yk[3];
        og_clip_fractions3(w[OW_Y], w[OW_Y2], Yk);
        cvm = Yk[0] * e->cv[0] + Yk[1] * e->cv[1] + Yk[2] * e->cv[2];
      }
      double mu = mix_alpha(e->mu, ncomp, w[OW_A], w[OW_A2]);
      double kc = mix_alpha(e->kc, ncomp, w[OW_A], w[OW_A2]) / cvm;
      l += 2.0 * (mu > kc ? mu : kc) / w[OW_RHO] * sdx2;
    }
    if (l > lam) lam = l;
  }
  return s->cfl / lam;
}

/* four-stage low-storage Runge-Kutta: q^(k) = q^n + a_k dt R(q^(k-1)) */
void og_lsrk(const og_scheme* s, double* q, int n, double dt, og_rhs_fn f, void* user)
{
  double* q0 = (double*)malloc(sizeof(double) * (size_t)n);
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  memcpy(q0, q, sizeof(double) * (size_t)n);
  for (int st = 0; st < 4; ++st) {
    f(q, r, n, user);
    for (int i = 0; i < n; ++i) q[i] = q0[i] + s->rk[st] * dt * r[i];
  }
  free(q0);
  free(r);
}

typedef struct { const og_grid* g; const og_eos* e; const og_scheme* s; int64_t step; int rc; } rhs_ctx;

static void rhs_cb(const double* q, double* r, int n, void* user)
{
  (void)n;
  rhs_ctx* c = (rhs_ctx*)user;
  if (c->rc) return;
  c->rc = og_rhs(c->g, c->e, c->s, q, c->step, r);
}

int og_step(const og_grid* g, const og_eos* e, const og_scheme* s, double* q,
            int64_t step, double* t, double t_end, double* dt_out)
{
  og_pad pd;
  og_pad_init(&pd, g);
  int n = (int)((size_t)og_nq(g, e) * pd.ncell);
  double dt = og_dt(g, e, s, q);
  if (!isfinite(dt)) { og_set_error("non-physical state at the start of a step"); return -2; }
  if (t_end > 0.0 && *t + dt > t_end) dt = t_end - *t;
  if (dt < 0.0) dt = 0.0;
  rhs_ctx c = {g, e, s, step, 0};
  og_lsrk(s, q, n, dt, rhs_cb, &c);
  if (c.rc) return c.rc;
  *t += dt;
  if (dt_out) *dt_out = dt;
  return 0;
}

int og_run(const og_grid* g, const og_eos* e, const og_scheme* s, double* q,
           int64_t step0, int nsteps, double* t, double t_end)
{
  for (int it = 0; it < nsteps; ++it) {
    int rc = og_step(g, e, s, q, step0 + it, t, t_end, NULL);
    if (rc) return rc;
  }
  return 0;
}

/* conserved totals: sum over cells of q times the cell volume, fixed order */
void og_totals(const og_grid* g, const og_eos* e, const double* q, double* out)
{
  og_pad pd;
  og_pad_init(&pd, g);
  size_t nc = pd.ncell;
  int nq = og_nq(g, e);
  double vol = 1.0;
  for (int d = 0; d < g->dim; ++d) vol *= g->dx[d];
  for (int f = 0; f < nq; ++f) {
    double acc = 0.0;
    for (size_t c = 0; c < nc; ++c) acc += q[f * nc + c];
    out[f] = acc * vol;
  }
}
