// fvm_baro.hip -- gfx950 kernels of the barotropic cavitation model
// (Section 2.2, eqs. 2-3 .. 2-7): a liquid that becomes a liquid-vapour
// mixture below its saturation pressure and one isothermal ideal gas (or two:
// the G2 instances), with no energy equation; face density by TDU (eq. 3-5)
// or, across liquid-vapour interface cells, by THINC of the density
// (eqs. 3-7, 3-8, Remarks 1-2).
//
// Storage of a cell, N_q = D + 2 (D + 3 with two gases):
//   0: rho (1 - xi - xi_2) - rref_L   liquid / mixture partial density minus a reference
//   1: rho xi                          gas partial density
//   2..1+D: rho u
//   2+D: rho xi_2                      second gas partial density (two gases)
// One fused kernel per Runge-Kutta stage on 1D/2D tiles, shaped like the
// four-equation kernel: tile + two-cell halo staged in LDS after the FP64
// closure p = f(rho, xi), sensors, x and y face sweeps (with the viscous
// stress of the mixture viscosity of eq. 2-8 when the fluids are viscous),
// CSF, body force, update, and in the last stage the CFL bound of the new state.  In 3D a
// closure kernel and a face kernel, as for the four-equation model.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "fvm_device.hpp"
#include "fvm_kernels.hpp"
#include "fvm_stage_common.hpp"
#include "fvm_stage3_prim.hpp"   // k_csf_zero

namespace fvm {

// ------------------------------------------------------------------ closure
// liquid (p >= p_sat, eq. 2-3) or liquid-vapour mixture (eq. 2-4) density
template <class R>
__device__ inline R baro_liq(const CaseC& C, R p)
{
  R c2 = p >= R(C.bt_ps) ? R(C.bt_cl2) : R(C.bt_cm2);
  return R(C.bt_rs) + fdiv(p - R(C.bt_ps), c2);
}

// density at (p, xi, xi_2): 1/rho = xi R T / p + xi_2 R_2 T_2 / p + (1 - xi - xi_2) / rho_L/M(p)
template <class R>
__device__ inline R baro_rho(const CaseC& C, R p, R Y, R Y2 = R(0))
{
  R v = R(0), l = R(1) - Y - Y2;
  if (Y != R(0)) v += Y * fdiv(R(C.bt_RT), p);
  if (Y2 != R(0)) v += Y2 * fdiv(R(C.bt_RT2), p);
  if (l != R(0)) v += fdiv(l, baro_liq<R>(C, p));
  return frcp(v);
}

struct PB { double p, c, aG, aV, aG2; };

// p = f(rho, xi): (p - a) rho_L/M(p) - b p = 0 with a = rho xi R T,
// b = (1 - xi) rho; the sign at p = p_sat selects the branch of rho_L/M, on
// which the equation is the quadratic p^2 + B p + C = 0 (K = rho_sat c^2 - p_sat,
// B = K - a - b c^2, C = -a K); its positive root without cancellation.
// Also the sound speed of impedances and CFL and the volume fractions
// alpha_G (eq. 2-6) and alpha_V (eq. 2-7, at most 0.995).
__device__ inline PB baro_closure(const CaseC& C, double rho, double Y, double Y2 = 0.0)
{
  // the gas fractions clipped to [0, 1] and rescaled where they sum above one;
  // with two gases a = rho (xi R T + xi_2 R_2 T_2), b = (1 - xi - xi_2) rho
  double y0, y1, y2;
  clip_fractions3(Y, Y2, y0, y1, y2);
  double a = rho * (y1 * C.bt_RT + y2 * C.bt_RT2), b = y0 * rho;
  double ps = C.bt_ps, rs = C.bt_rs;
  bool liq = (ps - a) * rs - b * ps <= 0.0;
  double c2 = liq ? C.bt_cl2 : C.bt_cm2;
  double K = rs * c2 - ps;
  double B = K - a - b * c2, Cc = -a * K;
  double s = sqrt(B * B - 4.0 * Cc);
  PB r;
  r.p = (B <= 0.0) ? 0.5 * (-B + s) : (-2.0 * Cc) / (B + s);
  r.c = (r.p >= ps) ? C.bt_c_hi : C.bt_c_lo;
  r.aG = (y1 == 0.0) ? 0.0 : rho * y1 * C.bt_RT / r.p;
  r.aG2 = (y2 == 0.0) ? 0.0 : rho * y2 * C.bt_RT2 / r.p;
  double rM = baro_liq<double>(C, r.p);
  double aV = (rM < rs) ? (1.0 - r.aG - r.aG2) * (rs - rM) / (rs - C.bt_rv) : 0.0;
  r.aV = aV > 0.995 ? 0.995 : (aV < 0.0 ? 0.0 : aV);
  return r;
}

// partial densities and momentum of a cell from (p, alpha_G, u[, alpha_G2]);
// G2: the second gas's partial density at q[2 + D]
template <int D, bool G2 = false>
__device__ inline void baro_from_prim(const CaseC& C, double p, double al, const double* u, double* q,
                                      double al2 = 0.0)
{
  double rG = p / C.bt_RT, rL = baro_liq<double>(C, p);
  q[0] = (1.0 - al - al2) * rL;
  q[1] = al * rG;
  double rho = q[0] + q[1];
  if constexpr (G2) {
    q[2 + D] = al2 * (p / C.bt_RT2);
    rho += q[2 + D];
  }
#pragma unroll
  for (int d = 0; d < D; ++d) q[2 + d] = rho * u[d];
}

// load one (possibly ghost) cell: physical partial densities and momentum
// (far-field and inflow states hold no second gas)
template <class S, int D, bool G2 = false>
__device__ inline void baro_load(const CaseC& C, const S* __restrict__ src, long long total, int gx, int gy,
                                 long long step, double* q)
{
  if (beyond_farfield<D>(C, gx, gy, 0)) {
    const double u0[3] = {0.0, 0.0, 0.0};
    baro_from_prim<D, G2>(C, C.ff_p, C.ff_alpha, u0, q);
    return;
  }
  bool fx = false, fy = false;
  int ix = gx, iy = gy;
  if (D >= 2) map_index(iy, C.n[1], C.bc[1][0], C.bc[1][1], fy);
  if (ix < 0 && C.bc[0][0] == BC_INFLOW) {
    double yy = (D >= 2) ? (iy + 0.5) * C.dx[1] - C.in_c0 : 0.0;
    if (D == 1 || fabs(yy) < C.in_radius) {
      double u[3] = {C.in_u, 0.0, 0.0};
      for (int c = 0; c < D; ++c)
        u[c] += C.in_noise * C.in_u *
                (2.0 * noise01(C.in_seed, (unsigned long long)step, (unsigned long long)iy, 0ull,
                               (unsigned long long)c) - 1.0);
      baro_from_prim<D, G2>(C, C.in_p, C.in_alpha, u, q);
      if (D >= 2 && fy) q[3] = -q[3];
      return;
    }
    ix = -1 - ix;
    fx = true;
  } else {
    map_index(ix, C.n[0], C.bc[0][0], C.bc[0][1], fx);
  }
  long long cell = C.off + ix + (long long)C.n[0] * iy;
  q[0] = (double)src[cell] + C.rref[0];
  q[1] = (double)src[total + cell];
#pragma unroll
  for (int d = 0; d < D; ++d) q[2 + d] = (double)src[(2 + d) * total + cell];
  if constexpr (G2) q[2 + D] = (double)src[(2 + D) * total + cell];
  if (fx) q[2] = -q[2];
  if (D >= 2 && fy) q[3] = -q[3];
}

// primitives of a loaded cell (G2: xi_2 from q[2 + D])
template <int D, bool G2 = false>
__device__ inline PB baro_prim(const CaseC& C, const double* q, double* u, double& rho, double& Y,
                               double& Y2)
{
  rho = q[0] + q[1];
  if constexpr (G2) rho += q[2 + D];
  double ir = 1.0 / rho;
  Y = q[1] * ir;
  Y2 = G2 ? q[2 + D] * ir : 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) u[d] = q[2 + d] * ir;
  return baro_closure(C, rho, Y, Y2);
}

template <int D>
__device__ inline PB baro_prim(const CaseC& C, const double* q, double* u, double& rho, double& Y)
{
  double Y2;
  return baro_prim<D, false>(C, q, u, rho, Y, Y2);
}

// ------------------------------------------------------------------ face flux
template <class R, int D>
struct BStencil {
  R u[D][4];
  R p[4], Y[4], r[4];
  R Y2[4];   // second gas fraction (two gases only)
  R c1, c2;
};

// One face between stencil cells 1 and 2 (Section 3.2/3.3, Appendix D, Section
// 3.4): impedances and p*, u* as in the four-equation model; xi limited, by
// THINC where the upwind cell is a gas interface cell (bit 0 of its
// eligibility), second-order central in the smooth branch; the face gas
// fraction taken in [0, 1]; face density rho(p*, xi_f) (TDU, eq. 3-5), or the
// THINC value of rho where the upwind cell is a liquid-vapour interface cell
// (bit 1); storage flux (m (1 - xi_f), m xi_f, m u_f + p* n), m = rho_f u*.
// A face with p* <= 0 has no density: its flux is NaN, which the closure of
// the updated cells reports.
template <class R, int D, int DIR, int LIM, bool G2 = false>
__device__ inline void baro_face(const SchemeC& S, const CaseC& C, const BStencil<R, D>& s, bool disc, int el,
                                 int er, R* F)
{
  const int lu = LIM ? int(LIM_KOREN) : S.lim_u;   // LIM = 1: the default limiters fixed
  const int ls = LIM ? int(LIM_MINMOD) : S.lim_s;
  R cm = fmax(s.c1, s.c2);
  R IL = (R(3) * s.r[1] + s.r[2]) * cm * R(0.25);
  R IR = (s.r[1] + R(3) * s.r[2]) * cm * R(0.25);
  R iI = frcp((s.r[1] + s.r[2]) * cm);
  R uf[D];
  R us, ps, Yf, Yf2 = R(0);
  bool left = true, lv = false;
  if (disc) {
    R uL[D], uR[D];
#pragma unroll
    for (int d = 0; d < D; ++d) recon<R>(lu, s.u[d][0], s.u[d][1], s.u[d][2], s.u[d][3], uL[d], uR[d]);
    R pL, pR, YL, YR, Y2L = R(0), Y2R = R(0);
    recon<R>(ls, s.p[0], s.p[1], s.p[2], s.p[3], pL, pR);
    recon<R>(ls, s.Y[0], s.Y[1], s.Y[2], s.Y[3], YL, YR);
    if constexpr (G2) recon<R>(ls, s.Y2[0], s.Y2[1], s.Y2[2], s.Y2[3], Y2L, Y2R);
    ps = R(0.5) * (pL + pR);
    us = (IL * uL[DIR] + IR * uR[DIR] + pL - pR) * iI;
    left = us >= R(0);
#pragma unroll
    for (int d = 0; d < D; ++d) uf[d] = left ? uL[d] : uR[d];
    Yf = left ? YL : YR;
    int eb = left ? el : er;
    if (S.thinc && (eb & 1))
      Yf = thinc_value<R>(S, left, left ? s.Y[0] : s.Y[1], left ? s.Y[1] : s.Y[2], left ? s.Y[2] : s.Y[3]);
    if constexpr (G2) {
      // the second gas fraction on its own, THINC where the upwind cell is one
      // of its interface cells (bit 2)
      Yf2 = left ? Y2L : Y2R;
      if (S.thinc && (eb & 4))
        Yf2 = thinc_value<R>(S, left, left ? s.Y2[0] : s.Y2[1], left ? s.Y2[1] : s.Y2[2], left ? s.Y2[2] : s.Y2[3]);
    }
    lv = S.thinc && (eb & 2);
  } else {
    const R c12 = R(1.0 / 12.0);
#pragma unroll
    for (int d = 0; d < D; ++d)
      uf[d] = (R(7) * (s.u[d][1] + s.u[d][2]) - s.u[d][0] - s.u[d][3]) * c12;
    ps = (R(7) * (s.p[1] + s.p[2]) - s.p[0] - s.p[3]) * c12;
    R d3p = s.p[3] - R(3) * s.p[2] + R(3) * s.p[1] - s.p[0];
    us = uf[DIR] + R(S.k3) * d3p * iI;
    Yf = R(0.5) * (s.Y[1] + s.Y[2]);
    if constexpr (G2) Yf2 = R(0.5) * (s.Y2[1] + s.Y2[2]);
  }
  // face gas fractions in [0, 1], two of them rescaled where they sum above one
  Yf = fmin(fmax(Yf, R(0)), R(1));
  if constexpr (G2) {
    Yf2 = fmin(fmax(Yf2, R(0)), R(1));
    R sum = Yf + Yf2;
    if (sum > R(1)) {
      R is = frcp(sum);
      Yf *= is;
      Yf2 *= is;
    }
  }
  R rf;
  if (lv) rf = thinc_value<R>(S, left, left ? s.r[0] : s.r[1], left ? s.r[1] : s.r[2], left ? s.r[2] : s.r[3]);
  else rf = baro_rho<R>(C, ps, Yf, Yf2);
  if (!(ps > R(0))) rf = R(__builtin_nan(""));
  R m = rf * us;
  F[0] = m * (R(1) - Yf - Yf2);
  F[1] = m * Yf;
#pragma unroll
  for (int d = 0; d < D; ++d) F[2 + d] = m * uf[d] + (d == DIR ? ps : R(0));
  if constexpr (G2) F[2 + D] = m * Yf2;
}

// THINC eligibility bits of the middle cell of (a, b, c): bit 0 gas fraction,
// bit 1 liquid-vapour interface (vapour fraction and density both monotone)
template <class R>
__device__ inline int baro_elig(R Ya, R Yb, R Yc, R va, R vb, R vc, R ra, R rb, R rc, R eps)
{
  int e = eligible<R>(Ya, Yb, Yc, eps) ? 1 : 0;
  if (eligible<R>(va, vb, vc, eps) && (rb - ra) * (rc - rb) > R(0)) e |= 2;
  return e;
}

// mixture viscosity of eq. 2-8,
// (1 - aG - aG2)[(1 - a_v)(1 + 5/2 a_v) mu_L + a_v mu_V] + aG mu_G + aG2 mu_G2: the
// bracket is the viscosity of the liquid-vapour part, so a_v = aV / (1 - aG - aG2)
// is the vapour share of that part (aV of eq. 2-7 is a share of the whole cell)
template <class R>
__device__ inline R baro_mu(const CaseC& C, R aG, R aV, R aG2 = R(0))
{
  R g = fmin(fmax(aG, R(0)), R(1));
  R g2 = fmin(fmax(aG2, R(0)), R(1));
  R sum = g + g2;
  if (sum > R(1)) {
    g = fdiv(g, sum);
    g2 = fdiv(g2, sum);
  }
  R m = fmax(R(1) - g - g2, R(0));
  R av = m > R(0) ? fmin(fmax(fdiv(aV, m), R(0)), R(1)) : R(0);
  return m * ((R(1) - av) * (R(1) + R(2.5) * av) * R(C.bt_mu_l) + av * R(C.bt_mu_v)) + g * R(C.bt_mu_g) +
         g2 * R(C.bt_mu_g2);
}

// Stress part of the momentum flux through the face between the LDS cells c
// and c + st[DIR] (eq. 2-2; the model has no energy equation): second-order
// central, normal derivatives from the two cells, transverse ones as the
// mean of the two cells' central differences, face viscosity the mean of the
// two cells' eq. 2-8 values.  tau = mu (grad u + grad u^T - 2/3 div u I),
// F_rho u -= tau . n.  U[a]: velocity component a; sA, sV: alpha_G, alpha_V.
template <class S, int D, int DIR>
__device__ inline void baro_visc(const CaseC& C, const S* const (&U)[D], const S* sA, const S* sV, int c,
                                 const int (&st)[D], S* F, const S* sA2 = nullptr)
{
  const int r = c + st[DIR];
  S g[D][D];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int b = 0; b < D; ++b) {
      if (b == DIR) g[a][b] = (U[a][r] - U[a][c]) * S(C.idx[DIR]);
      else g[a][b] = (U[a][c + st[b]] - U[a][c - st[b]] + U[a][r + st[b]] - U[a][r - st[b]]) * S(0.25 * C.idx[b]);
    }
  S div = S(0);
#pragma unroll
  for (int b = 0; b < D; ++b) div += g[b][b];
  const S mu = sA2 ? S(0.5) * (baro_mu<S>(C, sA[c], sV[c], sA2[c]) + baro_mu<S>(C, sA[r], sV[r], sA2[r]))
                   : S(0.5) * (baro_mu<S>(C, sA[c], sV[c]) + baro_mu<S>(C, sA[r], sV[r]));
#pragma unroll
  for (int a = 0; a < D; ++a) {
    S tau = mu * (g[a][DIR] + g[DIR][a]);
    if (a == DIR) tau -= S(2.0 / 3.0) * mu * div;
    F[2 + a] -= tau;
  }
}

// CFL rate of a cell: sum_d (|u_d| + c) / dx_d, plus 2 mu / rho sum_d 1/dx_d^2
// for a viscous mixture (explicit diffusion limit, mu of eq. 2-8)
template <int D>
__device__ inline double baro_cfl(const CaseC& C, const double* u, const PB& pb, double rho)
{
  double l = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) l += (fabs(u[d]) + pb.c) * C.idx[d];
  if (C.diff) l += 2.0 * baro_mu<double>(C, pb.aG, pb.aV, pb.aG2) / rho * C.sdx2;
  return l;
}

// ------------------------------------------------------------------ fused 1D/2D stage
template <class S, int D, int TX, int TY, int NT, int MINW, int LIM, bool G2>
__global__ __launch_bounds__(NT, MINW) void k_baro12(StageArgs a)
{
  static_assert(D == 1 || D == 2, "1D/2D kernel");
  static_assert(D == 2 || TY == 1, "1D tiles are one row");
  constexpr int HX = TX + 4, HY = (D == 2) ? TY + 4 : 1, NH = HX * HY;
  constexpr int NQ = D + 2 + (G2 ? 1 : 0);   // G2: a second gas, its partial density last
  constexpr int NC = TX * TY;
  constexpr int CPT = (NC + NT - 1) / NT;
  constexpr int NIT = (NH + NT - 1) / NT;
  constexpr int NFX = (TX + 1) * TY, NFY = (D == 2) ? TX * (TY + 1) : 0;
  constexpr int NF = NFX > NFY ? NFX : NFY;
  constexpr int OY = (D == 2) ? 2 : 0;
  constexpr int FX = TX + 2, FY = (D == 2) ? TY + 2 : 1;
  constexpr int VX = TX + 1, VY = (D == 2) ? TY + 1 : 1;
  static_assert(FX * FY + D * VX * VY <= NQ * NF, "CSF scratch fits in the flux buffer");

  __shared__ S s_rho[NH], s_u[NH], s_v[D == 2 ? NH : 1], s_p[NH], s_Y[NH], s_c[NH], s_a[NH], s_av[NH];
  __shared__ S s_Y2[G2 ? NH : 1], s_a2[G2 ? NH : 1];
  __shared__ unsigned char s_fl[NH];
  __shared__ S s_F[NQ][NF];
  __shared__ double s_red[NT / 64];

  const int4 tl = a.tiles[xcd_block(blockIdx.x, gridDim.x)];
  const CaseC& C = a.cases[tl.x];
  CaseDyn& dy = a.dyn[tl.x];
  const SchemeC& SC = a.sc;
  const int x0 = tl.y * TX, y0 = tl.z * TY;
  const int tid = threadIdx.x;
  const bool upd = a.stage >= 0;
  const long long step = upd ? dy.base + a.step_off : a.rhs_step;
  const S* __restrict__ src = (const S*)a.src;
  const long long T = a.total;

  S qn_reg[CPT][NQ];
  if (upd) {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      int cc = tid + k * NT;
      int gx = x0 + cc % TX, gy = y0 + cc / TX;
      bool own = cc < NC && gx < C.n[0] && (D == 1 || gy < C.n[1]);
      long long cell = C.off + (own ? gx + (long long)C.n[0] * gy : 0);
#pragma unroll
      for (int v = 0; v < NQ; ++v) qn_reg[k][v] = ((const S*)a.qn)[v * T + cell];
    }
  }

  // ---- tile + halo: loads, FP64 closure, primitives to LDS
  {
    double qv[NIT][NQ];
    if (halo_inside12<S, D>(C, x0, y0, TX, TY)) {
      // no ghost cell: straight loads at 32-bit byte offsets from the rows' bases
      const char* base[NQ];
#pragma unroll
      for (int v = 0; v < NQ; ++v) base[v] = (const char*)(src + v * T + C.off);
      const unsigned n0 = (unsigned)C.n[0];
      const unsigned org = (unsigned)(x0 - 2) + (D == 2 ? n0 * (unsigned)(y0 - 2) : 0u);
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        int h = tid + it * NT;
        if (h < NH) {
          const unsigned hx = h % HX, hy = h / HX;
          const unsigned off = (org + hx + n0 * hy) * (unsigned)sizeof(S);
#pragma unroll
          for (int v = 0; v < NQ; ++v) qv[it][v] = (double)*(const S*)(base[v] + off);
          qv[it][0] += C.rref[0];
        }
      }
    } else {
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        int h = tid + it * NT;
        if (h < NH) {
          int hx = h % HX, hy = h / HX;
          baro_load<S, D, G2>(C, src, T, x0 + hx - 2, (D == 2) ? y0 + hy - 2 : 0, step, qv[it]);
        }
      }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      int h = tid + it * NT;
      if (h < NH) {
        double u[D], rho, Y, Y2;
        PB pb = baro_prim<D, G2>(C, qv[it], u, rho, Y, Y2);
        s_rho[h] = S(rho);
        s_u[h] = S(u[0]);
        if (D == 2) s_v[h] = S(u[D - 1]);
        s_p[h] = S(pb.p);
        s_Y[h] = S(Y);
        s_c[h] = S(pb.c);
        s_a[h] = S(pb.aG);
        s_av[h] = S(pb.aV);
        if constexpr (G2) {
          s_Y2[h] = S(Y2);
          s_a2[h] = S(pb.aG2);
        }
      }
    }
  }
  __syncthreads();
  // total gas volume fraction and mass fraction of a staged cell
  auto aG = [&](int c) -> S {
    if constexpr (G2) return s_a[c] + s_a2[c];
    else return s_a[c];
  };
  auto YG = [&](int c) -> S {
    if constexpr (G2) return s_Y[c] + s_Y2[c];
    else return s_Y[c];
  };

  // ---- switching sensors (Appendix D: Ducros, gas and vapour volume fractions)
  if (SC.switching) {
    for (int h = tid; h < FX * FY; h += NT) {
      int lx = h % FX, ly = h / FX;
      int c = (ly + (D == 2 ? 1 : 0)) * HX + lx + 1;
      S idx2 = S(0.5 * C.idx[0]);
      S div = (s_u[c + 1] - s_u[c - 1]) * idx2, curl2 = S(0);
      S thg = fabs(aG(c) - aG(c - 1)) + fabs(aG(c + 1) - aG(c));
      S thv = fabs(s_av[c] - s_av[c - 1]) + fabs(s_av[c + 1] - s_av[c]);
      if (D == 2) {
        S idy2 = S(0.5 * C.idx[1]);
        S dvdy = (s_v[c + HX] - s_v[c - HX]) * idy2;
        S dvdx = (s_v[c + 1] - s_v[c - 1]) * idx2;
        S dudy = (s_u[c + HX] - s_u[c - HX]) * idy2;
        div += dvdy;
        S w = dvdx - dudy;
        curl2 = w * w;
        thg += fabs(aG(c) - aG(c - HX)) + fabs(aG(c + HX) - aG(c));
        thv += fabs(s_av[c] - s_av[c - HX]) + fabs(s_av[c + HX] - s_av[c]);
      }
      S thd = fdiv(div * div, div * div + curl2 + S(SC.eps_d));
      s_fl[c] = (thd > S(SC.th_d) || thv > S(SC.th_g) || thg > S(SC.th_g)) ? 1 : 0;
    }
    __syncthreads();
  }

  S R[CPT][NQ];
#pragma unroll
  for (int k = 0; k < CPT; ++k)
#pragma unroll
    for (int v = 0; v < NQ; ++v) R[k][v] = S(0);

  const S eps = S(SC.eps_int);
  // velocity arrays and LDS strides for the stress terms
  const S* U[D];
  int stv[D];
  U[0] = s_u;
  stv[0] = 1;
  if constexpr (D == 2) { U[1] = s_v; stv[1] = HX; }
  // stencil of the face between LDS cells c and c + st (cells c - st .. c + 2 st)
  auto stencil = [&](int c, int st, BStencil<S, D>& bs, int& el, int& er) {
    S av[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      int cm = c + (m - 1) * st;
      bs.u[0][m] = s_u[cm];
      if (D == 2) bs.u[D - 1][m] = s_v[cm];
      bs.p[m] = s_p[cm];
      bs.Y[m] = s_Y[cm];
      bs.r[m] = s_rho[cm];
      av[m] = s_av[cm];
      if constexpr (G2) bs.Y2[m] = s_Y2[cm];
    }
    bs.c1 = s_c[c];
    bs.c2 = s_c[c + st];
    el = baro_elig<S>(bs.Y[0], bs.Y[1], bs.Y[2], av[0], av[1], av[2], bs.r[0], bs.r[1], bs.r[2], eps);
    er = baro_elig<S>(bs.Y[1], bs.Y[2], bs.Y[3], av[1], av[2], av[3], bs.r[1], bs.r[2], bs.r[3], eps);
    if constexpr (G2) {
      // bit 2: interface cell of the second gas
      if (eligible<S>(bs.Y2[0], bs.Y2[1], bs.Y2[2], eps)) el |= 4;
      if (eligible<S>(bs.Y2[1], bs.Y2[2], bs.Y2[3], eps)) er |= 4;
    }
  };
  auto xface = [&](int f) {
    int i = f % (TX + 1), j = f / (TX + 1);
    int c = (j + OY) * HX + i + 1;
    BStencil<S, D> bs;
    int el, er;
    stencil(c, 1, bs, el, er);
    bool disc = !SC.switching || ((s_fl[c] | s_fl[c + 1]) != 0);
    S F[NQ];
    baro_face<S, D, 0, LIM, G2>(SC, C, bs, disc, el, er, F);
    if (C.diff) baro_visc<S, D, 0>(C, U, s_a, s_av, c, stv, F, G2 ? s_a2 : nullptr);
#pragma unroll
    for (int v = 0; v < NQ; ++v) s_F[v][f] = F[v];
  };
  for_faces<NFX, NT>(tid, xface);
  __syncthreads();
  {
    S ix = S(C.idx[0]);
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      int cc = tid + k * NT;
      if (cc < NC) {
        int f = (cc / TX) * (TX + 1) + cc % TX;
#pragma unroll
        for (int v = 0; v < NQ; ++v) R[k][v] += (s_F[v][f] - s_F[v][f + 1]) * ix;
      }
    }
  }
  if (D == 2) {
    __syncthreads();
    auto yface = [&](int f) {
      int i = f % TX, j = f / TX;
      int c = (j + 1) * HX + i + 2;
      BStencil<S, D> bs;
      int el, er;
      stencil(c, HX, bs, el, er);
      bool disc = !SC.switching || ((s_fl[c] | s_fl[c + HX]) != 0);
      S F[NQ];
      baro_face<S, D, D - 1, LIM, G2>(SC, C, bs, disc, el, er, F);
      if (C.diff) baro_visc<S, D, D - 1>(C, U, s_a, s_av, c, stv, F, G2 ? s_a2 : nullptr);
#pragma unroll
      for (int v = 0; v < NQ; ++v) s_F[v][f] = F[v];
    };
    for_faces<NFY, NT>(tid, yface);
    __syncthreads();
    S iy = S(C.idx[D - 1]);
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      int cc = tid + k * NT;
      if (cc < NC) {
        int f = cc;
#pragma unroll
        for (int v = 0; v < NQ; ++v) R[k][v] += (s_F[v][f] - s_F[v][f + TX]) * iy;
      }
    }
  }

  // ---- CSF (Section 3.5): kappa from the Gaussian-smoothed xi, force sigma kappa grad(alpha_G)
  if (SC.sigma > 0.0) {
    __syncthreads();
    S* s_H = &s_F[0][0];
    S* s_nx = s_H + FX * FY;
    S* s_ny = s_nx + VX * VY;
    for (int h = tid; h < FX * FY; h += NT) {
      int lx = h % FX, ly = h / FX;
      int c = (ly + (D == 2 ? 1 : 0)) * HX + lx + 1;
      S acc;
      if (D == 1) {
        acc = (YG(c - 1) + S(2) * YG(c) + YG(c + 1)) * S(0.25);
      } else {
        S r0 = YG(c - HX - 1) + S(2) * YG(c - HX) + YG(c - HX + 1);
        S r1 = YG(c - 1) + S(2) * YG(c) + YG(c + 1);
        S r2 = YG(c + HX - 1) + S(2) * YG(c + HX) + YG(c + HX + 1);
        acc = (r0 + S(2) * r1 + r2) * S(1.0 / 16.0);
      }
      s_H[h] = acc;
    }
    __syncthreads();
    S en = S(SC.eps_n * C.idx[0]);
    for (int h = tid; h < VX * VY; h += NT) {
      int vx = h % VX, vy = h / VX;
      int c = vy * FX + vx;
      S gx, gy = S(0);
      if (D == 1) {
        gx = (s_H[c + 1] - s_H[c]) * S(C.idx[0]);
      } else {
        gx = (s_H[c + 1] + s_H[c + FX + 1] - s_H[c] - s_H[c + FX]) * S(0.5 * C.idx[0]);
        gy = (s_H[c + FX] + s_H[c + FX + 1] - s_H[c] - s_H[c + 1]) * S(0.5 * C.idx[1]);
      }
      S inv = frcp(sqrt(gx * gx + gy * gy) + en);
      s_nx[h] = gx * inv;
      if (D == 2) s_ny[h] = gy * inv;
    }
    __syncthreads();
    S sig = S(SC.sigma);
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      int cc = tid + k * NT;
      if (cc < NC) {
        int i = cc % TX, j = cc / TX;
        int c = (j + OY) * HX + i + 2;
        if (D == 1) {
          S kap = -(s_nx[i + 1] - s_nx[i]) * S(C.idx[0]);
          R[k][2] += sig * kap * (aG(c + 1) - aG(c - 1)) * S(0.5 * C.idx[0]);
        } else {
          int v = (j + 1) * VX + (i + 1);
          S dnx = s_nx[v] + s_nx[v - VX] - s_nx[v - 1] - s_nx[v - VX - 1];
          S dny = s_ny[v] + s_ny[v - 1] - s_ny[v - VX] - s_ny[v - VX - 1];
          S kap = -(dnx * S(0.5 * C.idx[0]) + dny * S(0.5 * C.idx[1]));
          R[k][2] += sig * kap * (aG(c + 1) - aG(c - 1)) * S(0.5 * C.idx[0]);
          R[k][3] += sig * kap * (aG(c + HX) - aG(c - HX)) * S(0.5 * C.idx[1]);
        }
      }
    }
  }

  // ---- body force (eq. 2-2, source Q): rho g on the momentum
  if (SC.has_grav) {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      int cc = tid + k * NT;
      if (cc < NC) {
        int c = (cc / TX + OY) * HX + cc % TX + 2;
#pragma unroll
        for (int d = 0; d < D; ++d) R[k][2 + d] += s_rho[c] * S(SC.grav[d]);
      }
    }
  }

  // ---- output
  if (!upd) {
    // right-hand side in the conserved variables (rho, rho u, rho xi), FP64
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      int cc = tid + k * NT;
      int i = cc % TX, j = cc / TX;
      int gx = x0 + i, gy = y0 + j;
      if (cc < NC && gx < C.n[0] && (D == 1 || gy < C.n[1])) {
        const long long RS = C.ncell;
        long long cell = gx + (long long)C.n[0] * gy;
        double r0 = (double)R[k][0], r1 = (double)R[k][1];
        double r2 = G2 ? (double)R[k][NQ - 1] : 0.0;
        a.rhs_out[cell] = G2 ? r0 + r1 + r2 : r0 + r1;
#pragma unroll
        for (int d = 0; d < D; ++d) a.rhs_out[(1 + d) * RS + cell] = (double)R[k][2 + d];
        a.rhs_out[(1 + D) * RS + cell] = r1;
        if constexpr (G2) a.rhs_out[(2 + D) * RS + cell] = r2;
      }
    }
    return;
  }
  const double dt = step_dt(dy, step, SC.cfl, SC.t_end);
  if (a.stage == 0 && tl.y == 0 && tl.z == 0 && tl.w == 0 && tid == 0) step_scalars(dy, step, dt);
  S* dst = (S*)a.dst;
  const S adt = S(a.ak * dt);
  double lam = 0.0;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    int cc = tid + k * NT;
    int i = cc % TX, j = cc / TX;
    int gx = x0 + i, gy = y0 + j;
    if (cc < NC && gx < C.n[0] && (D == 1 || gy < C.n[1])) {
      long long cell = C.off + gx + (long long)C.n[0] * gy;
      S nv[NQ];
#pragma unroll
      for (int v = 0; v < NQ; ++v) {
        nv[v] = qn_reg[k][v] + adt * R[k][v];
        dst[v * T + cell] = nv[v];
      }
      if (a.stage == 3) {
        double q[NQ], u[D], rho, Y, Y2;
        q[0] = (double)nv[0] + C.rref[0];
#pragma unroll
        for (int v = 1; v < NQ; ++v) q[v] = (double)nv[v];
        PB pb = baro_prim<D, G2>(C, q, u, rho, Y, Y2);
        double l = baro_cfl<D>(C, u, pb, rho);
        if (!isfinite(l) || !isfinite(pb.p)) record_error(dy, ERR_NAN, cell - C.off, step);
        else if (!(rho > 0.0) || !(pb.p > 0.0)) record_error(dy, ERR_NONPHYS, cell - C.off, step);
        else lam = fmax(lam, l);
      }
    }
  }
  if (a.stage == 3) {
    lam = wave_max(lam);
    if ((tid & 63) == 0) s_red[tid >> 6] = lam;
    __syncthreads();
    if (tid == 0) {
      double m = s_red[0];
      for (int w = 1; w < NT / 64; ++w) m = fmax(m, s_red[w]);
      cfl_max(dy, (int)((step + 1) & 1), m);
    }
  }
}

// ------------------------------------------------------------------ per-cell kernels of one case
// G2 (two gases): alpha_G2 follows u in the primitive input, rho xi_2 is the
// last storage field
template <class S, int D, bool G2>
__global__ void k_baro_prim_to_state(const CaseC* cases, int icase, const double* __restrict__ prim,
                                     S* __restrict__ dst, long long total)
{
  constexpr int NQ = D + 2 + (G2 ? 1 : 0);
  const CaseC& C = cases[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= C.ncell) return;
  double u[3] = {0, 0, 0}, q[NQ];
  for (int d = 0; d < D; ++d) u[d] = prim[(3 + d) * C.ncell + c];
  double al2 = G2 ? prim[(3 + D) * C.ncell + c] : 0.0;
  baro_from_prim<D, G2>(C, prim[c], prim[2 * C.ncell + c], u, q, al2);
  long long g = C.off + c;
  dst[g] = S(q[0] - C.rref[0]);
  for (int v = 1; v < NQ; ++v) dst[v * total + g] = S(q[v]);
}

template <class S, int D, bool G2>
__global__ void k_baro_cons_to_state(const CaseC* cases, int icase, const double* __restrict__ qin,
                                     S* __restrict__ dst, long long total)
{
  const CaseC& C = cases[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= C.ncell) return;
  long long n = C.ncell, g = C.off + c;
  double rY = qin[(1 + D) * n + c];
  double rY2 = G2 ? qin[(2 + D) * n + c] : 0.0;
  dst[g] = S(qin[c] - rY - rY2 - C.rref[0]);
  dst[total + g] = S(rY);
  for (int d = 0; d < D; ++d) dst[(2 + d) * total + g] = S(qin[(1 + d) * n + c]);
  if constexpr (G2) dst[(2 + D) * total + g] = S(rY2);
}

template <class S, int D, bool G2>
__global__ void k_baro_state_to_cons(const CaseC* cases, int icase, const S* __restrict__ src,
                                     double* __restrict__ qout, long long total)
{
  const CaseC& C = cases[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= C.ncell) return;
  long long n = C.ncell, g = C.off + c;
  double rL = (double)src[g] + C.rref[0], rG = (double)src[total + g];
  double rG2 = G2 ? (double)src[(2 + D) * total + g] : 0.0;
  qout[c] = G2 ? rL + rG + rG2 : rL + rG;
  for (int d = 0; d < D; ++d) qout[(1 + d) * n + c] = (double)src[(2 + d) * total + g];
  qout[(1 + D) * n + c] = rG;
  if constexpr (G2) qout[(2 + D) * n + c] = rG2;
}

template <class S, int D, bool G2 = false>
__device__ inline void baro_own(const CaseC& C, const S* __restrict__ src, long long total, long long g, double* q)
{
  q[0] = (double)src[g] + C.rref[0];
  for (int v = 1; v < D + 2 + (G2 ? 1 : 0); ++v) q[v] = (double)src[v * total + g];
}

// primitive rows: rho, u, v, w, p, T (0), xi, c, alpha_G, xi_2, alpha_G2 (0 with one gas), alpha_V
template <class S, int D, bool G2>
__global__ void k_baro_state_to_prim(const CaseC* cases, int icase, const S* __restrict__ src,
                                     double* __restrict__ w, long long total)
{
  const CaseC& C = cases[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= C.ncell) return;
  long long n = C.ncell, g = C.off + c;
  double q[D + 3], u[D], rho, Y, Y2;
  baro_own<S, D, G2>(C, src, total, g, q);
  PB pb = baro_prim<D, G2>(C, q, u, rho, Y, Y2);
  w[c] = rho;
  for (int d = 0; d < 3; ++d) w[(1 + d) * n + c] = d < D ? u[d] : 0.0;
  w[4 * n + c] = pb.p;
  w[5 * n + c] = 0.0;
  w[6 * n + c] = Y;
  w[7 * n + c] = pb.c;
  w[8 * n + c] = pb.aG;
  w[9 * n + c] = Y2;
  w[10 * n + c] = pb.aG2;
  w[11 * n + c] = pb.aV;
}

template <class S, int D, bool G2>
__global__ __launch_bounds__(256) void k_baro_dt_init(const CaseC* cases, CaseDyn* dyn, int icase,
                                                      const S* __restrict__ src, long long total,
                                                      long long label_off)
{
  __shared__ double s_red[4];
  const CaseC& C = cases[icase];
  CaseDyn& dy = dyn[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double lam = 0.0;
  if (c < C.ncell) {
    double q[D + 3], u[D], rho, Y, Y2;
    baro_own<S, D, G2>(C, src, total, C.off + c, q);
    PB pb = baro_prim<D, G2>(C, q, u, rho, Y, Y2);
    double l = baro_cfl<D>(C, u, pb, rho);
    if (!isfinite(l) || !isfinite(pb.p)) record_error(dy, ERR_NAN, c, dy.base + label_off);
    else if (!(rho > 0.0) || !(pb.p > 0.0)) record_error(dy, ERR_NONPHYS, c, dy.base + label_off);
    else lam = l;
  }
  lam = wave_max(lam);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = lam;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
    cfl_max(dy, (int)(dy.base & 1), m);
  }
}

// deterministic conserved totals (rho, rho u, rho xi[, rho xi_2]) of one case, partial sums per block
template <class S, int D, bool G2>
__global__ __launch_bounds__(256) void k_baro_totals_part(const CaseC* cases, int icase, const S* __restrict__ src,
                                                          long long total, double* __restrict__ part)
{
  constexpr int NQ = D + 2 + (G2 ? 1 : 0);
  __shared__ double s[NQ][256];
  const CaseC& C = cases[icase];
  double acc[NQ];
  for (int v = 0; v < NQ; ++v) acc[v] = 0.0;
  for (long long c = blockIdx.x * 256ll + threadIdx.x; c < C.ncell; c += 256ll * gridDim.x) {
    long long g = C.off + c;
    double rL = (double)src[g] + C.rref[0], rG = (double)src[total + g];
    double rG2 = G2 ? (double)src[(2 + D) * total + g] : 0.0;
    acc[0] += G2 ? rL + rG + rG2 : rL + rG;
    for (int d = 0; d < D; ++d) acc[1 + d] += (double)src[(2 + d) * total + g];
    acc[1 + D] += rG;
    if constexpr (G2) acc[2 + D] += rG2;
  }
  for (int v = 0; v < NQ; ++v) s[v][threadIdx.x] = acc[v];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int v = 0; v < NQ; ++v) s[v][threadIdx.x] += s[v][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int v = 0; v < NQ; ++v) part[blockIdx.x * NQ + v] = s[v][0];
}

// ------------------------------------------------------------------ 3D: closure kernel + face kernel
// As for the four-equation model in 3D: the FP64 closure runs once per cell in
// its own kernel and writes the primitives in the storage precision; the face
// kernel stages tile + two-cell halo primitives in LDS.
// rho, u, v, w, p, xi, alpha_G, alpha_V [, c with FP32 storage] [, xi_2,
// alpha_G2 with two gases].  The sound speed is a function of p alone
// (baro_sound): the FP64 path recomputes it at the faces; the FP32 path keeps
// it as a stored field, which measured faster there.
template <class S, bool G2>
constexpr int nwb3() { return (sizeof(S) == 4 ? 9 : 8) + (G2 ? 2 : 0); }

// the sound speed of the closure at pressure p (the larger of the liquid and
// gas speeds above p_sat, of the mixture and gas speeds below)
template <class S>
__device__ inline S baro_sound(const CaseC& C, S p)
{
  return (p >= S(C.bt_ps)) ? S(C.bt_c_hi) : S(C.bt_c_lo);
}

// primitives of every owned cell; in the first stage of a step also the CFL
// bound of q^n and its checks (an error of the step before)
template <class S, int TX, int TY, int TZ, bool G2>
__global__ __launch_bounds__(256) void k_bprim3(StageArgs a, S* __restrict__ W)
{
  __shared__ double s_red[4];
  constexpr int NB = (TX * TY * TZ + 255) / 256;   // workgroups per tile
  const int bb = xcd_block(blockIdx.x, gridDim.x);
  const int4 tl = a.tiles[bb / NB];
  const CaseC& C = a.cases[tl.x];
  CaseDyn& dy = a.dyn[tl.x];
  const S* __restrict__ src = (const S*)a.src;
  const long long T = a.total;
  const bool first = a.stage == 0;
  const long long step = dy.base + a.step_off;
  double lam = 0.0;
  constexpr int NC = TX * TY * TZ;
  const int cc = (bb % NB) * 256 + threadIdx.x;
  const int i = cc % TX, j = (cc / TX) % TY, k = cc / (TX * TY);
  const int gx = tl.y * TX + i, gy = tl.z * TY + j, gz = tl.w * TZ + k;
  // this cell's total gas mass and volume fractions as the face kernel stages
  // them (storage precision, the two gases summed there)
  S yg = S(0), ag = S(0);
  const bool in = cc < NC && gx < C.n[0] && gy < C.n[1] && gz < C.n[2];
  if (in) {
    long long cell = C.off + gx + (long long)C.n[0] * (gy + (long long)C.n[1] * gz);
    constexpr int NQ = 5 + (G2 ? 1 : 0);
    double q[NQ], u[3], rho, Y, Y2;
    q[0] = (double)src[cell] + C.rref[0];
#pragma unroll
    for (int v = 1; v < NQ; ++v) q[v] = (double)src[v * T + cell];
    PB pb = baro_prim<3, G2>(C, q, u, rho, Y, Y2);
    W[cell] = S(rho);
    W[T + cell] = S(u[0]);
    W[2 * T + cell] = S(u[1]);
    W[3 * T + cell] = S(u[2]);
    W[4 * T + cell] = S(pb.p);
    W[5 * T + cell] = S(Y);
    constexpr int NW = nwb3<S, G2>();
    W[6 * T + cell] = S(pb.aG);
    W[7 * T + cell] = S(pb.aV);
    if constexpr (sizeof(S) == 4) W[8 * T + cell] = S(pb.c);
    yg = S(Y);
    ag = S(pb.aG);
    if constexpr (G2) {
      W[(NW - 2) * T + cell] = S(Y2);
      W[(NW - 1) * T + cell] = S(pb.aG2);
      yg = yg + S(Y2);
      ag = ag + S(pb.aG2);
    }
    if (first) {
      double l = baro_cfl<3>(C, u, pb, rho);
      if (!isfinite(l) || !isfinite(pb.p)) record_error(dy, ERR_NAN, cell - C.off, step - 1);
      else if (!(rho > 0.0) || !(pb.p > 0.0)) record_error(dy, ERR_NONPHYS, cell - C.off, step - 1);
      else lam = fmax(lam, l);
    }
  }
  if (first) {
    lam = wave_max(lam);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = lam;
    __syncthreads();
    if (threadIdx.x == 0) cfl_max(dy, (int)(step & 1), fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3])));
  }
  // with surface tension: this workgroup's (min, max) of both fractions, from
  // which k_csf_zero marks the face-kernel tiles whose CSF term is zero
  if (a.frac_ext && a.sc.sigma > 0.0) frac_extremes<S>(in, yg, ag, (S*)a.frac_ext + (long long)bb * 4);
}

template <class S, bool G2>
__device__ inline void bprim_of(const CaseC& C, const double* q, S* w)
{
  double u[3], rho, Y, Y2;
  PB pb = baro_prim<3, G2>(C, q, u, rho, Y, Y2);
  w[0] = S(rho); w[1] = S(u[0]); w[2] = S(u[1]); w[3] = S(u[2]);
  constexpr int NW = nwb3<S, G2>();
  w[4] = S(pb.p); w[5] = S(Y); w[6] = S(pb.aG); w[7] = S(pb.aV);
  if constexpr (sizeof(S) == 4) w[8] = S(pb.c);
  if constexpr (G2) {
    w[NW - 2] = S(Y2);
    w[NW - 1] = S(pb.aG2);
  }
}

// primitives of one (possibly ghost) cell (far-field and inflow states hold
// no second gas)
template <class S, bool G2>
__device__ inline void load_bprim3(const CaseC& C, const S* __restrict__ W, long long T, int gx, int gy, int gz,
                                   long long step, S* w)
{
  if (beyond_farfield<3>(C, gx, gy, gz)) {
    const double u0[3] = {0.0, 0.0, 0.0};
    double q[6];
    baro_from_prim<3, G2>(C, C.ff_p, C.ff_alpha, u0, q);
    bprim_of<S, G2>(C, q, w);
    return;
  }
  bool fx = false, fy = false, fz = false;
  int ix = gx, iy = gy, iz = gz;
  map_index(iy, C.n[1], C.bc[1][0], C.bc[1][1], fy);
  map_index(iz, C.n[2], C.bc[2][0], C.bc[2][1], fz);
  if (ix < 0 && C.bc[0][0] == BC_INFLOW) {
    double yy = (iy + 0.5) * C.dx[1] - C.in_c0;
    double zz = (iz + 0.5) * C.dx[2] - C.in_c1;
    if (sqrt(yy * yy + zz * zz) < C.in_radius) {
      double u[3] = {C.in_u, 0.0, 0.0}, q[6];
      for (int c = 0; c < 3; ++c)
        u[c] += C.in_noise * C.in_u *
                (2.0 * noise01(C.in_seed, (unsigned long long)step, (unsigned long long)iy,
                               (unsigned long long)iz, (unsigned long long)c) - 1.0);
      baro_from_prim<3, G2>(C, C.in_p, C.in_alpha, u, q);
      if (fy) q[3] = -q[3];
      if (fz) q[4] = -q[4];
      bprim_of<S, G2>(C, q, w);
      return;
    }
    ix = -1 - ix;
    fx = true;
  } else {
    map_index(ix, C.n[0], C.bc[0][0], C.bc[0][1], fx);
  }
  long long cell = C.off + ix + (long long)C.n[0] * (iy + (long long)C.n[1] * iz);
#pragma unroll
  for (int v = 0; v < nwb3<S, G2>(); ++v) w[v] = W[v * T + cell];
  if (fx) w[1] = -w[1];
  if (fy) w[2] = -w[2];
  if (fz) w[3] = -w[3];
}

template <class S, int TX, int TY, int TZ, int NT, int MINW, int LIM, bool G2>
__global__ __launch_bounds__(NT, MINW) void k_bface3(StageArgs a, const S* __restrict__ W)
{
  constexpr int HX = TX + 4, HY = TY + 4, HZ = TZ + 4, HXY = HX * HY, NH = HXY * HZ;
  constexpr int NWB3 = nwb3<S, G2>();
  constexpr int NQ = 5 + (G2 ? 1 : 0);
  constexpr int NC = TX * TY * TZ;
  constexpr int CPT = (NC + NT - 1) / NT;
  constexpr int NFX = (TX + 1) * TY * TZ, NFY = TX * (TY + 1) * TZ, NFZ = TX * TY * (TZ + 1);
  constexpr int NF = NFX > NFY ? (NFX > NFZ ? NFX : NFZ) : (NFY > NFZ ? NFY : NFZ);
  constexpr int FX = TX + 2, FY = TY + 2, FZ = TZ + 2, NFH = FX * FY * FZ;
  constexpr int VX = TX + 1, VY = TY + 1, VZ = TZ + 1, NV = VX * VY * VZ;
  constexpr int NBUF = (NQ * NF > NFH + 3 * NV) ? NQ * NF : NFH + 3 * NV;

  __shared__ S s_w[NWB3][NH];
  __shared__ unsigned char s_fl[NH];
  __shared__ S s_buf[NBUF];
  S(*s_F)[NF] = reinterpret_cast<S(*)[NF]>(s_buf);

  const int4 tl = a.tiles[xcd_block(blockIdx.x, gridDim.x)];
  const CaseC& C = a.cases[tl.x];
  CaseDyn& dy = a.dyn[tl.x];
  const SchemeC& SC = a.sc;
  const int x0 = tl.y * TX, y0 = tl.z * TY, z0 = tl.w * TZ;
  const int tid = threadIdx.x;
  const bool upd = a.stage >= 0;
  const long long step = upd ? dy.base + a.step_off : a.rhs_step;
  const long long T = a.total;
  S* s_rho = s_w[0];
  S* s_u = s_w[1];
  S* s_v = s_w[2];
  S* s_ww = s_w[3];
  S* s_p = s_w[4];
  S* s_Y = s_w[5];
  S* s_a = s_w[6];
  S* s_av = s_w[7];
  S* s_Y2 = G2 ? s_w[NWB3 - 2] : nullptr;
  S* s_a2 = G2 ? s_w[NWB3 - 1] : nullptr;
  // total gas volume fraction and gas mass fraction of a halo cell
  auto aG = [&](int c) { if constexpr (G2) return s_a[c] + s_a2[c]; else return s_a[c]; };
  auto YG = [&](int c) { if constexpr (G2) return s_Y[c] + s_Y2[c]; else return s_Y[c]; };

  auto owned = [&](int cc, int& gx, int& gy, int& gz) {
    int i = cc % TX, j = (cc / TX) % TY, k = cc / (TX * TY);
    gx = x0 + i; gy = y0 + j; gz = z0 + k;
    return cc < NC && gx < C.n[0] && gy < C.n[1] && gz < C.n[2];
  };

  S qn_reg[CPT][NQ];
  if (upd) {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      int gx, gy, gz;
      bool own = owned(tid + k * NT, gx, gy, gz);
      long long cell = C.off + (own ? gx + (long long)C.n[0] * (gy + (long long)C.n[1] * gz) : 0);
#pragma unroll
      for (int v = 0; v < NQ; ++v) qn_reg[k][v] = ((const S*)a.qn)[v * T + cell];
    }
  }

  if (halo_inside3<S>(C, x0, y0, z0, TX, TY, TZ)) {
    // no ghost cell: straight loads at 32-bit byte offsets from the rows' bases
    const char* base[NWB3];
#pragma unroll
    for (int v = 0; v < NWB3; ++v) base[v] = (const char*)(W + v * T + C.off);
    const unsigned n0 = (unsigned)C.n[0], n01 = n0 * (unsigned)C.n[1];
    const unsigned org = (unsigned)(x0 - 2) + n0 * (unsigned)(y0 - 2) + n01 * (unsigned)(z0 - 2);
#pragma unroll
    for (int it = 0; it < (NH + NT - 1) / NT; ++it) {
      const int h = tid + it * NT;
      if (h < NH) {
        const unsigned hx = h % HX, hy = (h / HX) % HY, hz = h / HXY;
        const unsigned off = (org + hx + n0 * hy + n01 * hz) * (unsigned)sizeof(S);
#pragma unroll
        for (int v = 0; v < NWB3; ++v) s_w[v][h] = *(const S*)(base[v] + off);
      }
    }
  } else {
    for (int h = tid; h < NH; h += NT) {
      int hx = h % HX, hy = (h / HX) % HY, hz = h / HXY;
      S w[NWB3];
      load_bprim3<S, G2>(C, W, T, x0 + hx - 2, y0 + hy - 2, z0 + hz - 2, step, w);
#pragma unroll
      for (int v = 0; v < NWB3; ++v) s_w[v][h] = w[v];
    }
  }
  __syncthreads();

  const int st[3] = {1, HX, HXY};
  // ---- switching sensors (Ducros, gas and vapour volume fractions) on tile + one halo layer
  if (SC.switching) {
    for (int h = tid; h < NFH; h += NT) {
      int lx = h % FX, ly = (h / FX) % FY, lz = h / (FX * FY);
      int c = (lz + 1) * HXY + (ly + 1) * HX + lx + 1;
      S g[3][3];
      const S* uu[3] = {s_u, s_v, s_ww};
#pragma unroll
      for (int comp = 0; comp < 3; ++comp)
#pragma unroll
        for (int d = 0; d < 3; ++d)
          g[comp][d] = (uu[comp][c + st[d]] - uu[comp][c - st[d]]) * S(0.5 * C.idx[d]);
      S div = g[0][0] + g[1][1] + g[2][2];
      S w0 = g[2][1] - g[1][2], w1 = g[0][2] - g[2][0], w2 = g[1][0] - g[0][1];
      S curl2 = w0 * w0 + w1 * w1 + w2 * w2;
      S thg = S(0), thv = S(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        thg += fabs(aG(c) - aG(c - st[d])) + fabs(aG(c + st[d]) - aG(c));
        thv += fabs(s_av[c] - s_av[c - st[d]]) + fabs(s_av[c + st[d]] - s_av[c]);
      }
      S thd = fdiv(div * div, div * div + curl2 + S(SC.eps_d));
      s_fl[c] = (thd > S(SC.th_d) || thv > S(SC.th_g) || thg > S(SC.th_g)) ? 1 : 0;
    }
    __syncthreads();
  }

  S R[CPT][NQ];
#pragma unroll
  for (int k = 0; k < CPT; ++k)
#pragma unroll
    for (int v = 0; v < NQ; ++v) R[k][v] = S(0);

  const S eps = S(SC.eps_int);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int EX = TX + (d == 0), EY = TY + (d == 1);
    const int NFD = d == 0 ? NFX : (d == 1 ? NFY : NFZ);
    const int sd = st[d];
    if (d > 0) __syncthreads();
    for (int f = tid; f < NFD; f += NT) {
      int i = f % EX, j = (f / EX) % EY, k = f / (EX * EY);
      int c = (k + 2) * HXY + (j + 2) * HX + (i + 2) - sd;   // lower cell of the face
      BStencil<S, 3> bs;
      S av[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        int cm = c + (m - 1) * sd;
        bs.u[0][m] = s_u[cm];
        bs.u[1][m] = s_v[cm];
        bs.u[2][m] = s_ww[cm];
        bs.p[m] = s_p[cm];
        bs.Y[m] = s_Y[cm];
        bs.r[m] = s_rho[cm];
        av[m] = s_av[cm];
        if constexpr (G2) bs.Y2[m] = s_Y2[cm];
      }
      if constexpr (sizeof(S) == 4) {
        bs.c1 = s_w[8][c];
        bs.c2 = s_w[8][c + sd];
      } else {
        bs.c1 = baro_sound<S>(C, s_p[c]);
        bs.c2 = baro_sound<S>(C, s_p[c + sd]);
      }
      int el = baro_elig<S>(bs.Y[0], bs.Y[1], bs.Y[2], av[0], av[1], av[2], bs.r[0], bs.r[1], bs.r[2], eps);
      int er = baro_elig<S>(bs.Y[1], bs.Y[2], bs.Y[3], av[1], av[2], av[3], bs.r[1], bs.r[2], bs.r[3], eps);
      if constexpr (G2) {
        if (eligible<S>(bs.Y2[0], bs.Y2[1], bs.Y2[2], eps)) el |= 4;
        if (eligible<S>(bs.Y2[1], bs.Y2[2], bs.Y2[3], eps)) er |= 4;
      }
      bool disc = !SC.switching || ((s_fl[c] | s_fl[c + sd]) != 0);
      S F[NQ];
      if (d == 0) baro_face<S, 3, 0, LIM, G2>(SC, C, bs, disc, el, er, F);
      else if (d == 1) baro_face<S, 3, 1, LIM, G2>(SC, C, bs, disc, el, er, F);
      else baro_face<S, 3, 2, LIM, G2>(SC, C, bs, disc, el, er, F);
      if (C.diff) {
        const S* U3[3] = {s_u, s_v, s_ww};
        if (d == 0) baro_visc<S, 3, 0>(C, U3, s_a, s_av, c, st, F, s_a2);
        else if (d == 1) baro_visc<S, 3, 1>(C, U3, s_a, s_av, c, st, F, s_a2);
        else baro_visc<S, 3, 2>(C, U3, s_a, s_av, c, st, F, s_a2);
      }
#pragma unroll
      for (int v = 0; v < NQ; ++v) s_F[v][f] = F[v];
    }
    __syncthreads();
    const S id = S(C.idx[d]);
#pragma unroll
    for (int kk = 0; kk < CPT; ++kk) {
      int cc = tid + kk * NT;
      if (cc < NC) {
        int i = cc % TX, j = (cc / TX) % TY, k = cc / (TX * TY);
        int f = (k * EY + j) * EX + i;
        int fn = f + (d == 0 ? 1 : (d == 1 ? EX : EX * EY));
#pragma unroll
        for (int v = 0; v < NQ; ++v) R[kk][v] += (s_F[v][f] - s_F[v][fn]) * id;
      }
    }
  }

  // ---- CSF (Section 3.5): 3D binomial kernel /64 of xi, vertex normals, kappa = -div n,
  // force sigma kappa grad(alpha_G) on the momentum
  // a tile whose staged gas fractions are all equal (marked by k_csf_zero from
  // the closure kernel of this stage, with its neighbours) gets exactly zero
  if (SC.sigma > 0.0 && !(a.csf_zero && a.frac_ext && a.csf_zero[xcd_block(blockIdx.x, gridDim.x)])) {
    __syncthreads();
    S* s_H = s_buf;
    S* s_n = s_H + NFH;
    for (int h = tid; h < NFH; h += NT) {
      int lx = h % FX, ly = (h / FX) % FY, lz = h / (FX * FY);
      int c = (lz + 1) * HXY + (ly + 1) * HX + lx + 1;
      S acc = S(0);
#pragma unroll
      for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dyy = -1; dyy <= 1; ++dyy) {
          S row = YG(c + dz * HXY + dyy * HX - 1) + S(2) * YG(c + dz * HXY + dyy * HX) +
                  YG(c + dz * HXY + dyy * HX + 1);
          acc += row * S((dz == 0 ? 2 : 1) * (dyy == 0 ? 2 : 1));
        }
      s_H[h] = acc * S(1.0 / 64.0);
    }
    __syncthreads();
    S en = S(SC.eps_n * C.idx[0]);
    for (int h = tid; h < NV; h += NT) {
      int vx = h % VX, vy = (h / VX) % VY, vz = h / (VX * VY);
      int c = (vz * FY + vy) * FX + vx;
      const int sx = 1, sy = FX, sz = FX * FY;
      S gx = (s_H[c + sx] + s_H[c + sx + sy] + s_H[c + sx + sz] + s_H[c + sx + sy + sz] -
              s_H[c] - s_H[c + sy] - s_H[c + sz] - s_H[c + sy + sz]) * S(0.25 * C.idx[0]);
      S gy = (s_H[c + sy] + s_H[c + sy + sx] + s_H[c + sy + sz] + s_H[c + sy + sx + sz] -
              s_H[c] - s_H[c + sx] - s_H[c + sz] - s_H[c + sx + sz]) * S(0.25 * C.idx[1]);
      S gz = (s_H[c + sz] + s_H[c + sz + sx] + s_H[c + sz + sy] + s_H[c + sz + sx + sy] -
              s_H[c] - s_H[c + sx] - s_H[c + sy] - s_H[c + sx + sy]) * S(0.25 * C.idx[2]);
      S inv = frcp(sqrt(gx * gx + gy * gy + gz * gz) + en);
      s_n[h] = gx * inv;
      s_n[NV + h] = gy * inv;
      s_n[2 * NV + h] = gz * inv;
    }
    __syncthreads();
    S sig = S(SC.sigma);
#pragma unroll
    for (int kk = 0; kk < CPT; ++kk) {
      int cc = tid + kk * NT;
      if (cc < NC) {
        int i = cc % TX, j = (cc / TX) % TY, k = cc / (TX * TY);
        int c = (k + 2) * HXY + (j + 2) * HX + i + 2;
        int v = ((k + 1) * VY + (j + 1)) * VX + (i + 1);
        const int vs[3] = {1, VX, VX * VY};
        S kap = S(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          int t1 = vs[(d + 1) % 3], t2 = vs[(d + 2) % 3];
          const S* nd = s_n + d * NV;
          S plus = nd[v] + nd[v - t1] + nd[v - t2] + nd[v - t1 - t2];
          S minus = nd[v - vs[d]] + nd[v - vs[d] - t1] + nd[v - vs[d] - t2] + nd[v - vs[d] - t1 - t2];
          kap += (plus - minus) * S(0.25 * C.idx[d]);
        }
        kap = -kap;
#pragma unroll
        for (int d = 0; d < 3; ++d) R[kk][2 + d] += sig * kap * (aG(c + st[d]) - aG(c - st[d])) * S(0.5 * C.idx[d]);
      }
    }
  }

  // ---- body force (eq. 2-2, source Q): rho g on the momentum
  if (SC.has_grav) {
#pragma unroll
    for (int kk = 0; kk < CPT; ++kk) {
      int cc = tid + kk * NT;
      if (cc < NC) {
        int i = cc % TX, j = (cc / TX) % TY, k = cc / (TX * TY);
        int c = (k + 2) * HXY + (j + 2) * HX + i + 2;
#pragma unroll
        for (int d = 0; d < 3; ++d) R[kk][2 + d] += s_rho[c] * S(SC.grav[d]);
      }
    }
  }

  if (!upd) {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      int gx, gy, gz;
      if (owned(tid + k * NT, gx, gy, gz)) {
        const long long RS = C.ncell;
        long long cell = gx + (long long)C.n[0] * (gy + (long long)C.n[1] * gz);
        double r0 = (double)R[k][0], r1 = (double)R[k][1];
        double r2 = G2 ? (double)R[k][NQ - 1] : 0.0;
        a.rhs_out[cell] = G2 ? r0 + r1 + r2 : r0 + r1;
#pragma unroll
        for (int d = 0; d < 3; ++d) a.rhs_out[(1 + d) * RS + cell] = (double)R[k][2 + d];
        a.rhs_out[4 * RS + cell] = r1;
        if constexpr (G2) a.rhs_out[5 * RS + cell] = r2;
      }
    }
    return;
  }
  const double dt = step_dt(dy, step, SC.cfl, SC.t_end);
  if (a.stage == 0 && tl.y == 0 && tl.z == 0 && tl.w == 0 && tid == 0) step_scalars(dy, step, dt);
  // the last stage writes q^(n+1); its CFL bound and checks come from the
  // closure kernel of the next step's first stage (or the end-of-run check)
  S* dst = (S*)a.dst;
  const S adt = S(a.ak * dt);
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    int gx, gy, gz;
    if (owned(tid + k * NT, gx, gy, gz)) {
      long long cell = C.off + gx + (long long)C.n[0] * (gy + (long long)C.n[1] * gz);
#pragma unroll
      for (int v = 0; v < NQ; ++v) dst[v * T + cell] = qn_reg[k][v] + adt * R[k][v];
    }
  }
}

// LDS bytes of the 3D face kernel (halo primitives, flags, flux / CSF buffer);
// a workgroup holds at most 160 KiB
template <class S, int TX, int TY, int TZ, bool G2>
constexpr long bld3()
{
  constexpr long NH = (long)(TX + 4) * (TY + 4) * (TZ + 4);
  constexpr long NFX = (long)(TX + 1) * TY * TZ, NFY = (long)TX * (TY + 1) * TZ, NFZ = (long)TX * TY * (TZ + 1);
  constexpr long NF = NFX > NFY ? (NFX > NFZ ? NFX : NFZ) : (NFY > NFZ ? NFY : NFZ);
  constexpr long NFH = (long)(TX + 2) * (TY + 2) * (TZ + 2), NV = (long)(TX + 1) * (TY + 1) * (TZ + 1);
  constexpr long NQ = 5 + (G2 ? 1 : 0);
  constexpr long NBUF = NQ * NF > NFH + 3 * NV ? NQ * NF : NFH + 3 * NV;
  return (long)sizeof(S) * (nwb3<S, G2>() * NH + NBUF) + NH;
}

template <class S, int TX, int TY, int TZ, bool G2>
constexpr bool bfits3() { return bld3<S, TX, TY, TZ, G2>() <= 160L * 1024; }

template <class S, int TX, int TY, int TZ, int NT, int MINW, bool G2>
static hipError_t launch_b3(const StageArgs& a, int ntiles, hipStream_t st)
{
  if constexpr (!bfits3<S, TX, TY, TZ, G2>()) {
    return hipErrorInvalidValue;
  } else {
    S* W = (S*)a.prim;
    constexpr int NB = (TX * TY * TZ + 255) / 256;
    hipLaunchKernelGGL((k_bprim3<S, TX, TY, TZ, G2>), dim3(ntiles * NB), dim3(256), 0, st, a, W);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.csf_zero && a.frac_ext && a.sc.sigma > 0.0) {
      hipLaunchKernelGGL((k_csf_zero<S, TX, TY, TZ, NB>), dim3((ntiles + 255) / 256), dim3(256), 0, st, a, ntiles,
                         (unsigned char*)a.csf_zero);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (fvm_default_limiters(a.sc))
      hipLaunchKernelGGL((k_bface3<S, TX, TY, TZ, NT, MINW, 1, G2>), dim3(ntiles), dim3(NT), 0, st, a, (const S*)W);
    else
      hipLaunchKernelGGL((k_bface3<S, TX, TY, TZ, NT, MINW, 0, G2>), dim3(ntiles), dim3(NT), 0, st, a, (const S*)W);
    return hipGetLastError();
  }
}

// the tile shapes (and indices) of the four-equation 3D kernels
template <class S, bool G2>
static hipError_t stage_b3(int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  switch (fvm_k_tile_row3(tile)) {
    case 0: return launch_b3<S, 8, 8, 4, 256, 2, G2>(a, ntiles, st);
    case 1: return launch_b3<S, 16, 8, 2, 256, 2, G2>(a, ntiles, st);
    case 2: return launch_b3<S, 8, 4, 4, 128, 2, G2>(a, ntiles, st);
    case 3: return launch_b3<S, 16, 4, 4, 256, 2, G2>(a, ntiles, st);
    case 4: return launch_b3<S, 8, 8, 8, 512, 1, G2>(a, ntiles, st);
    case 5: return launch_b3<S, 8, 8, 8, 768, 1, G2>(a, ntiles, st);
    case 6: return launch_b3<S, 8, 8, 8, 1024, 1, G2>(a, ntiles, st);
    case 7: return launch_b3<S, 8, 8, 4, 512, 1, G2>(a, ntiles, st);
    case 8: return launch_b3<S, 8, 4, 4, 256, 2, G2>(a, ntiles, st);
    case 9: return launch_b3<S, 8, 8, 8, 576, 1, G2>(a, ntiles, st);
  }
  return hipErrorInvalidValue;
}

// 1 if the 3D tile fits the LDS of a workgroup, 0 if not, -1 for no such tile
// (or a z-marching tile, which the barotropic model does not take)
template <class S, bool G2>
static int tile_okb3(int tile)
{
  switch (fvm_k_tile_row3(tile)) {
    case 0: case 7: return bfits3<S, 8, 8, 4, G2>();
    case 1: return bfits3<S, 16, 8, 2, G2>();
    case 2: case 8: return bfits3<S, 8, 4, 4, G2>();
    case 3: return bfits3<S, 16, 4, 4, G2>();
    case 4: case 5: case 6: case 9: return bfits3<S, 8, 8, 8, G2>();
  }
  return -1;
}

template <class S, int D, int TX, int TY, int NT, int MINW, bool G2>
static hipError_t launch_b(const StageArgs& a, int ntiles, hipStream_t st)
{
  if (fvm_default_limiters(a.sc))
    hipLaunchKernelGGL((k_baro12<S, D, TX, TY, NT, MINW, 1, G2>), dim3(ntiles), dim3(NT), 0, st, a);
  else
    hipLaunchKernelGGL((k_baro12<S, D, TX, TY, NT, MINW, 0, G2>), dim3(ntiles), dim3(NT), 0, st, a);
  return hipGetLastError();
}

// the same tile shapes (and indices) as the four-equation kernel
template <class S, bool G2>
static hipError_t stage_b(int dim, int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  if (dim == 1) {
    switch (tile) {
      case 0: return launch_b<S, 1, 256, 1, 256, 4, G2>(a, ntiles, st);
      case 1: return launch_b<S, 1, 128, 1, 128, 4, G2>(a, ntiles, st);
      case 2: return launch_b<S, 1, 128, 1, 256, 4, G2>(a, ntiles, st);
    }
  } else if (dim == 2) {
    switch (tile) {
      case 0: return launch_b<S, 2, 32, 8, 256, 4, G2>(a, ntiles, st);
      case 1: return launch_b<S, 2, 16, 8, 256, 4, G2>(a, ntiles, st);
      case 2: return launch_b<S, 2, 64, 4, 256, 4, G2>(a, ntiles, st);
      case 3: return launch_b<S, 2, 16, 16, 256, 4, G2>(a, ntiles, st);
      case 4: return launch_b<S, 2, 32, 16, 256, 2, G2>(a, ntiles, st);
      case 5: return launch_b<S, 2, 32, 4, 256, 4, G2>(a, ntiles, st);
      case 6: return launch_b<S, 2, 32, 8, 320, 5, G2>(a, ntiles, st);
      case 7: return launch_b<S, 2, 16, 16, 320, 5, G2>(a, ntiles, st);
      case 8: return launch_b<S, 2, 32, 8, 384, 6, G2>(a, ntiles, st);
      case 9: return launch_b<S, 2, 32, 16, 512, 4, G2>(a, ntiles, st);
      case 10: return launch_b<S, 2, 32, 32, 1024, 4, G2>(a, ntiles, st);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace fvm

using namespace fvm;

static unsigned blocks_b(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t fvm_kb_stage(int dim, int mixed, int g2, int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  if (dim == 3) {
    if (g2) return mixed ? stage_b3<float, true>(tile, a, ntiles, st) : stage_b3<double, true>(tile, a, ntiles, st);
    return mixed ? stage_b3<float, false>(tile, a, ntiles, st) : stage_b3<double, false>(tile, a, ntiles, st);
  }
  if (g2) return mixed ? stage_b<float, true>(dim, tile, a, ntiles, st) : stage_b<double, true>(dim, tile, a, ntiles, st);
  return mixed ? stage_b<float, false>(dim, tile, a, ntiles, st) : stage_b<double, false>(dim, tile, a, ntiles, st);
}

int fvm_kb_tile_ok3(int mixed, int g2, int tile)
{
  if (g2) return mixed ? tile_okb3<float, true>(tile) : tile_okb3<double, true>(tile);
  return mixed ? tile_okb3<float, false>(tile) : tile_okb3<double, false>(tile);
}

#define FVM_BDISPATCH_G(MIXED, DIM, G, CALL)                                            \
  do {                                                                                  \
    if (MIXED) {                                                                        \
      if (DIM == 1) { CALL(float, 1, G); } else if (DIM == 2) { CALL(float, 2, G); } else { CALL(float, 3, G); } \
    } else {                                                                            \
      if (DIM == 1) { CALL(double, 1, G); } else if (DIM == 2) { CALL(double, 2, G); } else { CALL(double, 3, G); } \
    }                                                                                   \
  } while (0)
#define FVM_BDISPATCH(MIXED, DIM, G2, CALL)                                             \
  do {                                                                                  \
    if (G2) FVM_BDISPATCH_G(MIXED, DIM, true, CALL);                                    \
    else FVM_BDISPATCH_G(MIXED, DIM, false, CALL);                                      \
  } while (0)

hipError_t fvm_kb_prim_to_state(int dim, int mixed, int g2, const CaseC* cases, int icase, long long ncell,
                                const double* prim, void* dst, long long total, hipStream_t st)
{
  if (dim < 1 || dim > 3) return hipErrorInvalidValue;
#define CALL(S, D, G) hipLaunchKernelGGL((k_baro_prim_to_state<S, D, G>), dim3(blocks_b(ncell, 256)), dim3(256), 0, st, cases, icase, prim, (S*)dst, total)
  FVM_BDISPATCH(mixed, dim, g2, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_kb_cons_to_state(int dim, int mixed, int g2, const CaseC* cases, int icase, long long ncell,
                                const double* q, void* dst, long long total, hipStream_t st)
{
  if (dim < 1 || dim > 3) return hipErrorInvalidValue;
#define CALL(S, D, G) hipLaunchKernelGGL((k_baro_cons_to_state<S, D, G>), dim3(blocks_b(ncell, 256)), dim3(256), 0, st, cases, icase, q, (S*)dst, total)
  FVM_BDISPATCH(mixed, dim, g2, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_kb_state_to_cons(int dim, int mixed, int g2, const CaseC* cases, int icase, long long ncell,
                                const void* src, double* q, long long total, hipStream_t st)
{
  if (dim < 1 || dim > 3) return hipErrorInvalidValue;
#define CALL(S, D, G) hipLaunchKernelGGL((k_baro_state_to_cons<S, D, G>), dim3(blocks_b(ncell, 256)), dim3(256), 0, st, cases, icase, (const S*)src, q, total)
  FVM_BDISPATCH(mixed, dim, g2, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_kb_state_to_prim(int dim, int mixed, int g2, const CaseC* cases, int icase, long long ncell,
                                const void* src, double* w, long long total, hipStream_t st)
{
  if (dim < 1 || dim > 3) return hipErrorInvalidValue;
#define CALL(S, D, G) hipLaunchKernelGGL((k_baro_state_to_prim<S, D, G>), dim3(blocks_b(ncell, 256)), dim3(256), 0, st, cases, icase, (const S*)src, w, total)
  FVM_BDISPATCH(mixed, dim, g2, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_kb_dt_init(int dim, int mixed, int g2, const CaseC* cases, CaseDyn* dyn, int icase, long long ncell,
                          const void* src, long long total, long long label_off, hipStream_t st)
{
  if (dim < 1 || dim > 3) return hipErrorInvalidValue;
#define CALL(S, D, G) hipLaunchKernelGGL((k_baro_dt_init<S, D, G>), dim3(blocks_b(ncell, 256)), dim3(256), 0, st, cases, dyn, icase, (const S*)src, total, label_off)
  FVM_BDISPATCH(mixed, dim, g2, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_kb_totals_part(int dim, int mixed, int g2, const CaseC* cases, int icase, const void* src, long long total,
                              double* part, int nblk, hipStream_t st)
{
  if (dim < 1 || dim > 3) return hipErrorInvalidValue;
#define CALL(S, D, G) hipLaunchKernelGGL((k_baro_totals_part<S, D, G>), dim3(nblk), dim3(256), 0, st, cases, icase, (const S*)src, total, part)
  FVM_BDISPATCH(mixed, dim, g2, CALL);
#undef CALL
  return hipGetLastError();
}
