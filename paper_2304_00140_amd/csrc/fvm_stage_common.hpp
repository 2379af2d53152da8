// fvm_stage_common.hpp -- device helpers shared by the fused stage kernels:
// ghost-cell generation from the boundary kinds, loading a cell, primitives of
// a cell, error recording, wavefront max and the per-step scalars.
#pragma once
#include <hip/hip_runtime.h>
#include "fvm_device.hpp"

namespace fvm {

// ------------------------------------------------------------------ ghost cells
__device__ inline void map_index(int& i, int n, int bclo, int bchi, bool& flip)
{
  if (i < 0) {
    if (bclo == BC_PERIODIC) i += n;
    else if (bclo == BC_WALL) { i = -1 - i; flip = true; }
    else i = 0;
  } else if (i >= n) {
    if (bchi == BC_PERIODIC) i -= n;
    else if (bchi == BC_WALL) { i = 2 * n - 1 - i; flip = true; }
    else i = n - 1;
  }
  i = min(max(i, 0), n - 1);   // cells beyond the stencil's reach (partial tiles)
}

// physical partial densities, momentum and gauge energy of a cell from its
// primitives (p, T, alpha_G, u); xi = alpha_G rho_G / rho at (p, T).  G2:
// three components, al2 = alpha of the second gas, whose partial density
// follows the energy (index 3 + D).
template <bool PRK, bool G2 = false>
__device__ inline void state_from_prim(const CaseC& C, double p, double T, double al, const double* u,
                                       int D, double* q, double al2 = 0.0)
{
  if constexpr (G2) {
    double r[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = (p + C.comp[k].pinf) / (C.comp[k].A * T);
    double rho = (1.0 - al - al2) * r[0] + al * r[1] + al2 * r[2];
    double ir = 1.0 / rho;
    double Y1 = al * r[1] * ir, Y2 = al2 * r[2] * ir;
    double vm, em;
    tdu3<double>(C, p, T, Y1, Y2, vm, em);
    double ke = 0.0;
    for (int d = 0; d < D; ++d) ke += u[d] * u[d];
    q[0] = rho - rho * Y1 - rho * Y2;
    q[1] = rho * Y1;
    for (int d = 0; d < D; ++d) q[2 + d] = rho * u[d];
    q[2 + D] = rho * (em + 0.5 * ke);
    q[3 + D] = rho * Y2;
    return;
  }
  double vL, eL, vG, eG;
  closure_fwd<PRK>(C, p, T, 0.0, vL, eL);
  closure_fwd<PRK>(C, p, T, 1.0, vG, eG);
  double rG = 1.0 / vG, rL = 1.0 / vL;
  double rho = al * rG + (1.0 - al) * rL;
  double Y = al * rG / rho;
  double vm, em;
  closure_fwd<PRK>(C, p, T, Y, vm, em);
  double ke = 0.0;
  for (int d = 0; d < D; ++d) ke += u[d] * u[d];
  q[0] = rho - rho * Y;
  q[1] = rho * Y;
  for (int d = 0; d < D; ++d) q[2 + d] = rho * u[d];
  q[2 + D] = rho * (em + 0.5 * ke);
}

// is the cell a ghost beyond a far-field side (in any direction)?
template <int D>
__device__ inline bool beyond_farfield(const CaseC& C, int gx, int gy, int gz)
{
  if (!C.any_ff) return false;
  bool f = (gx < 0 && C.bc[0][0] == BC_FARFIELD) || (gx >= C.n[0] && C.bc[0][1] == BC_FARFIELD);
  if (D >= 2) f = f || (gy < 0 && C.bc[1][0] == BC_FARFIELD) || (gy >= C.n[1] && C.bc[1][1] == BC_FARFIELD);
  if (D >= 3) f = f || (gz < 0 && C.bc[2][0] == BC_FARFIELD) || (gz >= C.n[2] && C.bc[2][1] == BC_FARFIELD);
  return f;
}

// true when the two-cell halo of the TX (x TY) tile at x0 (, y0) lies inside
// its case, so that no cell of it is a ghost, and every cell of the case sits
// within 32-bit byte offsets of its row's base (the loads of such a tile skip
// the boundary logic and address in 32 bits)
template <class S, int D>
__device__ inline bool halo_inside12(const CaseC& C, int x0, int y0, int TX, int TY)
{
  bool in = x0 >= 2 && x0 + TX + 2 <= C.n[0];
  if (D == 2) in = in && y0 >= 2 && y0 + TY + 2 <= C.n[1];
  return in && (long long)C.n[0] * (D == 2 ? C.n[1] : 1) * (long long)sizeof(S) <= 0xffffffffLL;
}

// true when the two-cell halo of the TX x TY x TZ tile at (x0, y0, z0) lies
// inside its case, so that no cell of it is a ghost, and every cell of the
// case sits within 32-bit byte offsets of its row's base (the loads of such a
// tile skip the boundary logic and address in 32 bits)
template <class S>
__device__ inline bool halo_inside3(const CaseC& C, int x0, int y0, int z0, int TX, int TY, int TZ)
{
  return x0 >= 2 && y0 >= 2 && z0 >= 2 && x0 + TX + 2 <= C.n[0] && y0 + TY + 2 <= C.n[1] &&
         z0 + TZ + 2 <= C.n[2] && (long long)C.n[0] * C.n[1] * C.n[2] * (long long)sizeof(S) <= 0xffffffffLL;
}

// load one (possibly ghost) cell: physical partial densities, momentum, gauge
// energy (and the second gas's partial density with G2)
template <class S, int D, bool PRK, bool G2 = false>
__device__ inline void load_cell(const CaseC& C, const S* __restrict__ src, long long total,
                                 int gx, int gy, int gz, long long step, double* q)
{
  if (beyond_farfield<D>(C, gx, gy, gz)) {
    const double u0[3] = {0.0, 0.0, 0.0};
    state_from_prim<PRK, G2>(C, C.ff_p, C.ff_T, C.ff_alpha, u0, D, q);
    return;
  }
  bool fx = false, fy = false, fz = false;
  int ix = gx, iy = gy, iz = gz;
  if (D >= 2) map_index(iy, C.n[1], C.bc[1][0], C.bc[1][1], fy);
  if (D >= 3) map_index(iz, C.n[2], C.bc[2][0], C.bc[2][1], fz);
  if (ix < 0 && C.bc[0][0] == BC_INFLOW) {
    double yy = (D >= 2) ? (iy + 0.5) * C.dx[1] - C.in_c0 : 0.0;
    double zz = (D >= 3) ? (iz + 0.5) * C.dx[2] - C.in_c1 : 0.0;
    if (D == 1 || sqrt(yy * yy + zz * zz) < C.in_radius) {
      double u[3] = {C.in_u, 0.0, 0.0};
      for (int c = 0; c < D; ++c)
        u[c] += C.in_noise * C.in_u *
                (2.0 * noise01(C.in_seed, (unsigned long long)step, (unsigned long long)iy,
                               (unsigned long long)iz, (unsigned long long)c) - 1.0);
      state_from_prim<PRK, G2>(C, C.in_p, C.in_T, C.in_alpha, u, D, q);
      if (D >= 2 && fy) q[3] = -q[3];
      if (D >= 3 && fz) q[4] = -q[4];
      return;
    }
    ix = -1 - ix;
    fx = true;
  } else {
    map_index(ix, C.n[0], C.bc[0][0], C.bc[0][1], fx);
  }
  long long cell = C.off + ix + (long long)C.n[0] * (iy + (long long)C.n[1] * iz);
  q[0] = (double)src[cell] + C.rref[0];
  q[1] = (double)src[total + cell] + C.rref[1];
#pragma unroll
  for (int d = 0; d < D; ++d) q[2 + d] = (double)src[(2 + d) * total + cell];
  q[2 + D] = (double)src[(2 + D) * total + cell];
  if constexpr (G2) q[3 + D] = (double)src[(3 + D) * total + cell] + C.rref[2];
  if (fx) q[2] = -q[2];
  if (D >= 2 && fy) q[3] = -q[3];
  if (D >= 3 && fz) q[4] = -q[4];
}

// primitives of a loaded cell
template <int D, bool PRK>
__device__ inline PT cell_prim(const CaseC& C, const double* q, double* u, double& rho, double& Y,
                               double Tw = 0.0, double pw = 0.0)
{
  rho = q[0] + q[1];
  double ir = frcp(rho);
  Y = q[1] * ir;
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) { u[d] = q[2 + d] * ir; ke += u[d] * u[d]; }
  double e = q[2 + D] * ir - 0.5 * ke;
  return closure<PRK>(C, rho, Y, e, Tw, pw);
}

// primitives of a loaded three-component cell (second gas at index 3 + D)
template <int D>
__device__ inline PT cell_prim3(const CaseC& C, const double* q, double* u, double& rho, double& Y,
                                double& Y2)
{
  rho = q[0] + q[1] + q[3 + D];
  double ir = frcp(rho);
  Y = q[1] * ir;
  Y2 = q[3 + D] * ir;
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) { u[d] = q[2 + d] * ir; ke += u[d] * u[d]; }
  double e = q[2 + D] * ir - 0.5 * ke;
  return closure3(C, rho, Y, Y2, e);
}

// either closure: G2 selects the three-component one
template <int D, bool PRK, bool G2>
__device__ inline PT cell_prim_any(const CaseC& C, const double* q, double* u, double& rho, double& Y,
                                   double& Y2)
{
  if constexpr (G2) return cell_prim3<D>(C, q, u, rho, Y, Y2);
  Y2 = 0.0;
  return cell_prim<D, PRK>(C, q, u, rho, Y);
}

__device__ inline void record_error(CaseDyn& dy, int code, long long cell, long long step)
{
  if (atomicCAS(&dy.err, 0, code) == 0) {
    dy.err_cell = cell;
    dy.err_step = step;
  }
}

__device__ inline double wave_max(double v)
{
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Apply fn to every face index f < NF, NT threads: the full rounds are taken two
// at a time with independent faces per thread, so that the two face
// evaluations interleave and hide each other's latency; the partial round last.
template <int NF, int NT, class Fn>
__device__ inline void for_faces(int tid, Fn&& fn)
{
  constexpr int FULL = NF / NT;
  int f = tid;
#pragma unroll 1
  for (int r = 0; r + 1 < FULL; r += 2, f += 2 * NT) {
    fn(f);
    fn(f + NT);
  }
  if (FULL & 1) {
    fn(f);
    f += NT;
  }
  if (f < NF) fn(f);
}

// dt of the step `step` of a case, identical in every workgroup of every stage:
// CFL / (max over cells of sum_d (|u_d| + c) / dx_d of q^n), shortened so that
// the step ends on t_end; NaN or a non-positive bound gives dt = 0
__device__ inline double step_dt(const CaseDyn& dy, long long step, double cfl, double t_end)
{
  int s = (int)(step & 1);
  unsigned long long mb = 0ull;
#pragma unroll
  for (int i = 0; i < NSLOT; ++i) mb = mb > dy.dtmax[s][i] ? mb : dy.dtmax[s][i];
  double lam = __longlong_as_double((long long)mb);
  double dt = cfl / lam;
  double t = dy.t[s];
  if (t_end > 0.0 && t + dt > t_end) dt = t_end - t;
  if (!(dt > 0.0) || !(dt < 1e300)) dt = 0.0;
  return dt;
}

// first workgroup of a case in the first stage: time at the end of the step,
// and the CFL slot of q^(n+1) cleared for the last stage's reduction
__device__ inline void step_scalars(CaseDyn& dy, long long step, double dt)
{
  int s = (int)(step & 1);
  dy.t[s ^ 1] = dy.t[s] + dt;
#pragma unroll
  for (int i = 0; i < NSLOT; ++i) dy.dtmax[s ^ 1][i] = 0ull;
  dy.dt_last = dt;
}

// ------------------------------------------------------------------ XCD-aware tile order
// Workgroups are dealt to the 8 XCDs round-robin (block b to XCD b % 8), and
// each XCD has its own L2.  Remapping block b to tile
//   (b % 8) * q + min(b % 8, r) + b / 8,   q = n / 8, r = n % 8,
// gives each XCD one contiguous run of tiles, so neighbouring tiles, whose
// halos overlap, are served by the same L2.  A permutation of [0, n).
__device__ inline int xcd_block(int b, int n)
{
  constexpr int NX = 8;
  int q = n / NX, r = n % NX, k = b % NX;
  return k * q + (k < r ? k : r) + b / NX;
}

// ------------------------------------------------------------------ viscous stress, heat conduction
// transport coefficient of a cell from its gas volume fraction: eq. (2-8) with
// one gas and no vapour, (1 - alpha_G) v0 + alpha_G v1
template <class S>
__device__ inline S mix_alpha(double v0, double v1, S a)
{
  S ac = a < S(0) ? S(0) : (a > S(1) ? S(1) : a);
  return (S(1) - ac) * S(v0) + ac * S(v1);
}

// three components: (1 - alpha_1 - alpha_2) v0 + alpha_1 v1 + alpha_2 v2, the
// fractions clipped into [0, 1] and rescaled when they sum above one
template <class S>
__device__ inline S mix_alpha3(double v0, double v1, double v2, S a, S b)
{
  S ac = a < S(0) ? S(0) : (a > S(1) ? S(1) : a);
  S bc = b < S(0) ? S(0) : (b > S(1) ? S(1) : b);
  S sum = ac + bc;
  if (sum > S(1)) { ac = ac / sum; bc = bc / sum; }
  return (S(1) - ac - bc) * S(v0) + ac * S(v1) + bc * S(v2);
}

// Stress part of the flux of eq. (2-2) through the face between the LDS cells
// c and c + st[DIR], second-order central: normal derivatives from the two
// cells, transverse ones as the mean of the two cells' central differences,
// face coefficients and face velocity as the two cells' mean.
//   tau = mu (grad u + grad u^T - 2/3 div u I);  F_rho u -= tau . n,
//   F_rho E -= u . tau . n + kc dT/dn.
// U[a]: LDS array of velocity component a; st: LDS strides of the directions.
template <class S, int D, int DIR, bool G2 = false>
__device__ inline void visc_flux(const CaseC& C, const S* const (&U)[D], const S* sT, const S* sA, int c,
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
  const S aL = sA[c], aR = sA[r];
  S mu, kc;
  if constexpr (G2) {
    const S bL = sA2[c], bR = sA2[r];
    const Comp* k = C.comp;
    mu = S(0.5) * (mix_alpha3<S>(k[0].mu, k[1].mu, k[2].mu, aL, bL) + mix_alpha3<S>(k[0].mu, k[1].mu, k[2].mu, aR, bR));
    kc = S(0.5) * (mix_alpha3<S>(k[0].kc, k[1].kc, k[2].kc, aL, bL) + mix_alpha3<S>(k[0].kc, k[1].kc, k[2].kc, aR, bR));
  } else {
    mu = S(0.5) * (mix_alpha<S>(C.comp[0].mu, C.comp[1].mu, aL) + mix_alpha<S>(C.comp[0].mu, C.comp[1].mu, aR));
    kc = S(0.5) * (mix_alpha<S>(C.comp[0].kc, C.comp[1].kc, aL) + mix_alpha<S>(C.comp[0].kc, C.comp[1].kc, aR));
  }
  S work = S(0);
#pragma unroll
  for (int a = 0; a < D; ++a) {
    S tau = mu * (g[a][DIR] + g[DIR][a]);
    if (a == DIR) tau -= S(2.0 / 3.0) * mu * div;
    F[2 + a] -= tau;
    work += S(0.5) * (U[a][c] + U[a][r]) * tau;
  }
  F[2 + D] -= work + kc * (sT[r] - sT[c]) * S(C.idx[DIR]);
}

// CFL rate of a cell: sum_d (|u_d| + c) / dx_d, plus 2 nu sum_d 1/dx_d^2 with
// nu = max(mu, kc / cv) / rho (cv mixed by mass fraction) for viscous or
// conducting fluids (explicit diffusion limit)
template <int D, bool G2 = false>
__device__ inline double cfl_rate(const CaseC& C, const double* u, const PT& pt, double rho, double Y,
                                  double Y2 = 0.0)
{
  double l = 0.0;
#pragma unroll
  for (int d = 0; d < D; ++d) l += (fabs(u[d]) + pt.c) * C.idx[d];
  if (C.diff) {
    double cvm, mu, kc;
    const Comp* k = C.comp;
    if constexpr (G2) {
      double y0, y1, y2;
      clip_fractions3(Y, Y2, y0, y1, y2);
      cvm = y0 * k[0].cv + y1 * k[1].cv + y2 * k[2].cv;
      mu = mix_alpha3<double>(k[0].mu, k[1].mu, k[2].mu, pt.alpha, pt.alpha2);
      kc = mix_alpha3<double>(k[0].kc, k[1].kc, k[2].kc, pt.alpha, pt.alpha2) / cvm;
    } else {
      double Yc = Y < 0.0 ? 0.0 : (Y > 1.0 ? 1.0 : Y);
      cvm = (1.0 - Yc) * k[0].cv + Yc * k[1].cv;
      mu = mix_alpha<double>(k[0].mu, k[1].mu, pt.alpha);
      kc = mix_alpha<double>(k[0].kc, k[1].kc, pt.alpha) / cvm;
    }
    l += 2.0 * (mu > kc ? mu : kc) / rho * C.sdx2;
  }
  return l;
}

// fold a workgroup's CFL bound into its slot: one unsigned 64-bit atomic max
// with no return value (a non-negative double orders like its bit pattern);
// spreading the workgroups over NSLOT slots keeps the contention per address
// low, and a read of the slot first to skip the atomic was measured slower
// (the load's latency lands on the last wave of every workgroup)
__device__ inline void cfl_max(CaseDyn& dy, int s, double m)
{
  unsigned long long bits = (unsigned long long)__double_as_longlong(m);
  atomicMax(&dy.dtmax[s][blockIdx.x % NSLOT], bits);
}

}  // namespace fvm
