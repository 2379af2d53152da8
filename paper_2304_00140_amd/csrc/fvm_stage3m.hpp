// fvm_stage3m.hpp -- 3D stage as one kernel per Runge-Kutta stage that marches
// along z through a column of tiles (two-component closures: stiffened-gas
// pair or Peng-Robinson gas; inviscid, with or without gravity, CSF and
// sensor switching; the default limiter pair).
//
// A workgroup owns a TX x TY column of cells and a chunk of ZC planes.  It
// walks the planes upwards keeping three planes of primitives (k, k+1, k+2)
// with the two-cell x-y halo of the four-cell stencil (Fig. 3.1) in LDS; the
// FP64 closure inversion of each new plane is done once per staged cell, so
// q^(k-1) is read from HBM once per cell and stage (plus the x-y halo, which
// neighbouring workgroups of the same XCD share through L2).  Per plane:
//   A  closure of plane k+2 (ghosts from the boundary kinds) -> LDS ring;
//   B  sensors (Appendix D) and the Gaussian-smoothed mass fraction (eq. 3-9,
//      /64) of plane k+1 on the one-cell halo;
//   C  vertex normals between planes k and k+1; every x and y face of plane k
//      (flux to LDS); the z face k+1/2 of each owned column (flux kept in
//      registers, where it is the lower face of plane k+1 next);
//   D  divergence, CSF (kappa from the normals below and above the plane),
//      body force, update of plane k; the last stage also inverts the closure
//      of q^(n+1) for the CFL bound of the next step and its checks.
// The column values of plane k-1 that the z faces need are kept in
// registers, so the ring holds three planes.
#pragma once
#include <hip/hip_runtime.h>
#include "fvm_device.hpp"
#include "fvm_kernels.hpp"
#include "fvm_stage_common.hpp"
#include "fvm_stage3_prim.hpp"

namespace fvm {

// FUSED: the closure of each staged cell is computed here from q^(k-1);
// otherwise the primitives come from the buffer a.prim that the closure
// kernel k_prim3 wrote for this stage (ghosts from the boundary kinds either
// way), and k_prim3 also supplies the CFL bound of q^n at the first stage.
template <class S, int TX, int TY, int ZC, int MINW, bool PRK, int LIM, bool FUSED>
__global__ __launch_bounds__(TX * TY, MINW) void k_march3(StageArgs a)
{
  constexpr int NT = TX * TY;
  constexpr int HX = TX + 4, HY = TY + 4, NH = HX * HY;   // plane with the two-cell halo
  constexpr int FX = TX + 2, FY = TY + 2, NH1 = FX * FY;  // plane with a one-cell halo
  constexpr int VX = TX + 1, VY = TY + 1, NV = VX * VY;   // vertices of a plane
  constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1), NF = NFX + NFY;
  constexpr int NQ = 6;
  constexpr int NW = 9;    // rho, u, v, w, p, T, xi, c, alpha_G
  constexpr int NIT = (NH + NT - 1) / NT;
  enum { WR = 0, WU = 1, WV = 2, WW = 3, WP = 4, WT = 5, WY = 6, WC = 7, WA = 8 };

  __shared__ S s_w[3][NW][NH];
  __shared__ unsigned char s_fl[2][NH1];
  __shared__ S s_H[2][NH1];
  __shared__ S s_n[2][3][NV];
  __shared__ S s_F[NQ][NF];
  __shared__ double s_red[NT / 64];

  const int4 tl = a.tiles[xcd_block(blockIdx.x, gridDim.x)];
  const CaseC& C = a.cases[tl.x];
  CaseDyn& dy = a.dyn[tl.x];
  const SchemeC& SC = a.sc;
  const int x0 = tl.y * TX, y0 = tl.z * TY, z0 = tl.w * ZC;
  const int z1 = min(z0 + ZC, C.n[2]);
  const int tid = threadIdx.x;
  const int ti = tid % TX, tj = tid / TX;
  const int gx = x0 + ti, gy = y0 + tj;
  const bool own_xy = gx < C.n[0] && gy < C.n[1];
  const bool upd = a.stage >= 0;
  const long long step = upd ? dy.base + a.step_off : a.rhs_step;
  const S* __restrict__ src = (const S*)a.src;
  const S* __restrict__ qn = (const S*)a.qn;
  const long long T = a.total;
  const bool sw = SC.switching != 0;
  const bool csf = SC.sigma > 0.0;
  const S eps = S(SC.eps_int);
  const int cown = (tj + 2) * HX + ti + 2;        // owned cell in the two-cell-halo plane
  const int c1own = (tj + 1) * FX + ti + 1;       // owned cell in the one-cell-halo plane
  // ring slot of plane z: planes z0-2, z0-1, z0 take slots 0, 1, 2, then cyclic
  auto slot = [&](int z) { return (z - z0 + 2) % 3; };
  auto par = [&](int z) { return (z - z0 + 2) & 1; };   // flags, smoothed xi: slot of plane z

  // ---- staging of plane z on the two-cell x-y halo into ring slot sl: the
  // FP64 closure of each staged cell (FUSED), or the primitives k_prim3 wrote
  // (ghosts from the boundary kinds either way); all loads of a thread first
  auto stage_plane = [&](int z, int sl) {
    if constexpr (!FUSED) {
      const S* __restrict__ W = (const S*)a.prim;
      S w[NIT][NW];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        int h = tid + it * NT;
        if (h < NH) load_prim3<S, PRK, false>(C, W, T, x0 + h % HX - 2, y0 + h / HX - 2, z, step, w[it]);
      }
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        int h = tid + it * NT;
        if (h < NH) {
#pragma unroll
          for (int v = 0; v < NW; ++v) s_w[sl][v][h] = w[it][v];
        }
      }
      return;
    }
    double qv[NIT][NQ];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      int h = tid + it * NT;
      if (h < NH) load_cell<S, 3, PRK>(C, src, T, x0 + h % HX - 2, y0 + h / HX - 2, z, step, qv[it]);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      int h = tid + it * NT;
      if (h < NH) {
        double u[3], rho, Y;
        PT pt = cell_prim<3, PRK>(C, qv[it], u, rho, Y);
        s_w[sl][WR][h] = S(rho);
        s_w[sl][WU][h] = S(u[0]);
        s_w[sl][WV][h] = S(u[1]);
        s_w[sl][WW][h] = S(u[2]);
        s_w[sl][WP][h] = S(pt.p);
        s_w[sl][WT][h] = S(pt.T);
        s_w[sl][WY][h] = S(Y);
        s_w[sl][WC][h] = S(pt.c);
        s_w[sl][WA][h] = S(pt.alpha);
      }
    }
  };

  // ---- sensors (eq. D.4) and the smoothed mass fraction of plane z (slots of
  // planes z-1, z, z+1 given) on the one-cell halo
  auto sensors_gauss = [&](int z, int sm, int s0, int sp) {
    const int st[2] = {1, HX};
    for (int h1 = tid; h1 < NH1; h1 += NT) {
      int lx = h1 % FX, ly = h1 / FX;
      int c = (ly + 1) * HX + lx + 1;
      if (sw) {
        S g[3][3];
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) {
#pragma unroll
          for (int d = 0; d < 2; ++d)
            g[comp][d] = (s_w[s0][WU + comp][c + st[d]] - s_w[s0][WU + comp][c - st[d]]) * S(0.5 * C.idx[d]);
          g[comp][2] = (s_w[sp][WU + comp][c] - s_w[sm][WU + comp][c]) * S(0.5 * C.idx[2]);
        }
        S div = g[0][0] + g[1][1] + g[2][2];
        S w0 = g[2][1] - g[1][2], w1 = g[0][2] - g[2][0], w2 = g[1][0] - g[0][1];
        S curl2 = w0 * w0 + w1 * w1 + w2 * w2;
        const S* al = s_w[s0][WA];
        S thg = S(0);
#pragma unroll
        for (int d = 0; d < 2; ++d) thg += fabs(al[c] - al[c - st[d]]) + fabs(al[c + st[d]] - al[c]);
        thg += fabs(al[c] - s_w[sm][WA][c]) + fabs(s_w[sp][WA][c] - al[c]);
        S thd = fdiv(div * div, div * div + curl2 + S(SC.eps_d));
        s_fl[par(z)][h1] = (thd > S(SC.th_d) || thg > S(SC.th_g)) ? 1 : 0;
      }
      if (csf) {
        // binomial 1-2-1 kernel in each direction (eq. 3-9), /64
        const int sl3[3] = {sm, s0, sp};
        S acc = S(0);
#pragma unroll
        for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
          for (int dyy = -1; dyy <= 1; ++dyy) {
            const S* Yp = s_w[sl3[dz + 1]][WY];
            S row = Yp[c + dyy * HX - 1] + S(2) * Yp[c + dyy * HX] + Yp[c + dyy * HX + 1];
            acc += row * S((dz == 0 ? 2 : 1) * (dyy == 0 ? 2 : 1));
          }
        s_H[par(z)][h1] = acc * S(1.0 / 64.0);
      }
    }
  };

  // ---- unit normals at the vertices between planes z and z+1, from the
  // smoothed mass fraction of the 2 x 2 x 2 cells around each vertex
  auto normals = [&](int z) {
    const S* lo = s_H[par(z)];
    const S* hi = s_H[par(z + 1)];
    S* n = &s_n[par(z)][0][0];
    const S en = S(SC.eps_n * C.idx[0]);
    for (int v = tid; v < NV; v += NT) {
      int vx = v % VX, vy = v / VX;      // upper corner of the cell (vx - 1, vy - 1) of plane z
      int c = vy * FX + vx;              // that cell in the one-cell-halo plane
      S gxv = (lo[c + 1] + lo[c + 1 + FX] + hi[c + 1] + hi[c + 1 + FX] - lo[c] - lo[c + FX] - hi[c] - hi[c + FX]) *
              S(0.25 * C.idx[0]);
      S gyv = (lo[c + FX] + lo[c + FX + 1] + hi[c + FX] + hi[c + FX + 1] - lo[c] - lo[c + 1] - hi[c] - hi[c + 1]) *
              S(0.25 * C.idx[1]);
      S gzv = (hi[c] + hi[c + 1] + hi[c + FX] + hi[c + FX + 1] - lo[c] - lo[c + 1] - lo[c + FX] - lo[c + FX + 1]) *
              S(0.25 * C.idx[2]);
      S inv = frcp(sqrt(gxv * gxv + gyv * gyv + gzv * gzv) + en);
      n[v] = gxv * inv;
      n[NV + v] = gyv * inv;
      n[2 * NV + v] = gzv * inv;
    }
  };

  // column values of the owned cell's plane below the ring (z faces)
  struct Col { S u[3], p, T, Y, a; };
  auto col_from = [&](int sl) {
    Col k;
#pragma unroll
    for (int d = 0; d < 3; ++d) k.u[d] = s_w[sl][WU + d][cown];
    k.p = s_w[sl][WP][cown];
    k.T = s_w[sl][WT][cown];
    k.Y = s_w[sl][WY][cown];
    k.a = s_w[sl][WA][cown];
    return k;
  };

  // z face between plane z (slot s0) and z+1 (slot s1), stencil planes z-1
  // (registers), z, z+1, z+2 (slot s2)
  auto zface = [&](const Col& km, int z, int s0, int s1, int s2, S* F) {
    Stencil<S, 3> st;
    const int sl[3] = {s0, s1, s2};
#pragma unroll
    for (int d = 0; d < 3; ++d) st.u[d][0] = km.u[d];
    st.p[0] = km.p;
    st.T[0] = km.T;
    st.Y[0] = km.Y;
#pragma unroll
    for (int m = 1; m < 4; ++m) {
#pragma unroll
      for (int d = 0; d < 3; ++d) st.u[d][m] = s_w[sl[m - 1]][WU + d][cown];
      st.p[m] = s_w[sl[m - 1]][WP][cown];
      st.T[m] = s_w[sl[m - 1]][WT][cown];
      st.Y[m] = s_w[sl[m - 1]][WY][cown];
    }
    st.rho1 = s_w[s0][WR][cown];
    st.rho2 = s_w[s1][WR][cown];
    st.c1 = s_w[s0][WC][cown];
    st.c2 = s_w[s1][WC][cown];
    bool disc = !sw || ((s_fl[par(z)][c1own] | s_fl[par(z + 1)][c1own]) != 0);
    face_flux<S, 3, 2, PRK, false, LIM>(SC, C, st, disc, eligible(st.Y[0], st.Y[1], st.Y[2], eps),
                                        eligible(st.Y[1], st.Y[2], st.Y[3], eps), F);
  };

  // x or y face f of plane z (slot s0) into the LDS flux buffer
  auto xyface = [&](int f, int z, int s0) {
    Stencil<S, 3> st;
    S F[NQ];
    const S* w = &s_w[s0][0][0];
    if (f < NFX) {
      int i = f % (TX + 1), j = f / (TX + 1);
      int c = (j + 2) * HX + i + 1;            // lower cell of the face
#pragma unroll
      for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int d = 0; d < 3; ++d) st.u[d][m] = w[(WU + d) * NH + c - 1 + m];
        st.p[m] = w[WP * NH + c - 1 + m];
        st.T[m] = w[WT * NH + c - 1 + m];
        st.Y[m] = w[WY * NH + c - 1 + m];
      }
      st.rho1 = w[WR * NH + c];
      st.rho2 = w[WR * NH + c + 1];
      st.c1 = w[WC * NH + c];
      st.c2 = w[WC * NH + c + 1];
      int c1 = (j + 1) * FX + i;
      bool disc = !sw || ((s_fl[par(z)][c1] | s_fl[par(z)][c1 + 1]) != 0);
      face_flux<S, 3, 0, PRK, false, LIM>(SC, C, st, disc, eligible(st.Y[0], st.Y[1], st.Y[2], eps),
                                          eligible(st.Y[1], st.Y[2], st.Y[3], eps), F);
    } else {
      int g = f - NFX;
      int i = g % TX, j = g / TX;
      int c = (j + 1) * HX + i + 2;            // lower cell of the face
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        int cm = c + (m - 1) * HX;
#pragma unroll
        for (int d = 0; d < 3; ++d) st.u[d][m] = w[(WU + d) * NH + cm];
        st.p[m] = w[WP * NH + cm];
        st.T[m] = w[WT * NH + cm];
        st.Y[m] = w[WY * NH + cm];
      }
      st.rho1 = w[WR * NH + c];
      st.rho2 = w[WR * NH + c + HX];
      st.c1 = w[WC * NH + c];
      st.c2 = w[WC * NH + c + HX];
      int c1 = j * FX + i + 1;
      bool disc = !sw || ((s_fl[par(z)][c1] | s_fl[par(z)][c1 + FX]) != 0);
      face_flux<S, 3, 1, PRK, false, LIM>(SC, C, st, disc, eligible(st.Y[0], st.Y[1], st.Y[2], eps),
                                          eligible(st.Y[1], st.Y[2], st.Y[3], eps), F);
    }
#pragma unroll
    for (int v = 0; v < NQ; ++v) s_F[v][f] = F[v];
  };

  // ---------------------------------------------------------------- prologue
  // planes z0-2 .. z0+1, the sensors and smoothed xi of z0-1 and z0, the
  // normals between them and the z face z0-1/2
  stage_plane(z0 - 2, 0);
  stage_plane(z0 - 1, 1);
  stage_plane(z0, 2);
  __syncthreads();
  sensors_gauss(z0 - 1, 0, 1, 2);
  Col km2 = col_from(0);
  __syncthreads();
  stage_plane(z0 + 1, 0);
  __syncthreads();
  sensors_gauss(z0, 1, 2, 0);
  __syncthreads();
  if (csf) normals(z0 - 1);
  S Flo[NQ];
  zface(km2, z0 - 1, 1, 2, 0, Flo);
  Col km1 = col_from(1);
  __syncthreads();

  const double dt = upd ? step_dt(dy, step, SC.cfl, SC.t_end) : 0.0;
  if (upd && a.stage == 0 && tl.y == 0 && tl.z == 0 && tl.w == 0 && tid == 0) step_scalars(dy, step, dt);
  S* dst = (S*)a.dst;
  double* rhs_out = a.rhs_out;
  const S adt = S(a.ak * dt);
  double lam = 0.0;

  // ---------------------------------------------------------------- march
  for (int k = z0; k < z1; ++k) {
    const int s0 = slot(k), s1 = slot(k + 1), s2 = slot(k + 2);
    const long long cell = C.off + gx + (long long)C.n[0] * (gy + (long long)C.n[1] * k);
    S qn_reg[NQ];
    if (upd && own_xy) {
#pragma unroll
      for (int v = 0; v < NQ; ++v) qn_reg[v] = qn[v * T + cell];
    }
    // A
    stage_plane(k + 2, s2);
    __syncthreads();
    // B
    sensors_gauss(k + 1, s0, s1, s2);
    __syncthreads();
    // C
    if (csf) normals(k);
    for (int f = tid; f < 2 * NT && f < NF; f += NT) xyface(f, k, s0);
    S Fhi[NQ];
    zface(km1, k, s0, s1, s2, Fhi);
    for (int f = tid + 2 * NT; f < NF; f += NT) xyface(f, k, s0);
    __syncthreads();
    // D
    S R[NQ];
    {
      const int fx = tj * (TX + 1) + ti, fy = NFX + tj * TX + ti;
      const S ix = S(C.idx[0]), iy = S(C.idx[1]), iz = S(C.idx[2]);
#pragma unroll
      for (int v = 0; v < NQ; ++v)
        R[v] = (s_F[v][fx] - s_F[v][fx + 1]) * ix + (s_F[v][fy] - s_F[v][fy + TX]) * iy + (Flo[v] - Fhi[v]) * iz;
    }
    const S* al = s_w[s0][WA];
    if (csf) {
      const S* nd = &s_n[par(k - 1)][0][0];
      const S* nu = &s_n[par(k)][0][0];
      const int vi = (tj + 1) * VX + ti + 1;   // upper corner of the owned cell
      S kap = S(0);
      {
        const S* a0 = nu;
        const S* b0 = nd;
        S plus = a0[vi] + a0[vi - VX] + b0[vi] + b0[vi - VX];
        S minus = a0[vi - 1] + a0[vi - 1 - VX] + b0[vi - 1] + b0[vi - 1 - VX];
        kap += (plus - minus) * S(0.25 * C.idx[0]);
      }
      {
        const S* a1 = nu + NV;
        const S* b1 = nd + NV;
        S plus = a1[vi] + b1[vi] + a1[vi - 1] + b1[vi - 1];
        S minus = a1[vi - VX] + b1[vi - VX] + a1[vi - VX - 1] + b1[vi - VX - 1];
        kap += (plus - minus) * S(0.25 * C.idx[1]);
      }
      {
        const S* a2 = nu + 2 * NV;
        const S* b2 = nd + 2 * NV;
        S plus = a2[vi] + a2[vi - 1] + a2[vi - VX] + a2[vi - 1 - VX];
        S minus = b2[vi] + b2[vi - 1] + b2[vi - VX] + b2[vi - 1 - VX];
        kap += (plus - minus) * S(0.25 * C.idx[2]);
      }
      kap = -kap;
      const S sig = S(SC.sigma);
      S Sd[3];
      Sd[0] = sig * kap * (al[cown + 1] - al[cown - 1]) * S(0.5 * C.idx[0]);
      Sd[1] = sig * kap * (al[cown + HX] - al[cown - HX]) * S(0.5 * C.idx[1]);
      Sd[2] = sig * kap * (s_w[s1][WA][cown] - km1.a) * S(0.5 * C.idx[2]);
      S se = S(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        R[2 + d] += Sd[d];
        se += s_w[s0][WU + d][cown] * Sd[d];
      }
      R[5] += se;
    }
    if (SC.has_grav) {
      S rho = s_w[s0][WR][cown], pw = S(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        S gd = S(SC.grav[d]);
        R[2 + d] += rho * gd;
        pw += s_w[s0][WU + d][cown] * gd;
      }
      R[5] += rho * pw;
    }
    if (own_xy) {
      if (!upd) {
        const long long RS = C.ncell;
        const long long cl = cell - C.off;
        double r0 = (double)R[0], r1 = (double)R[1];
        rhs_out[cl] = r0 + r1;
#pragma unroll
        for (int d = 0; d < 3; ++d) rhs_out[(1 + d) * RS + cl] = (double)R[2 + d];
        rhs_out[4 * RS + cl] = (double)R[5] + C.Q[0] * r0 + C.Q[1] * r1;
        rhs_out[5 * RS + cl] = r1;
      } else {
        S nv[NQ];
#pragma unroll
        for (int v = 0; v < NQ; ++v) {
          nv[v] = qn_reg[v] + adt * R[v];
          dst[v * T + cell] = nv[v];
        }
        if (FUSED && a.stage == 3) {
          double q[NQ], u[3], rho, Y;
          q[0] = (double)nv[0] + C.rref[0];
          q[1] = (double)nv[1] + C.rref[1];
#pragma unroll
          for (int v = 2; v < NQ; ++v) q[v] = (double)nv[v];
          PT pt = cell_prim<3, PRK>(C, q, u, rho, Y);
          double l = cfl_rate<3>(C, u, pt, rho, Y);
          if (!isfinite(l) || !isfinite(pt.p)) record_error(dy, ERR_NAN, cell - C.off, step);
          else if (!(rho > 0.0) || !(pt.T > 0.0) || !pt.ok) record_error(dy, ERR_NONPHYS, cell - C.off, step);
          else lam = fmax(lam, l);
        }
      }
    }
    // the owned column of plane k is the lower stencil cell of the next z face
    km1 = col_from(s0);
#pragma unroll
    for (int v = 0; v < NQ; ++v) Flo[v] = Fhi[v];
    __syncthreads();
  }
  if (FUSED && upd && a.stage == 3) {
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

// z-marching tile shapes (tx, ty, planes per workgroup); threads = tx * ty
constexpr int TILESM[][3] = {{32, 8, 32}, {16, 16, 32}, {32, 8, 64}, {16, 8, 32}, {32, 4, 32}};
constexpr int NTM = sizeof(TILESM) / sizeof(TILESM[0]);

}  // namespace fvm
