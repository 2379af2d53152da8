// fvm_stage12.hpp -- the fused 1D/2D stage kernel (one Runge-Kutta stage per
// launch, Algorithm 1) and its tile dispatch, shared by the translation units
// that instantiate it with run-time limiters and with the default limiters
// fixed at compile time (LIM = 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "fvm_device.hpp"
#include "fvm_kernels.hpp"
#include "fvm_stage_common.hpp"

namespace fvm {

// ------------------------------------------------------------------ fused 1D/2D stage
// One fused kernel per Runge-Kutta stage (Algorithm 1): a workgroup owns a
// tile of cells, stages the tile plus the two-cell halo of the four-cell
// stencil (Fig. 3.1) in LDS after inverting the closure in FP64 for every
// staged cell, evaluates the sensors (Appendix D), every face flux of the tile
// once (Section 3.2/3.3), the CSF source (Section 3.5) and writes
// q^(k) = q^n + a_k dt R.  Ghost cells are generated from the boundary kinds
// while loading; the last stage also reduces the CFL bound of the new state
// (wavefront shuffle -> LDS -> one atomicMax per workgroup) and flags cells
// that left the closure's domain.  Batches of cases run through the same
// kernels via a tile table (case, tile coordinates).
// Tile TX x TY cells, NT threads (NT may exceed TX*TY: then several threads
// share the halo and face work of fewer cells).  MINW: waves per SIMD the
// register budget is held to.
template <class S, int D, int TX, int TY, int NT, int MINW, bool PRK, bool G2, int LIM>
__global__ __launch_bounds__(NT, MINW) void k_stage12(StageArgs a)
{
  static_assert(D == 1 || D == 2, "1D/2D kernel");
  static_assert(D == 2 || TY == 1, "1D tiles are one row");
  constexpr int HX = TX + 4, HY = (D == 2) ? TY + 4 : 1, NH = HX * HY;
  constexpr int NQ = D + 3 + (G2 ? 1 : 0);   // G2: second gas, its partial density last
  constexpr int NC = TX * TY;
  constexpr int CPT = (NC + NT - 1) / NT;
  constexpr int NIT = (NH + NT - 1) / NT;
  constexpr int NFX = (TX + 1) * TY, NFY = (D == 2) ? TX * (TY + 1) : 0;
  constexpr int NF = NFX > NFY ? NFX : NFY;
  constexpr int OY = (D == 2) ? 2 : 0;          // halo offset in y
  constexpr int FX = TX + 2, FY = (D == 2) ? TY + 2 : 1;   // tile + one halo layer
  constexpr int VX = TX + 1, VY = (D == 2) ? TY + 1 : 1;   // vertices
  static_assert(FX * FY + D * VX * VY <= NQ * NF, "CSF scratch fits in the flux buffer");

  __shared__ S s_rho[NH], s_u[NH], s_v[D == 2 ? NH : 1], s_p[NH], s_T[NH], s_Y[NH], s_c[NH], s_a[NH];
  __shared__ S s_Y2[G2 ? NH : 1], s_a2[G2 ? NH : 1];
  // specific internal energy, staged for the internal-energy face closure
  // (run-time limiter kernels only)
  __shared__ S s_e[(LIM == 0 && !G2) ? NH : 1];
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

  // ---- q^n of the owned cells, fetched early so its latency overlaps the stencil work
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

  // ---- tile + halo: all loads first, then the FP64 closure inversion, primitives to LDS
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
          qv[it][1] += C.rref[1];
          if constexpr (G2) qv[it][3 + D] += C.rref[2];
        }
      }
    } else {
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        int h = tid + it * NT;
        if (h < NH) {
          int hx = h % HX, hy = h / HX;
          load_cell<S, D, PRK, G2>(C, src, T, x0 + hx - 2, (D == 2) ? y0 + hy - 2 : 0, 0, step, qv[it]);
        }
      }
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      int h = tid + it * NT;
      if (h < NH) {
        double u[D], rho, Y, Y2;
        PT pt = cell_prim_any<D, PRK, G2>(C, qv[it], u, rho, Y, Y2);
        s_rho[h] = S(rho);
        s_u[h] = S(u[0]);
        if (D == 2) s_v[h] = S(u[D - 1]);
        s_p[h] = S(pt.p);
        s_T[h] = S(pt.T);
        s_Y[h] = S(Y);
        s_c[h] = S(pt.c);
        s_a[h] = S(pt.alpha);
        if constexpr (G2) {
          s_Y2[h] = S(Y2);
          s_a2[h] = S(pt.alpha2);
        }
        if constexpr (LIM == 0 && !G2) {
          if (SC.recon_e) {
            // e in the unshifted gauge (the FP32 storage gauge subtracts
            // sum_k xi_k Q_k, which the face would otherwise reconstruct
            // apart from xi)
            double ke = u[0] * u[0];
            if (D == 2) ke += u[D - 1] * u[D - 1];
            s_e[h] = S(qv[it][2 + D] * frcp(rho) - 0.5 * ke + (1.0 - Y) * C.Q[0] + Y * C.Q[1]);
          }
        }
      }
    }
  }
  __syncthreads();
  // the thermal variable a face reconstructs: T, or e with the internal-energy
  // face closure
  const S* s_th = s_T;
  if constexpr (LIM == 0 && !G2) {
    if (SC.recon_e) s_th = s_e;
  }
  // total gas volume fraction and mass fraction of a staged cell
  auto aG = [&](int c) -> S {
    if constexpr (G2) return s_a[c] + s_a2[c];
    else return s_a[c];
  };
  auto YG = [&](int c) -> S {
    if constexpr (G2) return s_Y[c] + s_Y2[c];
    else return s_Y[c];
  };

  // ---- switching sensors (Appendix D) on tile + one halo layer
  if (SC.switching) {
    for (int h = tid; h < FX * FY; h += NT) {
      int lx = h % FX, ly = h / FX;
      int c = (ly + (D == 2 ? 1 : 0)) * HX + lx + 1;
      S idx2 = S(0.5 * C.idx[0]);
      S dudx = (s_u[c + 1] - s_u[c - 1]) * idx2;
      S div = dudx, curl2 = S(0);
      S thg = fabs(aG(c) - aG(c - 1)) + fabs(aG(c + 1) - aG(c));
      if (D == 2) {
        S idy2 = S(0.5 * C.idx[1]);
        S dvdy = (s_v[c + HX] - s_v[c - HX]) * idy2;
        S dvdx = (s_v[c + 1] - s_v[c - 1]) * idx2;
        S dudy = (s_u[c + HX] - s_u[c - HX]) * idy2;
        div += dvdy;
        S w = dvdx - dudy;
        curl2 = w * w;
        thg += fabs(aG(c) - aG(c - HX)) + fabs(aG(c + HX) - aG(c));
      }
      S thd = fdiv(div * div, div * div + curl2 + S(SC.eps_d));
      s_fl[c] = (thd > S(SC.th_d) || thg > S(SC.th_g)) ? 1 : 0;
    }
    __syncthreads();
  }

  S R[CPT][NQ];
#pragma unroll
  for (int k = 0; k < CPT; ++k)
#pragma unroll
    for (int v = 0; v < NQ; ++v) R[k][v] = S(0);

  const S eps = S(SC.eps_int);
  // velocity arrays and LDS strides for the stress terms and the body force
  const S* U[D];
  int stv[D];
  U[0] = s_u;
  stv[0] = 1;
  if constexpr (D == 2) { U[1] = s_v; stv[1] = HX; }
  // ---- x faces: face i-1/2 of tile column i = 0..TX, between LDS cells c and c+1
  auto xface = [&](int f) {
    int i = f % (TX + 1), j = f / (TX + 1);
    int c = (j + OY) * HX + i + 1;
    Stencil<S, D> st;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      st.u[0][m] = s_u[c - 1 + m];
      if (D == 2) st.u[D - 1][m] = s_v[c - 1 + m];
      st.p[m] = s_p[c - 1 + m];
      st.T[m] = s_th[c - 1 + m];
      st.Y[m] = s_Y[c - 1 + m];
      if constexpr (G2) st.Y2[m] = s_Y2[c - 1 + m];
    }
    st.rho1 = s_rho[c]; st.rho2 = s_rho[c + 1];
    st.c1 = s_c[c]; st.c2 = s_c[c + 1];
    bool disc = !SC.switching || ((s_fl[c] | s_fl[c + 1]) != 0);
    S F[NQ];
    bool sl2 = false, sr2 = false;
    if constexpr (G2) {
      sl2 = eligible(st.Y2[0], st.Y2[1], st.Y2[2], eps);
      sr2 = eligible(st.Y2[1], st.Y2[2], st.Y2[3], eps);
    }
    face_flux<S, D, 0, PRK, G2, LIM>(SC, C, st, disc, eligible(st.Y[0], st.Y[1], st.Y[2], eps),
                                eligible(st.Y[1], st.Y[2], st.Y[3], eps), F, sl2, sr2);
    if (C.diff) visc_flux<S, D, 0, G2>(C, U, s_T, s_a, c, stv, F, s_a2);
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
      Stencil<S, D> st;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        int cm = c + (m - 1) * HX;
        st.u[0][m] = s_u[cm];
        st.u[D - 1][m] = s_v[cm];
        st.p[m] = s_p[cm];
        st.T[m] = s_th[cm];
        st.Y[m] = s_Y[cm];
        if constexpr (G2) st.Y2[m] = s_Y2[cm];
      }
      st.rho1 = s_rho[c]; st.rho2 = s_rho[c + HX];
      st.c1 = s_c[c]; st.c2 = s_c[c + HX];
      bool disc = !SC.switching || ((s_fl[c] | s_fl[c + HX]) != 0);
      S F[NQ];
      bool sl2 = false, sr2 = false;
      if constexpr (G2) {
        sl2 = eligible(st.Y2[0], st.Y2[1], st.Y2[2], eps);
        sr2 = eligible(st.Y2[1], st.Y2[2], st.Y2[3], eps);
      }
      face_flux<S, D, D - 1, PRK, G2, LIM>(SC, C, st, disc, eligible(st.Y[0], st.Y[1], st.Y[2], eps),
                                      eligible(st.Y[1], st.Y[2], st.Y[3], eps), F, sl2, sr2);
      if (C.diff) visc_flux<S, D, D - 1, G2>(C, U, s_T, s_a, c, stv, F, s_a2);
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
        int f = cc;   // j * TX + i
#pragma unroll
        for (int v = 0; v < NQ; ++v) R[k][v] += (s_F[v][f] - s_F[v][f + TX]) * iy;
      }
    }
  }

  // ---- CSF: kappa from the Gaussian-smoothed xi with vertex normals, force sigma kappa grad(alpha_G)
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
      int vx = h % VX, vy = h / VX;      // vertex at the upper corner of tile cell (vx-1, vy-1)
      int c = vy * FX + vx;              // s_H index of cell (vx-1, vy-1)
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
        S kap, Sx, Sy = S(0);
        if (D == 1) {
          kap = -(s_nx[i + 1] - s_nx[i]) * S(C.idx[0]);
          Sx = sig * kap * (aG(c + 1) - aG(c - 1)) * S(0.5 * C.idx[0]);
        } else {
          int v = (j + 1) * VX + (i + 1);   // vertex (i, j) = upper corner of cell (i, j)
          S dnx = s_nx[v] + s_nx[v - VX] - s_nx[v - 1] - s_nx[v - VX - 1];
          S dny = s_ny[v] + s_ny[v - 1] - s_ny[v - VX] - s_ny[v - VX - 1];
          kap = -(dnx * S(0.5 * C.idx[0]) + dny * S(0.5 * C.idx[1]));
          Sx = sig * kap * (aG(c + 1) - aG(c - 1)) * S(0.5 * C.idx[0]);
          Sy = sig * kap * (aG(c + HX) - aG(c - HX)) * S(0.5 * C.idx[1]);
        }
        R[k][2] += Sx;
        S se = s_u[c] * Sx;
        if (D == 2) { R[k][3] += Sy; se += s_v[c] * Sy; }
        R[k][2 + D] += se;
      }
    }
  }

  // ---- body force (eq. 2-2, source Q): rho g on the momentum, rho u . g on the energy
  if (SC.has_grav) {
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      int cc = tid + k * NT;
      if (cc < NC) {
        int c = (cc / TX + OY) * HX + cc % TX + 2;
        S rho = s_rho[c], pw = S(0);
#pragma unroll
        for (int d = 0; d < D; ++d) {
          S gd = S(SC.grav[d]);
          R[k][2 + d] += rho * gd;
          pw += U[d][c] * gd;
        }
        R[k][2 + D] += rho * pw;
      }
    }
  }

  // ---- output
  if (!upd) {
    // right-hand side in the conserved variables (rho, rho u, rho E, rho xi), FP64,
    // in the caller's layout [N_q][ncell] of this case
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
        double rE = (double)R[k][2 + D] + C.Q[0] * r0 + C.Q[1] * r1;
        a.rhs_out[(1 + D) * RS + cell] = G2 ? rE + C.Q[2] * r2 : rE;
        a.rhs_out[(2 + D) * RS + cell] = r1;
        if constexpr (G2) a.rhs_out[(3 + D) * RS + cell] = r2;
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
        q[1] = (double)nv[1] + C.rref[1];
#pragma unroll
        for (int v = 2; v < NQ; ++v) q[v] = (double)nv[v];
        if constexpr (G2) q[NQ - 1] += C.rref[2];
        PT pt = cell_prim_any<D, PRK, G2>(C, q, u, rho, Y, Y2);
        double l = cfl_rate<D, G2>(C, u, pt, rho, Y, Y2);
        bool finite = isfinite(l) && isfinite(pt.p);
        if (!finite) record_error(dy, ERR_NAN, cell - C.off, step);
        else if (!(rho > 0.0) || !(pt.T > 0.0) || !pt.ok) record_error(dy, ERR_NONPHYS, cell - C.off, step);
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

template <class S, int D, int TX, int TY, int NT, int MINW, bool PRK, bool G2, int LIM>
static hipError_t launch12(const StageArgs& a, int ntiles, hipStream_t st)
{
  // the Peng-Robinson closure needs more registers than the stiffened-gas one
  constexpr int W = PRK ? 1 : MINW;
  hipLaunchKernelGGL((k_stage12<S, D, TX, TY, NT, W, PRK, G2, LIM>), dim3(ntiles), dim3(NT), 0, st, a);
  return hipGetLastError();
}

// tile index -> instantiation (the shapes of the tile tables in fvm_kernels.hip)
template <class S, bool PRK, bool G2, int LIM>
static hipError_t stage12(int dim, int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  if (dim == 1) {
    switch (tile) {
      case 0: return launch12<S, 1, 256, 1, 256, 4, PRK, G2, LIM>(a, ntiles, st);
      case 1: return launch12<S, 1, 128, 1, 128, 4, PRK, G2, LIM>(a, ntiles, st);
      case 2: return launch12<S, 1, 128, 1, 256, 4, PRK, G2, LIM>(a, ntiles, st);
    }
  } else {
    switch (tile) {
      case 0: return launch12<S, 2, 32, 8, 256, 4, PRK, G2, LIM>(a, ntiles, st);
      case 1: return launch12<S, 2, 16, 8, 256, 4, PRK, G2, LIM>(a, ntiles, st);
      case 2: return launch12<S, 2, 64, 4, 256, 4, PRK, G2, LIM>(a, ntiles, st);
      case 3: return launch12<S, 2, 16, 16, 256, 4, PRK, G2, LIM>(a, ntiles, st);
      case 4: return launch12<S, 2, 32, 16, 256, 2, PRK, G2, LIM>(a, ntiles, st);
      case 5: return launch12<S, 2, 32, 4, 256, 4, PRK, G2, LIM>(a, ntiles, st);
      // every x and every y face of the tile in one round of threads
      case 6: return launch12<S, 2, 32, 8, 320, 5, PRK, G2, LIM>(a, ntiles, st);
      case 7: return launch12<S, 2, 16, 16, 320, 5, PRK, G2, LIM>(a, ntiles, st);
      case 8: return launch12<S, 2, 32, 8, 384, 6, PRK, G2, LIM>(a, ntiles, st);
      // larger tiles: a smaller halo share (1.41 and 1.27 staged cells per cell)
      // at the same four waves per SIMD
      case 9: return launch12<S, 2, 32, 16, 512, 4, PRK, G2, LIM>(a, ntiles, st);
      case 10: return launch12<S, 2, 32, 32, 1024, 4, PRK, G2, LIM>(a, ntiles, st);
    }
  }
  return hipErrorInvalidValue;
}

// kind: FVM_KIND_SG (stiffened-gas pair), FVM_KIND_PR (Peng-Robinson
// component 1) or FVM_KIND_THREE (liquid and two ideal gases)
template <int LIM>
static hipError_t stage12_any(int dim, int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  if (mixed) {
    if (kind == FVM_KIND_THREE) return stage12<float, false, true, LIM>(dim, tile, a, ntiles, st);
    return kind == FVM_KIND_PR ? stage12<float, true, false, LIM>(dim, tile, a, ntiles, st)
                               : stage12<float, false, false, LIM>(dim, tile, a, ntiles, st);
  }
  if (kind == FVM_KIND_THREE) return stage12<double, false, true, LIM>(dim, tile, a, ntiles, st);
  return kind == FVM_KIND_PR ? stage12<double, true, false, LIM>(dim, tile, a, ntiles, st)
                             : stage12<double, false, false, LIM>(dim, tile, a, ntiles, st);
}

}  // namespace fvm
