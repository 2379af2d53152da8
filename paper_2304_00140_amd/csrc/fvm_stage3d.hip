// fvm_stage3d.hip -- 3D stage: closure kernel + LDS-tiled face/update kernel.
//
// In 3D the halo of a tile is large (a 2-cell halo around 8x8x4 cells holds
// 4.5 cells per owned cell), and the method is bound by arithmetic, so the
// FP64 closure inversion runs once per cell in its own kernel and writes the
// primitives (rho, u, v, w, p, T, xi, c, alpha_G) in the storage precision;
// the face kernel stages tile + halo primitives in LDS (ghosts generated from
// the boundary kinds), evaluates the sensors, every face flux once (x, y, z
// sweeps), the CSF source with the 3D Gaussian kernel (/64) and vertex normals
// of the 2x2x2 cell blocks, and the stage update.  G2: three components (a
// liquid and two gases); the second gas adds its partial density as the last
// storage field and (xi_2, alpha_2) as primitive rows 9 and 10.
#include <hip/hip_runtime.h>
#include "fvm_device.hpp"
#include "fvm_kernels.hpp"
#include "fvm_stage_common.hpp"
#include "fvm_stage3_prim.hpp"

namespace fvm {

template <class S, int TX, int TY, int TZ, int NT, int MINW, bool PRK, bool G2, int LIM>
__global__ __launch_bounds__(NT, MINW) void k_face3(StageArgs a, const S* __restrict__ W)
{
  constexpr int HX = TX + 4, HY = TY + 4, HZ = TZ + 4, HXY = HX * HY, NH = HXY * HZ;
  constexpr int NQ = G2 ? 7 : 6;   // G2: the second gas's partial density last
  constexpr int NW3 = nw3<G2>();
  constexpr int NC = TX * TY * TZ;
  constexpr int CPT = (NC + NT - 1) / NT;
  constexpr int NFX = (TX + 1) * TY * TZ, NFY = TX * (TY + 1) * TZ, NFZ = TX * TY * (TZ + 1);
  constexpr int NF = NFX > NFY ? (NFX > NFZ ? NFX : NFZ) : (NFY > NFZ ? NFY : NFZ);
  constexpr int FX = TX + 2, FY = TY + 2, FZ = TZ + 2, NFH = FX * FY * FZ;   // tile + one halo layer
  constexpr int VX = TX + 1, VY = TY + 1, VZ = TZ + 1, NV = VX * VY * VZ;    // vertices
  constexpr int NBUF = (NQ * NF > NFH + 3 * NV) ? NQ * NF : NFH + 3 * NV;   // fluxes, then CSF scratch

  __shared__ S s_w[NW3][NH];
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
  S* s_T = s_w[5];
  S* s_Y = s_w[6];
  S* s_c = s_w[7];
  S* s_a = s_w[8];
  S* s_Y2 = G2 ? s_w[NW3 - 2] : nullptr;
  S* s_a2 = G2 ? s_w[NW3 - 1] : nullptr;
  // total gas volume fraction and mass fraction of a staged cell
  auto aG = [&](int c) -> S {
    if constexpr (G2) return s_a[c] + s_a2[c];
    else return s_a[c];
  };
  auto YG = [&](int c) -> S {
    if constexpr (G2) return s_Y[c] + s_Y2[c];
    else return s_Y[c];
  };

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

  // ---- tile + halo primitives into LDS
  if (halo_inside3<S>(C, x0, y0, z0, TX, TY, TZ)) {
    // no ghost cell: straight loads at 32-bit byte offsets from the rows' bases
    const char* base[NW3];
#pragma unroll
    for (int v = 0; v < NW3; ++v) base[v] = (const char*)(W + v * T + C.off);
    const unsigned n0 = (unsigned)C.n[0], n01 = n0 * (unsigned)C.n[1];
    const unsigned org = (unsigned)(x0 - 2) + n0 * (unsigned)(y0 - 2) + n01 * (unsigned)(z0 - 2);
    // unrolled, so that the loads of every pass are in flight together
#pragma unroll
    for (int it = 0; it < (NH + NT - 1) / NT; ++it) {
      const int h = tid + it * NT;
      if (h < NH) {
        const unsigned hx = h % HX, hy = (h / HX) % HY, hz = h / HXY;
        const unsigned off = (org + hx + n0 * hy + n01 * hz) * (unsigned)sizeof(S);
#pragma unroll
        for (int v = 0; v < NW3; ++v) s_w[v][h] = *(const S*)(base[v] + off);
      }
    }
  } else {
    for (int h = tid; h < NH; h += NT) {
      int hx = h % HX, hy = (h / HX) % HY, hz = h / HXY;
      S w[NW3];
      load_prim3<S, PRK, G2>(C, W, T, x0 + hx - 2, y0 + hy - 2, z0 + hz - 2, step, w);
#pragma unroll
      for (int v = 0; v < NW3; ++v) s_w[v][h] = w[v];
    }
  }
  __syncthreads();

  const int st[3] = {1, HX, HXY};
  // ---- switching sensors on tile + one halo layer
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
      S thg = S(0);
#pragma unroll
      for (int d = 0; d < 3; ++d) thg += fabs(aG(c) - aG(c - st[d])) + fabs(aG(c + st[d]) - aG(c));
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
  const S* U[3] = {s_u, s_v, s_ww};
  // ---- faces along d: face at the lower side of tile cell (i, j, k) with index
  // i running to TX (d = 0), j to TY (d = 1) or k to TZ (d = 2)
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int EX = TX + (d == 0), EY = TY + (d == 1);
    const int NFD = d == 0 ? NFX : (d == 1 ? NFY : NFZ);
    const int sd = st[d];
    if (d > 0) __syncthreads();
    for (int f = tid; f < NFD; f += NT) {
      int i = f % EX, j = (f / EX) % EY, k = f / (EX * EY);
      int c = (k + 2) * HXY + (j + 2) * HX + (i + 2) - sd;   // lower cell of the face
      Stencil<S, 3> sten;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        int cm = c + (m - 1) * sd;
        sten.u[0][m] = s_u[cm];
        sten.u[1][m] = s_v[cm];
        sten.u[2][m] = s_ww[cm];
        sten.p[m] = s_p[cm];
        sten.T[m] = s_T[cm];
        sten.Y[m] = s_Y[cm];
        if constexpr (G2) sten.Y2[m] = s_Y2[cm];
      }
      sten.rho1 = s_rho[c]; sten.rho2 = s_rho[c + sd];
      sten.c1 = s_c[c]; sten.c2 = s_c[c + sd];
      bool disc = !SC.switching || ((s_fl[c] | s_fl[c + sd]) != 0);
      bool sl = eligible(sten.Y[0], sten.Y[1], sten.Y[2], eps);
      bool sr = eligible(sten.Y[1], sten.Y[2], sten.Y[3], eps);
      bool sl2 = false, sr2 = false;
      if constexpr (G2) {
        sl2 = eligible(sten.Y2[0], sten.Y2[1], sten.Y2[2], eps);
        sr2 = eligible(sten.Y2[1], sten.Y2[2], sten.Y2[3], eps);
      }
      S F[NQ];
      if (d == 0) face_flux<S, 3, 0, PRK, G2, LIM>(SC, C, sten, disc, sl, sr, F, sl2, sr2);
      else if (d == 1) face_flux<S, 3, 1, PRK, G2, LIM>(SC, C, sten, disc, sl, sr, F, sl2, sr2);
      else face_flux<S, 3, 2, PRK, G2, LIM>(SC, C, sten, disc, sl, sr, F, sl2, sr2);
      if (C.diff) {
        if (d == 0) visc_flux<S, 3, 0, G2>(C, U, s_T, s_a, c, st, F, s_a2);
        else if (d == 1) visc_flux<S, 3, 1, G2>(C, U, s_T, s_a, c, st, F, s_a2);
        else visc_flux<S, 3, 2, G2>(C, U, s_T, s_a, c, st, F, s_a2);
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

  // ---- CSF (Section 3.5): 3D binomial kernel /64, vertex normals, kappa = -div n
  // a tile whose staged gas fractions are all equal (marked by the closure
  // kernel of this stage, with its neighbours) gets exactly zero from it
  if (SC.sigma > 0.0 && !(a.csf_zero && a.frac_ext && a.csf_zero[xcd_block(blockIdx.x, gridDim.x)])) {
    __syncthreads();
    S* s_H = s_buf;
    S* s_n = s_H + NFH;    // [3][NV]
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
      int vx = h % VX, vy = (h / VX) % VY, vz = h / (VX * VY);   // upper corner of tile cell (vx-1, vy-1, vz-1)
      int c = (vz * FY + vy) * FX + vx;                           // s_H index of that cell
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
        int v = ((k + 1) * VY + (j + 1)) * VX + (i + 1);   // vertex (i, j, k): upper corner of the cell
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
        S se = S(0);
        const S* uu[3] = {s_u, s_v, s_ww};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          S Sd = sig * kap * (aG(c + st[d]) - aG(c - st[d])) * S(0.5 * C.idx[d]);
          R[kk][2 + d] += Sd;
          se += uu[d][c] * Sd;
        }
        R[kk][5] += se;
      }
    }
  }

  // ---- body force (eq. 2-2, source Q): rho g on the momentum, rho u . g on the energy
  if (SC.has_grav) {
#pragma unroll
    for (int kk = 0; kk < CPT; ++kk) {
      int cc = tid + kk * NT;
      if (cc < NC) {
        int i = cc % TX, j = (cc / TX) % TY, k = cc / (TX * TY);
        int c = (k + 2) * HXY + (j + 2) * HX + i + 2;
        S rho = s_rho[c], pw = S(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          S gd = S(SC.grav[d]);
          R[kk][2 + d] += rho * gd;
          pw += U[d][c] * gd;
        }
        R[kk][5] += rho * pw;
      }
    }
  }

  // ---- output
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
        double rE = (double)R[k][5] + C.Q[0] * r0 + C.Q[1] * r1;
        a.rhs_out[4 * RS + cell] = G2 ? rE + C.Q[2] * r2 : rE;
        a.rhs_out[5 * RS + cell] = r1;
        if constexpr (G2) a.rhs_out[6 * RS + cell] = r2;
      }
    }
    return;
  }
  const double dt = step_dt(dy, step, SC.cfl, SC.t_end);
  if (a.stage == 0 && tl.y == 0 && tl.z == 0 && tl.w == 0 && tid == 0) step_scalars(dy, step, dt);
  // the last stage writes q^(n+1); its CFL bound and its checks come from the
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

// LDS of a face-kernel tile: primitives of tile + halo, flags, flux / CSF buffer
template <class S, int TX, int TY, int TZ, bool G2>
constexpr long long lds3()
{
  constexpr long long NH = (TX + 4LL) * (TY + 4) * (TZ + 4);
  constexpr long long NF1 = (TX + 1LL) * TY * TZ, NF2 = TX * (TY + 1LL) * TZ, NF3 = TX * TY * (TZ + 1LL);
  constexpr long long NF = NF1 > NF2 ? (NF1 > NF3 ? NF1 : NF3) : (NF2 > NF3 ? NF2 : NF3);
  constexpr long long NFH = (TX + 2LL) * (TY + 2) * (TZ + 2), NV = (TX + 1LL) * (TY + 1) * (TZ + 1);
  constexpr long long NQ = G2 ? 7 : 6;
  constexpr long long NB = NQ * NF > NFH + 3 * NV ? NQ * NF : NFH + 3 * NV;
  return (nw3<G2>() * NH + NB) * (long long)sizeof(S) + NH;
}

// whether a tile's face kernel fits the 160 KiB of LDS of a workgroup
template <class S, int TX, int TY, int TZ, bool G2>
constexpr bool fits3() { return lds3<S, TX, TY, TZ, G2>() <= 160LL * 1024; }

template <class S, int TX, int TY, int TZ, int NT, int MINW, bool PRK, bool G2, int LIM>
static hipError_t launch3(const StageArgs& a, int ntiles, hipStream_t st)
{
  if constexpr (!fits3<S, TX, TY, TZ, G2>()) {
    return hipErrorInvalidValue;   // rejected on the host before any launch (fvm_k_tile_ok3)
  } else {
    // the Peng-Robinson face kernels ask for as many waves per SIMD as the
    // workgroups that the LDS of the tile admits per CU hold, within what the
    // kernel's registers allow without large spills (4 waves in FP32 storage,
    // 3 in FP64), so the register budget does not become the tighter limit
    constexpr long long LDS_CU = 160LL * 1024;
    constexpr int WG_LDS = (int)(LDS_CU / lds3<S, TX, TY, TZ, G2>());
    constexpr int WPS = (NT / 64 + 3) / 4;
    constexpr int CAP = sizeof(S) == 4 ? 4 : 3;
    constexpr int NWG = WG_LDS < CAP / WPS ? WG_LDS : CAP / WPS;
    constexpr int WOCC = (NWG > 1 ? NWG : 1) * WPS;
    constexpr int Wv = PRK ? WOCC : MINW;
    S* W = (S*)a.prim;
    constexpr int PB = (TX * TY * TZ + 255) / 256;
    hipLaunchKernelGGL((k_prim3<S, TX, TY, TZ, PRK, G2>), dim3(ntiles * PB), dim3(256), 0, st, a, W);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.csf_zero && a.frac_ext && a.sc.sigma > 0.0) {
      hipLaunchKernelGGL((k_csf_zero<S, TX, TY, TZ, PB>), dim3((ntiles + 255) / 256), dim3(256), 0, st, a, ntiles,
                         (unsigned char*)a.csf_zero);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_face3<S, TX, TY, TZ, NT, Wv, PRK, G2, LIM>), dim3(ntiles), dim3(NT), 0, st, a,
                       (const S*)W);
    return hipGetLastError();
  }
}

}  // namespace fvm

using namespace fvm;

// (tx, ty, tz, threads).  Rows 5-9 give the 8x8x8 and 8x8x4 / 8x4x4 tiles
// more threads than cells: up to one thread per face of a direction, so each
// direction's faces take one pass, and more waves per SIMD to hide latency
// where the LDS of the tile admits only one or two workgroups per CU.
static const int TILES3[][4] = {{8, 8, 4, 256}, {16, 8, 2, 256}, {8, 4, 4, 128}, {16, 4, 4, 256}, {8, 8, 8, 512},
                                {8, 8, 8, 768}, {8, 8, 8, 1024}, {8, 8, 4, 512}, {8, 4, 4, 256}, {8, 8, 8, 576}};
static const int NT3 = sizeof(TILES3) / sizeof(TILES3[0]);
// 3D tile numbering: rows 0-4 of the closure + face kernel pair, then the
// z-marching kernel's tiles (two-component inviscid closures only), then rows
// 5-9 of the pair
static const int NP3A = 5;

static int march_index3(int t)
{
  int m = t - NP3A;
  return (m >= 0 && m < fvm_k_tile_count_m3()) ? m : -1;
}

// TILES3 row of a 3D tile index, -1 for a z-marching tile or no tile
static int pair_row3(int t)
{
  if (t < 0) return -1;
  if (t < NP3A) return t;
  int r = t - fvm_k_tile_count_m3();
  return (r >= NP3A && r < NT3) ? r : -1;
}

int fvm_k_tile_is_m3(int t) { return march_index3(t) >= 0; }

int fvm_k_tile_row3(int t) { return pair_row3(t); }

int fvm_k_tile_march3(int t)
{
  int m = march_index3(t);
  return m < 0 ? -1 : (m < fvm_k_tile_count_m3() / 2 ? 0 : 1);
}

int fvm_k_tile_count3() { return NT3 + fvm_k_tile_count_m3(); }

int fvm_k_tile_shape3(int t, int* tx, int* ty, int* nt)
{
  int m = march_index3(t);
  if (m >= 0) {
    int zc;
    return fvm_k_tile_shape_m3(m, tx, ty, nt, &zc);
  }
  int r = pair_row3(t);
  if (r < 0) return -1;
  *tx = TILES3[r][0];
  *ty = TILES3[r][1];
  *nt = TILES3[r][3];
  return 0;
}

int fvm_k_tile_zchunk3(int t)
{
  int m = march_index3(t);
  if (m >= 0) {
    int tx, ty, nt, zc;
    return fvm_k_tile_shape_m3(m, &tx, &ty, &nt, &zc) ? 1 : zc;
  }
  int r = pair_row3(t);
  return r >= 0 ? TILES3[r][2] : 1;
}

template <class S, bool PRK, bool G2, int LIM>
static hipError_t stage3(int row, const StageArgs& a, int ntiles, hipStream_t st)
{
  switch (row) {
    case 0: return launch3<S, 8, 8, 4, 256, 2, PRK, G2, LIM>(a, ntiles, st);
    case 1: return launch3<S, 16, 8, 2, 256, 2, PRK, G2, LIM>(a, ntiles, st);
    case 2: return launch3<S, 8, 4, 4, 128, 2, PRK, G2, LIM>(a, ntiles, st);
    case 3: return launch3<S, 16, 4, 4, 256, 2, PRK, G2, LIM>(a, ntiles, st);
    case 4: return launch3<S, 8, 8, 8, 512, 1, PRK, G2, LIM>(a, ntiles, st);
    case 5: return launch3<S, 8, 8, 8, 768, 1, PRK, G2, LIM>(a, ntiles, st);
    case 6: return launch3<S, 8, 8, 8, 1024, 1, PRK, G2, LIM>(a, ntiles, st);
    case 7: return launch3<S, 8, 8, 4, 512, 1, PRK, G2, LIM>(a, ntiles, st);
    case 8: return launch3<S, 8, 4, 4, 256, 2, PRK, G2, LIM>(a, ntiles, st);
    case 9: return launch3<S, 8, 8, 8, 576, 1, PRK, G2, LIM>(a, ntiles, st);
  }
  return hipErrorInvalidValue;
}

template <class S, bool G2>
static bool tile_ok3(int row)
{
  switch (row) {
    case 0: case 7: return fits3<S, 8, 8, 4, G2>();
    case 1: return fits3<S, 16, 8, 2, G2>();
    case 2: case 8: return fits3<S, 8, 4, 4, G2>();
    case 3: return fits3<S, 16, 4, 4, G2>();
    case 4: case 5: case 6: case 9: return fits3<S, 8, 8, 8, G2>();
  }
  return false;
}

// kind: FVM_KIND_SG, FVM_KIND_PR or FVM_KIND_THREE
template <int LIM>
static hipError_t stage3_any(int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  if (mixed) {
    if (kind == FVM_KIND_THREE) return stage3<float, false, true, LIM>(tile, a, ntiles, st);
    return kind == FVM_KIND_PR ? stage3<float, true, false, LIM>(tile, a, ntiles, st)
                               : stage3<float, false, false, LIM>(tile, a, ntiles, st);
  }
  if (kind == FVM_KIND_THREE) return stage3<double, false, true, LIM>(tile, a, ntiles, st);
  return kind == FVM_KIND_PR ? stage3<double, true, false, LIM>(tile, a, ntiles, st)
                             : stage3<double, false, false, LIM>(tile, a, ntiles, st);
}

// the default limiters (Koren, Minmod) as compile-time constants, any others at run time
hipError_t fvm_k_stage3(int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  int m = march_index3(tile);
  if (m >= 0) {
    if (kind != FVM_KIND_SG && kind != FVM_KIND_PR) return hipErrorInvalidValue;
    return fvm_k_stage_m3(mixed, kind, m, a, ntiles, st);
  }
  int r = pair_row3(tile);
  if (r < 0) return hipErrorInvalidValue;
  if (fvm_default_limiters(a.sc)) return stage3_any<1>(mixed, kind, r, a, ntiles, st);
  return stage3_any<0>(mixed, kind, r, a, ntiles, st);
}

// whether the face kernel of a 3D tile fits the LDS of a workgroup for this
// precision and closure kind (the three-component FP64 tile of 8x8x8 cells
// does not)
int fvm_k_tile_ok3(int mixed, int kind, int tile)
{
  if (march_index3(tile) >= 0) return kind == FVM_KIND_SG || kind == FVM_KIND_PR;
  int r = pair_row3(tile);
  if (r < 0) return 0;
  bool g2 = kind == FVM_KIND_THREE;
  if (mixed) return g2 ? tile_ok3<float, true>(r) : tile_ok3<float, false>(r);
  return g2 ? tile_ok3<double, true>(r) : tile_ok3<double, false>(r);
}
