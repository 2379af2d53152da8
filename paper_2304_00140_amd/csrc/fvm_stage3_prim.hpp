// fvm_stage3_prim.hpp -- 3D closure kernel: the primitives of every cell of a
// tile in the storage precision (rho, u, v, w, p, T, xi, c, alpha_G; with a
// second gas also xi_2, alpha_2), and the loader of one (possibly ghost) cell's
// primitives that the face kernels use.
#pragma once
#include <hip/hip_runtime.h>
#include "fvm_device.hpp"
#include "fvm_kernels.hpp"
#include "fvm_stage_common.hpp"

namespace fvm {

// primitive rows: rho, u, v, w, p, T, xi, c, alpha_G (+ xi_2, alpha_2 with G2)
template <bool G2>
constexpr int nw3() { return G2 ? 11 : 9; }

// the value of the lowest active lane of the wave
template <class S>
__device__ inline S first_lane(S v)
{
  if constexpr (sizeof(S) == 4) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
  } else {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
  }
}

// (min, max) of a 256-thread workgroup's gas mass fractions yg and volume
// fractions ag over its cells with in == true, stored as out[0..3] = (min yg,
// max yg, min ag, max ag) where they are uniform; a workgroup whose cells
// differ (a NaN counts) stores the whole line, one without cells the empty
// interval.  Each wave compares its cells with its first one (a ballot, no
// shuffles); called by all threads of the workgroup
template <class S>
__device__ inline void frac_extremes(bool in, S yg, S ag, S* out)
{
  __shared__ S s_ext[4][4];
  const S inf = S(INFINITY);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_ext[w][0] = inf; s_ext[w][1] = -inf; s_ext[w][2] = inf; s_ext[w][3] = -inf;
  }
  if (in) {
    const S y0 = first_lane(yg), a0 = first_lane(ag);
    const unsigned long long diff = __ballot(!(yg == y0) || !(ag == a0));
    const unsigned long long act = __ballot(1);
    if (__lane_id() == __ffsll((long long)act) - 1) {
      if (diff) {
        s_ext[w][0] = -inf; s_ext[w][1] = inf; s_ext[w][2] = -inf; s_ext[w][3] = inf;
      } else {
        s_ext[w][0] = y0; s_ext[w][1] = y0; s_ext[w][2] = a0; s_ext[w][3] = a0;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int m = threadIdx.x;
    S r = s_ext[0][m];
#pragma unroll
    for (int v = 1; v < 4; ++v) r = (m & 1) ? fmax(r, s_ext[v][m]) : fmin(r, s_ext[v][m]);
    out[m] = r;
  }
}

// primitives of every owned cell of the tile (a Peng-Robinson closure starts
// its Newton iterations from the cell's previous primitives, which the paper
// suggests for convergence speed).  In the first stage of a step
// the cells hold q^n, so this kernel also folds the CFL bound of q^n into the
// case's slot for this step (read by the face kernel of the same stage) and
// reports a non-finite or non-physical q^n as an error of the step before.
// Four waves per SIMD: the Peng-Robinson closure fits 127 VGPRs without
// spills (it took 133, three waves, when left free)
template <class S, int TX, int TY, int TZ, bool PRK, bool G2>
__global__ __launch_bounds__(256, 4) void k_prim3(StageArgs a, S* __restrict__ W)
{
  __shared__ double s_red[4];
  // PB workgroups of 256 threads per tile, one cell per thread
  constexpr int PB = (TX * TY * TZ + 255) / 256;
  const int bb = xcd_block(blockIdx.x, gridDim.x);
  const int4 tl = a.tiles[bb / PB];
  const CaseC& C = a.cases[tl.x];
  CaseDyn& dy = a.dyn[tl.x];
  const S* __restrict__ src = (const S*)a.src;
  const long long T = a.total;
  const bool first = a.stage == 0;
  const long long step = dy.base + a.step_off;
  double lam = 0.0;
  constexpr int NC = TX * TY * TZ;
  const int cc = (bb % PB) * 256 + threadIdx.x;
  const int i = cc % TX, j = (cc / TX) % TY, k = cc / (TX * TY);
  const int gx = tl.y * TX + i, gy = tl.z * TY + j, gz = tl.w * TZ + k;
  // this cell's total gas mass and volume fractions as the face kernel stages
  // them (storage precision, the two gases summed there)
  S yg = S(0), ag = S(0);
  const bool in = cc < NC && gx < C.n[0] && gy < C.n[1] && gz < C.n[2];
  if (in) {
    long long cell = C.off + gx + (long long)C.n[0] * (gy + (long long)C.n[1] * gz);
    double q[G2 ? 7 : 6], u[3], rho, Y, Y2 = 0.0;
    q[0] = (double)src[cell] + C.rref[0];
    q[1] = (double)src[T + cell] + C.rref[1];
#pragma unroll
    for (int v = 2; v < 6; ++v) q[v] = (double)src[v * T + cell];
    PT pt;
    if constexpr (G2) {
      q[6] = (double)src[6 * T + cell] + C.rref[2];
      pt = cell_prim3<3>(C, q, u, rho, Y, Y2);
    } else {
      // the Peng-Robinson Newton starts from this cell's (p, T) of the previous
      // stage, still in the primitive buffer (zero before the first stage)
      double Tw = 0.0, pw = 0.0;
      if constexpr (PRK) {
        Tw = (double)W[5 * T + cell];
        pw = (double)W[4 * T + cell];
      }
      pt = cell_prim<3, PRK>(C, q, u, rho, Y, Tw, pw);
    }
    W[cell] = S(rho);
    W[T + cell] = S(u[0]);
    W[2 * T + cell] = S(u[1]);
    W[3 * T + cell] = S(u[2]);
    W[4 * T + cell] = S(pt.p);
    W[5 * T + cell] = S(pt.T);
    W[6 * T + cell] = S(Y);
    W[7 * T + cell] = S(pt.c);
    W[8 * T + cell] = S(pt.alpha);
    yg = S(Y);
    ag = S(pt.alpha);
    if constexpr (G2) {
      W[9 * T + cell] = S(Y2);
      W[10 * T + cell] = S(pt.alpha2);
      yg = yg + S(Y2);
      ag = ag + S(pt.alpha2);
    }
    if (first) {
      double l = cfl_rate<3, G2>(C, u, pt, rho, Y, Y2);
      if (!isfinite(l) || !isfinite(pt.p)) record_error(dy, ERR_NAN, cell - C.off, step - 1);
      else if (!(rho > 0.0) || !(pt.T > 0.0) || !pt.ok) record_error(dy, ERR_NONPHYS, cell - C.off, step - 1);
      else lam = fmax(lam, l);
    }
  }
  if (first) {
    lam = wave_max(lam);
    if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = lam;
    __syncthreads();
    if (threadIdx.x == 0) cfl_max(dy, (int)(step & 1), fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3])));
  }
  // with surface tension: the extremes (min, max) of the two fractions over this
  // workgroup's cells, from which the CSF mark of each face-kernel tile follows
  if (a.frac_ext && a.sc.sigma > 0.0) frac_extremes<S>(in, yg, ag, (S*)a.frac_ext + (long long)bb * 4);
}

// per tile-table entry of the face kernel: 1 when the tiles around it (itself
// included, at most 27) hold one value of each gas fraction, so that the CSF
// term of the tile is exactly zero (zero normals of a uniform smoothed
// fraction, zero volume-fraction differences).  Where the tile's two-cell halo
// crosses a zero-gradient or slip-wall side, its ghost cells copy or mirror
// cells of the tile and its neighbours, so the neighbours that exist decide;
// across a periodic, inflow or far-field side (ghosts from elsewhere) the tile
// keeps its CSF term.  PB closure workgroups per tile, each with its extremes
template <class S, int TX, int TY, int TZ, int PB>
__global__ __launch_bounds__(256) void k_csf_zero(StageArgs a, int ntiles, unsigned char* out)
{
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= ntiles) return;
  const int4 tl = a.tiles[e];
  const CaseC& C = a.cases[tl.x];
  const int t[3] = {tl.y, tl.z, tl.w}, ext3[3] = {TX, TY, TZ};
  int lo[3], hi[3];
  bool ok = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int x0 = t[d] * ext3[d];
    lo[d] = (t[d] > 0) ? -1 : 0;
    hi[d] = (t[d] < C.tiles[d] - 1) ? 1 : 0;
    const bool below = x0 < 2, above = x0 + ext3[d] + 2 > C.n[d];
    if (below && !(C.bc[d][0] == BC_ZEROGRAD || C.bc[d][0] == BC_WALL)) ok = false;
    if (above && !(C.bc[d][1] == BC_ZEROGRAD || C.bc[d][1] == BC_WALL)) ok = false;
  }
  unsigned char z = 0;
  if (ok) {
    const S* ext = (const S*)a.frac_ext;
    const S inf = S(INFINITY);
    S ylo = inf, yhi = -inf, alo = inf, ahi = -inf;
    for (int dk = lo[2]; dk <= hi[2]; ++dk)
      for (int dj = lo[1]; dj <= hi[1]; ++dj)
        for (int di = lo[0]; di <= hi[0]; ++di) {
          const int ni = t[0] + di, sl = ni / C.xslab, w = min(C.xslab, C.tiles[0] - sl * C.xslab);
          const long long n = C.tile0 + (long long)sl * C.xslab * C.tiles[1] * C.tiles[2] +
                              ((long long)(t[2] + dk) * C.tiles[1] + (t[1] + dj)) * w + (ni - sl * C.xslab);
#pragma unroll
          for (int b = 0; b < PB; ++b) {
            const S* x = ext + (n * PB + b) * 4;
            ylo = fmin(ylo, x[0]);
            yhi = fmax(yhi, x[1]);
            alo = fmin(alo, x[2]);
            ahi = fmax(ahi, x[3]);
          }
        }
    z = (ylo == yhi && alo == ahi) ? 1 : 0;
  }
  out[e] = z;
}

// primitives of one (possibly ghost) cell
template <class S, bool PRK, bool G2>
__device__ inline void load_prim3(const CaseC& C, const S* __restrict__ W, long long T, int gx, int gy, int gz,
                                  long long step, S* w)
{
  // far-field and inflow states hold no second gas
  if (beyond_farfield<3>(C, gx, gy, gz)) {
    double u0[3] = {0.0, 0.0, 0.0}, q[G2 ? 7 : 6], uu[3], rho, Y, Y2;
    state_from_prim<PRK, G2>(C, C.ff_p, C.ff_T, C.ff_alpha, u0, 3, q);
    PT pt = cell_prim_any<3, PRK, G2>(C, q, uu, rho, Y, Y2);
    w[0] = S(rho); w[1] = S(uu[0]); w[2] = S(uu[1]); w[3] = S(uu[2]);
    w[4] = S(pt.p); w[5] = S(pt.T); w[6] = S(Y); w[7] = S(pt.c); w[8] = S(pt.alpha);
    if constexpr (G2) { w[9] = S(Y2); w[10] = S(pt.alpha2); }
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
      double u[3] = {C.in_u, 0.0, 0.0}, q[G2 ? 7 : 6], uu[3], rho, Y, Y2;
      for (int c = 0; c < 3; ++c)
        u[c] += C.in_noise * C.in_u *
                (2.0 * noise01(C.in_seed, (unsigned long long)step, (unsigned long long)iy,
                               (unsigned long long)iz, (unsigned long long)c) - 1.0);
      state_from_prim<PRK, G2>(C, C.in_p, C.in_T, C.in_alpha, u, 3, q);
      PT pt = cell_prim_any<3, PRK, G2>(C, q, uu, rho, Y, Y2);
      w[0] = S(rho);
      w[1] = S(uu[0]);
      w[2] = S(fy ? -uu[1] : uu[1]);
      w[3] = S(fz ? -uu[2] : uu[2]);
      w[4] = S(pt.p); w[5] = S(pt.T); w[6] = S(Y); w[7] = S(pt.c); w[8] = S(pt.alpha);
      if constexpr (G2) { w[9] = S(Y2); w[10] = S(pt.alpha2); }
      return;
    }
    ix = -1 - ix;
    fx = true;
  } else {
    map_index(ix, C.n[0], C.bc[0][0], C.bc[0][1], fx);
  }
  long long cell = C.off + ix + (long long)C.n[0] * (iy + (long long)C.n[1] * iz);
#pragma unroll
  for (int v = 0; v < nw3<G2>(); ++v) w[v] = W[v * T + cell];
  if (fx) w[1] = -w[1];
  if (fy) w[2] = -w[2];
  if (fz) w[3] = -w[3];
}

}  // namespace fvm
