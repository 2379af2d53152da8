// fvm_kernels.hip -- gfx950 kernels of the solver: the stage dispatch, the
// run-time-limiter instantiations of the fused 1D/2D stage kernel
// (fvm_stage12.hpp), the per-step counter, the per-cell conversion, time-step
// and totals kernels and the storage-shift kernel.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "fvm_device.hpp"
#include "fvm_kernels.hpp"
#include "fvm_stage_common.hpp"
#include "fvm_stage12.hpp"

namespace fvm {


// ------------------------------------------------------------------ per-chunk step counter
__global__ void k_advance(CaseDyn* dyn, int ncases, int nsteps)
{
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncases) dyn[c].base += nsteps;
}

// ------------------------------------------------------------------ per-cell kernels of one case
// G2: three components; the second gas's partial density is the last storage
// field, the last conserved field is rho xi_2 and alpha_2 follows u in the
// primitive input
template <class S, int D, bool PRK, bool G2>
__global__ void k_prim_to_state(const CaseC* cases, int icase, const double* __restrict__ prim,
                                S* __restrict__ dst, long long total)
{
  constexpr int NQ = D + 3 + (G2 ? 1 : 0);
  const CaseC& C = cases[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= C.ncell) return;
  double u[3] = {0, 0, 0}, q[NQ];
  for (int d = 0; d < D; ++d) u[d] = prim[(3 + d) * C.ncell + c];
  double al2 = G2 ? prim[(3 + D) * C.ncell + c] : 0.0;
  state_from_prim<PRK, G2>(C, prim[c], prim[C.ncell + c], prim[2 * C.ncell + c], u, D, q, al2);
  long long g = C.off + c;
  dst[g] = S(q[0] - C.rref[0]);
  dst[total + g] = S(q[1] - C.rref[1]);
  for (int v = 2; v < D + 3; ++v) dst[v * total + g] = S(q[v]);
  if constexpr (G2) dst[(NQ - 1) * total + g] = S(q[NQ - 1] - C.rref[2]);
}

template <class S, int D, bool G2>
__global__ void k_cons_to_state(const CaseC* cases, int icase, const double* __restrict__ qin,
                                S* __restrict__ dst, long long total)
{
  const CaseC& C = cases[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= C.ncell) return;
  long long n = C.ncell, g = C.off + c;
  double rho = qin[c], rY = qin[(2 + D) * n + c];
  double rY2 = G2 ? qin[(3 + D) * n + c] : 0.0;
  double rL = G2 ? rho - rY - rY2 : rho - rY, rG = rY;
  dst[g] = S(rL - C.rref[0]);
  dst[total + g] = S(rG - C.rref[1]);
  for (int d = 0; d < D; ++d) dst[(2 + d) * total + g] = S(qin[(1 + d) * n + c]);
  double E = qin[(1 + D) * n + c] - C.Q[0] * rL - C.Q[1] * rG;
  if constexpr (G2) {
    dst[(2 + D) * total + g] = S(E - C.Q[2] * rY2);
    dst[(3 + D) * total + g] = S(rY2 - C.rref[2]);
  } else {
    dst[(2 + D) * total + g] = S(E);
  }
}

template <class S, int D, bool G2>
__global__ void k_state_to_cons(const CaseC* cases, int icase, const S* __restrict__ src,
                                double* __restrict__ qout, long long total)
{
  const CaseC& C = cases[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= C.ncell) return;
  long long n = C.ncell, g = C.off + c;
  double rL = (double)src[g] + C.rref[0], rG = (double)src[total + g] + C.rref[1];
  double r2 = G2 ? (double)src[(3 + D) * total + g] + C.rref[2] : 0.0;
  qout[c] = G2 ? rL + rG + r2 : rL + rG;
  for (int d = 0; d < D; ++d) qout[(1 + d) * n + c] = (double)src[(2 + d) * total + g];
  double E = (double)src[(2 + D) * total + g] + C.Q[0] * rL + C.Q[1] * rG;
  qout[(1 + D) * n + c] = G2 ? E + C.Q[2] * r2 : E;
  qout[(2 + D) * n + c] = rG;
  if constexpr (G2) qout[(3 + D) * n + c] = r2;
}

// load the storage of one interior cell (physical partial densities)
template <class S, int D, bool G2>
__device__ inline void load_own(const CaseC& C, const S* __restrict__ src, long long total, long long g,
                                double* q)
{
  q[0] = (double)src[g] + C.rref[0];
  q[1] = (double)src[total + g] + C.rref[1];
  for (int v = 2; v < D + 3; ++v) q[v] = (double)src[v * total + g];
  if constexpr (G2) q[D + 3] = (double)src[(D + 3) * total + g] + C.rref[2];
}

// primitives rows: rho, u, v, w, p, T, xi_1, c, alpha_1 (+ xi_2, alpha_2 with G2)
template <class S, int D, bool PRK, bool G2>
__global__ void k_state_to_prim(const CaseC* cases, int icase, const S* __restrict__ src,
                                double* __restrict__ w, long long total)
{
  constexpr int NQ = D + 3 + (G2 ? 1 : 0);
  const CaseC& C = cases[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= C.ncell) return;
  long long n = C.ncell, g = C.off + c;
  double q[NQ], u[D], rho, Y, Y2;
  load_own<S, D, G2>(C, src, total, g, q);
  PT pt = cell_prim_any<D, PRK, G2>(C, q, u, rho, Y, Y2);
  w[c] = rho;
  for (int d = 0; d < 3; ++d) w[(1 + d) * n + c] = d < D ? u[d] : 0.0;
  w[4 * n + c] = pt.p;
  w[5 * n + c] = pt.T;
  w[6 * n + c] = Y;
  w[7 * n + c] = pt.c;
  w[8 * n + c] = pt.alpha;
  if constexpr (G2) {
    w[9 * n + c] = Y2;
    w[10 * n + c] = pt.alpha2;
  }
}

// CFL bound of the current state of one case into dtmax[step & 1]
template <class S, int D, bool PRK, bool G2>
__global__ __launch_bounds__(256) void k_dt_init(const CaseC* cases, CaseDyn* dyn, int icase,
                                                 const S* __restrict__ src, long long total, long long label_off)
{
  constexpr int NQ = D + 3 + (G2 ? 1 : 0);
  __shared__ double s_red[4];
  const CaseC& C = cases[icase];
  CaseDyn& dy = dyn[icase];
  long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  double lam = 0.0;
  if (c < C.ncell) {
    long long g = C.off + c;
    double q[NQ], u[D], rho, Y, Y2;
    load_own<S, D, G2>(C, src, total, g, q);
    PT pt = cell_prim_any<D, PRK, G2>(C, q, u, rho, Y, Y2);
    double l = cfl_rate<D, G2>(C, u, pt, rho, Y, Y2);
    if (!isfinite(l) || !isfinite(pt.p)) record_error(dy, ERR_NAN, c, dy.base + label_off);
    else if (!(rho > 0.0) || !(pt.T > 0.0) || !pt.ok) record_error(dy, ERR_NONPHYS, c, dy.base + label_off);
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

// deterministic conserved totals of one case: fixed-shape tree per block, then one block
template <class S, int D, bool G2>
__global__ __launch_bounds__(256) void k_totals_part(const CaseC* cases, int icase, const S* __restrict__ src,
                                                     long long total, double* __restrict__ part)
{
  constexpr int NQ = D + 3 + (G2 ? 1 : 0);
  __shared__ double s[NQ][256];
  const CaseC& C = cases[icase];
  double acc[NQ];
  for (int v = 0; v < NQ; ++v) acc[v] = 0.0;
  for (long long c = blockIdx.x * 256ll + threadIdx.x; c < C.ncell; c += 256ll * gridDim.x) {
    long long g = C.off + c;
    double rL = (double)src[g] + C.rref[0], rG = (double)src[total + g] + C.rref[1];
    double r2 = G2 ? (double)src[(3 + D) * total + g] + C.rref[2] : 0.0;
    acc[0] += G2 ? rL + rG + r2 : rL + rG;
    for (int d = 0; d < D; ++d) acc[1 + d] += (double)src[(2 + d) * total + g];
    double E = (double)src[(2 + D) * total + g] + C.Q[0] * rL + C.Q[1] * rG;
    acc[1 + D] += G2 ? E + C.Q[2] * r2 : E;
    acc[2 + D] += rG;
    if constexpr (G2) acc[3 + D] += r2;
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

__global__ void k_totals_final(const double* __restrict__ part, int nblk, int nq, double vol, double* out)
{
  int v = threadIdx.x;
  if (v >= nq) return;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += part[b * nq + v];
  out[v] = acc * vol;
}

// ------------------------------------------------------------------ host-side launchers

}  // namespace fvm

using namespace fvm;

// tile tables: (tx, ty, threads, waves per SIMD targeted by the register budget)
static const int TILES1[][4] = {{256, 1, 256, 4}, {128, 1, 128, 4}, {128, 1, 256, 4}};
static const int TILES2[][4] = {{32, 8, 256, 4}, {16, 8, 256, 4}, {64, 4, 256, 4},
                                {16, 16, 256, 4}, {32, 16, 256, 2}, {32, 4, 256, 4},
                                {32, 8, 320, 5}, {16, 16, 320, 5}, {32, 8, 384, 6},
                                {32, 16, 512, 4}, {32, 32, 1024, 4}};
static const int NT1 = sizeof(TILES1) / sizeof(TILES1[0]);
static const int NT2 = sizeof(TILES2) / sizeof(TILES2[0]);

int fvm_k_tile_count(int dim)
{
  if (dim == 1) return NT1;
  if (dim == 2) return NT2;
  if (dim == 3) return fvm_k_tile_count3();
  return 0;
}

int fvm_k_tile_shape(int dim, int t, int* tx, int* ty, int* nt)
{
  if (dim == 1 && t >= 0 && t < NT1) { *tx = TILES1[t][0]; *ty = TILES1[t][1]; *nt = TILES1[t][2]; return 0; }
  if (dim == 2 && t >= 0 && t < NT2) { *tx = TILES2[t][0]; *ty = TILES2[t][1]; *nt = TILES2[t][2]; return 0; }
  if (dim == 3) return fvm_k_tile_shape3(t, tx, ty, nt);
  return -1;
}


// kind: closure of the batch, FVM_KIND_SG (stiffened-gas pair), FVM_KIND_PR
// (Peng-Robinson component 1), FVM_KIND_THREE (liquid and two ideal gases) or
// FVM_KIND_BARO / FVM_KIND_BARO2 (barotropic model, one or two gases)
hipError_t fvm_k_stage(int dim, int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  if (kind >= FVM_KIND_BARO) return fvm_kb_stage(dim, mixed, kind == FVM_KIND_BARO2, tile, a, ntiles, st);
  if (dim == 3) return fvm_k_stage3(mixed, kind, tile, a, ntiles, st);
  if (fvm_default_limiters(a.sc)) return fvm_k_stage12_deflim(dim, mixed, kind, tile, a, ntiles, st);
  return stage12_any<0>(dim, mixed, kind, tile, a, ntiles, st);
}

hipError_t fvm_k_advance(CaseDyn* dyn, int ncases, int nsteps, hipStream_t st)
{
  hipLaunchKernelGGL(k_advance, dim3((ncases + 63) / 64), dim3(64), 0, st, dyn, ncases, nsteps);
  return hipGetLastError();
}

#define FVM_DISPATCH_D(S, DIM, KIND, CALL)                                            \
  do {                                                                                \
    if (DIM == 1) {                                                                   \
      if (KIND == FVM_KIND_THREE) { CALL(S, 1, false, true); }                        \
      else if (KIND == FVM_KIND_PR) { CALL(S, 1, true, false); }                      \
      else { CALL(S, 1, false, false); }                                              \
    } else if (DIM == 2) {                                                            \
      if (KIND == FVM_KIND_THREE) { CALL(S, 2, false, true); }                        \
      else if (KIND == FVM_KIND_PR) { CALL(S, 2, true, false); }                      \
      else { CALL(S, 2, false, false); }                                              \
    } else {                                                                          \
      if (KIND == FVM_KIND_THREE) { CALL(S, 3, false, true); }                        \
      else if (KIND == FVM_KIND_PR) { CALL(S, 3, true, false); }                      \
      else { CALL(S, 3, false, false); }                                              \
    }                                                                                 \
  } while (0)
#define FVM_DISPATCH(MIXED, DIM, KIND, CALL)                                          \
  do {                                                                                \
    if (MIXED) FVM_DISPATCH_D(float, DIM, KIND, CALL);                                \
    else FVM_DISPATCH_D(double, DIM, KIND, CALL);                                     \
  } while (0)

static unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t fvm_k_prim_to_state(int dim, int mixed, int kind, const CaseC* cases, int icase, long long ncell,
                               const double* prim, void* dst, long long total, hipStream_t st)
{
  if (kind >= FVM_KIND_BARO) return fvm_kb_prim_to_state(dim, mixed, kind == FVM_KIND_BARO2, cases, icase, ncell, prim, dst, total, st);
#define CALL(S, D, P, G) hipLaunchKernelGGL((k_prim_to_state<S, D, P, G>), dim3(blocks_for(ncell, 256)), dim3(256), 0, st, cases, icase, prim, (S*)dst, total)
  FVM_DISPATCH(mixed, dim, kind, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_k_cons_to_state(int dim, int mixed, int kind, const CaseC* cases, int icase, long long ncell,
                               const double* q, void* dst, long long total, hipStream_t st)
{
  if (kind >= FVM_KIND_BARO) return fvm_kb_cons_to_state(dim, mixed, kind == FVM_KIND_BARO2, cases, icase, ncell, q, dst, total, st);
#define CALL(S, D, P, G) hipLaunchKernelGGL((k_cons_to_state<S, D, G>), dim3(blocks_for(ncell, 256)), dim3(256), 0, st, cases, icase, q, (S*)dst, total)
  FVM_DISPATCH(mixed, dim, kind, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_k_state_to_cons(int dim, int mixed, int kind, const CaseC* cases, int icase, long long ncell,
                               const void* src, double* q, long long total, hipStream_t st)
{
  if (kind >= FVM_KIND_BARO) return fvm_kb_state_to_cons(dim, mixed, kind == FVM_KIND_BARO2, cases, icase, ncell, src, q, total, st);
#define CALL(S, D, P, G) hipLaunchKernelGGL((k_state_to_cons<S, D, G>), dim3(blocks_for(ncell, 256)), dim3(256), 0, st, cases, icase, (const S*)src, q, total)
  FVM_DISPATCH(mixed, dim, kind, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_k_state_to_prim(int dim, int mixed, int kind, const CaseC* cases, int icase, long long ncell,
                               const void* src, double* w, long long total, hipStream_t st)
{
  if (kind >= FVM_KIND_BARO) return fvm_kb_state_to_prim(dim, mixed, kind == FVM_KIND_BARO2, cases, icase, ncell, src, w, total, st);
#define CALL(S, D, P, G) hipLaunchKernelGGL((k_state_to_prim<S, D, P, G>), dim3(blocks_for(ncell, 256)), dim3(256), 0, st, cases, icase, (const S*)src, w, total)
  FVM_DISPATCH(mixed, dim, kind, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_k_dt_init(int dim, int mixed, int kind, const CaseC* cases, CaseDyn* dyn, int icase, long long ncell,
                         const void* src, long long total, long long label_off, hipStream_t st)
{
  if (kind >= FVM_KIND_BARO)
    return fvm_kb_dt_init(dim, mixed, kind == FVM_KIND_BARO2, cases, dyn, icase, ncell, src, total, label_off, st);
#define CALL(S, D, P, G) hipLaunchKernelGGL((k_dt_init<S, D, P, G>), dim3(blocks_for(ncell, 256)), dim3(256), 0, st, cases, dyn, icase, (const S*)src, total, label_off)
  FVM_DISPATCH(mixed, dim, kind, CALL);
#undef CALL
  return hipGetLastError();
}

hipError_t fvm_k_totals(int dim, int mixed, int kind, const CaseC* cases, int icase, long long ncell, const void* src,
                        long long total, double* part, int nblk, double vol, double* out, hipStream_t st)
{
  if (kind >= FVM_KIND_BARO) {
    hipError_t e = fvm_kb_totals_part(dim, mixed, kind == FVM_KIND_BARO2, cases, icase, src, total, part, nblk, st);
    if (e != hipSuccess) return e;
  } else {
#define CALL(S, D, P, G) hipLaunchKernelGGL((k_totals_part<S, D, G>), dim3(nblk), dim3(256), 0, st, cases, icase, (const S*)src, total, part)
    FVM_DISPATCH(mixed, dim, kind, CALL);
#undef CALL
  }
  int nq = dim + (kind == FVM_KIND_BARO ? 2 : (kind == FVM_KIND_BARO2 ? 3 : (kind == FVM_KIND_THREE ? 4 : 3)));
  hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, st, part, nblk, nq, vol, out);
  return hipGetLastError();
}

// storage shifts: partial densities and energies of the pure components at
// (p_ref, T_ref): out[6c + k] = rho_k, out[6c + 3 + k] = e_k (k = 2 only with
// three components)
template <bool PRK>
__global__ void k_ref_shift(const CaseC* cases, int ncases, double* out, const double* pT)
{
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncases) return;
  const CaseC& C = cases[c];
  double p = pT[2 * c], T = pT[2 * c + 1];
  double v0, e0, v1, e1;
  closure_fwd<PRK>(C, p, T, 0.0, v0, e0);
  closure_fwd<PRK>(C, p, T, 1.0, v1, e1);
  double r2 = 0.0, e2 = 0.0;
  if (C.ncomp == 3) {
    const Comp& k = C.comp[2];
    double v2 = k.A * T / (p + k.pinf);
    r2 = 1.0 / v2;
    e2 = k.cv * T + k.pinf * v2 + k.qs;
  }
  out[6 * c] = 1.0 / v0;
  out[6 * c + 1] = 1.0 / v1;
  out[6 * c + 2] = r2;
  out[6 * c + 3] = e0;
  out[6 * c + 4] = e1;
  out[6 * c + 5] = e2;
}

hipError_t fvm_k_ref_shift(const CaseC* cases, int ncases, double* out, const double* pT, hipStream_t st)
{
  hipLaunchKernelGGL((k_ref_shift<true>), dim3((ncases + 63) / 64), dim3(64), 0, st, cases, ncases, out, pT);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(st);
}
