// fvm_stage3m.hip -- instantiation of the fused z-marching 3D stage (the
// closure computed in the kernel for every staged cell).
#include "fvm_stage3m.hpp"

namespace fvm {

template <class S, int TX, int TY, int ZC, int MINW, bool PRK>
static hipError_t launch_m3f(const StageArgs& a, int ntiles, hipStream_t st)
{
  hipLaunchKernelGGL((k_march3<S, TX, TY, ZC, MINW, PRK, 1, true>), dim3(ntiles), dim3(TX * TY), 0, st, a);
  return hipGetLastError();
}

template <class S, bool PRK>
static hipError_t stage_m3f(int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  constexpr int W64 = sizeof(S) == 8 ? 1 : 2;
  switch (tile) {
    case 0: return launch_m3f<S, TILESM[0][0], TILESM[0][1], TILESM[0][2], W64, PRK>(a, ntiles, st);
    case 1: return launch_m3f<S, TILESM[1][0], TILESM[1][1], TILESM[1][2], W64, PRK>(a, ntiles, st);
    case 2: return launch_m3f<S, TILESM[2][0], TILESM[2][1], TILESM[2][2], W64, PRK>(a, ntiles, st);
    case 3: return launch_m3f<S, TILESM[3][0], TILESM[3][1], TILESM[3][2], 2, PRK>(a, ntiles, st);
    case 4: return launch_m3f<S, TILESM[4][0], TILESM[4][1], TILESM[4][2], 2, PRK>(a, ntiles, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fvm

using namespace fvm;

// z-marching tiles: shapes 0 .. NTM-1 with the closure in the kernel, then
// the same shapes after the closure kernel k_prim3 (fvm_stage3mp.hip)
int fvm_k_tile_count_m3() { return 2 * NTM; }

int fvm_k_tile_shape_m3(int t, int* tx, int* ty, int* nt, int* zc)
{
  if (t < 0 || t >= 2 * NTM) return -1;
  const int s = t % NTM;
  *tx = TILESM[s][0];
  *ty = TILESM[s][1];
  *nt = TILESM[s][0] * TILESM[s][1];
  *zc = TILESM[s][2];
  return 0;
}

// kind: FVM_KIND_SG or FVM_KIND_PR (two components, inviscid); the default
// limiters (Koren for velocities, Minmod for p, T, xi) only
hipError_t fvm_k_stage_m3(int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  const bool pr = kind == FVM_KIND_PR;
  if (!fvm_default_limiters(a.sc) || tile < 0 || tile >= 2 * NTM) return hipErrorInvalidValue;
  if (tile >= NTM) return fvm_k_stage_m3p(mixed, kind, tile - NTM, a, ntiles, st);
  if (mixed) return pr ? stage_m3f<float, true>(tile, a, ntiles, st) : stage_m3f<float, false>(tile, a, ntiles, st);
  return pr ? stage_m3f<double, true>(tile, a, ntiles, st) : stage_m3f<double, false>(tile, a, ntiles, st);
}
