// fvm_stage3mp.hip -- instantiation of the z-marching 3D stage that reads
// the primitives the closure kernel k_prim3 writes once per cell and stage.
#include "fvm_stage3m.hpp"

namespace fvm {

template <class S, int TX, int TY, int ZC, int MINW, bool PRK>
static hipError_t launch_m3p(const StageArgs& a, int ntiles, hipStream_t st)
{
  S* W = (S*)a.prim;
  constexpr int PB = (TX * TY * ZC + 255) / 256;
  hipLaunchKernelGGL((k_prim3<S, TX, TY, ZC, PRK, false>), dim3(ntiles * PB), dim3(256), 0, st, a, W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_march3<S, TX, TY, ZC, MINW, PRK, 1, false>), dim3(ntiles), dim3(TX * TY), 0, st, a);
  return hipGetLastError();
}

template <class S, bool PRK>
static hipError_t stage_m3p(int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  constexpr int W64 = sizeof(S) == 8 ? 1 : 2;
  switch (tile) {
    case 0: return launch_m3p<S, TILESM[0][0], TILESM[0][1], TILESM[0][2], W64, PRK>(a, ntiles, st);
    case 1: return launch_m3p<S, TILESM[1][0], TILESM[1][1], TILESM[1][2], W64, PRK>(a, ntiles, st);
    case 2: return launch_m3p<S, TILESM[2][0], TILESM[2][1], TILESM[2][2], W64, PRK>(a, ntiles, st);
    case 3: return launch_m3p<S, TILESM[3][0], TILESM[3][1], TILESM[3][2], 2, PRK>(a, ntiles, st);
    case 4: return launch_m3p<S, TILESM[4][0], TILESM[4][1], TILESM[4][2], 2, PRK>(a, ntiles, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace fvm

using namespace fvm;

hipError_t fvm_k_stage_m3p(int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st)
{
  const bool pr = kind == FVM_KIND_PR;
  if (mixed) return pr ? stage_m3p<float, true>(tile, a, ntiles, st) : stage_m3p<float, false>(tile, a, ntiles, st);
  return pr ? stage_m3p<double, true>(tile, a, ntiles, st) : stage_m3p<double, false>(tile, a, ntiles, st);
}
