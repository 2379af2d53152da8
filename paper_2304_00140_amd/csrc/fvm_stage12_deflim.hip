// fvm_stage12_deflim.hip -- the fused 1D/2D stage kernels instantiated with
// the default limiters (Koren for velocities, Minmod for p, T, xi) as
// compile-time constants: no branch on the limiter kind at each slope.  Its
// own translation unit so that the two instantiation sets compile in parallel.
#include "fvm_stage12.hpp"

hipError_t fvm_k_stage12_deflim(int dim, int mixed, int kind, int tile, const StageArgs& a, int ntiles,
                                hipStream_t st)
{
  return fvm::stage12_any<1>(dim, mixed, kind, tile, a, ntiles, st);
}
