// fvm_stage3d.hip -- fused 3D stage kernel (placeholder until the marching kernel lands)
#include <hip/hip_runtime.h>
#include "fvm_kernels.hpp"

int fvm_k_tile_count3() { return 0; }
int fvm_k_tile_shape3(int, int*, int*, int*) { return -1; }
int fvm_k_tile_zchunk3(int) { return 1; }
hipError_t fvm_k_stage3(int, int, int, const StageArgs&, int, hipStream_t) { return hipErrorInvalidValue; }
