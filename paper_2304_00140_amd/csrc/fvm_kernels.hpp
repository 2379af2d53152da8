// fvm_kernels.hpp -- launch interface between the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "fvm_device.hpp"

struct StageArgs {
  const fvm::CaseC* cases;
  fvm::CaseDyn* dyn;
  const int4* tiles;          // (case, tile x, tile y, tile z) per workgroup
  const void* src;            // q^(k-1), storage variables [N_q][total]
  const void* qn;             // q^n
  void* dst;                  // q^(k)
  void* prim;                 // 3D: primitives of q^(k-1) [9][total] (three components: [11][total]), storage precision
  long long total;            // field stride (cells of all cases)
  double* rhs_out;            // stage < 0: R in conserved variables [N_q][total]
  long long rhs_step;         // stage < 0: step number for the inflow noise
  int step_off;               // stage >= 0: step index relative to CaseDyn::base
  int stage;                  // 0..3, or -1 for a bare right-hand side
  double ak;                  // stage coefficient
  fvm::SchemeC sc;
  // 3D four-equation pair: per tile-table entry, 1 when the CSF term of the
  // tile is exactly zero (its staged gas fractions are uniform), written each
  // stage from the closure kernel's per-tile extremes (frac_ext); null: the
  // face kernel evaluates the term everywhere
  const unsigned char* csf_zero;
  void* frac_ext;
};

// closure of a batch: stiffened-gas pair, Peng-Robinson component 1, a
// liquid with two ideal gases (three components, one more storage field), or
// the barotropic model (no energy field; its own kernels, 1D/2D)
enum { FVM_KIND_SG = 0, FVM_KIND_PR = 1, FVM_KIND_THREE = 2, FVM_KIND_BARO = 3, FVM_KIND_BARO2 = 4 };

// the scheme uses the default limiters (Koren for velocities, Minmod for the
// thermodynamic variables) and reconstructs T: the stage kernels then take
// the limiters as compile-time constants instead of branching on the limiter
// kind at every slope (the internal-energy face closure runs in the run-time
// limiter kernels)
inline bool fvm_default_limiters(const fvm::SchemeC& s)
{
  return s.lim_u == fvm::LIM_KOREN && s.lim_s == fvm::LIM_MINMOD && !s.recon_e;
}

int fvm_k_tile_count(int dim);
int fvm_k_tile_shape(int dim, int tile, int* tx, int* ty, int* nt);
int fvm_k_tile_count3();
int fvm_k_tile_shape3(int tile, int* tx, int* ty, int* nt);
// 3D tiles march along z over this many planes per workgroup
int fvm_k_tile_zchunk3(int tile);

hipError_t fvm_k_stage(int dim, int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st);
// 1D/2D stage kernels with the default limiters fixed (fvm_stage12_deflim.hip)
hipError_t fvm_k_stage12_deflim(int dim, int mixed, int kind, int tile, const StageArgs& a, int ntiles,
                                hipStream_t st);
hipError_t fvm_k_stage3(int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st);
// z-marching 3D stage (fvm_stage3m.hip), two-component inviscid closures; its
// tiles follow the closure + face kernel pair's in the 3D tile numbering
int fvm_k_tile_count_m3();
int fvm_k_tile_shape_m3(int tile, int* tx, int* ty, int* nt, int* zc);
hipError_t fvm_k_stage_m3(int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st);
// the same shapes after the closure kernel k_prim3 (fvm_stage3mp.hip)
hipError_t fvm_k_stage_m3p(int mixed, int kind, int tile, const StageArgs& a, int ntiles, hipStream_t st);
// whether a 3D tile index is one of the z-marching kernel's
int fvm_k_tile_is_m3(int tile);
// -1 for a closure + face pair tile, 0 for a z-marching tile with the closure
// fused, 1 for one after the closure kernel
int fvm_k_tile_march3(int tile);
// shape row (0-9) of a 3D tile index of the closure + face kernel pair, which
// the barotropic 3D kernels share; -1 for a z-marching tile or no tile
int fvm_k_tile_row3(int tile);
int fvm_k_tile_ok3(int mixed, int kind, int tile);
hipError_t fvm_k_advance(fvm::CaseDyn* dyn, int ncases, int nsteps, hipStream_t st);
hipError_t fvm_k_prim_to_state(int dim, int mixed, int kind, const fvm::CaseC* cases, int icase, long long ncell,
                               const double* prim, void* dst, long long total, hipStream_t st);
hipError_t fvm_k_cons_to_state(int dim, int mixed, int kind, const fvm::CaseC* cases, int icase, long long ncell,
                               const double* q, void* dst, long long total, hipStream_t st);
hipError_t fvm_k_state_to_cons(int dim, int mixed, int kind, const fvm::CaseC* cases, int icase, long long ncell,
                               const void* src, double* q, long long total, hipStream_t st);
hipError_t fvm_k_state_to_prim(int dim, int mixed, int kind, const fvm::CaseC* cases, int icase, long long ncell,
                               const void* src, double* w, long long total, hipStream_t st);
// CFL bound of the current state into the slot of the next step, and its
// checks; an error is reported as one of step (base + label_off)
hipError_t fvm_k_dt_init(int dim, int mixed, int kind, const fvm::CaseC* cases, fvm::CaseDyn* dyn, int icase,
                         long long ncell, const void* src, long long total, long long label_off, hipStream_t st);
hipError_t fvm_k_totals(int dim, int mixed, int kind, const fvm::CaseC* cases, int icase, long long ncell, const void* src,
                        long long total, double* part, int nblk, double vol, double* out, hipStream_t st);
hipError_t fvm_k_ref_shift(const fvm::CaseC* cases_in, int ncases, double* out /* [ncases][6] */,
                           const double* pT /* [ncases][2] */, hipStream_t st);

// barotropic model (fvm_baro.hip), 1D and 2D
hipError_t fvm_kb_stage(int dim, int mixed, int g2, int tile, const StageArgs& a, int ntiles, hipStream_t st);
int fvm_kb_tile_ok3(int mixed, int g2, int tile);
hipError_t fvm_kb_prim_to_state(int dim, int mixed, int g2, const fvm::CaseC* cases, int icase, long long ncell,
                                const double* prim, void* dst, long long total, hipStream_t st);
hipError_t fvm_kb_cons_to_state(int dim, int mixed, int g2, const fvm::CaseC* cases, int icase, long long ncell,
                                const double* q, void* dst, long long total, hipStream_t st);
hipError_t fvm_kb_state_to_cons(int dim, int mixed, int g2, const fvm::CaseC* cases, int icase, long long ncell,
                                const void* src, double* q, long long total, hipStream_t st);
hipError_t fvm_kb_state_to_prim(int dim, int mixed, int g2, const fvm::CaseC* cases, int icase, long long ncell,
                                const void* src, double* w, long long total, hipStream_t st);
hipError_t fvm_kb_dt_init(int dim, int mixed, int g2, const fvm::CaseC* cases, fvm::CaseDyn* dyn, int icase,
                          long long ncell, const void* src, long long total, long long label_off, hipStream_t st);
hipError_t fvm_kb_totals_part(int dim, int mixed, int g2, const fvm::CaseC* cases, int icase, const void* src,
                              long long total, double* part, int nblk, hipStream_t st);
