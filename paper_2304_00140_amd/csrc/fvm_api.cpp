// fvm_api.cpp -- C ABI of the solver (include/fvm.h): validation, device
// buffers, the case and tile tables, stage sequencing and HIP-graph replay.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fvm.h"
#include "fvm_kernels.hpp"

using fvm::CaseC;
using fvm::CaseDyn;
using fvm::Comp;
using fvm::SchemeC;

struct fvm_batch {
  int ncases = 0, dim = 0, mixed = 0, kind = FVM_KIND_SG, nq = 0, ncomp = 2;
  hipStream_t st = nullptr;
  std::vector<CaseC> hc;
  std::vector<double> vol;
  CaseC* dc = nullptr;
  CaseDyn* dd = nullptr;
  int4* dtiles = nullptr;
  int ntiles = 0, tile = 0;
  long long total = 0;
  size_t esz = 8;
  void* q[3] = {nullptr, nullptr, nullptr};
  void* prim = nullptr;       // 3D: primitives of the stage input
  void* fext = nullptr;       // 3D pair tiles: gas-fraction extremes per closure workgroup
  unsigned char* czero = nullptr;   // and the per-tile marks of a zero CSF term
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  double* dpart = nullptr;
  double* dout = nullptr;
  SchemeC sc{};
  double rk[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int gsteps = 0;
  double gtend = -1.0;
  std::vector<char> has_state;
  std::string err;
};

struct fvm_ctx {
  fvm_batch* b = nullptr;
};

static int fail(fvm_batch* b, int code, const std::string& msg)
{
  if (b) b->err = msg;
  return code;
}

#define HIPCHECK(b, call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail((b), FVM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));          \
  } while (0)

// ------------------------------------------------------------------ descriptors -> tables
// baro: the barotropic model, whose far-field and inflow states need no
// temperature but a positive pressure
static int check_grid(fvm_batch* b, const fvm_grid_desc* g, bool baro)
{
  if (!g) return fail(b, FVM_EINVAL, "grid descriptor is NULL");
  if (g->dim < 1 || g->dim > 3) return fail(b, FVM_EINVAL, "dim must be 1, 2 or 3");
  for (int d = 0; d < 3; ++d) {
    if (d < g->dim) {
      if (g->n[d] < 2) return fail(b, FVM_EINVAL, "n[d] >= 2 is needed in every used direction");
      if (!(g->dx[d] > 0.0)) return fail(b, FVM_EINVAL, "dx[d] must be > 0");
      for (int s = 0; s < 2; ++s) {
        int k = g->bc[d][s];
        if (k < 0 || k > 4) return fail(b, FVM_EINVAL, "unknown boundary kind");
        if (k == FVM_BC_FARFIELD && !((baro ? g->ff_p > 0.0 : g->ff_T > 0.0) && g->ff_alpha >= 0.0 &&
                                      g->ff_alpha <= 1.0))
          return fail(b, FVM_EINVAL, baro ? "far-field state needs ff_p > 0 and 0 <= ff_alpha <= 1"
                                          : "far-field state needs ff_T > 0 and 0 <= ff_alpha <= 1");
        if (k == FVM_BC_INFLOW && !(d == 0 && s == 0)) return fail(b, FVM_EINVAL, "inflow only at the x-min side");
      }
      if ((g->bc[d][0] == FVM_BC_PERIODIC) != (g->bc[d][1] == FVM_BC_PERIODIC))
        return fail(b, FVM_EINVAL, "periodic boundaries come in pairs");
    } else if (g->n[d] != 1) {
      return fail(b, FVM_EINVAL, "n[d] must be 1 in unused directions");
    }
  }
  if (g->bc[0][0] == FVM_BC_INFLOW && !(baro ? g->in_p > 0.0 : (g->in_p > -1e300 && g->in_T > 0.0)))
    return fail(b, FVM_EINVAL, baro ? "inflow state needs in_p > 0" : "inflow state needs in_T > 0");
  return FVM_OK;
}

static int eos_ncomp(const fvm_eos_desc* e) { return e->ncomp == 3 ? 3 : 2; }

static int check_eos(fvm_batch* b, const fvm_eos_desc* e)
{
  if (!e) return fail(b, FVM_EINVAL, "eos descriptor is NULL");
  if (e->model != FVM_MODEL_FOUR_EQ && e->model != FVM_MODEL_BAROTROPIC)
    return fail(b, FVM_EINVAL, "unknown model");
  if (e->model == FVM_MODEL_BAROTROPIC) {
    if (e->ncomp != 0 && e->ncomp != 2 && e->ncomp != 3)
      return fail(b, FVM_EINVAL, "the barotropic model has one gas (ncomp 2) or two (ncomp 3)");
    if (e->ncomp == 3 && (!(e->bt_RT2 > 0.0) || !std::isfinite(e->bt_RT2)))
      return fail(b, FVM_EINVAL, "a second gas in the barotropic model needs RT2 > 0");
    if (!(e->bt_rho_sat > 0.0) || !(e->bt_p_sat > 0.0) || !(e->bt_c_liq > 0.0) || !(e->bt_RT > 0.0) ||
        !(e->bt_rho_vap >= 0.0) || !(e->bt_rho_vap < e->bt_rho_sat) || !std::isfinite(e->bt_rho_sat) ||
        !std::isfinite(e->bt_p_sat) || !std::isfinite(e->bt_c_liq) || !std::isfinite(e->bt_RT))
      return fail(b, FVM_EINVAL, "barotropic model needs rho_sat, p_sat, c_liq, RT > 0 and 0 <= rho_vap < rho_sat");
    for (int k = 0; k < 3; ++k)
      if (e->kc[k] != 0.0 || (k == 2 && e->ncomp != 3 && e->mu[k] != 0.0))
        return fail(b, FVM_EINVAL,
                    "the barotropic model has no heat conduction (kc = 0) and viscosities mu[0], mu[1] (mu[2] with a "
                    "second gas)");
    if (!(e->mu[0] >= 0.0 && e->mu[0] < 1e300) || !(e->mu[1] >= 0.0 && e->mu[1] < 1e300) ||
        !(e->mu[2] >= 0.0 && e->mu[2] < 1e300) || !(e->bt_mu_vap >= 0.0 && e->bt_mu_vap < 1e300))
      return fail(b, FVM_EINVAL, "viscosities must be finite and >= 0");
    return FVM_OK;
  }
  if (e->ncomp != 0 && e->ncomp != 2 && e->ncomp != 3) return fail(b, FVM_EINVAL, "ncomp must be 2 or 3");
  const int nc = eos_ncomp(e);
  if (nc == 3) {
    for (int k = 0; k < 3; ++k)
      if (e->kind[k] != FVM_EOS_SG) return fail(b, FVM_EINVAL, "three components are all stiffened gases");
    if (e->pinf[1] != 0.0 || e->pinf[2] != 0.0)
      return fail(b, FVM_EINVAL, "the gases of a three-component closure are ideal (pinf = 0)");
  }
  for (int k = 0; k < nc; ++k) {
    if (e->kind[k] == FVM_EOS_SG) {
      if (!(e->gamma[k] > 1.0) || !(e->cv[k] > 0.0) || !(e->pinf[k] >= 0.0))
        return fail(b, FVM_EINVAL, "stiffened gas needs gamma > 1, cv > 0, pinf >= 0");
    } else if (e->kind[k] == FVM_EOS_PR) {
      if (k != 1) return fail(b, FVM_EINVAL, "a Peng-Robinson fluid is supported as component 1 only");
      int ns = e->pr_ns[k];
      if (ns < 1 || ns > FVM_MAXSPEC || !(e->cv[k] > 0.0)) return fail(b, FVM_EINVAL, "bad Peng-Robinson description");
      for (int a = 0; a < ns; ++a)
        if (!(e->pr_Tc[k][a] > 0 && e->pr_pc[k][a] > 0 && e->pr_M[k][a] > 0 && e->pr_vc[k][a] > 0 &&
              e->pr_Zc[k][a] > 0 && e->pr_X[k][a] >= 0))
          return fail(b, FVM_EINVAL, "bad Peng-Robinson species data");
    } else {
      return fail(b, FVM_EINVAL, "unknown closure kind");
    }
    if (!(e->mu[k] >= 0.0 && e->mu[k] < 1e300) || !(e->kc[k] >= 0.0 && e->kc[k] < 1e300))
      return fail(b, FVM_EINVAL, "viscosity and conductivity must be finite and >= 0");
  }
  return FVM_OK;
}

static int check_scheme(fvm_batch* b, const fvm_scheme_desc* s)
{
  if (!s) return fail(b, FVM_EINVAL, "scheme descriptor is NULL");
  if (s->lim_u < 0 || s->lim_u > 7 || s->lim_s < 0 || s->lim_s > 7) return fail(b, FVM_EINVAL, "unknown limiter");
  if (!(s->cfl > 0.0) || !(s->sigma >= 0.0) || !(s->beta > 0.0) || !(s->thinc_gamma >= 0.0) ||
      !(s->eps_normal > 0.0))
    return fail(b, FVM_EINVAL, "scheme parameters out of range");
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(s->gravity[d])) return fail(b, FVM_EINVAL, "gravity must be finite");
  if (s->thermal != 0 && s->thermal != 1) return fail(b, FVM_EINVAL, "thermal must be 0 or 1");
  return FVM_OK;
}

// the internal-energy face closure is built for the two-component
// stiffened-gas closure in 1D and 2D
static int check_thermal(fvm_batch* b, const fvm_scheme_desc* s, int dim, int kind)
{
  if (s->thermal == 1 && (dim == 3 || kind != FVM_KIND_SG))
    return fail(b, FVM_EINVAL,
                "the internal-energy face closure (thermal = 1) takes the two-component stiffened-gas closure in 1D "
                "and 2D");
  return FVM_OK;
}

static void fill_comp(Comp& c, const fvm_eos_desc* e, int k)
{
  std::memset(&c, 0, sizeof c);
  c.kind = e->kind[k];
  c.cv = e->cv[k];
  c.qs = e->q[k];
  if (c.kind == FVM_EOS_SG) {
    c.gamma = e->gamma[k];
    c.pinf = e->pinf[k];
  } else {
    const double R = fvm::R_UNIV;
    int ns = e->pr_ns[k];
    double bb = 0.0, M = 0.0;
    for (int a = 0; a < ns; ++a) {
      bb += e->pr_X[k][a] * 0.077796 * R * e->pr_Tc[k][a] / e->pr_pc[k][a];
      M += e->pr_X[k][a] * e->pr_M[k][a];
    }
    int np = 0;
    for (int a = 0; a < ns; ++a)
      for (int be = a; be < ns; ++be) {
        double Tc = std::sqrt(e->pr_Tc[k][a] * e->pr_Tc[k][be]) * (1.0 - e->pr_kij[k][a][be]);
        double cr = 0.5 * (std::cbrt(e->pr_vc[k][a]) + std::cbrt(e->pr_vc[k][be]));
        double vc = cr * cr * cr;
        double Zc = 0.5 * (e->pr_Zc[k][a] + e->pr_Zc[k][be]);
        double pc = Zc * R * Tc / vc;
        double w = 0.5 * (e->pr_omega[k][a] + e->pr_omega[k][be]);
        c.pcc[np] = 0.37464 + 1.5422 * w - 0.26992 * w * w;
        c.pa0[np] = 0.457236 * (R * Tc) * (R * Tc) / pc;
        c.prs[np] = 1.0 / std::sqrt(Tc);
        c.pw[np] = e->pr_X[k][a] * e->pr_X[k][be] * (a == be ? 1.0 : 2.0);
        ++np;
      }
    c.npair = np;
    c.b = bb;
    c.M = M;
    // sum_q w_q a0_q (A_q - B_q s)^2 with A_q = 1 + c_q, B_q = c_q / sqrt(Tc_q), s = sqrt(T)
    c.pa_0 = c.pa_1 = c.pa_2 = 0.0;
    for (int q = 0; q < np; ++q) {
      double w = c.pw[q] * c.pa0[q], A = 1.0 + c.pcc[q], B = c.pcc[q] * c.prs[q];
      c.pa_0 += w * A * A;
      c.pa_1 += 2.0 * w * A * B;
      c.pa_2 += w * B * B;
    }
    c.iM = 1.0 / M;
    c.ikb = 1.0 / (2.0 * fvm::SQRT2 * bb * M);
    c.gam_ig = 1.0 + R / (M * c.cv);
    c.gamma = c.gam_ig;   // used only by the sound-speed bound of the ideal stand-in
    c.pinf = 0.0;
  }
  c.A = (c.gamma - 1.0) * c.cv;
  c.Cp = c.gamma * c.cv;
  c.c2T = c.gamma * (c.gamma - 1.0) * c.cv;
  c.mu = e->mu[k];
  c.kc = e->kc[k];
}

static int build_tiles(fvm_batch* b)
{
  int tx, ty, nt;
  if (fvm_k_tile_shape(b->dim, b->tile, &tx, &ty, &nt)) return fail(b, FVM_EINVAL, "bad tile index");
  int zc = (b->dim == 3) ? fvm_k_tile_zchunk3(b->tile) : 1;
  std::vector<int4> t;
  for (int c = 0; c < b->ncases; ++c) {
    CaseC& C = b->hc[c];
    C.tiles[0] = (C.n[0] + tx - 1) / tx;
    C.tiles[1] = (b->dim >= 2) ? (C.n[1] + ty - 1) / ty : 1;
    C.tiles[2] = (b->dim >= 3) ? (C.n[2] + zc - 1) / zc : 1;
    C.tile0 = (int)t.size();
    // 3D: up to eight x slabs one after another, each in (z, y, x) order with
    // x fastest, so that the contiguous run of the table each XCD takes is a
    // slab across the whole y-z section (a jet along x lands on every XCD
    // alike); a slab spans at least 64 cells in x, so that the tiles resident
    // together still read rows of 64 cells or more
    C.xslab = (b->dim == 3) ? std::max((C.tiles[0] + 7) / 8, (64 + tx - 1) / tx) : C.tiles[0];
    for (int s0 = 0; s0 < C.tiles[0]; s0 += C.xslab) {
      const int s1 = std::min(C.tiles[0], s0 + C.xslab);
      for (int k = 0; k < C.tiles[2]; ++k)
        for (int j = 0; j < C.tiles[1]; ++j)
          for (int i = s0; i < s1; ++i) t.push_back(make_int4(c, i, j, k));
    }
  }
  if (b->dtiles) (void)hipFree(b->dtiles);
  b->dtiles = nullptr;
  if (b->fext) (void)hipFree(b->fext);
  if (b->czero) (void)hipFree(b->czero);
  b->fext = nullptr;
  b->czero = nullptr;
  b->ntiles = (int)t.size();
  HIPCHECK(b, hipMalloc(&b->dtiles, sizeof(int4) * t.size()));
  if (b->dim == 3 && !fvm_k_tile_is_m3(b->tile)) {
    // the closure + face pair (four-equation or barotropic): (min, max) of both
    // gas fractions per closure workgroup (256 cells; FP64-sized entries) and
    // one mark per tile, from which the face kernel skips a CSF term that is
    // exactly zero
    const size_t pb = ((size_t)tx * ty * zc + 255) / 256;
    HIPCHECK(b, hipMalloc(&b->fext, sizeof(double) * 4 * pb * t.size()));
    HIPCHECK(b, hipMalloc((void**)&b->czero, t.size()));
  }
  HIPCHECK(b, hipMemcpy(b->dtiles, t.data(), sizeof(int4) * t.size(), hipMemcpyHostToDevice));
  HIPCHECK(b, hipMemcpy(b->dc, b->hc.data(), sizeof(CaseC) * b->hc.size(), hipMemcpyHostToDevice));
  return FVM_OK;
}

static void drop_graph(fvm_batch* b)
{
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->gsteps = 0;
}

static int ensure_scratch(fvm_batch* b, size_t bytes)
{
  if (bytes <= b->scratch_bytes) return FVM_OK;
  if (b->scratch) (void)hipFree(b->scratch);
  b->scratch = nullptr;
  b->scratch_bytes = 0;
  if (hipMalloc(&b->scratch, bytes) != hipSuccess) return fail(b, FVM_ENOMEM, "scratch allocation failed");
  b->scratch_bytes = bytes;
  return FVM_OK;
}

static void batch_free(fvm_batch* b)
{
  if (!b) return;
  drop_graph(b);
  for (int i = 0; i < 3; ++i)
    if (b->q[i]) (void)hipFree(b->q[i]);
  if (b->prim) (void)hipFree(b->prim);
  if (b->fext) (void)hipFree(b->fext);
  if (b->czero) (void)hipFree(b->czero);
  if (b->dc) (void)hipFree(b->dc);
  if (b->dd) (void)hipFree(b->dd);
  if (b->dtiles) (void)hipFree(b->dtiles);
  if (b->scratch) (void)hipFree(b->scratch);
  if (b->dpart) (void)hipFree(b->dpart);
  if (b->dout) (void)hipFree(b->dout);
  delete b;
}

// one case's constants from its descriptors (validated): grid, boundary data,
// closure components; rows start at field offset `off`.  Reports the number of
// components, whether the barotropic model is used and whether component 1 is
// a Peng-Robinson fluid.  No storage shifts (FP64 storage); the caller adds
// them for FP32 storage.
static int describe_case(fvm_batch* b, CaseC& C, const fvm_grid_desc* g, const fvm_eos_desc* eos, long long off,
                         double* vol_out, int* nc_out, int* baro_out, int* pr_out)
{
  int rc;
  if (!eos) return fail(b, FVM_EINVAL, "eos descriptor is NULL");
  if ((rc = check_grid(b, g, eos->model == FVM_MODEL_BAROTROPIC))) return rc;
  if ((rc = check_eos(b, eos))) return rc;
  const int nc = eos_ncomp(eos);
  const int baro = eos->model == FVM_MODEL_BAROTROPIC;
  std::memset(&C, 0, sizeof C);
  C.dim = g->dim;
  long long n = 1;
  double vol = 1.0;
  for (int d = 0; d < 3; ++d) {
    C.n[d] = g->n[d];
    C.dx[d] = d < g->dim ? g->dx[d] : 1.0;
    C.idx[d] = 1.0 / C.dx[d];
    C.bc[d][0] = g->bc[d][0];
    C.bc[d][1] = g->bc[d][1];
    n *= g->n[d];
    if (d < g->dim) vol *= g->dx[d];
  }
  if (vol_out) *vol_out = vol;
  C.ncell = n;
  C.off = off;
  C.in_p = g->in_p; C.in_T = g->in_T; C.in_alpha = g->in_alpha; C.in_u = g->in_u;
  C.in_radius = g->in_radius; C.in_c0 = g->in_center[0]; C.in_c1 = g->in_center[1];
  C.in_noise = g->in_noise; C.in_seed = g->in_seed;
  C.ff_p = g->ff_p; C.ff_T = g->ff_T; C.ff_alpha = g->ff_alpha;
  C.any_ff = 0;
  for (int d = 0; d < g->dim; ++d)
    for (int sd = 0; sd < 2; ++sd) C.any_ff |= (g->bc[d][sd] == FVM_BC_FARFIELD);
  C.ncomp = nc;
  C.sdx2 = 0.0;
  for (int d = 0; d < g->dim; ++d) C.sdx2 += C.idx[d] * C.idx[d];
  *nc_out = nc;
  *baro_out = baro;
  *pr_out = 0;
  if (baro) {
    const fvm_eos_desc& e = *eos;
    C.model = 1;
    C.bt_rs = e.bt_rho_sat;
    C.bt_ps = e.bt_p_sat;
    C.bt_cl2 = e.bt_c_liq * e.bt_c_liq;
    C.bt_cm2 = e.bt_p_sat / e.bt_rho_sat;
    C.bt_rv = e.bt_rho_vap;
    C.bt_RT = e.bt_RT;
    C.bt_RT2 = nc == 3 ? e.bt_RT2 : 0.0;
    double cg = std::sqrt(e.bt_RT > C.bt_RT2 ? e.bt_RT : C.bt_RT2), cm = std::sqrt(C.bt_cm2);
    C.bt_c_hi = e.bt_c_liq > cg ? e.bt_c_liq : cg;
    C.bt_c_lo = cm > cg ? cm : cg;
    C.bt_mu_l = e.mu[0];
    C.bt_mu_g = e.mu[1];
    C.bt_mu_v = e.bt_mu_vap;
    C.bt_mu_g2 = nc == 3 ? e.mu[2] : 0.0;
    C.diff = (e.mu[0] > 0.0 || e.mu[1] > 0.0 || C.bt_mu_g2 > 0.0 || e.bt_mu_vap > 0.0) ? 1 : 0;
    return FVM_OK;
  }
  for (int k = 0; k < nc; ++k) fill_comp(C.comp[k], eos, k);
  C.diff = 0;
  for (int k = 0; k < nc; ++k)
    if (eos->mu[k] > 0.0 || eos->kc[k] > 0.0) C.diff = 1;
  if (C.comp[1].kind == FVM_EOS_PR) *pr_out = 1;
  return FVM_OK;
}

static void fill_scheme(SchemeC& S, double* rk, const fvm_scheme_desc* s, int dim)
{
  std::memset(&S, 0, sizeof S);
  S.switching = s->switching; S.lim_u = s->lim_u; S.lim_s = s->lim_s; S.thinc = s->thinc;
  S.beta = s->beta; S.thinc_gamma = s->thinc_gamma; S.eps_int = s->eps_interface;
  S.th_d = s->theta_ducros; S.th_g = s->theta_gas; S.eps_d = s->eps_ducros; S.k3 = s->kappa3;
  S.sigma = s->sigma; S.eps_n = s->eps_normal; S.cfl = s->cfl;
  S.tanh_b = std::tanh(s->beta); S.icosh_b = 1.0 / std::cosh(s->beta); S.itanh_b = 1.0 / std::tanh(s->beta);
  S.t_end = 0.0;
  S.has_grav = 0;
  for (int d = 0; d < 3; ++d) {
    S.grav[d] = d < dim ? s->gravity[d] : 0.0;
    if (S.grav[d] != 0.0) S.has_grav = 1;
  }
  S.recon_e = s->thermal;
  for (int i = 0; i < 4; ++i) rk[i] = s->rk[i];
}

static int batch_create(fvm_batch** out, int ncases, const fvm_grid_desc* grids, const fvm_eos_desc* eos,
                        const fvm_scheme_desc* s, int precision, void* stream, std::string* errout)
{
  fvm_batch* b = new fvm_batch();
  auto bail = [&](int rc) {
    if (errout) *errout = b->err;
    batch_free(b);
    return rc;
  };
  if (!out) return bail(fail(b, FVM_EINVAL, "out is NULL"));
  *out = nullptr;
  if (ncases < 1 || !grids || !eos) return bail(fail(b, FVM_EINVAL, "need at least one case"));
  if (precision != FVM_FP64 && precision != FVM_MIXED) return bail(fail(b, FVM_EINVAL, "unknown precision"));
  int rc = check_scheme(b, s);
  if (rc) return bail(rc);
  b->ncases = ncases;
  b->dim = grids[0].dim;
  b->mixed = precision == FVM_MIXED;
  b->esz = b->mixed ? sizeof(float) : sizeof(double);
  b->st = (hipStream_t)stream;
  b->hc.resize(ncases);
  b->vol.resize(ncases);
  b->has_state.assign(ncases, 0);
  long long off = 0;
  for (int c = 0; c < ncases; ++c) {
    int nc = 0, baro = 0, pr = 0;
    if ((rc = describe_case(b, b->hc[c], &grids[c], &eos[c], off, &b->vol[c], &nc, &baro, &pr))) return bail(rc);
    if (grids[c].dim != b->dim) return bail(fail(b, FVM_EINVAL, "all cases of a batch share the dimension"));
    if (c == 0) b->ncomp = nc;
    if (nc != b->ncomp) return bail(fail(b, FVM_EINVAL, "all cases of a batch share the number of components"));
    if (c == 0) b->kind = baro ? FVM_KIND_BARO : FVM_KIND_SG;
    if (baro != (b->kind >= FVM_KIND_BARO)) return bail(fail(b, FVM_EINVAL, "all cases of a batch share the model"));
    if (pr) b->kind = FVM_KIND_PR;
    off += (b->hc[c].ncell + 63) / 64 * 64;   // keep every case's rows starting on a 64-word boundary
  }
  if (b->ncomp == 3) b->kind = (b->kind == FVM_KIND_BARO) ? FVM_KIND_BARO2 : FVM_KIND_THREE;
  b->nq = (b->kind >= FVM_KIND_BARO) ? b->dim + b->ncomp : b->dim + b->ncomp + 1;
  if ((rc = check_thermal(b, s, b->dim, b->kind))) return bail(rc);
  b->total = off;
  fill_scheme(b->sc, b->rk, s, b->dim);

  // device tables
  HIPCHECK(b, hipMalloc(&b->dc, sizeof(CaseC) * ncases));
  HIPCHECK(b, hipMalloc(&b->dd, sizeof(CaseDyn) * ncases));
  HIPCHECK(b, hipMemset(b->dd, 0, sizeof(CaseDyn) * ncases));
  HIPCHECK(b, hipMemcpy(b->dc, b->hc.data(), sizeof(CaseC) * ncases, hipMemcpyHostToDevice));

  // storage shifts: rho_k(p_ref, T_ref) and e_k(p_ref, T_ref), evaluated by the device closure
  {
    std::vector<double> pT(2 * ncases), sh(6 * ncases);
    bool any = false;
    for (int c = 0; c < ncases; ++c) {
      pT[2 * c] = eos[c].p_ref;
      pT[2 * c + 1] = eos[c].T_ref;
      any = any || (eos[c].T_ref > 0.0);
    }
    if (b->kind >= FVM_KIND_BARO) any = false;
    if (any && b->mixed) {
      if ((rc = ensure_scratch(b, sizeof(double) * 8 * ncases))) return bail(rc);
      double* dpT = (double*)b->scratch;
      double* dsh = dpT + 2 * ncases;
      HIPCHECK(b, hipMemcpy(dpT, pT.data(), sizeof(double) * 2 * ncases, hipMemcpyHostToDevice));
      HIPCHECK(b, fvm_k_ref_shift(b->dc, ncases, dsh, dpT, nullptr));
      HIPCHECK(b, hipMemcpy(sh.data(), dsh, sizeof(double) * 6 * ncases, hipMemcpyDeviceToHost));
    }
    for (int c = 0; c < ncases; ++c) {
      CaseC& C = b->hc[c];
      if (b->kind >= FVM_KIND_BARO) {
        // FP32 storage keeps the liquid's partial density relative to the
        // liquid density at p_ref (eq. 2-3 / 2-4); the gas is unshifted
        double pr = eos[c].p_ref, rl = 0.0;
        if (b->mixed && pr > 0.0 && std::isfinite(pr)) {
          double c2 = pr >= C.bt_ps ? C.bt_cl2 : C.bt_cm2;
          rl = (double)(float)(C.bt_rs + (pr - C.bt_ps) / c2);
        }
        C.rref[0] = rl;
        continue;
      }
      // FP64 storage needs no shift; FP32 storage shifts the partial density of
      // stiff components (pinf > 0, where one FP32 ulp of density is a large
      // pressure) and the energy of both components.  Gases keep their
      // partial density unshifted so that trace amounts keep full relative
      // precision.
      const int nc = b->ncomp;
      bool on = b->mixed && eos[c].T_ref > 0.0;
      for (int k = 0; k < nc; ++k) on = on && std::isfinite(sh[6 * c + k]) && std::isfinite(sh[6 * c + 3 + k]);
      for (int k = 0; k < nc; ++k) {
        bool stiff = eos[c].kind[k] == FVM_EOS_SG && eos[c].pinf[k] > 0.0;
        double rref = (on && stiff) ? sh[6 * c + k] : 0.0;
        double qs = on ? eos[c].q[k] - sh[6 * c + 3 + k] : eos[c].q[k];
        if (b->mixed) { rref = (double)(float)rref; qs = (double)(float)qs; }
        C.rref[k] = rref;
        C.comp[k].qs = qs;
        C.Q[k] = eos[c].q[k] - qs;
      }
    }
  }

  size_t bytes = (size_t)b->nq * (size_t)b->total * b->esz;
  for (int i = 0; i < 3; ++i) {
    if (hipMalloc(&b->q[i], bytes) != hipSuccess) return bail(fail(b, FVM_ENOMEM, "state allocation failed"));
    HIPCHECK(b, hipMemset(b->q[i], 0, bytes));
  }
  if (b->dim == 3) {
    // rho, u, v, w, p, T, xi, c, alpha (+ xi_2, alpha_2 with three components)
    // (barotropic: rho, u, v, w, p, xi, alpha_G, alpha_V, c in FP32 + xi_2, alpha_G2 with two gases)
    const size_t rows = (b->kind == FVM_KIND_THREE || b->kind == FVM_KIND_BARO2) ? 11 : 9;
    if (hipMalloc(&b->prim, rows * (size_t)b->total * b->esz) != hipSuccess)
      return bail(fail(b, FVM_ENOMEM, "primitive buffer allocation failed"));
    // zero T: the first closure of a Peng-Robinson cell takes the ideal-gas start
    HIPCHECK(b, hipMemset(b->prim, 0, rows * (size_t)b->total * b->esz));
  }
  HIPCHECK(b, hipMalloc(&b->dpart, sizeof(double) * 1024 * 8));
  HIPCHECK(b, hipMalloc(&b->dout, sizeof(double) * 16));
  b->tile = 0;
  if ((rc = build_tiles(b))) return bail(rc);
  *out = b;
  return FVM_OK;
}

// ------------------------------------------------------------------ stepping
static StageArgs stage_args(fvm_batch* b)
{
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  a.cases = b->dc;
  a.dyn = b->dd;
  a.tiles = b->dtiles;
  a.total = b->total;
  a.prim = b->prim;
  a.sc = b->sc;
  a.frac_ext = b->fext;
  a.csf_zero = b->czero;
  return a;
}

// the four stage launches of step `off` of the current chunk (dt, t and the
// step number are derived on the device from CaseDyn)
static hipError_t launch_stages(fvm_batch* b, int off, double t_end, hipEvent_t* ev = nullptr)
{
  StageArgs a = stage_args(b);
  a.sc.t_end = t_end;
  a.step_off = off;
  void* src[4] = {b->q[0], b->q[1], b->q[2], b->q[1]};
  void* dst[4] = {b->q[1], b->q[2], b->q[1], b->q[0]};
  for (int k = 0; k < 4; ++k) {
    a.src = src[k];
    a.qn = b->q[0];
    a.dst = dst[k];
    a.stage = k;
    a.ak = b->rk[k];
    hipError_t e;
    if (ev && (e = hipEventRecord(ev[2 * k], b->st)) != hipSuccess) return e;
    e = fvm_k_stage(b->dim, b->mixed, b->kind, b->tile, a, b->ntiles, b->st);
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[2 * k + 1], b->st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// a chunk of n steps followed by the device-side step counter update
static hipError_t launch_chunk(fvm_batch* b, int n, double t_end)
{
  for (int i = 0; i < n; ++i) {
    hipError_t e = launch_stages(b, i, t_end);
    if (e != hipSuccess) return e;
  }
  return fvm_k_advance(b->dd, b->ncases, n, b->st);
}

static int all_state(fvm_batch* b)
{
  for (int c = 0; c < b->ncases; ++c)
    if (!b->has_state[c]) return fail(b, FVM_ESTATE, "a case has no state yet");
  return FVM_OK;
}

static int check_errors(fvm_batch* b, int* icase = nullptr)
{
  std::vector<CaseDyn> d(b->ncases);
  HIPCHECK(b, hipMemcpy(d.data(), b->dd, sizeof(CaseDyn) * b->ncases, hipMemcpyDeviceToHost));
  for (int c = 0; c < b->ncases; ++c)
    if (d[c].err) {
      if (icase) *icase = c;
      char msg[160];
      std::snprintf(msg, sizeof msg, "case %d: %s at cell %lld, step %lld", c,
                    d[c].err == FVM_ENAN ? "NaN/Inf" : "non-physical state", d[c].err_cell, d[c].err_step);
      return fail(b, d[c].err, msg);
    }
  return FVM_OK;
}

// 3D: the last stage does not inspect q^(n+1) (the next step's closure kernel
// does), so the state a run ends on is checked here
static hipError_t end_check(fvm_batch* b)
{
  if (b->dim != 3) return hipSuccess;
  for (int c = 0; c < b->ncases; ++c) {
    hipError_t e = fvm_k_dt_init(b->dim, b->mixed, b->kind, b->dc, b->dd, c, b->hc[c].ncell, b->q[0], b->total, -1,
                                 b->st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static int run_steps(fvm_batch* b, int n, double t_end)
{
  int rc = all_state(b);
  if (rc) return rc;
  const int chunk = 50;
  bool use_graph = b->st != nullptr && n >= chunk;
  int done = 0;
  if (use_graph) {
    if (!b->gexec || b->gsteps != chunk || b->gtend != t_end) {
      drop_graph(b);
      HIPCHECK(b, hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
      hipError_t e = launch_chunk(b, chunk, t_end);
      hipGraph_t g = nullptr;
      hipError_t e2 = hipStreamEndCapture(b->st, &g);
      if (e != hipSuccess) return fail(b, FVM_EHIP, std::string("launch during capture: ") + hipGetErrorString(e));
      if (e2 != hipSuccess) return fail(b, FVM_EHIP, std::string("capture: ") + hipGetErrorString(e2));
      b->graph = g;
      HIPCHECK(b, hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
      b->gsteps = chunk;
      b->gtend = t_end;
    }
    for (; done + chunk <= n; done += chunk) HIPCHECK(b, hipGraphLaunch(b->gexec, b->st));
  }
  if (done < n) HIPCHECK(b, launch_chunk(b, n - done, t_end));
  HIPCHECK(b, end_check(b));
  HIPCHECK(b, hipStreamSynchronize(b->st));
  return check_errors(b);
}

static int set_from_device_cons(fvm_batch* b, int c, const double* qdev)
{
  const CaseC& C = b->hc[c];
  HIPCHECK(b, fvm_k_cons_to_state(b->dim, b->mixed, b->kind, b->dc, c, C.ncell, qdev, b->q[0], b->total, b->st));
  return FVM_OK;
}

static int finish_set(fvm_batch* b, int c)
{
  const CaseC& C = b->hc[c];
  CaseDyn z;
  std::memset(&z, 0, sizeof z);
  HIPCHECK(b, hipMemcpyAsync(b->dd + c, &z, sizeof z, hipMemcpyHostToDevice, b->st));
  HIPCHECK(b, fvm_k_dt_init(b->dim, b->mixed, b->kind, b->dc, b->dd, c, C.ncell, b->q[0], b->total, 0, b->st));
  HIPCHECK(b, hipStreamSynchronize(b->st));
  b->has_state[c] = 1;
  int rc = check_errors(b);
  if (rc) b->has_state[c] = 0;
  return rc;
}

static int batch_init_primitive(fvm_batch* b, int c, const double* prim)
{
  if (c < 0 || c >= b->ncases || !prim) return fail(b, FVM_EINVAL, "bad case or NULL array");
  const CaseC& C = b->hc[c];
  size_t bytes = sizeof(double) * (3 + b->dim + (b->ncomp == 3 ? 1 : 0)) * (size_t)C.ncell;
  int rc = ensure_scratch(b, bytes);
  if (rc) return rc;
  HIPCHECK(b, hipMemcpyAsync(b->scratch, prim, bytes, hipMemcpyHostToDevice, b->st));
  HIPCHECK(b, fvm_k_prim_to_state(b->dim, b->mixed, b->kind, b->dc, c, C.ncell, (const double*)b->scratch,
                                  b->q[0], b->total, b->st));
  return finish_set(b, c);
}

static int batch_set_state(fvm_batch* b, int c, const double* q, bool device)
{
  if (c < 0 || c >= b->ncases || !q) return fail(b, FVM_EINVAL, "bad case or NULL array");
  const CaseC& C = b->hc[c];
  size_t bytes = sizeof(double) * b->nq * (size_t)C.ncell;
  const double* qd = q;
  if (!device) {
    int rc = ensure_scratch(b, bytes);
    if (rc) return rc;
    HIPCHECK(b, hipMemcpyAsync(b->scratch, q, bytes, hipMemcpyHostToDevice, b->st));
    qd = (const double*)b->scratch;
  }
  int rc = set_from_device_cons(b, c, qd);
  if (rc) return rc;
  return finish_set(b, c);
}

static int batch_get_state(fvm_batch* b, int c, double* q, bool device)
{
  if (c < 0 || c >= b->ncases || !q) return fail(b, FVM_EINVAL, "bad case or NULL array");
  if (!b->has_state[c]) return fail(b, FVM_ESTATE, "no state set");
  const CaseC& C = b->hc[c];
  size_t bytes = sizeof(double) * b->nq * (size_t)C.ncell;
  double* qd = q;
  if (!device) {
    int rc = ensure_scratch(b, bytes);
    if (rc) return rc;
    qd = (double*)b->scratch;
  }
  HIPCHECK(b, fvm_k_state_to_cons(b->dim, b->mixed, b->kind, b->dc, c, C.ncell, b->q[0], qd, b->total, b->st));
  if (!device) HIPCHECK(b, hipMemcpyAsync(q, qd, bytes, hipMemcpyDeviceToHost, b->st));
  HIPCHECK(b, hipStreamSynchronize(b->st));
  return FVM_OK;
}

static int batch_totals(fvm_batch* b, int c, double* out)
{
  if (c < 0 || c >= b->ncases || !out) return fail(b, FVM_EINVAL, "bad case or NULL array");
  if (!b->has_state[c]) return fail(b, FVM_ESTATE, "no state set");
  const CaseC& C = b->hc[c];
  int nblk = (int)std::min<long long>(1024, (C.ncell + 255) / 256);
  HIPCHECK(b, fvm_k_totals(b->dim, b->mixed, b->kind, b->dc, c, C.ncell, b->q[0], b->total, b->dpart, nblk, b->vol[c],
                           b->dout, b->st));
  HIPCHECK(b, hipMemcpyAsync(out, b->dout, sizeof(double) * b->nq, hipMemcpyDeviceToHost, b->st));
  HIPCHECK(b, hipStreamSynchronize(b->st));
  return FVM_OK;
}

static int time_stages(fvm_batch* b, int steps, double* ms)
{
  int rc = all_state(b);
  if (rc) return rc;
  if (steps < 1 || !ms) return fail(b, FVM_EINVAL, "steps >= 1 and an output array are needed");
  std::vector<hipEvent_t> ev(8 * steps);
  for (auto& e : ev) HIPCHECK(b, hipEventCreate(&e));
  for (int s = 0; s < steps; ++s) HIPCHECK(b, launch_stages(b, s, 0.0, &ev[8 * s]));
  HIPCHECK(b, fvm_k_advance(b->dd, b->ncases, steps, b->st));
  HIPCHECK(b, end_check(b));
  HIPCHECK(b, hipStreamSynchronize(b->st));
  for (int k = 0; k < 4; ++k) ms[k] = 0.0;
  for (int s = 0; s < steps; ++s)
    for (int k = 0; k < 4; ++k) {
      float t = 0.f;
      HIPCHECK(b, hipEventElapsedTime(&t, ev[8 * s + 2 * k], ev[8 * s + 2 * k + 1]));
      ms[k] += t / steps;
    }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return check_errors(b);
}

// ------------------------------------------------------------------ C ABI: single case
extern "C" {

static thread_local std::string g_create_err;

int fvm_version(void) { return FVM_VERSION; }

int fvm_create(fvm_ctx** out, const fvm_grid_desc* g, const fvm_eos_desc* e, const fvm_scheme_desc* s,
               int precision, void* stream)
{
  if (!out) return FVM_EINVAL;
  *out = nullptr;
  fvm_batch* b = nullptr;
  int rc = batch_create(&b, 1, g, e, s, precision, stream, &g_create_err);
  if (rc) return rc;
  fvm_ctx* c = new fvm_ctx();
  c->b = b;
  *out = c;
  return FVM_OK;
}

void fvm_destroy(fvm_ctx* ctx)
{
  if (!ctx) return;
  if (ctx->b) (void)hipStreamSynchronize(ctx->b->st);
  batch_free(ctx->b);
  delete ctx;
}

const char* fvm_last_error(const fvm_ctx* ctx)
{
  if (!ctx || !ctx->b) return g_create_err.c_str();
  return ctx->b->err.c_str();
}

#define CTX_CHECK(ctx) \
  if (!(ctx) || !(ctx)->b) return FVM_EINVAL

int fvm_init_primitive(fvm_ctx* ctx, const double* prim_host)
{
  CTX_CHECK(ctx);
  return batch_init_primitive(ctx->b, 0, prim_host);
}

int fvm_set_state(fvm_ctx* ctx, const double* q_host)
{
  CTX_CHECK(ctx);
  return batch_set_state(ctx->b, 0, q_host, false);
}

int fvm_set_state_device(fvm_ctx* ctx, const double* q_dev)
{
  CTX_CHECK(ctx);
  return batch_set_state(ctx->b, 0, q_dev, true);
}

int fvm_get_state(fvm_ctx* ctx, double* q_host)
{
  CTX_CHECK(ctx);
  return batch_get_state(ctx->b, 0, q_host, false);
}

int fvm_get_state_device(fvm_ctx* ctx, double* q_dev)
{
  CTX_CHECK(ctx);
  return batch_get_state(ctx->b, 0, q_dev, true);
}

int fvm_get_primitive(fvm_ctx* ctx, double* w_host)
{
  CTX_CHECK(ctx);
  fvm_batch* b = ctx->b;
  if (!w_host) return fail(b, FVM_EINVAL, "NULL array");
  if (!b->has_state[0]) return fail(b, FVM_ESTATE, "no state set");
  const CaseC& C = b->hc[0];
  size_t rows = b->kind >= FVM_KIND_BARO ? 12 : (b->ncomp == 3 ? 11 : 9);
  size_t bytes = sizeof(double) * rows * (size_t)C.ncell;
  int rc = ensure_scratch(b, bytes);
  if (rc) return rc;
  HIPCHECK(b, fvm_k_state_to_prim(b->dim, b->mixed, b->kind, b->dc, 0, C.ncell, b->q[0], (double*)b->scratch,
                                  b->total, b->st));
  HIPCHECK(b, hipMemcpyAsync(w_host, b->scratch, bytes, hipMemcpyDeviceToHost, b->st));
  HIPCHECK(b, hipStreamSynchronize(b->st));
  return FVM_OK;
}

int fvm_rhs(fvm_ctx* ctx, const double* q_dev_in, double* r_dev_out, int64_t step)
{
  CTX_CHECK(ctx);
  fvm_batch* b = ctx->b;
  if (!q_dev_in || !r_dev_out) return fail(b, FVM_EINVAL, "NULL device array");
  const CaseC& C = b->hc[0];
  // the input goes to the first stage buffer; the case's own state q^n is untouched
  HIPCHECK(b, fvm_k_cons_to_state(b->dim, b->mixed, b->kind, b->dc, 0, C.ncell, q_dev_in, b->q[1], b->total, b->st));
  StageArgs a = stage_args(b);
  a.src = b->q[1];
  a.qn = b->q[1];
  a.dst = nullptr;
  a.stage = -1;
  a.rhs_out = r_dev_out;
  a.rhs_step = step;
  HIPCHECK(b, fvm_k_stage(b->dim, b->mixed, b->kind, b->tile, a, b->ntiles, b->st));
  HIPCHECK(b, hipStreamSynchronize(b->st));
  return FVM_OK;
}

int fvm_step(fvm_ctx* ctx, double* dt_out, double* t_out)
{
  CTX_CHECK(ctx);
  int rc = run_steps(ctx->b, 1, 0.0);
  double t, dt;
  int64_t n;
  fvm_clock(ctx, &t, &dt, &n);
  if (dt_out) *dt_out = dt;
  if (t_out) *t_out = t;
  return rc;
}

int fvm_n_steps(fvm_ctx* ctx, int n, double t_end, double* t_out)
{
  CTX_CHECK(ctx);
  if (n < 0) return fail(ctx->b, FVM_EINVAL, "n < 0");
  int rc = run_steps(ctx->b, n, t_end);
  if (t_out) {
    double dt;
    int64_t k;
    fvm_clock(ctx, t_out, &dt, &k);
  }
  return rc;
}

int fvm_clock(fvm_ctx* ctx, double* t, double* dt, int64_t* steps)
{
  CTX_CHECK(ctx);
  fvm_batch* b = ctx->b;
  CaseDyn d;
  HIPCHECK(b, hipMemcpy(&d, b->dd, sizeof d, hipMemcpyDeviceToHost));
  if (t) *t = d.t[d.base & 1];
  if (dt) *dt = d.dt_last;
  if (steps) *steps = d.base;
  return FVM_OK;
}

int fvm_totals(fvm_ctx* ctx, double* out)
{
  CTX_CHECK(ctx);
  return batch_totals(ctx->b, 0, out);
}

int fvm_error_info(fvm_ctx* ctx, int* code, int64_t* cell, int64_t* step)
{
  CTX_CHECK(ctx);
  CaseDyn d;
  HIPCHECK(ctx->b, hipMemcpy(&d, ctx->b->dd, sizeof d, hipMemcpyDeviceToHost));
  if (code) *code = d.err;
  if (cell) *cell = d.err_cell;
  if (step) *step = d.err_step;
  return FVM_OK;
}

int fvm_tile_count(int dim) { return fvm_k_tile_count(dim); }

int fvm_tile_kernels(int dim, int tile)
{
  if (dim < 1 || dim > 3 || tile < 0 || tile >= fvm_k_tile_count(dim)) return FVM_EINVAL;
  if (dim < 3) return FVM_TK_STAGE;
  int m = fvm_k_tile_march3(tile);
  return m < 0 ? FVM_TK_PAIR : (m == 0 ? FVM_TK_MARCH : FVM_TK_PRIM_MARCH);
}

int fvm_tile_shape(int dim, int tile, int* tx, int* ty, int* threads)
{
  int a, b2, c;
  if (fvm_k_tile_shape(dim, tile, &a, &b2, &c)) return FVM_EINVAL;
  if (tx) *tx = a;
  if (ty) *ty = b2;
  if (threads) *threads = c;
  return FVM_OK;
}

// a tile index that exists and whose kernels fit this batch's closure and precision
static int check_tile(fvm_batch* b, int tile)
{
  if (tile < 0 || tile >= fvm_k_tile_count(b->dim)) return fail(b, FVM_EINVAL, "bad tile index");
  if (b->dim == 3 && fvm_k_tile_is_m3(tile)) {
    bool ok = (b->kind == FVM_KIND_SG || b->kind == FVM_KIND_PR) && fvm_default_limiters(b->sc);
    for (const CaseC& C : b->hc) ok = ok && !C.diff;
    if (!ok)
      return fail(b, FVM_EINVAL,
                  "the z-marching 3D tiles take two-component inviscid closures (stiffened gas or Peng-Robinson) "
                  "with the default limiters");
    return FVM_OK;
  }
  if (b->dim == 3 && b->kind == FVM_KIND_THREE && !fvm_k_tile_ok3(b->mixed, b->kind, tile))
    return fail(b, FVM_EINVAL, "this 3D tile does not fit the LDS of a workgroup with three components in FP64");
  if (b->dim == 3 && b->kind == FVM_KIND_BARO2 && fvm_kb_tile_ok3(b->mixed, 1, tile) != 1)
    return fail(b, FVM_EINVAL, "this 3D tile does not fit the LDS of a workgroup with two gases in FP64");
  return FVM_OK;
}

int fvm_set_tile(fvm_ctx* ctx, int tile)
{
  CTX_CHECK(ctx);
  fvm_batch* b = ctx->b;
  int rc = check_tile(b, tile);
  if (rc) return rc;
  drop_graph(b);
  b->tile = tile;
  return build_tiles(b);
}

int fvm_time_stages(fvm_ctx* ctx, int steps, double* ms_per_stage)
{
  CTX_CHECK(ctx);
  return time_stages(ctx->b, steps, ms_per_stage);
}

// ------------------------------------------------------------------ C ABI: batches
int fvm_batch_create(fvm_batch** out, int ncases, const fvm_grid_desc* grids, const fvm_eos_desc* eos,
                     const fvm_scheme_desc* s, int precision, void* stream)
{
  return batch_create(out, ncases, grids, eos, s, precision, stream, &g_create_err);
}

void fvm_batch_destroy(fvm_batch* b)
{
  if (b) (void)hipStreamSynchronize(b->st);
  batch_free(b);
}

const char* fvm_batch_last_error(const fvm_batch* b) { return b ? b->err.c_str() : g_create_err.c_str(); }

int fvm_batch_init_primitive(fvm_batch* b, int icase, const double* prim_host)
{
  if (!b) return FVM_EINVAL;
  return batch_init_primitive(b, icase, prim_host);
}

int fvm_batch_set_state(fvm_batch* b, int icase, const double* q_host)
{
  if (!b) return FVM_EINVAL;
  return batch_set_state(b, icase, q_host, false);
}

int fvm_batch_get_state(fvm_batch* b, int icase, double* q_host)
{
  if (!b) return FVM_EINVAL;
  return batch_get_state(b, icase, q_host, false);
}

int fvm_batch_n_steps(fvm_batch* b, int n, double* t_out)
{
  if (!b) return FVM_EINVAL;
  if (n < 0) return fail(b, FVM_EINVAL, "n < 0");
  int rc = run_steps(b, n, 0.0);
  if (t_out) {
    std::vector<CaseDyn> d(b->ncases);
    HIPCHECK(b, hipMemcpy(d.data(), b->dd, sizeof(CaseDyn) * b->ncases, hipMemcpyDeviceToHost));
    for (int c = 0; c < b->ncases; ++c) t_out[c] = d[c].t[d[c].base & 1];
  }
  return rc;
}

int fvm_batch_totals(fvm_batch* b, int icase, double* out)
{
  if (!b) return FVM_EINVAL;
  return batch_totals(b, icase, out);
}

int fvm_batch_error_info(fvm_batch* b, int* code, int* icase, int64_t* cell, int64_t* step)
{
  if (!b) return FVM_EINVAL;
  std::vector<CaseDyn> d(b->ncases);
  HIPCHECK(b, hipMemcpy(d.data(), b->dd, sizeof(CaseDyn) * b->ncases, hipMemcpyDeviceToHost));
  if (code) *code = 0;
  for (int c = 0; c < b->ncases; ++c)
    if (d[c].err) {
      if (code) *code = d[c].err;
      if (icase) *icase = c;
      if (cell) *cell = d[c].err_cell;
      if (step) *step = d[c].err_step;
      break;
    }
  return FVM_OK;
}

int fvm_batch_time_stages(fvm_batch* b, int steps, double* ms_per_stage)
{
  if (!b) return FVM_EINVAL;
  return time_stages(b, steps, ms_per_stage);
}

int fvm_batch_set_tile(fvm_batch* b, int tile)
{
  if (!b) return FVM_EINVAL;
  int rc = check_tile(b, tile);
  if (rc) return rc;
  drop_graph(b);
  b->tile = tile;
  return build_tiles(b);
}

int64_t fvm_batch_cells(fvm_batch* b)
{
  if (!b) return -1;
  long long n = 0;
  for (const CaseC& C : b->hc) n += C.ncell;
  return n;
}

}  // extern "C"

// ------------------------------------------------------------------ allocation-free right-hand side
// Workspace of fvm_rhs_noalloc: the case and tile tables, the FP64 storage
// copy of the input and (3D) the primitive rows, in one file-scope device
// array.  Every GPU the library runs on holds its own copy until the process
// ends; in host code the array's name is only a stand-in, so its device
// address is looked up once per device and kept in g_noalloc_ptr.
static __device__ __align__(256) unsigned char scratch[FVM_NOALLOC_SCRATCH_BYTES];

static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[64];

static int noalloc_base(void** out, std::string& err)
{
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return FVM_EHIP;
  }
  if (dev < 0 || dev >= 64) {
    err = "device index out of range for the allocation-free workspace";
    return FVM_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return FVM_EHIP;
    }
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return FVM_OK;
}

// case table (by value), zeroed per-case scalars, the tile table of one case
// ((case 0, i, j, k), i fastest) and zeroed rows [zero0, zero0 + nzero) of the
// 3D primitive buffer (a zero temperature makes a Peng-Robinson closure start
// from its ideal-gas stand-in); no memset or copy nodes
__global__ void k_noalloc_setup(CaseC c, CaseC* dc, CaseDyn* dd, int4* tiles, int ntiles, int t0, int t1,
                                double* zero0, long long nzero)
{
  const long long tid = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const long long nth = (long long)gridDim.x * blockDim.x;
  if (tid == 0) {
    *dc = c;
    unsigned char* z = reinterpret_cast<unsigned char*>(dd);
    for (size_t i = 0; i < sizeof(CaseDyn); ++i) z[i] = 0;
  }
  for (long long i = tid; i < ntiles; i += nth)
    tiles[i] = make_int4(0, (int)(i % t0), (int)((i / t0) % t1), (int)(i / ((long long)t0 * t1)));
  for (long long i = tid; i < nzero; i += nth) zero0[i] = 0.0;
}

static size_t align256(size_t n) { return (n + 255) / 256 * 256; }

extern "C" int fvm_rhs_noalloc(const fvm_grid_desc* g, const fvm_eos_desc* e, const fvm_scheme_desc* s,
                               const double* q_dev_in, double* r_dev_out, int64_t step, void* stream)
{
  fvm_batch eb;   // error messages only (its containers stay empty)
  auto bail = [&](int rc) {
    g_create_err = eb.err;
    return rc;
  };
  if (!q_dev_in || !r_dev_out) return bail(fail(&eb, FVM_EINVAL, "NULL device array"));
  int rc = check_scheme(&eb, s);
  if (rc) return bail(rc);
  CaseC C;
  int nc = 0, baro = 0, pr = 0;
  if ((rc = describe_case(&eb, C, g, e, 0, nullptr, &nc, &baro, &pr))) return bail(rc);
  const int dim = C.dim;
  const int kind = baro ? (nc == 3 ? FVM_KIND_BARO2 : FVM_KIND_BARO)
                        : (nc == 3 ? FVM_KIND_THREE : (pr ? FVM_KIND_PR : FVM_KIND_SG));
  const int nq = baro ? dim + nc : dim + nc + 1;
  if ((rc = check_thermal(&eb, s, dim, kind))) return bail(rc);
  const int tile = 0;
  int tx, ty, nt;
  if (fvm_k_tile_shape(dim, tile, &tx, &ty, &nt)) return bail(fail(&eb, FVM_EINVAL, "bad tile"));
  const int zc = dim == 3 ? fvm_k_tile_zchunk3(tile) : 1;
  C.tiles[0] = (C.n[0] + tx - 1) / tx;
  C.tiles[1] = dim >= 2 ? (C.n[1] + ty - 1) / ty : 1;
  C.tiles[2] = dim >= 3 ? (C.n[2] + zc - 1) / zc : 1;
  C.tile0 = 0;
  C.xslab = C.tiles[0];   // one slab: the table this path builds runs x fastest over the whole case
  const long long ntiles = (long long)C.tiles[0] * C.tiles[1] * C.tiles[2];
  const long long total = (C.ncell + 63) / 64 * 64;
  const size_t rows = (kind == FVM_KIND_THREE || kind == FVM_KIND_BARO2) ? 11 : 9;
  const size_t oD = align256(sizeof(CaseC));
  const size_t oT = oD + align256(sizeof(CaseDyn));
  const size_t oQ = oT + align256(sizeof(int4) * (size_t)ntiles);
  const size_t oP = oQ + align256(sizeof(double) * (size_t)nq * (size_t)total);
  const size_t end = oP + (dim == 3 ? sizeof(double) * rows * (size_t)total : 0);
  if (end > (size_t)FVM_NOALLOC_SCRATCH_BYTES || ntiles > 0x7fffffffLL) {
    char msg[200];
    std::snprintf(msg, sizeof msg, "case needs %zu bytes of workspace; the allocation-free right-hand side has %zu",
                  end, (size_t)FVM_NOALLOC_SCRATCH_BYTES);
    return bail(fail(&eb, FVM_EINVAL, msg));
  }
  void* base = nullptr;
  if ((rc = noalloc_base(&base, eb.err))) return bail(rc);
  char* p = static_cast<char*>(base);
  CaseC* dc = reinterpret_cast<CaseC*>(p);
  CaseDyn* dd = reinterpret_cast<CaseDyn*>(p + oD);
  int4* dt = reinterpret_cast<int4*>(p + oT);
  double* q = reinterpret_cast<double*>(p + oQ);
  double* prim = dim == 3 ? reinterpret_cast<double*>(p + oP) : nullptr;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_noalloc_setup, dim3(256), dim3(256), 0, st, C, dc, dd, dt, (int)ntiles, C.tiles[0], C.tiles[1],
                     prim, dim == 3 ? (long long)rows * total : 0LL);
  hipError_t he = hipGetLastError();
  if (he == hipSuccess) he = fvm_k_cons_to_state(dim, 0, kind, dc, 0, C.ncell, q_dev_in, q, total, st);
  if (he != hipSuccess) return bail(fail(&eb, FVM_EHIP, std::string("launch: ") + hipGetErrorString(he)));
  StageArgs a;
  std::memset(&a, 0, sizeof a);
  double rk[4];
  fill_scheme(a.sc, rk, s, dim);
  a.cases = dc;
  a.dyn = dd;
  a.tiles = dt;
  a.total = total;
  a.prim = prim;
  a.src = q;
  a.qn = q;
  a.dst = nullptr;
  a.stage = -1;
  a.rhs_out = r_dev_out;
  a.rhs_step = step;
  he = fvm_k_stage(dim, 0, kind, tile, a, (int)ntiles, st);
  if (he != hipSuccess) return bail(fail(&eb, FVM_EHIP, std::string("stage launch: ") + hipGetErrorString(he)));
  return FVM_OK;
}
