// Internal declarations of the hfv library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hfv.h"

namespace hfv {

__host__ __device__ constexpr int binom(int n, int k) {
  int r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}
// Non-constant unknowns of a degree-r polynomial in d dimensions (Section 2.1).
__host__ __device__ constexpr int n_unknowns(int d, int r) { return binom(r + d, d) - 1; }
__host__ __device__ constexpr int nf_max(int d) { return d == 2 ? 4 : 6; }

// Exponents of the monomials of degree lo..hi, ordered by degree and then in
// descending lexicographic order (the hierarchical basis order).
template <int DIM, int LO, int HI>
struct Exps {
  static constexpr int count() { return binom(HI + DIM, DIM) - (LO > 0 ? binom(LO - 1 + DIM, DIM) : 0); }
  int e[count() > 0 ? count() : 1][DIM];
  constexpr Exps() : e{} {
    int k = 0;
    for (int deg = LO; deg <= HI; ++deg) {
      if (DIM == 2) {
        for (int a = deg; a >= 0; --a) {
          e[k][0] = a;
          e[k][DIM - 1] = deg - a;
          ++k;
        }
      } else {
        for (int a = deg; a >= 0; --a)
          for (int b = deg - a; b >= 0; --b) {
            e[k][0] = a;
            e[k][1 % DIM] = b;
            e[k][DIM - 1] = deg - a - b;
            ++k;
          }
      }
    }
  }
};

// Device tables of one context.  Per-cell arrays are [row][n_cells] so that
// consecutive cells are consecutive in memory.
template <typename T>
struct Tables {
  int *sten = nullptr;     // [M][N]
  T *P = nullptr;          // [K][M][N]   pseudo-inverse times |V_m'|
  T *psibar = nullptr;     // [K][N]
  T *gpxi = nullptr;       // [NGPC][DIM][N] Gauss points in the cell frame
  uint8_t *ngp = nullptr;  // [N]
  int *nbr = nullptr;      // [NFM][N]   face neighbours, -1 at boundaries
  uint8_t *nfc = nullptr;  // [N]
  T *thr = nullptr;        // [N]  NAD deactivation threshold (kappa h)^n
  T *veps2 = nullptr;      // [N]  Venkatakrishnan limiter eps^2 = (kappa h)^3
  T *OI = nullptr;         // [K(K+1)/2][N]
  T *OIc = nullptr;        // [N][K(K+1)/2]  cell-major copy (CWENOZ over sparse lists)
  int *dsten = nullptr;    // [NFM][Md][N]
  T *Pdir = nullptr;       // [NFM][DIM][Md][N]
  // cell-major copies for the class-list kernels over sparse lists
  int *dstenC = nullptr;   // [N][NFM][Md]
  T *PdirC = nullptr;      // [N][NFM][DIM][Md]
  T *psibarC = nullptr;    // [N][K]
  T *gpxiC = nullptr;      // [N][NGPC][DIM]
  int *mstenC = nullptr;   // [N][NFM]
  T *PmusC = nullptr;      // [N][DIM][NFM]
  int *nbrC = nullptr;     // [N][NFM]
  uint8_t *ndir = nullptr; // [N]
  int *msten = nullptr;    // [NFM][N]
  T *Pmus = nullptr;       // [DIM][NFM][N]
  uint8_t *nmus = nullptr; // [N]
  // faces
  T *fnormal = nullptr;    // [DIM][NF]
  int *gp_off = nullptr;   // [NF+1]
  T *gpw = nullptr;        // [NGPT] weight x surface Jacobian
  int *face_cells = nullptr; // [2][NF]
  int *fgb = nullptr;      // [NF] first local Gauss-point slot of the face in its owner (bits 0-7) and
                           //      neighbour (bits 8-15) cell; the owner's slot again at boundaries
  int *cf_off = nullptr;   // [N+1]
  int *cf = nullptr;       // [..] face | (side << 31)
  T *ivol = nullptr;       // [N]
  T *hinv = nullptr;       // [N]  1 / h_c (gradients in physical units)
  T *linv = nullptr;       // [NF] 1 / (distance between the face's two cell centres); 0 at boundaries
  // adjoint: positions inside the central stencil and its transpose
  uint8_t *dpos = nullptr;  // [NFM][Md][N] directional member -> central slot
  uint8_t *mpos = nullptr;  // [NFM][N]     MUSCL member -> central slot
  uint8_t *nbpos = nullptr; // [NFM][N]     face neighbour -> central slot (255: none)
  int *inv_off = nullptr;   // [N+1]  cells whose central stencil holds cell j
  int *inv_idx = nullptr;   // [N*M]  m * N + i, ordered by (i, m)
};

struct Params {
  int order_r, mode, riemann, form, limiter, cvars, viscous;
  double gamma, alpha_m, beta_m, alpha_w, beta_w, kappa, n_exp, lam1p, eps_w, b_w, theta, tvd_eps;
  double mu0, T0, suth_S, prandtl, visc_alpha;
};

}  // namespace hfv

constexpr int RED_BLOCKS = 1024;

struct hfv_ctx {
  int dim = 0, r = 0, prec = 64, N = 0, NF = 0, NGPT = 0, NGPC = 0, K = 0, M = 0, Md = 0, NFM = 0, nvar = 0;
  hfv::Params p{};
  hfv::Tables<double> t64;
  hfv::Tables<float> t32;
  // double geometry kept for queries: [DIM+2][N] centroid, volume, h
  double *geom = nullptr;
  // workspace
  uint8_t *own = nullptr;      // [N]
  uint8_t *cls_ws = nullptr;   // [N]
  int *lists = nullptr;        // [3][N] CWENOZ, MUSCL, first order
  int *counts = nullptr;       // [8] list lengths at 1 + list index
  void *coef = nullptr;        // [K][nvar][N] central fits kept by the linear pass for CWENOZ
  void *fs_ws = nullptr;       // [NGPC][nvar][N] Gauss-point states, cell-major
  void *fflux = nullptr;       // [nvar][NF]
  void *vgrad = nullptr;       // viscous: fit gradients at the Gauss-point slots [N][NGPC][dim][nvar]
  double *red = nullptr;       // [RED_BLOCKS] per-block partial results of reductions
  void *noalloc_scratch = nullptr;  // this device's static scratch array (hfv_residual_noalloc)
  void *vjp_C = nullptr;       // adjoint: per stencil slot contributions [M][N][nvar]
  void *vjp_S = nullptr;       // adjoint: self contributions [nvar][N]
  void *vjp_gfs = nullptr;     // adjoint: Gauss-point state cotangents [NGPC][nvar][N]
  bool vjp_ok = false;
  std::string vjp_why;
  size_t table_bytes = 0;
  // launch configuration
  int lanes = 1, block = 256, list_blocks = 2048;
  int lin_split = 0, lin_lanes = 4;  // linear kernel: 0 variables, 1 stencil members, 2 unknowns per lane
  int cw_reuse = 0;                  // CWENOZ starts from the linear pass's central fit
  int fused_residual = 0;            // one owner-computes residual kernel instead of flux + gather
  int xcd_remap = 1;                 // XCD-contiguous block order (block_id)
  int muscl_lanes = 0;               // lanes per cell of the MUSCL pass (0: lanes)
  int merged_lists = 0;              // MUSCL and first-order lists served by the CWENOZ launch
  int lists_cm = 0;                  // class-list kernels read the cell-major table copies
  int device = 0, n_cu = 256;
  // kernel timing (hfv_profile_*)
  struct ProfEv {
    int slot;
    hipEvent_t a, b;
  };
  std::vector<ProfEv> prof_pool;
  int prof_next = 0, prof_mask = 0;
  std::vector<void *> allocs;
  std::string err;
};

namespace hfv {

hfv_status setup_tables(hfv_ctx *ctx, const hfv_mesh *mesh, const hfv_stencils *st, hipStream_t s);
hfv_status run_reconstruct(hfv_ctx *ctx, const void *U, void *fs, uint8_t *cls, hipStream_t s,
                           void *margin = nullptr);
hfv_status run_reconstruct_frozen(hfv_ctx *ctx, const void *U, void *fs, const uint8_t *cls, hipStream_t s);
hfv_status run_class_lists(hfv_ctx *ctx, const uint8_t *cls, hipStream_t s);
hfv_status run_residual_tail(hfv_ctx *ctx, const void *fs, void *R, hipStream_t s);
hfv_status run_vjp(hfv_ctx *ctx, const void *U, const uint8_t *cls, const void *fs, const void *gR, void *gU,
                   hipStream_t s);
hfv_status dev_alloc(hfv_ctx *ctx, void **p, size_t bytes);
// viscous fluxes (hfv_visc.cpp): the central fit of every cell kept in
// ctx->coef (for the modes without a linear pass), and F_v subtracted from
// the integrated face fluxes
hfv_status run_keep_fits(hfv_ctx *ctx, const void *U, hipStream_t s);
hfv_status run_viscous_flux(hfv_ctx *ctx, const void *fs, void *Ff, hipStream_t s);

// Brackets one kernel launch with HIP events when its slot is being timed.
struct ProfScope {
  hfv_ctx *ctx;
  hipStream_t s;
  int idx = -1;
  ProfScope(hfv_ctx *c, int slot, hipStream_t st) : ctx(c), s(st) {
    if ((c->prof_mask >> slot) & 1 && c->prof_next < (int)c->prof_pool.size()) {
      idx = c->prof_next++;
      c->prof_pool[idx].slot = slot;
      (void)hipEventRecord(c->prof_pool[idx].a, s);
    }
  }
  ~ProfScope() {
    if (idx >= 0) (void)hipEventRecord(ctx->prof_pool[idx].b, s);
  }
};

}  // namespace hfv

#define HFV_HIP(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) {                                                           \
      ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                   \
      return HFV_ERR_HIP;                                                             \
    }                                                                                 \
  } while (0)
