// C ABI of the hfv library: argument validation, ownership, dispatch.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "hfv_internal.hpp"

namespace hfv {
hfv_status refresh_thresholds(hfv_ctx *ctx, hipStream_t s);
}

using namespace hfv;

static thread_local std::string g_create_err;

// Scratch of hfv_residual_noalloc: a fixed array in the library's code
// object, one copy per device, held until the process ends.  Host code never
// uses its name as an address: the device address of each device's copy is
// looked up once, with that device current, and kept in g_scratch_addr.
static __device__ __align__(256) unsigned char scratch[HFV_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// Device address of `device`'s scratch array (the current device at create).
hfv_status scratch_address(int device, void **out, std::string &err) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return err = "device ordinal out of range", HFV_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return HFV_ERR_HIP;
    }
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return HFV_OK;
}

constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of scratch hfv_residual_noalloc carves for a context: own classes
// [N], class lists [3][N], list lengths [8], face fluxes [nvar][NF].
size_t noalloc_bytes(const hfv_ctx *ctx) {
  const size_t ts = ctx->prec == 64 ? 8 : 4, N = (size_t)ctx->N;
  return align256(N) + align256(sizeof(int) * 3 * N) + align256(sizeof(int) * 8) +
         align256(ts * ctx->nvar * (size_t)ctx->NF);
}
}  // namespace

static const int kTypeDim[6] = {2, 2, 3, 3, 3, 3};
static const int kTypeNv[6] = {3, 4, 4, 5, 6, 8};
static const int kTypeNf[6] = {3, 4, 4, 5, 5, 6};

static hfv_status check_params(const hfv_params *p, std::string &err) {
  if (!(p->gamma > 1.0)) return err = "gamma must exceed 1", HFV_ERR_PARAM;
  if (!(p->lambda1_prime > 1.0)) return err = "lambda1_prime must exceed 1", HFV_ERR_PARAM;
  if (!(p->alpha_m >= 0.0) || !(p->beta_m >= 0.0) || !(p->alpha_w >= 0.0))
    return err = "NAD margins alpha_m, beta_m, alpha_w must be non-negative", HFV_ERR_PARAM;
  if (!std::isfinite(p->beta_w)) return err = "beta_w must be finite", HFV_ERR_PARAM;
  if (!(p->kappa >= 0.0) || !(p->n_exp > 0.0)) return err = "deactivation needs kappa >= 0, n > 0", HFV_ERR_PARAM;
  if (!(p->eps_w > 0.0) || !(p->b_w > 0.0)) return err = "CWENOZ eps and b must be positive", HFV_ERR_PARAM;
  if (!(p->tvd_theta > 0.0) || !(p->tvd_eps > 0.0)) return err = "Harten theta and eps must be positive", HFV_ERR_PARAM;
  if (p->scheme_mode < 0 || p->scheme_mode > 3) return err = "unknown scheme_mode", HFV_ERR_PARAM;
  if (p->riemann < 0 || p->riemann > 1) return err = "unknown riemann solver", HFV_ERR_PARAM;
  if (p->cweno_form < 0 || p->cweno_form > 1) return err = "unknown cweno_form", HFV_ERR_PARAM;
  if (p->limiter != HFV_LIM_BJ && p->limiter != HFV_LIM_VENKAT) return err = "unknown limiter", HFV_ERR_PARAM;
  if (p->cweno_vars != HFV_CONSERVED && p->cweno_vars != HFV_CHARACTERISTIC)
    return err = "unknown cweno_vars", HFV_ERR_PARAM;
  if (p->viscous != 0 && p->viscous != 1) return err = "viscous must be 0 or 1", HFV_ERR_PARAM;
  if (p->viscous && (!(p->mu0 >= 0.0) || !(p->T0 > 0.0) || !(p->sutherland_S >= 0.0) || !(p->prandtl > 0.0) ||
                     !(p->visc_alpha >= 0.0) || !std::isfinite(p->mu0) || !std::isfinite(p->visc_alpha)))
    return err = "viscous fluxes need mu0 >= 0, T0 > 0, sutherland_S >= 0, prandtl > 0, visc_alpha >= 0",
           HFV_ERR_PARAM;
  return HFV_OK;
}

static void copy_params(hfv_ctx *ctx, const hfv_params *p) {
  ctx->p.order_r = p->order_r;
  ctx->p.mode = p->scheme_mode;
  ctx->p.riemann = p->riemann;
  ctx->p.form = p->cweno_form;
  ctx->p.limiter = p->limiter;
  ctx->p.cvars = p->cweno_vars;
  ctx->p.viscous = p->viscous;
  ctx->p.mu0 = p->mu0;
  ctx->p.T0 = p->T0;
  ctx->p.suth_S = p->sutherland_S;
  ctx->p.prandtl = p->prandtl;
  ctx->p.visc_alpha = p->visc_alpha;
  ctx->p.gamma = p->gamma;
  ctx->p.alpha_m = p->alpha_m;
  ctx->p.beta_m = p->beta_m;
  ctx->p.alpha_w = p->alpha_w;
  ctx->p.beta_w = p->beta_w;
  ctx->p.kappa = p->kappa;
  ctx->p.n_exp = p->n_exp;
  ctx->p.lam1p = p->lambda1_prime;
  ctx->p.eps_w = p->eps_w;
  ctx->p.b_w = p->b_w;
  ctx->p.theta = p->tvd_theta;
  ctx->p.tvd_eps = p->tvd_eps;
}

static hfv_status validate(const hfv_mesh *m, const hfv_stencils *st, const hfv_params *p, std::string &err) {
  if (!m || !st || !p) return err = "NULL mesh, stencils or params", HFV_ERR_PARAM;
  hfv_status e = check_params(p, err);
  if (e != HFV_OK) return e;
  const int d = m->dim;
  if (d != 2 && d != 3) return err = "dim must be 2 or 3", HFV_ERR_PARAM;
  if (p->order_r < 1 || p->order_r > (d == 2 ? 6 : 4))
    return err = d == 2 ? "order_r must be in 1..6 in 2D" : "order_r must be in 1..4 in 3D", HFV_ERR_PARAM;
  if (p->precision != 64 && p->precision != 32) return err = "precision must be 64 or 32", HFV_ERR_DTYPE;
  if (m->n_cells <= 0 || m->n_faces <= 0 || m->n_vertices <= 0) return err = "empty mesh", HFV_ERR_MESH;
  if (!m->vertices || !m->cell_type || !m->cell_vtx_off || !m->cell_vtx || !m->face_cells || !m->face_vtx_off ||
      !m->face_vtx)
    return err = "NULL mesh array", HFV_ERR_MESH;
  if (m->face_shift && !m->period) return err = "face_shift given without period", HFV_ERR_MESH;
  const int N = m->n_cells, NF = m->n_faces, NFM = nf_max(d), K = n_unknowns(d, p->order_r);
  if ((long)N * 2 * K * 8 > (1L << 46)) return err = "mesh too large", HFV_ERR_MESH;
  if (m->cell_vtx_off[0] != 0) return err = "cell_vtx_off[0] must be 0", HFV_ERR_MESH;
  for (int c = 0; c < N; ++c) {
    int t = m->cell_type[c];
    if (t < 0 || t > 5 || kTypeDim[t] != d) return err = "bad cell type at cell " + std::to_string(c), HFV_ERR_MESH;
    if (m->cell_vtx_off[c + 1] - m->cell_vtx_off[c] != kTypeNv[t])
      return err = "vertex count does not match type at cell " + std::to_string(c), HFV_ERR_MESH;
  }
  for (long i = 0; i < m->cell_vtx_off[N]; ++i)
    if (m->cell_vtx[i] < 0 || m->cell_vtx[i] >= m->n_vertices) return err = "cell vertex out of range", HFV_ERR_MESH;
  std::vector<int> nfc(N, 0);
  if (m->face_vtx_off[0] != 0) return err = "face_vtx_off[0] must be 0", HFV_ERR_MESH;
  for (int f = 0; f < NF; ++f) {
    int l = m->face_cells[2 * f], r = m->face_cells[2 * f + 1];
    if (l < 0 || l >= N || r < -1 || r >= N) return err = "face_cells out of range at face " + std::to_string(f), HFV_ERR_MESH;
    nfc[l]++;
    if (r >= 0) nfc[r]++;
    int nv = m->face_vtx_off[f + 1] - m->face_vtx_off[f];
    if ((d == 2 && nv != 2) || (d == 3 && nv != 3 && nv != 4))
      return err = "bad face vertex count at face " + std::to_string(f), HFV_ERR_MESH;
    for (int k = m->face_vtx_off[f]; k < m->face_vtx_off[f + 1]; ++k)
      if (m->face_vtx[k] < 0 || m->face_vtx[k] >= m->n_vertices) return err = "face vertex out of range", HFV_ERR_MESH;
  }
  for (int c = 0; c < N; ++c)
    if (nfc[c] != kTypeNf[(int)m->cell_type[c]])
      return err = "cell " + std::to_string(c) + " has " + std::to_string(nfc[c]) + " faces", HFV_ERR_MESH;
  if (st->M != 2 * K) return err = "central stencil size must be 2K = " + std::to_string(2 * K), HFV_ERR_MESH;
  if (st->nf_max != NFM || st->Md != 2 * d) return err = "stencil strides do not match dim", HFV_ERR_MESH;
  if (!st->central || !st->dir || !st->n_dir || !st->muscl || !st->n_muscl) return err = "NULL stencil array", HFV_ERR_MESH;
  if ((st->central_shift || st->dir_shift || st->muscl_shift) && !m->period)
    return err = "stencil shifts given without period", HFV_ERR_MESH;
  for (long i = 0; i < (long)N * st->M; ++i)
    if (st->central[i] < 0 || st->central[i] >= N) return err = "central stencil entry out of range", HFV_ERR_MESH;
  for (int c = 0; c < N; ++c) {
    if (st->n_dir[c] < 1 || st->n_dir[c] > NFM) return err = "n_dir out of range at cell " + std::to_string(c), HFV_ERR_MESH;
    if (st->n_muscl[c] < d || st->n_muscl[c] > NFM) return err = "n_muscl out of range at cell " + std::to_string(c), HFV_ERR_MESH;
    for (int s = 0; s < st->n_dir[c]; ++s)
      for (int q = 0; q < st->Md; ++q) {
        int v = st->dir[((long)c * NFM + s) * st->Md + q];
        if (v < 0 || v >= N) return err = "directional stencil entry out of range at cell " + std::to_string(c), HFV_ERR_MESH;
      }
    for (int q = 0; q < st->n_muscl[c]; ++q) {
      int v = st->muscl[(long)c * NFM + q];
      if (v < 0 || v >= N) return err = "MUSCL stencil entry out of range at cell " + std::to_string(c), HFV_ERR_MESH;
    }
  }
  return HFV_OK;
}

extern "C" {

// The viscous fluxes' gradient buffer of FP64 contexts ([N][NGPC][dim][nvar]):
// allocated once, at create or when hfv_set_params first turns the viscous
// fluxes on (FP32 contexts evaluate the gradients in the face kernel).
static hfv_status viscous_buffer(hfv_ctx *ctx) {
  if (ctx->vgrad || ctx->prec != 64) return HFV_OK;
  const size_t ts = ctx->prec == 64 ? 8 : 4;
  return dev_alloc(ctx, &ctx->vgrad, ts * (size_t)ctx->NGPC * ctx->dim * ctx->nvar * ctx->N);
}

hfv_status hfv_create(const hfv_mesh *mesh, const hfv_stencils *st, const hfv_params *p, void *stream,
                      hfv_ctx **out) {
  if (!out) return HFV_ERR_PARAM;
  *out = nullptr;
  g_create_err.clear();
  hfv_status e = validate(mesh, st, p, g_create_err);
  if (e != HFV_OK) return e;
  hfv_ctx *ctx = new (std::nothrow) hfv_ctx();
  if (!ctx) return g_create_err = "host allocation failed", HFV_ERR_OOM;
  const int d = mesh->dim;
  ctx->dim = d;
  ctx->r = p->order_r;
  ctx->prec = p->precision;
  ctx->N = mesh->n_cells;
  ctx->NF = mesh->n_faces;
  ctx->K = n_unknowns(d, p->order_r);
  ctx->M = 2 * ctx->K;
  ctx->Md = 2 * d;
  ctx->NFM = nf_max(d);
  ctx->nvar = d + 2;
  ctx->lanes = d + 2;
  ctx->lin_lanes = d + 2;
  copy_params(ctx, p);
  hipStream_t s = (hipStream_t)stream;
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    g_create_err = "no HIP device";
    delete ctx;
    return HFV_ERR_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) ctx->n_cu = prop.multiProcessorCount;
  ctx->list_blocks = 8 * ctx->n_cu;
  e = scratch_address(ctx->device, &ctx->noalloc_scratch, ctx->err);
  if (e == HFV_OK) e = setup_tables(ctx, mesh, st, s);
  if (e == HFV_OK) {
    const size_t ts = ctx->prec == 64 ? 8 : 4;
    const int N = ctx->N;
    if ((e = dev_alloc(ctx, (void **)&ctx->own, N)) == HFV_OK &&
        (e = dev_alloc(ctx, (void **)&ctx->cls_ws, N)) == HFV_OK &&
        (e = dev_alloc(ctx, (void **)&ctx->lists, sizeof(int) * 3 * (size_t)N)) == HFV_OK &&
        (e = dev_alloc(ctx, (void **)&ctx->counts, sizeof(int) * 8)) == HFV_OK &&
        (e = dev_alloc(ctx, &ctx->coef, ts * ctx->K * ctx->nvar * (size_t)N)) == HFV_OK &&
        (e = dev_alloc(ctx, &ctx->fs_ws, ts * ctx->nvar * (size_t)ctx->NGPC * ctx->N)) == HFV_OK &&
        (e = dev_alloc(ctx, &ctx->fflux, ts * ctx->nvar * (size_t)ctx->NF)) == HFV_OK &&
        (e = dev_alloc(ctx, (void **)&ctx->red, sizeof(double) * RED_BLOCKS)) == HFV_OK &&
        (!ctx->p.viscous || (e = viscous_buffer(ctx)) == HFV_OK)) {
      if (hipMemsetAsync(ctx->counts, 0, sizeof(int) * 8, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        ctx->err = "workspace initialisation failed";
        e = HFV_ERR_HIP;
      }
    }
  }
  if (e != HFV_OK) {
    g_create_err = ctx->err;
    hfv_destroy(ctx);
    return e;
  }
  *out = ctx;
  return HFV_OK;
}

hfv_status hfv_set_params(hfv_ctx *ctx, const hfv_params *p) {
  if (!ctx || !p) return HFV_ERR_PARAM;
  if (p->order_r != ctx->r || p->precision != ctx->prec) {
    ctx->err = "order_r and precision are fixed at create";
    return HFV_ERR_PARAM;
  }
  hfv_status e = check_params(p, ctx->err);
  if (e != HFV_OK) return e;
  const bool thr = p->kappa != ctx->p.kappa || p->n_exp != ctx->p.n_exp;
  if (p->viscous && (e = viscous_buffer(ctx)) != HFV_OK) return e;   // before anything changes
  copy_params(ctx, p);
  if (thr) {
    e = refresh_thresholds(ctx, nullptr);
    if (e != HFV_OK) return e;
    if (hipDeviceSynchronize() != hipSuccess) return ctx->err = "threshold refresh failed", HFV_ERR_HIP;
  }
  return HFV_OK;
}

hfv_status hfv_set_launch(hfv_ctx *ctx, const hfv_launch *c) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!c) return ctx->err = "NULL launch configuration", HFV_ERR_PARAM;
  const int lanes = c->lanes_per_cell;
  if (!(lanes == 1 || lanes == ctx->nvar || (ctx->dim == 2 && lanes == 2)))
    return ctx->err = "lanes_per_cell must be 1 or nvar (or 2 in 2D)", HFV_ERR_PARAM;
  if (c->block % 64 != 0 || c->block < 64 || c->block > 256)
    return ctx->err = "block must be 64, 128, 192 or 256", HFV_ERR_PARAM;
  if (c->list_blocks < 0) return ctx->err = "list_blocks must be >= 0", HFV_ERR_PARAM;
  if (c->linear_split < 0 || c->linear_split > 2) return ctx->err = "linear_split must be 0, 1 or 2", HFV_ERR_PARAM;
  const int ll = c->linear_lanes;
  if (c->linear_split == 0 && !(ll == 1 || ll == ctx->nvar || (ctx->dim == 2 && ll == 2)))
    return ctx->err = "linear_lanes must be 1 or nvar (or 2 in 2D) with the variable split", HFV_ERR_PARAM;
  if (c->linear_split != 0 && ll != 2 && ll != 4 && ll != 8)
    return ctx->err = "linear_lanes must be 2, 4 or 8 with the member or unknown split", HFV_ERR_PARAM;
  if (c->cwenoz_reuse != 0 && c->cwenoz_reuse != 1) return ctx->err = "cwenoz_reuse must be 0 or 1", HFV_ERR_PARAM;
  if (c->fused_residual != 0 && c->fused_residual != 1)
    return ctx->err = "fused_residual must be 0 or 1", HFV_ERR_PARAM;
  if (c->xcd_remap != 0 && c->xcd_remap != 1) return ctx->err = "xcd_remap must be 0 or 1", HFV_ERR_PARAM;
  const int ml = c->muscl_lanes;
  if (!(ml == 0 || ml == 1 || ml == ctx->nvar || (ctx->dim == 2 && ml == 2)))
    return ctx->err = "muscl_lanes must be 0, 1 or nvar (or 2 in 2D)", HFV_ERR_PARAM;
  if (c->merged_lists != 0 && c->merged_lists != 1) return ctx->err = "merged_lists must be 0 or 1", HFV_ERR_PARAM;
  if (c->lists_cell_major != 0 && c->lists_cell_major != 1)
    return ctx->err = "lists_cell_major must be 0 or 1", HFV_ERR_PARAM;
  ctx->lanes = lanes;
  ctx->block = c->block;
  ctx->list_blocks = c->list_blocks;
  ctx->lin_split = c->linear_split;
  ctx->lin_lanes = c->linear_lanes;
  ctx->cw_reuse = c->cwenoz_reuse;
  ctx->fused_residual = c->fused_residual;
  ctx->xcd_remap = c->xcd_remap;
  ctx->muscl_lanes = c->muscl_lanes;
  ctx->merged_lists = c->merged_lists;
  ctx->lists_cm = c->lists_cell_major;
  return HFV_OK;
}

hfv_status hfv_get_launch(const hfv_ctx *ctx, hfv_launch *c) {
  if (!ctx || !c) return HFV_ERR_PARAM;
  c->lanes_per_cell = ctx->lanes;
  c->block = ctx->block;
  c->list_blocks = ctx->list_blocks;
  c->linear_split = ctx->lin_split;
  c->linear_lanes = ctx->lin_lanes;
  c->cwenoz_reuse = ctx->cw_reuse;
  c->fused_residual = ctx->fused_residual;
  c->xcd_remap = ctx->xcd_remap;
  c->muscl_lanes = ctx->muscl_lanes;
  c->merged_lists = ctx->merged_lists;
  c->lists_cell_major = ctx->lists_cm;
  return HFV_OK;
}

hfv_status hfv_reconstruct(hfv_ctx *ctx, const void *U, void *fs, uint8_t *cls, void *near_margin, void *stream) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!U || !fs || !cls) return ctx->err = "NULL device pointer", HFV_ERR_PARAM;
  return run_reconstruct(ctx, U, fs, cls, (hipStream_t)stream, near_margin);
}

hfv_status hfv_residual(hfv_ctx *ctx, const void *U, void *R, void *fs, uint8_t *cls, void *stream) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!U || !R) return ctx->err = "NULL device pointer", HFV_ERR_PARAM;
  hipStream_t s = (hipStream_t)stream;
  void *f = fs ? fs : ctx->fs_ws;
  uint8_t *c = cls ? cls : ctx->cls_ws;
  hfv_status e = run_reconstruct(ctx, U, f, c, s);
  if (e != HFV_OK) return e;
  return run_residual_tail(ctx, f, R, s);
}

hfv_status hfv_residual_noalloc(hfv_ctx *ctx, const void *U, void *R, void *fs, uint8_t *cls, void *stream) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!U || !R || !fs || !cls) return ctx->err = "NULL device pointer", HFV_ERR_PARAM;
  const size_t need = noalloc_bytes(ctx);
  if (need > (size_t)HFV_NOALLOC_SCRATCH_BYTES) {
    ctx->err = "hfv_residual_noalloc needs " + std::to_string(need) + " bytes of scratch for this mesh, more than its " +
               std::to_string((size_t)HFV_NOALLOC_SCRATCH_BYTES) + "-byte maximum";
    return HFV_ERR_PARAM;
  }
  if (!ctx->noalloc_scratch) return ctx->err = "scratch array address unknown", HFV_ERR_STATE;
  if (ctx->p.viscous) return ctx->err = "hfv_residual_noalloc computes inviscid residuals only", HFV_ERR_STATE;
  // The same kernels as hfv_residual, with the workspace they write carved
  // from the scratch array; the context's own workspace is put back on every
  // return path.  The kernels clear the list lengths themselves (the first
  // block of the linear pass, or a fill kernel), so nothing needs zeroing here.
  struct Swap {
    hfv_ctx *c;
    uint8_t *own;
    int *lists, *counts;
    void *coef, *fflux;
    ~Swap() {
      c->own = own;
      c->lists = lists;
      c->counts = counts;
      c->coef = coef;
      c->fflux = fflux;
    }
  } keep{ctx, ctx->own, ctx->lists, ctx->counts, ctx->coef, ctx->fflux};
  unsigned char *b = (unsigned char *)ctx->noalloc_scratch;
  const size_t N = (size_t)ctx->N;
  ctx->own = b;
  b += align256(N);
  ctx->lists = (int *)b;
  b += align256(sizeof(int) * 3 * N);
  ctx->counts = (int *)b;
  b += align256(sizeof(int) * 8);
  ctx->fflux = b;
  ctx->coef = nullptr;  // CWENOZ refits its central polynomial (no kept fits)
  hipStream_t s = (hipStream_t)stream;
  hfv_status e = run_reconstruct(ctx, U, fs, cls, s);
  if (e != HFV_OK) return e;
  return run_residual_tail(ctx, fs, R, s);
}

hfv_status hfv_residual_frozen(hfv_ctx *ctx, const void *U, const uint8_t *cls, void *R, void *stream) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!U || !cls || !R) return ctx->err = "NULL device pointer", HFV_ERR_PARAM;
  hipStream_t s = (hipStream_t)stream;
  hfv_status e = run_reconstruct_frozen(ctx, U, ctx->fs_ws, cls, s);
  if (e != HFV_OK) return e;
  return run_residual_tail(ctx, ctx->fs_ws, R, s);
}

hfv_status hfv_residual_vjp(hfv_ctx *ctx, const void *U, const uint8_t *cls, const void *gR, void *gU,
                            void *stream) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!U || !cls || !gR || !gU) return ctx->err = "NULL device pointer", HFV_ERR_PARAM;
  return run_vjp(ctx, U, cls, nullptr, gR, gU, (hipStream_t)stream);
}

hfv_status hfv_residual_vjp_states(hfv_ctx *ctx, const void *U, const uint8_t *cls, const void *face_states,
                                   const void *gR, void *gU, void *stream) {
  if (!ctx) return HFV_ERR_PARAM;
  if (!U || !cls || !face_states || !gR || !gU) return ctx->err = "NULL device pointer", HFV_ERR_PARAM;
  return run_vjp(ctx, U, cls, face_states, gR, gU, (hipStream_t)stream);
}

hfv_status hfv_query(const hfv_ctx *ctx, int32_t what, int64_t *out) {
  if (!ctx || !out) return HFV_ERR_PARAM;
  switch (what) {
    case HFV_Q_N_CELLS: *out = ctx->N; return HFV_OK;
    case HFV_Q_N_FACES: *out = ctx->NF; return HFV_OK;
    case HFV_Q_N_GP: *out = ctx->NGPT; return HFV_OK;
    case HFV_Q_NVAR: *out = ctx->nvar; return HFV_OK;
    case HFV_Q_K: *out = ctx->K; return HFV_OK;
    case HFV_Q_M: *out = ctx->M; return HFV_OK;
    case HFV_Q_PRECISION: *out = ctx->prec; return HFV_OK;
    case HFV_Q_DIM: *out = ctx->dim; return HFV_OK;
    case HFV_Q_TABLE_BYTES: *out = (int64_t)ctx->table_bytes; return HFV_OK;
    case HFV_Q_NGP_CELL_MAX: *out = ctx->NGPC; return HFV_OK;
    case HFV_Q_NOALLOC_BYTES: *out = (int64_t)noalloc_bytes(ctx); return HFV_OK;
    case HFV_Q_COUNT_CWENOZ:
    case HFV_Q_COUNT_MUSCL:
    case HFV_Q_COUNT_FIRST: {
      int c[8];
      // the counters may be written by work on any of the caller's streams
      if (hipDeviceSynchronize() != hipSuccess) return HFV_ERR_HIP;
      if (hipMemcpy(c, ctx->counts, sizeof c, hipMemcpyDeviceToHost) != hipSuccess) return HFV_ERR_HIP;
      *out = c[1 + what - HFV_Q_COUNT_CWENOZ];
      return HFV_OK;
    }
  }
  return HFV_ERR_PARAM;
}

hfv_status hfv_copy_table(const hfv_ctx *ctx, int32_t which, void *dst, int64_t bytes) {
  if (!ctx || !dst) return HFV_ERR_PARAM;
  const size_t ts = ctx->prec == 64 ? 8 : 4;
  const size_t N = ctx->N;
  const void *src = nullptr;
  size_t n = 0;
  const bool d64 = ctx->prec == 64;
  switch (which) {
    case HFV_T_PINV: src = d64 ? (const void *)ctx->t64.P : ctx->t32.P; n = ts * ctx->K * ctx->M * N; break;
    case HFV_T_OI: src = d64 ? (const void *)ctx->t64.OI : ctx->t32.OI; n = ts * ctx->K * (ctx->K + 1) / 2 * N; break;
    case HFV_T_PSIBAR: src = d64 ? (const void *)ctx->t64.psibar : ctx->t32.psibar; n = ts * ctx->K * N; break;
    case HFV_T_GEOM: src = ctx->geom; n = 8 * (ctx->dim + 2) * N; break;
    case HFV_T_PDIR: src = d64 ? (const void *)ctx->t64.Pdir : ctx->t32.Pdir; n = ts * ctx->NFM * ctx->dim * ctx->Md * N; break;
    case HFV_T_PMUS: src = d64 ? (const void *)ctx->t64.Pmus : ctx->t32.Pmus; n = ts * ctx->dim * ctx->NFM * N; break;
    case HFV_T_FACE_SLOTS: src = d64 ? ctx->t64.fgb : ctx->t32.fgb; n = sizeof(int) * (size_t)ctx->NF; break;
    case HFV_T_GP_XI: src = d64 ? (const void *)ctx->t64.gpxi : ctx->t32.gpxi; n = ts * ctx->NGPC * ctx->dim * N; break;
    default: return HFV_ERR_PARAM;
  }
  if ((int64_t)n != bytes) return HFV_ERR_PARAM;
  if (hipMemcpy(dst, src, n, hipMemcpyDeviceToHost) != hipSuccess) return HFV_ERR_HIP;
  return HFV_OK;
}

hfv_status hfv_profile_enable(hfv_ctx *ctx, int32_t capacity, int32_t slot_mask) {
  if (!ctx || capacity < 0) return HFV_ERR_PARAM;
  for (auto &e : ctx->prof_pool) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  ctx->prof_pool.clear();
  ctx->prof_next = 0;
  ctx->prof_mask = capacity > 0 ? slot_mask : 0;
  for (int i = 0; i < capacity; ++i) {
    hfv_ctx::ProfEv e{0, nullptr, nullptr};
    // timing-only events: no system-scope fence, so recording one does not
    // write back and invalidate the caches in the middle of the step
    if (hipEventCreateWithFlags(&e.a, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&e.b, hipEventDisableSystemFence) != hipSuccess) {
      ctx->err = "hipEventCreate failed";
      return HFV_ERR_HIP;
    }
    ctx->prof_pool.push_back(e);
  }
  return HFV_OK;
}

hfv_status hfv_profile_read(hfv_ctx *ctx, double *ms_sum, int64_t *launches) {
  if (!ctx || !ms_sum || !launches) return HFV_ERR_PARAM;
  for (int i = 0; i < HFV_NSLOTS; ++i) {
    ms_sum[i] = 0;
    launches[i] = 0;
  }
  for (int i = 0; i < ctx->prof_next; ++i) {
    auto &e = ctx->prof_pool[i];
    if (hipEventSynchronize(e.b) != hipSuccess) return ctx->err = "hipEventSynchronize failed", HFV_ERR_HIP;
    float ms = 0;
    if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) return ctx->err = "hipEventElapsedTime failed", HFV_ERR_HIP;
    ms_sum[e.slot] += ms;
    launches[e.slot] += 1;
  }
  ctx->prof_next = 0;
  return HFV_OK;
}

const char *hfv_last_error(const hfv_ctx *ctx) { return ctx ? ctx->err.c_str() : g_create_err.c_str(); }

void hfv_destroy(hfv_ctx *ctx) {
  if (!ctx) return;
  for (auto &e : ctx->prof_pool) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (void *p : ctx->allocs) (void)hipFree(p);
  delete ctx;
}

}  // extern "C"
