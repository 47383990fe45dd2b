// kp_api.cpp -- host side of the C ABI declared in include/polrad.h:
// argument validation, device buffers owned by a context, kernel launches,
// timing with HIP events recorded on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/polrad.h"
#include "kp_internal.hpp"

using namespace kp;

// Device scratch of kp_run_static, the entry point that allocates nothing:
// its counters and small tables (first KP_STATIC_HEAD bytes) and its step-1
// tally (the next KP_STATIC_TALLY bytes).  Each device the library runs on
// holds its own copy until the process ends.  In host code `scratch` names
// a host-side stand-in: the device address of a device's copy comes from
// hipGetSymbolAddress (scratch_address below) and only that address is ever
// passed to a kernel or a copy.
namespace {
constexpr size_t KP_STATIC_HEAD = size_t(1) << 20;
constexpr size_t KP_STATIC_TALLY = size_t(256) << 20;
constexpr int KP_MAX_DEVICES = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[KP_STATIC_HEAD + KP_STATIC_TALLY];

namespace {
std::mutex g_scratch_mu;
bool g_scratch_done[KP_MAX_DEVICES] = {};
hipError_t g_scratch_err[KP_MAX_DEVICES] = {};
unsigned char* g_scratch_ptr[KP_MAX_DEVICES] = {};

// Device address of `scratch` on `device`, looked up once per device with
// that device current (called from kp_create).
hipError_t scratch_address(int device, unsigned char** out) {
  *out = nullptr;
  if (device < 0 || device >= KP_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? (unsigned char*)p : nullptr;
    g_scratch_done[device] = true;
  }
  *out = g_scratch_ptr[device];
  return g_scratch_err[device];
}
}  // namespace

struct kp_ctx {
  int device = 0;
  int cu_count = 0;
  std::string err;
  // grid
  bool have_grid = false;
  kp_grid grid{};
  uint64_t ncell = 0;
  float* d_rho = nullptr;   // active pointers (owned or borrowed)
  float* d_bhat = nullptr;  // [3][ncell] or null
  float* own_rho = nullptr;
  float* own_bhat = nullptr;
  // dust, source, views
  std::vector<kp_dust> dust;
  bool have_source = false;
  kp_source src{};
  std::vector<kp_view> views;
  std::vector<ViewDev> hviews;
  ViewDev* d_views = nullptr;
  size_t d_views_n = 0;
  std::vector<DustDev> hdust;
  DustDev* d_dust = nullptr;
  size_t d_dust_n = 0;
  // results
  double* d_tally = nullptr;
  size_t tally_n = 0;      // doubles allocated
  int tally_lambda = 0;    // wavelengths of the last step 1
  int tally_ts = 16;       // per-cell stride (doubles) of the last step 1
  int tally_nc = 9;        // components kept per cell
  bool have_tally = false;
  double* d_images = nullptr;
  size_t images_n = 0;
  bool have_images = false;
  size_t images_valid_n = 0;
  StatsDev* d_stats = nullptr;
  unsigned long long* d_counter = nullptr;
  unsigned long long* d_bad = nullptr;
  TraceDev* d_traces = nullptr;
  size_t traces_n = 0;
  size_t traces_valid = 0;
  kp_stats stats{};
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // this device's copy of the static scratch (kp_run_static), or null
  unsigned char* scratch = nullptr;
  hipError_t scratch_err = hipSuccess;
  // thermal emission of the dust (source kind 2): source function
  // [n_lambda][ncell], the per-wavelength luminosity tables built from it,
  // and each wavelength's total luminosity
  bool have_emission = false;
  int em_nl = 0;
  float* d_em_B = nullptr;
  double* d_em_cdf = nullptr;
  size_t em_cdf_n = 0;
  uint32_t* d_em_guide = nullptr;
  size_t em_guide_n = 0;
  double* d_em_partial = nullptr;
  size_t em_partial_n = 0;
  bool em_ready = false;  // tables match the current grid, dust and source function
  std::vector<double> em_L;
  // composite mesh (kp_set_mesh): the tree and per-leaf origins and levels on
  // the device; grid then holds the root-cell box
  bool have_mesh = false;
  kp_mesh mesh{};
  int32_t* d_child = nullptr;
  int32_t* d_leaf_of_node = nullptr;
  int32_t* d_leaf_org = nullptr;  // [leaves][4]
  int nfine[3] = {0, 0, 0};
  // tabulated scattering of every wavelength (kp_set_dust_tables): one
  // device array holding the normalised tables [n_lambda][n][6], the node
  // cosines [n] and the cumulative envelope masses [n_lambda][n]
  bool have_tables = false;
  int tab_nt = 0;
  double* d_tab = nullptr;
  size_t tab_n = 0;
  int32_t* d_tab_guide = nullptr;  // [8 (n - 1)] node interval of each cos Theta bin
  size_t tab_guide_n = 0;
  // the last step 1 tallied the per-view source [lambda][cell][view][4]
  // (tabulated grains) instead of coherency blocks
  bool tally_views = false;
  int tally_nv = 0;
  // peel-off images of the last step 1 run with peel_off
  double* d_peel = nullptr;
  size_t peel_n = 0;
  size_t peel_valid_n = 0;  // 0: the last step 1 formed none
};

namespace {

kp_status fail(kp_ctx* c, kp_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
kp_status fail(kp_ctx* c, kp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

kp_status hip_fail(kp_ctx* c, hipError_t e, const char* what) {
  return fail(c, e == hipErrorOutOfMemory ? KP_ERR_OOM : KP_ERR_DEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

#define KP_HIP(call, what)                        \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
  } while (0)

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

bool is_sphere(const kp_dust& d) {
  return d.a_perp[0] == d.a_par[0] && d.a_perp[1] == d.a_par[1];
}

template <typename T>
kp_status ensure(kp_ctx* ctx, T** p, size_t* have, size_t need, const char* what) {
  if (*have >= need && *p) return KP_OK;
  if (*p) { (void)hipFree(*p); *p = nullptr; *have = 0; }
  if (need == 0) return KP_OK;
  hipError_t e = hipMalloc((void**)p, need * sizeof(T));
  if (e != hipSuccess) { *p = nullptr; return hip_fail(ctx, e, what); }
  *have = need;
  return KP_OK;
}

void release_grid(kp_ctx* ctx) {
  for (int32_t** q : {&ctx->d_child, &ctx->d_leaf_of_node, &ctx->d_leaf_org}) {
    if (*q) (void)hipFree(*q);
    *q = nullptr;
  }
  ctx->have_mesh = false;
  if (ctx->own_rho) (void)hipFree(ctx->own_rho);
  if (ctx->own_bhat) (void)hipFree(ctx->own_bhat);
  ctx->own_rho = ctx->own_bhat = nullptr;
  ctx->d_rho = ctx->d_bhat = nullptr;
  ctx->have_grid = false;
  ctx->have_tally = false;
  ctx->have_images = false;
  // a source function belongs to the grid it was given for
  if (ctx->d_em_B) (void)hipFree(ctx->d_em_B);
  ctx->d_em_B = nullptr;
  ctx->have_emission = false;
  ctx->em_ready = false;
}

kp_status check_grid(kp_ctx* ctx, const kp_grid* g) {
  if (!g) return fail(ctx, KP_ERR_ARG, "grid is NULL");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(ctx, KP_ERR_ARG, "grid dimensions must be >= 1");
  if (!(g->dx > 0.0) || !std::isfinite(g->dx)) return fail(ctx, KP_ERR_ARG, "dx must be finite and > 0");
  if (!std::isfinite(g->x0) || !std::isfinite(g->y0) || !std::isfinite(g->z0))
    return fail(ctx, KP_ERR_ARG, "grid origin must be finite");
  if (g->boundary < 0 || g->boundary > 6)
    return fail(ctx, KP_ERR_ARG, "boundary must be a mask of periodic axes in 0..6 (7 leaves no open face)");
  const double n = (double)g->nx * g->ny * g->nz;
  if (n > 4.0e9) return fail(ctx, KP_ERR_ARG, "grid has more than 4e9 cells");
  return KP_OK;
}

void fill_view(const kp_view& v, ViewDev& o) {
  o.ox = std::sin(v.theta) * std::cos(v.phi);
  o.oy = std::sin(v.theta) * std::sin(v.phi);
  o.oz = std::cos(v.theta);
  const double r2 = o.ox * o.ox + o.oy * o.oy, st = std::sqrt(r2);
  double cp = 1.0, sp = 0.0;
  if (r2 > 8.673617379884035e-19) { cp = o.ox / st; sp = o.oy / st; }
  o.tx = o.oz * cp; o.ty = o.oz * sp; o.tz = -st;
  o.px = -sp; o.py = cp; o.pz = 0.0;
  o.half_width = v.half_width;
}

// per-wavelength constants in cell units
void fill_dust(const kp_ctx* ctx, const uint64_t* counts, std::vector<DustDev>& out) {
  const double dx = ctx->grid.dx;
  const double lum = ctx->src.lum;
  out.resize(ctx->dust.size());
  uint64_t first = 0;
  for (size_t l = 0; l < ctx->dust.size(); ++l) {
    const kp_dust& d = ctx->dust[l];
    DustDev& o = out[l];
    std::memset(&o, 0, sizeof o);
    o.ks_cell = d.kappa_sca * dx;
    o.ka_cell = d.kappa_abs * dx;
    o.ke_cell = (d.kappa_sca + d.kappa_abs) * dx;
    o.kext = d.kappa_sca + d.kappa_abs;
    o.sphere = (is_sphere(d) || ctx->have_tables) ? 1 : 0;
    if (ctx->have_tables) {
      const size_t nl = ctx->dust.size(), nt = (size_t)ctx->tab_nt;
      o.tab_n = ctx->tab_nt;
      o.tab = ctx->d_tab + l * nt * 6;
      o.tab_mu = ctx->d_tab + nl * nt * 6;
      o.tab_cum = ctx->d_tab + nl * nt * 6 + nt + l * nt;
      o.tab_guide = ctx->d_tab_guide;
      o.tab_g = 8 * (ctx->tab_nt - 1);
    }
    if (o.sphere) {
      o.ap_re = o.aa_re = 1.0;
      o.ap_im = o.aa_im = 0.0;
    } else {
      o.ap_re = d.a_perp[0]; o.ap_im = d.a_perp[1];
      o.aa_re = d.a_par[0]; o.aa_im = d.a_par[1];
    }
    const double cavg = (2.0 * o.ap_im + o.aa_im) / 3.0;
    o.inv2cavg = o.sphere ? 0.0 : 1.0 / (2.0 * cavg);
    o.alpha3_scale = d.alpha3_scale;
    const double ap2 = o.ap_re * o.ap_re + o.ap_im * o.ap_im;
    const double aa2 = o.aa_re * o.aa_re + o.aa_im * o.aa_im;
    const double np = (2.0 * ap2 + aa2) / 3.0;
    o.pfac = 3.0 / (8.0 * M_PI * np);
    o.bound_fac = o.pfac * (ap2 > aa2 ? ap2 : aa2);
    o.ap2_np = ap2 / np;
    o.aa2_np = aa2 / np;
    o.count = counts ? counts[l] : 0;
    o.first = first;
    const double L = ctx->src.kind == 2 ? (l < ctx->em_L.size() ? ctx->em_L[l] : 0.0) : lum;
    o.w0 = o.count ? L / (double)o.count : 0.0;
    first += o.count;
  }
}

kp_status upload_small(kp_ctx* ctx, hipStream_t s) {
  kp_status st = ensure(ctx, &ctx->d_dust, &ctx->d_dust_n, ctx->hdust.size(), "dust table");
  if (st) return st;
  st = ensure(ctx, &ctx->d_views, &ctx->d_views_n, ctx->hviews.size(), "view table");
  if (st) return st;
  KP_HIP(hipMemcpyAsync(ctx->d_dust, ctx->hdust.data(), ctx->hdust.size() * sizeof(DustDev),
                        hipMemcpyHostToDevice, s), "dust upload");
  KP_HIP(hipMemcpyAsync(ctx->d_views, ctx->hviews.data(), ctx->hviews.size() * sizeof(ViewDev),
                        hipMemcpyHostToDevice, s), "view upload");
  return KP_OK;
}

MeshDev mesh_dev(const kp_ctx* ctx) {
  MeshDev m{};
  if (!ctx->have_mesh) return m;
  m.child = ctx->d_child;
  m.leaf_of_node = ctx->d_leaf_of_node;
  m.leaf_org = ctx->d_leaf_org;
  m.rx = ctx->mesh.rx; m.ry = ctx->mesh.ry; m.rz = ctx->mesh.rz;
  m.block = ctx->mesh.block;
  m.max_level = ctx->mesh.max_level;
  for (int k = 0; k < 3; ++k) m.nfine[k] = ctx->nfine[k];
  m.fine = std::ldexp(ctx->mesh.dx, -ctx->mesh.max_level);
  return m;
}

kp_status check_ready(kp_ctx* ctx) {
  if (!ctx->have_grid) return fail(ctx, KP_ERR_STATE, "kp_set_grid has not been called");
  if (ctx->dust.empty()) return fail(ctx, KP_ERR_STATE, "kp_set_dust has not been called");
  if (!ctx->have_source) return fail(ctx, KP_ERR_STATE, "kp_set_source has not been called");
  if (ctx->views.empty()) return fail(ctx, KP_ERR_STATE, "kp_set_views has not been called");
  if (ctx->grid.boundary) {
    // with periodic axes a camera ray ends only at an open face: its path
    // through the open extent is at most n_a / |om_a| cell lengths for every
    // open axis a
    const int n[3] = {ctx->grid.nx, ctx->grid.ny, ctx->grid.nz};
    for (size_t v = 0; v < ctx->hviews.size(); ++v) {
      const double om[3] = {ctx->hviews[v].ox, ctx->hviews[v].oy, ctx->hviews[v].oz};
      double cells = INFINITY;
      for (int k = 0; k < 3; ++k)
        if (!((ctx->grid.boundary >> k) & 1) && om[k] != 0.0) cells = std::fmin(cells, n[k] / std::fabs(om[k]));
      if (!(cells <= (double)KP_MAX_STEPS))
        return fail(ctx, KP_ERR_ARG, "view %zu: its rays cross more than 2^24 cell lengths of the periodic "
                    "grid before reaching an open face", v);
    }
  }
  if (ctx->src.kind == 2) {
    if (!ctx->have_emission)
      return fail(ctx, KP_ERR_STATE, "thermal emission source: kp_set_emission has not been called for this grid");
    if (ctx->em_nl != (int)ctx->dust.size())
      return fail(ctx, KP_ERR_ARG, "kp_set_emission gave %d wavelengths, kp_set_dust %zu", ctx->em_nl,
                  ctx->dust.size());
    return KP_OK;
  }
  const kp_grid& g = ctx->grid;
  const double lo[3] = {g.x0, g.y0, g.z0};
  const int n[3] = {g.nx, g.ny, g.nz};
  for (int k = 0; k < 3; ++k)
    if (!(ctx->src.pos[k] >= lo[k] && ctx->src.pos[k] <= lo[k] + n[k] * g.dx))
      return fail(ctx, KP_ERR_ARG, "source position lies outside the grid box");
  return KP_OK;
}

// Tally layout of the loaded grid: slots per wavelength and bricks along x
// and y (tally_slot); a composite mesh keeps its cell order.
struct TallyLayout {
  uint64_t nslot;
  int tbx, tby;
};
TallyLayout tally_layout(const kp_ctx* ctx) {
  if (ctx->have_mesh) return TallyLayout{ctx->ncell, 0, 0};
  const kp_grid& g = ctx->grid;
  return TallyLayout{tally_slots(g.nx, g.ny, g.nz), (g.nx + 3) / 4, (g.ny + 3) / 4};
}

// Step 2.  With user_source the source is the per-view array d_S (the
// caller's, or the per-view tally of tabulated grains when from_tally),
// else the coherency tally d_tally; the dust's thermal term is added for a
// thermal source unless the caller supplied the source.
kp_status image_launch(kp_ctx* ctx, bool user_source, const double* d_S, double* d_out,
                       int n_lambda, hipStream_t s, const DustDev* d_dust, const ViewDev* d_views,
                       const double* d_tally, bool from_tally = false) {
  ImageArgs a{};
  a.rho = ctx->d_rho;
  if (ctx->d_bhat) {
    a.bx = ctx->d_bhat;
    a.by = ctx->d_bhat + ctx->ncell;
    a.bz = ctx->d_bhat + 2 * ctx->ncell;
  }
  a.nx = ctx->grid.nx; a.ny = ctx->grid.ny; a.nz = ctx->grid.nz;
  a.x0 = ctx->grid.x0; a.y0 = ctx->grid.y0; a.z0 = ctx->grid.z0; a.dx = ctx->grid.dx;
  a.dust = d_dust;
  a.views = d_views;
  a.n_views = (int)ctx->views.size();
  a.n_lambda = n_lambda;
  a.npx = ctx->views[0].npx;
  a.npy = ctx->views[0].npy;
  a.tally = d_tally;
  a.user_S = d_S;
  a.images = d_out;
  a.ncell = ctx->ncell;
  // the tally and the per-view tally are in the tally layout, a caller's
  // source array in cell order
  const TallyLayout tl = tally_layout(ctx);
  const bool slots = !user_source || from_tally;
  a.nslot = slots ? tl.nslot : ctx->ncell;
  a.tbx = slots ? tl.tbx : 0;
  a.tby = slots ? tl.tby : 0;
  a.em_B = ((!user_source || from_tally) && ctx->src.kind == 2) ? ctx->d_em_B : nullptr;
  a.boundary = ctx->grid.boundary;
  a.mesh = mesh_dev(ctx);
  // every wavelength shares the grain model kind of wavelength 0 for the
  // kernel choice; mixed sphere / non-sphere tables use the general kernel
  bool sphere = true;
  for (int l = 0; l < n_lambda; ++l) sphere = sphere && ctx->hdust[l].sphere;
  KP_HIP(hipEventRecord(ctx->ev[2], s), "event record");
  // tabulated grains are randomly oriented: the alignment directions do not
  // enter their extinction
  const bool aligned = ctx->d_bhat != nullptr && !ctx->have_tables;
  KP_HIP(launch_image(a, aligned, sphere, user_source, ctx->have_mesh, s), "imaging kernel launch");
  KP_HIP(hipEventRecord(ctx->ev[3], s), "event record");
  return KP_OK;
}

bool all_spheres(const kp_ctx* ctx) {
  for (const kp_dust& d : ctx->dust)
    if (!is_sphere(d)) return false;
  return true;
}

// The luminosity tables of the dust's thermal emission for every wavelength
// (cdf, guide) and each wavelength's total luminosity, rebuilt when the
// grid, the dust or the source function changed.  May allocate.
kp_status prepare_emission(kp_ctx* ctx, hipStream_t s) {
  if (ctx->em_ready) return KP_OK;
  const int nl = (int)ctx->dust.size();
  const uint64_t n = ctx->ncell;
  kp_status st = ensure(ctx, &ctx->d_em_cdf, &ctx->em_cdf_n, (size_t)nl * n, "emission table");
  if (st) return st;
  if ((st = ensure(ctx, &ctx->d_em_guide, &ctx->em_guide_n, (size_t)nl * (n + 1), "emission guide")))
    return st;
  if ((st = ensure(ctx, &ctx->d_em_partial, &ctx->em_partial_n, (size_t)emission_blocks(n),
                   "emission scan")))
    return st;
  const double vol = ctx->grid.dx * ctx->grid.dx * ctx->grid.dx;
  ctx->em_L.assign(nl, 0.0);
  for (int l = 0; l < nl; ++l) {
    const double fac = 4.0 * M_PI * ctx->dust[l].kappa_abs * vol;
    const uint64_t b3 = ctx->have_mesh ? (uint64_t)ctx->mesh.block * ctx->mesh.block * ctx->mesh.block : 1;
    KP_HIP(launch_emission_table(ctx->d_rho, ctx->d_em_B + (size_t)l * n, fac,
                                 ctx->have_mesh ? ctx->d_leaf_org : nullptr, b3, n, ctx->d_em_partial,
                                 ctx->d_em_cdf + (size_t)l * n, ctx->d_em_guide + (size_t)l * (n + 1), s),
           "emission table launch");
    KP_HIP(hipMemcpyAsync(&ctx->em_L[l], ctx->d_em_cdf + (size_t)l * n + (n - 1), sizeof(double),
                          hipMemcpyDeviceToHost, s), "emission luminosity readback");
  }
  KP_HIP(hipStreamSynchronize(s), "emission tables");
  for (int l = 0; l < nl; ++l)
    if (!(ctx->em_L[l] > 0.0) || !std::isfinite(ctx->em_L[l]))
      return fail(ctx, KP_ERR_ARG, "wavelength %d: the dust's thermal luminosity is %g (needs rho kappa_abs B > 0 "
                  "somewhere)", l, ctx->em_L[l]);
  ctx->em_ready = true;
  return KP_OK;
}

// Checks of a step-1 call (kp_transport, kp_run, kp_run_static) before any
// launch; *total receives the packet count over all wavelengths.
kp_status check_run_args(kp_ctx* ctx, const uint64_t* counts, const kp_opts* o, uint64_t* total_out) {
  kp_status st = check_ready(ctx);
  if (st) return st;
  if (!counts || !o) return fail(ctx, KP_ERR_ARG, "packets or options are NULL");
  const int nl = (int)ctx->dust.size();
  uint64_t total = 0;
  for (int l = 0; l < nl; ++l) {
    if (counts[l] > (1ull << 40)) return fail(ctx, KP_ERR_ARG, "packet count of wavelength %d too large", l);
    total += counts[l];
  }
  if (total == 0) return fail(ctx, KP_ERR_ARG, "no packets");
  if (o->tally_mode != 0) return fail(ctx, KP_ERR_ARG, "tally_mode must be 0");
  if (o->max_events < 1 || o->max_events > (1 << 30)) return fail(ctx, KP_ERR_ARG, "max_events out of range");
  if (!(o->rr_wmin >= 0.0) || !std::isfinite(o->rr_wmin) ||
      (o->rr_wmin > 0.0 && !(o->rr_psurv > 0.0 && o->rr_psurv <= 1.0)))
    return fail(ctx, KP_ERR_ARG, "roulette parameters out of range");
  if (o->trace_packets > 0 && o->trace_stride < 1) return fail(ctx, KP_ERR_ARG, "trace_stride must be >= 1");
  const int bs = o->block_size ? o->block_size : 256;
  if (bs < 64 || bs > 256 || bs % 64) return fail(ctx, KP_ERR_ARG, "block_size must be 64, 128, 192 or 256");
  if (o->blocks_per_cu < 0 || o->blocks_per_cu > 64) return fail(ctx, KP_ERR_ARG, "blocks_per_cu out of range");
  if (o->transport_fp64 < 0 || o->transport_fp64 > 2) return fail(ctx, KP_ERR_ARG, "transport_fp64 must be 0, 1 or 2");
  if (o->scatter_batch < 0 || o->scatter_batch > 64) return fail(ctx, KP_ERR_ARG, "scatter_batch must be in 0..64");
  if (o->scatter_wait < 0 || o->scatter_wait > 1024) return fail(ctx, KP_ERR_ARG, "scatter_wait must be in 0..1024");
  if (o->peel_off != 0 && o->peel_off != 1) return fail(ctx, KP_ERR_ARG, "peel_off must be 0 or 1");
  if (o->peel_off && ctx->grid.boundary)
    return fail(ctx, KP_ERR_ARG, "peel-off imaging needs open boundaries (boundary 0)");
  *total_out = total;
  return KP_OK;
}

// Device buffers of one step-1 launch.
struct RunBuffers {
  DustDev* dust;                 // per-wavelength constants (uploaded by the caller)
  double* tally;                 // [lambda][cell][stride]
  StatsDev* stats;
  unsigned long long* counter;   // work counter of the persistent launch
  TraceDev* traces;              // [lambda][trace_packets] or null
  const ViewDev* views;          // camera table (uploaded by the caller)
  double* peel;                  // [lambda][view][4][npy][npx] peel-off images, or null
};

// Step 1 on prepared buffers: tally and counters cleared by kernels, the
// persistent transport launch, then (after a synchronise) the counters
// copied into ctx->stats.  Arguments are already checked.
kp_status transport_launch(kp_ctx* ctx, const kp_opts* o, uint64_t total, const RunBuffers& b,
                           hipStream_t s) {
  const int nl = (int)ctx->dust.size();
  const bool all_sphere = all_spheres(ctx);
  const bool tab = ctx->have_tables;
  const size_t trace_need = (size_t)nl * o->trace_packets;
  const int npx = ctx->views[0].npx, npy = ctx->views[0].npy, nv = (int)ctx->views.size();
  const TallyLayout tl = tally_layout(ctx);
  if (tab)
    KP_HIP(launch_fill_zero(b.tally, (size_t)nl * tl.nslot * nv * 4 * sizeof(double), s), "tally clear");
  else
    KP_HIP(launch_tally_init(b.tally, ctx->d_rho, ctx->d_bhat,
                             ctx->d_bhat ? ctx->d_bhat + ctx->ncell : nullptr,
                             ctx->d_bhat ? ctx->d_bhat + 2 * ctx->ncell : nullptr, ctx->ncell, nl, all_sphere,
                             tl.nslot, ctx->grid.nx, ctx->grid.ny, tl.tbx, tl.tby, s),
           "tally initialisation");
  KP_HIP(launch_fill_zero(b.stats, sizeof(StatsDev), s), "stats clear");
  KP_HIP(launch_fill_zero(b.counter, sizeof(unsigned long long), s), "counter clear");
  if (trace_need) KP_HIP(launch_fill_zero(b.traces, trace_need * sizeof(TraceDev), s), "trace clear");
  if (b.peel)
    KP_HIP(launch_fill_zero(b.peel, (size_t)nl * nv * 4 * npx * npy * sizeof(double), s), "peel-off clear");

  TransportArgs a{};
  a.rho = ctx->d_rho;
  if (ctx->d_bhat) {
    a.bx = ctx->d_bhat;
    a.by = ctx->d_bhat + ctx->ncell;
    a.bz = ctx->d_bhat + 2 * ctx->ncell;
  }
  a.nx = ctx->grid.nx; a.ny = ctx->grid.ny; a.nz = ctx->grid.nz;
  a.x0 = ctx->grid.x0; a.y0 = ctx->grid.y0; a.z0 = ctx->grid.z0; a.dx = ctx->grid.dx;
  a.dust = b.dust;
  a.n_lambda = nl;
  a.total = total;
  a.src_kind = ctx->src.kind;
  a.sx = ctx->src.pos[0]; a.sy = ctx->src.pos[1]; a.sz = ctx->src.pos[2];
  a.dx_ = ctx->src.dir[0]; a.dy_ = ctx->src.dir[1]; a.dz_ = ctx->src.dir[2];
  a.seed = o->seed;
  a.rr_wmin = o->rr_wmin;
  a.rr_psurv = o->rr_psurv;
  a.max_events = (int)o->max_events;
  a.tally = b.tally;
  a.ncell = ctx->ncell;
  a.nslot = tl.nslot;
  a.tbx = tl.tbx;
  a.tby = tl.tby;
  a.counter = b.counter;
  a.stats = b.stats;
  a.traces = b.traces;
  a.trace_count = o->trace_packets;
  a.trace_stride = o->trace_stride ? o->trace_stride : 1;
  a.scatter_batch = o->scatter_batch ? o->scatter_batch : 8;
  a.scatter_wait = o->scatter_wait ? o->scatter_wait : 16;
  if (ctx->src.kind == 2) {
    a.em_cdf = ctx->d_em_cdf;
    a.em_guide = ctx->d_em_guide;
  }
  a.boundary = ctx->grid.boundary;
  a.mesh = mesh_dev(ctx);
  a.views = b.views;
  a.n_views = nv;
  if (b.peel) {
    a.npx = npx;
    a.npy = npy;
    a.peel = b.peel;
  }

  const bool sphere = all_sphere || tab;
  const bool aligned = ctx->d_bhat != nullptr && !tab;
  // automatic precision: FP64 polarisation arithmetic for dichroic (aligned,
  // non-spherical) grains, FP32 otherwise
  const bool fp64 = o->transport_fp64 == 1 || (o->transport_fp64 == 0 && aligned && !sphere);
  const int bs = o->block_size ? o->block_size : 256;
  int bpc = o->blocks_per_cu;
  if (bpc == 0) {
    bpc = transport_max_blocks_per_cu(fp64, aligned, sphere, b.peel != nullptr, tab, ctx->have_mesh, bs);
    if (bpc < 1) bpc = 1;
    if (bpc > 8) bpc = 8;
  }
  uint64_t blocks = (uint64_t)ctx->cu_count * bpc;
  const uint64_t need_blocks = (total + bs - 1) / bs;
  if (blocks > need_blocks) blocks = need_blocks;
  KP_HIP(hipEventRecord(ctx->ev[0], s), "event record");
  KP_HIP(launch_transport(a, fp64, aligned, sphere, b.peel != nullptr, tab, ctx->have_mesh, (int)blocks, bs, s),
         "transport kernel launch");
  KP_HIP(hipEventRecord(ctx->ev[1], s), "event record");
  KP_HIP(hipStreamSynchronize(s), "transport kernel");

  StatsDev h{};
  KP_HIP(hipMemcpy(&h, b.stats, sizeof h, hipMemcpyDeviceToHost), "stats readback");
  kp_stats& r = ctx->stats;
  std::memset(&r, 0, sizeof r);
  r.cell_steps = (int64_t)h.cell_steps; r.scatterings = (int64_t)h.scatterings;
  r.trials = (int64_t)h.trials; r.rr_kills = (int64_t)h.rr_kills;
  r.rr_survivals = (int64_t)h.rr_survivals; r.escaped = (int64_t)h.escaped;
  r.budget = (int64_t)h.budget; r.numeric = (int64_t)h.numeric; r.packets = (int64_t)h.packets;
  r.tally_flushes = (int64_t)h.tally_flushes;
  r.e_emitted = h.e_emitted; r.e_escaped = h.e_escaped; r.e_absorbed = h.e_absorbed;
  r.e_rr_killed = h.e_rr_killed; r.e_rr_gained = h.e_rr_gained; r.e_budget = h.e_budget;
  r.e_scat_delta = h.e_scat_delta;
  float ms = 0.0f;
  KP_HIP(hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]), "event timing");
  r.ms_transport = ms;
  if (r.packets != (int64_t)total)
    return fail(ctx, KP_ERR_DEVICE, "transport finished %lld of %llu packets", (long long)r.packets,
                (unsigned long long)total);
  if (r.numeric) return fail(ctx, KP_ERR_NUMERIC, "%lld packets reached a non-finite state", (long long)r.numeric);
  if (o->strict && r.budget) return fail(ctx, KP_ERR_BUDGET, "%lld packets hit the event cap", (long long)r.budget);
  return KP_OK;
}

}  // namespace

extern "C" {

kp_status kp_create(int device, kp_ctx** out) {
  if (!out) return KP_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return KP_ERR_DEVICE;
  if (device < 0 || device >= n) return KP_ERR_ARG;
  kp_ctx* ctx = new (std::nothrow) kp_ctx();
  if (!ctx) return KP_ERR_OOM;
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete ctx; return KP_ERR_DEVICE; }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) { delete ctx; return KP_ERR_DEVICE; }
  ctx->cu_count = prop.multiProcessorCount;
  ctx->scratch_err = scratch_address(device, &ctx->scratch);
  for (auto& e : ctx->ev)
    if (hipEventCreate(&e) != hipSuccess) { kp_destroy(ctx); return KP_ERR_DEVICE; }
  if (hipMalloc(&ctx->d_stats, sizeof(StatsDev)) != hipSuccess ||
      hipMalloc(&ctx->d_counter, sizeof(unsigned long long)) != hipSuccess ||
      hipMalloc(&ctx->d_bad, sizeof(unsigned long long)) != hipSuccess) {
    kp_destroy(ctx);
    return KP_ERR_OOM;
  }
  *out = ctx;
  return KP_OK;
}

void kp_destroy(kp_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  release_grid(ctx);
  for (void* p : {(void*)ctx->d_views, (void*)ctx->d_dust, (void*)ctx->d_tally,
                  (void*)ctx->d_images, (void*)ctx->d_stats, (void*)ctx->d_counter,
                  (void*)ctx->d_bad, (void*)ctx->d_traces, (void*)ctx->d_em_cdf,
                  (void*)ctx->d_em_guide, (void*)ctx->d_em_partial, (void*)ctx->d_peel,
                  (void*)ctx->d_tab, (void*)ctx->d_tab_guide})
    if (p) (void)hipFree(p);
  for (auto& e : ctx->ev)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

const char* kp_last_error(const kp_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

kp_status kp_set_grid(kp_ctx* ctx, const kp_grid* g, const float* rho, const float* bhat) {
  if (!ctx) return KP_ERR_ARG;
  kp_status st = check_grid(ctx, g);
  if (st) return st;
  if (!rho) return fail(ctx, KP_ERR_ARG, "rho is NULL");
  const uint64_t n = (uint64_t)g->nx * g->ny * g->nz;
  for (uint64_t i = 0; i < n; ++i)
    if (!(rho[i] >= 0.0f) || !std::isfinite(rho[i]))
      return fail(ctx, KP_ERR_ARG, "rho[%llu] is negative or not finite", (unsigned long long)i);
  if (bhat)
    for (uint64_t i = 0; i < n; ++i) {
      const double b = std::sqrt((double)bhat[i] * bhat[i] + (double)bhat[n + i] * bhat[n + i] +
                                 (double)bhat[2 * n + i] * bhat[2 * n + i]);
      if (!(std::fabs(b - 1.0) <= 1e-5))
        return fail(ctx, KP_ERR_ARG, "bhat[:, %llu] is not a unit vector", (unsigned long long)i);
    }
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  release_grid(ctx);
  KP_HIP(hipMalloc(&ctx->own_rho, n * sizeof(float)), "rho allocation");
  KP_HIP(hipMemcpy(ctx->own_rho, rho, n * sizeof(float), hipMemcpyHostToDevice), "rho upload");
  if (bhat) {
    KP_HIP(hipMalloc(&ctx->own_bhat, 3 * n * sizeof(float)), "bhat allocation");
    KP_HIP(hipMemcpy(ctx->own_bhat, bhat, 3 * n * sizeof(float), hipMemcpyHostToDevice), "bhat upload");
  }
  ctx->d_rho = ctx->own_rho;
  ctx->d_bhat = ctx->own_bhat;
  ctx->grid = *g;
  ctx->ncell = n;
  ctx->have_grid = true;
  return KP_OK;
}

kp_status kp_set_grid_device(kp_ctx* ctx, const kp_grid* g, const float* d_rho, const float* d_bhat) {
  if (!ctx) return KP_ERR_ARG;
  kp_status st = check_grid(ctx, g);
  if (st) return st;
  if (!d_rho) return fail(ctx, KP_ERR_ARG, "rho is NULL");
  const uint64_t n = (uint64_t)g->nx * g->ny * g->nz;
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  KP_HIP(hipMemset(ctx->d_bad, 0, sizeof(unsigned long long)), "validation reset");
  KP_HIP(launch_validate(d_rho, d_bhat, d_bhat ? d_bhat + n : nullptr,
                         d_bhat ? d_bhat + 2 * n : nullptr, n, ctx->d_bad, 0), "validation launch");
  unsigned long long bad = 0;
  KP_HIP(hipMemcpy(&bad, ctx->d_bad, sizeof bad, hipMemcpyDeviceToHost), "validation readback");
  if (bad) return fail(ctx, KP_ERR_ARG, "%llu grid values are invalid (negative/non-finite rho or non-unit bhat)", bad);
  release_grid(ctx);
  ctx->d_rho = const_cast<float*>(d_rho);
  ctx->d_bhat = const_cast<float*>(d_bhat);
  ctx->grid = *g;
  ctx->ncell = n;
  ctx->have_grid = true;
  return KP_OK;
}

kp_status kp_set_mesh(kp_ctx* ctx, const kp_mesh* m, const int32_t* child, const float* rho,
                      const float* bhat) {
  if (!ctx) return KP_ERR_ARG;
  if (!m || !child || !rho) return fail(ctx, KP_ERR_ARG, "mesh, child or rho is NULL");
  if (m->rx < 1 || m->ry < 1 || m->rz < 1 || m->block < 1 || m->block > 64)
    return fail(ctx, KP_ERR_ARG, "root blocks must be >= 1 per axis and block in 1..64");
  if (m->max_level < 0 || m->max_level > 16) return fail(ctx, KP_ERR_ARG, "max_level must be in 0..16");
  if (!(m->dx > 0.0) || !std::isfinite(m->dx) || !std::isfinite(m->x0) || !std::isfinite(m->y0) ||
      !std::isfinite(m->z0))
    return fail(ctx, KP_ERR_ARG, "dx must be finite and > 0 and the corner finite");
  const int64_t full = (int64_t)m->block << m->max_level;
  const int64_t R = (int64_t)m->rx * m->ry * m->rz;
  const int64_t ext[3] = {m->rx * full, m->ry * full, m->rz * full};
  for (int k = 0; k < 3; ++k)
    if (ext[k] > ((int64_t)1 << 30)) return fail(ctx, KP_ERR_ARG, "the box exceeds 2^30 finest cells along an axis");
  if (m->n_nodes < R || m->n_nodes > (1 << 30)) return fail(ctx, KP_ERR_ARG, "n_nodes must cover the root blocks");
  // parents, levels and origins of every node; children after their parent
  const int32_t N = m->n_nodes;
  std::vector<int32_t> parents(N, 0), lev(N, 0);
  std::vector<int64_t> org(3 * (size_t)N, 0);
  for (int64_t r = 0; r < R; ++r) {
    org[3 * r] = (r % m->rx) * full;
    org[3 * r + 1] = ((r / m->rx) % m->ry) * full;
    org[3 * r + 2] = (r / ((int64_t)m->rx * m->ry)) * full;
  }
  for (int32_t i = 0; i < N; ++i) {
    const int32_t c = child[i];
    if (c == -1) continue;
    if (c < R || c <= i || (int64_t)c + 8 > N || lev[i] + 1 > m->max_level)
      return fail(ctx, KP_ERR_ARG, "node %d: child index %d invalid (before its parent, past the list or "
                  "deeper than max_level)", i, c);
    const int64_t half = full >> (lev[i] + 1);
    for (int k = 0; k < 8; ++k) {
      if (parents[c + k]++) return fail(ctx, KP_ERR_ARG, "node %d has two parents", c + k);
      lev[c + k] = lev[i] + 1;
      org[3 * (size_t)(c + k)] = org[3 * (size_t)i] + ((k & 1) ? half : 0);
      org[3 * (size_t)(c + k) + 1] = org[3 * (size_t)i + 1] + ((k & 2) ? half : 0);
      org[3 * (size_t)(c + k) + 2] = org[3 * (size_t)i + 2] + ((k & 4) ? half : 0);
    }
  }
  for (int32_t i = (int32_t)R; i < N; ++i)
    if (parents[i] != 1) return fail(ctx, KP_ERR_ARG, "node %d is nobody's child", i);
  std::vector<int32_t> leaf_of_node(N, -1), leaf_org;
  int64_t nleaf = 0;
  for (int32_t i = 0; i < N; ++i) {
    if (child[i] != -1) continue;
    leaf_of_node[i] = (int32_t)nleaf++;
    leaf_org.insert(leaf_org.end(), {(int32_t)org[3 * (size_t)i], (int32_t)org[3 * (size_t)i + 1],
                                     (int32_t)org[3 * (size_t)i + 2], lev[i]});
  }
  const uint64_t B3 = (uint64_t)m->block * m->block * m->block;
  const uint64_t n = (uint64_t)nleaf * B3;
  if ((double)n > 4.0e9) return fail(ctx, KP_ERR_ARG, "the mesh has more than 4e9 cells");
  for (uint64_t i = 0; i < n; ++i)
    if (!(rho[i] >= 0.0f) || !std::isfinite(rho[i]))
      return fail(ctx, KP_ERR_ARG, "rho[%llu] is negative or not finite", (unsigned long long)i);
  if (bhat)
    for (uint64_t i = 0; i < n; ++i) {
      const double b = std::sqrt((double)bhat[i] * bhat[i] + (double)bhat[n + i] * bhat[n + i] +
                                 (double)bhat[2 * n + i] * bhat[2 * n + i]);
      if (!(std::fabs(b - 1.0) <= 1e-5))
        return fail(ctx, KP_ERR_ARG, "bhat[:, %llu] is not a unit vector", (unsigned long long)i);
    }
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  release_grid(ctx);
  KP_HIP(hipMalloc(&ctx->own_rho, n * sizeof(float)), "rho allocation");
  KP_HIP(hipMemcpy(ctx->own_rho, rho, n * sizeof(float), hipMemcpyHostToDevice), "rho upload");
  if (bhat) {
    KP_HIP(hipMalloc(&ctx->own_bhat, 3 * n * sizeof(float)), "bhat allocation");
    KP_HIP(hipMemcpy(ctx->own_bhat, bhat, 3 * n * sizeof(float), hipMemcpyHostToDevice), "bhat upload");
  }
  KP_HIP(hipMalloc(&ctx->d_child, N * sizeof(int32_t)), "mesh allocation");
  KP_HIP(hipMalloc(&ctx->d_leaf_of_node, N * sizeof(int32_t)), "mesh allocation");
  KP_HIP(hipMalloc(&ctx->d_leaf_org, leaf_org.size() * sizeof(int32_t)), "mesh allocation");
  KP_HIP(hipMemcpy(ctx->d_child, child, N * sizeof(int32_t), hipMemcpyHostToDevice), "mesh upload");
  KP_HIP(hipMemcpy(ctx->d_leaf_of_node, leaf_of_node.data(), N * sizeof(int32_t), hipMemcpyHostToDevice),
         "mesh upload");
  KP_HIP(hipMemcpy(ctx->d_leaf_org, leaf_org.data(), leaf_org.size() * sizeof(int32_t), hipMemcpyHostToDevice),
         "mesh upload");
  ctx->d_rho = ctx->own_rho;
  ctx->d_bhat = ctx->own_bhat;
  ctx->grid = kp_grid{m->rx * m->block, m->ry * m->block, m->rz * m->block, m->x0, m->y0, m->z0, m->dx, 0};
  ctx->ncell = n;
  ctx->mesh = *m;
  for (int k = 0; k < 3; ++k) ctx->nfine[k] = (int)ext[k];
  ctx->have_mesh = true;
  ctx->have_grid = true;
  return KP_OK;
}

kp_status kp_set_dust(kp_ctx* ctx, int32_t n_lambda, const kp_dust* d) {
  if (!ctx) return KP_ERR_ARG;
  if (n_lambda < 1 || n_lambda > 1024 || !d) return fail(ctx, KP_ERR_ARG, "n_lambda must be in 1..1024");
  for (int l = 0; l < n_lambda; ++l) {
    const kp_dust& x = d[l];
    if (!(x.kappa_sca >= 0.0) || !(x.kappa_abs >= 0.0) || !std::isfinite(x.kappa_sca) ||
        !std::isfinite(x.kappa_abs) || !(x.kappa_sca + x.kappa_abs > 0.0))
      return fail(ctx, KP_ERR_ARG, "dust %d: opacities must be finite, >= 0, with a positive sum", l);
    const double v[5] = {x.a_perp[0], x.a_perp[1], x.a_par[0], x.a_par[1], x.alpha3_scale};
    for (double t : v)
      if (!std::isfinite(t)) return fail(ctx, KP_ERR_ARG, "dust %d: non-finite polarizability", l);
    if (!is_sphere(x)) {
      if (!(2.0 * x.a_perp[1] + x.a_par[1] > 0.0) || x.a_perp[1] < 0.0 || x.a_par[1] < 0.0)
        return fail(ctx, KP_ERR_ARG, "dust %d: aligned grains need Im(a) >= 0 with a positive average", l);
    } else if (x.a_perp[0] == 0.0 && x.a_perp[1] == 0.0) {
      return fail(ctx, KP_ERR_ARG, "dust %d: zero polarizability", l);
    }
  }
  ctx->dust.assign(d, d + n_lambda);
  ctx->have_tally = false;
  ctx->have_images = false;
  ctx->em_ready = false;
  ctx->have_tables = false;  // tables belong to the dust they were given for
  return KP_OK;
}

kp_status kp_set_dust_tables(kp_ctx* ctx, int32_t n_lambda, int32_t n_theta, const double* Z) {
  if (!ctx) return KP_ERR_ARG;
  if (n_lambda == 0 && !Z) {
    ctx->have_tables = false;
    ctx->have_tally = false;
    ctx->have_images = false;
    return KP_OK;
  }
  if (ctx->dust.empty()) return fail(ctx, KP_ERR_STATE, "kp_set_dust has not been called");
  if (n_lambda != (int)ctx->dust.size() || !Z)
    return fail(ctx, KP_ERR_ARG, "tables for %d wavelengths given, kp_set_dust set %zu", n_lambda, ctx->dust.size());
  if (n_theta < 2 || n_theta > 65536) return fail(ctx, KP_ERR_ARG, "n_theta must be in 2..65536");
  const size_t nl = (size_t)n_lambda, nt = (size_t)n_theta;
  std::vector<double> h(nl * nt * 6 + nt + nl * nt);
  double* mu = h.data() + nl * nt * 6;
  double* cum = mu + nt;
  for (size_t j = 0; j < nt; ++j) mu[j] = std::cos((double)j * M_PI / (double)(nt - 1));
  for (size_t l = 0; l < nl; ++l) {
    const double* z = Z + l * nt * 6;
    for (size_t j = 0; j < nt; ++j)
      for (int k = 0; k < 6; ++k)
        if (!std::isfinite(z[6 * j + k]) || std::fabs(z[6 * j + k]) > z[6 * j])
          return fail(ctx, KP_ERR_ARG, "table %zu, node %zu: element %d is not finite or exceeds S11 in "
                      "magnitude", l, j, k);
    // 2 pi times the integral of S11 over cos Theta, exact for S11 linear in
    // cos Theta on each interval
    double sum = 0.0;
    for (size_t j = 0; j + 1 < nt; ++j) sum += 0.5 * (z[6 * j] + z[6 * (j + 1)]) * (mu[j] - mu[j + 1]);
    const double N = 2.0 * M_PI * sum;
    if (!(N > 0.0) || !std::isfinite(N)) return fail(ctx, KP_ERR_ARG, "table %zu: S11 integrates to %g", l, N);
    double* t = h.data() + l * nt * 6;
    for (size_t i = 0; i < nt * 6; ++i) t[i] = z[i] / N;
    double* c = cum + l * nt;
    c[0] = 0.0;
    for (size_t j = 0; j + 1 < nt; ++j) c[j + 1] = c[j] + std::fmax(t[6 * j], t[6 * (j + 1)]) * (mu[j] - mu[j + 1]);
  }
  // guide: bin b of G = 8 (n - 1) uniform bins of cos Theta from 1 down to -1
  // holds the interval j (mu_j+1 <= mu <= mu_j) of its upper end 1 - 2 b / G
  const int G = 8 * (n_theta - 1);
  std::vector<int32_t> guide(G);
  for (int b = 0, j = 0; b < G; ++b) {
    const double top = 1.0 - 2.0 * b / G;
    while (j < n_theta - 2 && mu[j + 1] >= top) ++j;
    guide[b] = j;
  }
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  kp_status st = ensure(ctx, &ctx->d_tab, &ctx->tab_n, h.size(), "table allocation");
  if (st) return st;
  if ((st = ensure(ctx, &ctx->d_tab_guide, &ctx->tab_guide_n, guide.size(), "table guide allocation"))) return st;
  KP_HIP(hipMemcpy(ctx->d_tab, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice), "table upload");
  KP_HIP(hipMemcpy(ctx->d_tab_guide, guide.data(), guide.size() * sizeof(int32_t), hipMemcpyHostToDevice),
         "table guide upload");
  ctx->tab_nt = n_theta;
  ctx->have_tables = true;
  ctx->have_tally = false;
  ctx->have_images = false;
  return KP_OK;
}

kp_status kp_set_source(kp_ctx* ctx, const kp_source* s) {
  if (!ctx) return KP_ERR_ARG;
  if (!s) return fail(ctx, KP_ERR_ARG, "source is NULL");
  if (s->kind < 0 || s->kind > 2) return fail(ctx, KP_ERR_ARG, "source kind must be 0, 1 or 2");
  if (s->kind != 2 && (!finite3(s->pos) || !std::isfinite(s->lum) || !(s->lum > 0.0)))
    return fail(ctx, KP_ERR_ARG, "source position/luminosity invalid");
  kp_source c = *s;
  if (s->kind == 1) {
    if (!finite3(s->dir)) return fail(ctx, KP_ERR_ARG, "pencil direction not finite");
    const double n = std::sqrt(s->dir[0] * s->dir[0] + s->dir[1] * s->dir[1] + s->dir[2] * s->dir[2]);
    if (!(n > 0.0)) return fail(ctx, KP_ERR_ARG, "pencil direction is zero");
    for (int k = 0; k < 3; ++k) c.dir[k] = s->dir[k] / n;
  }
  if (s->kind == 2) c.lum = 0.0;  // the dust's luminosity comes from the grid
  ctx->src = c;
  ctx->have_source = true;
  return KP_OK;
}

kp_status kp_set_emission(kp_ctx* ctx, int32_t n_lambda, const float* B) {
  if (!ctx) return KP_ERR_ARG;
  if (!ctx->have_grid) return fail(ctx, KP_ERR_STATE, "kp_set_grid has not been called");
  if (n_lambda < 1 || n_lambda > 1024 || !B) return fail(ctx, KP_ERR_ARG, "n_lambda must be in 1..1024");
  const uint64_t n = ctx->ncell;
  const size_t total = (size_t)n_lambda * n;
  for (size_t i = 0; i < total; ++i)
    if (!(B[i] >= 0.0f) || !std::isfinite(B[i]))
      return fail(ctx, KP_ERR_ARG, "B[%zu] is negative or not finite", i);
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  if (ctx->d_em_B) (void)hipFree(ctx->d_em_B);
  ctx->d_em_B = nullptr;
  ctx->have_emission = false;
  ctx->em_ready = false;
  KP_HIP(hipMalloc(&ctx->d_em_B, total * sizeof(float)), "emission allocation");
  KP_HIP(hipMemcpy(ctx->d_em_B, B, total * sizeof(float), hipMemcpyHostToDevice), "emission upload");
  ctx->em_nl = n_lambda;
  ctx->have_emission = true;
  ctx->have_images = false;
  return KP_OK;
}

kp_status kp_set_views(kp_ctx* ctx, int32_t n_views, const kp_view* v) {
  if (!ctx) return KP_ERR_ARG;
  if (n_views < 1 || n_views > 4096 || !v) return fail(ctx, KP_ERR_ARG, "n_views must be in 1..4096");
  for (int k = 0; k < n_views; ++k) {
    if (!std::isfinite(v[k].theta) || !std::isfinite(v[k].phi) || !(v[k].half_width > 0.0) ||
        !std::isfinite(v[k].half_width))
      return fail(ctx, KP_ERR_ARG, "view %d: invalid direction or half width", k);
    if (v[k].npx < 1 || v[k].npy < 1 || v[k].npx > 16384 || v[k].npy > 16384)
      return fail(ctx, KP_ERR_ARG, "view %d: npx, npy must be in 1..16384", k);
    if (v[k].npx != v[0].npx || v[k].npy != v[0].npy)
      return fail(ctx, KP_ERR_ARG, "all views must share npx and npy");
  }
  ctx->views.assign(v, v + n_views);
  ctx->hviews.resize(n_views);
  for (int k = 0; k < n_views; ++k) fill_view(v[k], ctx->hviews[k]);
  ctx->have_images = false;
  ctx->peel_valid_n = 0;
  if (ctx->tally_views) ctx->have_tally = false;  // a per-view tally belongs to its cameras
  return KP_OK;
}

kp_status kp_transport(kp_ctx* ctx, const uint64_t* counts, const kp_opts* o, void* stream) {
  if (!ctx) return KP_ERR_ARG;
  uint64_t total = 0;
  kp_status st = check_run_args(ctx, counts, o, &total);
  if (st) return st;
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int nl = (int)ctx->dust.size();
  const bool all_sphere = all_spheres(ctx);
  const int ts = tally_stride(all_sphere);
  const uint64_t nslot = tally_layout(ctx).nslot;
  const size_t tally_need = ctx->have_tables ? (size_t)nl * nslot * ctx->views.size() * 4
                                             : (size_t)nl * nslot * ts;
  const size_t trace_need = (size_t)nl * o->trace_packets;
  const size_t peel_need =
      o->peel_off ? (size_t)nl * ctx->views.size() * 4 * ctx->views[0].npx * ctx->views[0].npy : 0;
  size_t free_b = 0, total_b = 0;
  KP_HIP(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
  size_t extra = (tally_need > ctx->tally_n ? tally_need * 8 : 0) +
                 (trace_need > ctx->traces_n ? trace_need * sizeof(TraceDev) : 0) +
                 (peel_need > ctx->peel_n ? peel_need * 8 : 0);
  if (extra > free_b) return fail(ctx, KP_ERR_OOM, "tally needs %zu bytes, %zu free", extra, free_b);
  if ((st = ensure(ctx, &ctx->d_tally, &ctx->tally_n, tally_need, "tally allocation"))) return st;
  if ((st = ensure(ctx, &ctx->d_traces, &ctx->traces_n, trace_need, "trace allocation"))) return st;
  if ((st = ensure(ctx, &ctx->d_peel, &ctx->peel_n, peel_need, "peel-off allocation"))) return st;
  ctx->peel_valid_n = 0;
  if (ctx->src.kind == 2 && (st = prepare_emission(ctx, s))) return st;
  fill_dust(ctx, counts, ctx->hdust);
  if ((st = upload_small(ctx, s))) return st;
  const RunBuffers buf{ctx->d_dust, ctx->d_tally, ctx->d_stats, ctx->d_counter, ctx->d_traces,
                       ctx->d_views, o->peel_off ? ctx->d_peel : nullptr};
  st = transport_launch(ctx, o, total, buf, s);
  if (st == KP_ERR_DEVICE || st == KP_ERR_OOM) return st;
  ctx->peel_valid_n = peel_need;
  ctx->tally_views = ctx->have_tables;
  ctx->tally_nv = (int)ctx->views.size();
  ctx->tally_lambda = nl;
  ctx->tally_ts = ts;
  ctx->tally_nc = tally_components(all_sphere);
  ctx->have_tally = true;
  ctx->have_images = false;
  ctx->traces_valid = trace_need;
  return st;
}

kp_status kp_image(kp_ctx* ctx, void* stream) {
  if (!ctx) return KP_ERR_ARG;
  if (!ctx->have_tally) return fail(ctx, KP_ERR_STATE, "no step-1 tally: call kp_transport first");
  kp_status st = check_ready(ctx);
  if (st) return st;
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int nl = ctx->tally_lambda;
  const size_t need = (size_t)nl * ctx->views.size() * 4 * ctx->views[0].npx * ctx->views[0].npy;
  if ((st = ensure(ctx, &ctx->d_images, &ctx->images_n, need, "image allocation"))) return st;
  if ((st = upload_small(ctx, s))) return st;
  if (ctx->tally_views) {
    if (!ctx->have_tables || ctx->tally_nv != (int)ctx->views.size())
      return fail(ctx, KP_ERR_STATE, "the per-view tally no longer matches the dust tables or cameras");
    st = image_launch(ctx, true, ctx->d_tally, ctx->d_images, nl, s, ctx->d_dust, ctx->d_views, nullptr, true);
  } else {
    st = image_launch(ctx, false, nullptr, ctx->d_images, nl, s, ctx->d_dust, ctx->d_views, ctx->d_tally);
  }
  if (st) return st;
  KP_HIP(hipStreamSynchronize(s), "imaging kernel");
  float ms = 0.0f;
  KP_HIP(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]), "event timing");
  ctx->stats.ms_image = ms;
  ctx->have_images = true;
  ctx->images_valid_n = need;
  return KP_OK;
}

kp_status kp_run(kp_ctx* ctx, const uint64_t* counts, const kp_opts* o, void* stream) {
  kp_status st = kp_transport(ctx, counts, o, stream);
  if (st != KP_OK && st != KP_ERR_NUMERIC && st != KP_ERR_BUDGET) return st;
  kp_status st2 = kp_image(ctx, stream);
  return st2 != KP_OK ? st2 : st;
}

kp_status kp_run_static(kp_ctx* ctx, const uint64_t* counts, const kp_opts* o, double* d_images,
                        size_t n, void* stream) {
  if (!ctx) return KP_ERR_ARG;
  uint64_t total = 0;
  kp_status st = check_run_args(ctx, counts, o, &total);
  if (st) return st;
  if (o->trace_packets) return fail(ctx, KP_ERR_ARG, "kp_run_static records no traces: trace_packets must be 0");
  if (o->peel_off) return fail(ctx, KP_ERR_ARG, "kp_run_static forms no peel-off images: peel_off must be 0");
  if (ctx->src.kind == 2 && !ctx->em_ready)
    return fail(ctx, KP_ERR_STATE, "thermal emission: its luminosity tables are built by kp_run or kp_transport; "
                "call one of them once after kp_set_emission, kp_set_dust or kp_set_grid");
  if (!ctx->scratch)
    return fail(ctx, KP_ERR_DEVICE, "static scratch of device %d unavailable: %s", ctx->device,
                hipGetErrorString(ctx->scratch_err));
  const int nl = (int)ctx->dust.size();
  const int nv = (int)ctx->views.size();
  const size_t img_need = (size_t)nl * nv * 4 * ctx->views[0].npx * ctx->views[0].npy;
  if (!d_images || n != img_need) return fail(ctx, KP_ERR_ARG, "destination must hold %zu doubles", img_need);
  const bool all_sphere = all_spheres(ctx);
  const size_t cell_bytes = ctx->have_tables ? (size_t)nv * 4 * sizeof(double)
                                             : (size_t)tally_stride(all_sphere) * sizeof(double);
  const uint64_t nslot = tally_layout(ctx).nslot;
  const size_t tally_bytes = (size_t)nl * nslot * cell_bytes;
  if (tally_bytes > KP_STATIC_TALLY)
    return fail(ctx, KP_ERR_ARG, "the tally needs %zu bytes, more than the %zu of the static scratch "
                "(%d wavelengths x %llu cell slots x %zu B): use kp_run", tally_bytes, KP_STATIC_TALLY, nl,
                (unsigned long long)nslot, cell_bytes);
  // head of the scratch: stats at 0, work counter at 256, the dust table at
  // 512, the camera table after it (at most 1024 x 144 B + 4096 x 80 B)
  const size_t dust_off = 512, dust_bytes = (size_t)nl * sizeof(DustDev);
  const size_t view_off = (dust_off + dust_bytes + 255) & ~size_t(255);
  const size_t view_bytes = (size_t)nv * sizeof(ViewDev);
  static_assert(512 + 1024 * sizeof(DustDev) + 256 + 4096 * sizeof(ViewDev) <= KP_STATIC_HEAD,
                "tables fit the head of the static scratch");
  unsigned char* base = ctx->scratch;
  StatsDev* d_stats = (StatsDev*)base;
  unsigned long long* d_counter = (unsigned long long*)(base + 256);
  DustDev* d_dust = (DustDev*)(base + dust_off);
  ViewDev* d_views = (ViewDev*)(base + view_off);
  double* d_tally = (double*)(base + KP_STATIC_HEAD);
  static_assert(sizeof(StatsDev) <= 256, "stats fit their slot");

  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  fill_dust(ctx, counts, ctx->hdust);
  KP_HIP(hipMemcpyAsync(d_dust, ctx->hdust.data(), dust_bytes, hipMemcpyHostToDevice, s), "dust upload");
  KP_HIP(hipMemcpyAsync(d_views, ctx->hviews.data(), view_bytes, hipMemcpyHostToDevice, s), "view upload");
  const RunBuffers buf{d_dust, d_tally, d_stats, d_counter, nullptr, d_views, nullptr};
  st = transport_launch(ctx, o, total, buf, s);
  if (st == KP_ERR_DEVICE || st == KP_ERR_OOM) return st;
  kp_status st2 = ctx->have_tables
                      ? image_launch(ctx, true, d_tally, d_images, nl, s, d_dust, d_views, nullptr, true)
                      : image_launch(ctx, false, nullptr, d_images, nl, s, d_dust, d_views, d_tally);
  if (st2) return st2;
  KP_HIP(hipStreamSynchronize(s), "imaging kernel");
  float ms = 0.0f;
  KP_HIP(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]), "event timing");
  ctx->stats.ms_image = ms;
  return st;
}

kp_status kp_image_source(kp_ctx* ctx, const double* d_S, double* d_out, void* stream) {
  if (!ctx) return KP_ERR_ARG;
  kp_status st = check_ready(ctx);
  if (st) return st;
  if (!d_S || !d_out) return fail(ctx, KP_ERR_ARG, "source or output is NULL");
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  std::vector<uint64_t> ones(ctx->dust.size(), 1);
  fill_dust(ctx, ones.data(), ctx->hdust);
  if ((st = upload_small(ctx, s))) return st;
  if ((st = image_launch(ctx, true, d_S, d_out, 1, s, ctx->d_dust, ctx->d_views, ctx->d_tally))) return st;
  KP_HIP(hipStreamSynchronize(s), "imaging kernel");
  float ms = 0.0f;
  KP_HIP(hipEventElapsedTime(&ms, ctx->ev[2], ctx->ev[3]), "event timing");
  ctx->stats.ms_image = ms;
  return KP_OK;
}

kp_status kp_get_images(kp_ctx* ctx, double* out, size_t n) {
  if (!ctx) return KP_ERR_ARG;
  if (!ctx->have_images) return fail(ctx, KP_ERR_STATE, "no images: call kp_run or kp_image first");
  if (!out || n != ctx->images_valid_n) return fail(ctx, KP_ERR_ARG, "destination must hold %zu doubles", ctx->images_valid_n);
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  KP_HIP(hipMemcpy(out, ctx->d_images, n * sizeof(double), hipMemcpyDeviceToHost), "image copy");
  return KP_OK;
}

kp_status kp_get_images_device(kp_ctx* ctx, double* d_out, size_t n, void* stream) {
  if (!ctx) return KP_ERR_ARG;
  if (!ctx->have_images) return fail(ctx, KP_ERR_STATE, "no images: call kp_run or kp_image first");
  if (!d_out || n != ctx->images_valid_n) return fail(ctx, KP_ERR_ARG, "destination must hold %zu doubles", ctx->images_valid_n);
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  KP_HIP(hipMemcpyAsync(d_out, ctx->d_images, n * sizeof(double), hipMemcpyDeviceToDevice,
                        (hipStream_t)stream), "image copy");
  return KP_OK;
}

kp_status kp_get_peel_images(kp_ctx* ctx, double* out, size_t n) {
  if (!ctx) return KP_ERR_ARG;
  if (!ctx->peel_valid_n)
    return fail(ctx, KP_ERR_STATE, "no peel-off images: the last step 1 ran without peel_off");
  if (!out || n != ctx->peel_valid_n)
    return fail(ctx, KP_ERR_ARG, "destination must hold %zu doubles", ctx->peel_valid_n);
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  KP_HIP(hipMemcpy(out, ctx->d_peel, n * sizeof(double), hipMemcpyDeviceToHost), "peel-off copy");
  return KP_OK;
}

// Copy of the last step 1's tally to the host in cell order: per (wavelength,
// cell) the first `keep` of the `stride` doubles at its tally slot, into
// rows of `row` doubles (zero past `keep`).
kp_status copy_tally_cells(kp_ctx* ctx, double* out, size_t row, size_t stride, size_t keep) {
  const TallyLayout tl = tally_layout(ctx);
  const size_t nl = (size_t)ctx->tally_lambda;
  std::vector<double> h;
  try {
    h.resize(nl * tl.nslot * stride);
  } catch (const std::bad_alloc&) {
    return fail(ctx, KP_ERR_OOM, "host copy of the tally (%zu doubles)", nl * tl.nslot * stride);
  }
  KP_HIP(hipMemcpy(h.data(), ctx->d_tally, h.size() * sizeof(double), hipMemcpyDeviceToHost), "tally copy");
  const int nx = ctx->grid.nx, ny = ctx->grid.ny;
  for (size_t l = 0; l < nl; ++l)
    for (uint64_t c = 0; c < ctx->ncell; ++c) {
      const uint64_t ck = tl.tbx ? c / ((uint64_t)nx * ny) : 0, r = tl.tbx ? c - ck * (uint64_t)nx * ny : 0;
      const uint64_t sl = tally_slot(c, (int)(r % nx), (int)(r / nx), (int)ck, tl.tbx, tl.tby);
      const double* src = h.data() + (l * tl.nslot + sl) * stride;
      double* dst = out + (l * ctx->ncell + c) * row;
      for (size_t k = 0; k < row; ++k) dst[k] = k < keep ? src[k] : 0.0;
    }
  return KP_OK;
}

kp_status kp_get_view_tally(kp_ctx* ctx, double* out, size_t n) {
  if (!ctx) return KP_ERR_ARG;
  if (!ctx->have_tally || !ctx->tally_views)
    return fail(ctx, KP_ERR_STATE, "no per-view tally: the last step 1 (kp_transport with tabulated grains) "
                "is missing or tallied coherencies");
  const size_t need = (size_t)ctx->tally_lambda * ctx->ncell * ctx->tally_nv * 4;
  if (!out || n != need) return fail(ctx, KP_ERR_ARG, "destination must hold %zu doubles", need);
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  return copy_tally_cells(ctx, out, (size_t)ctx->tally_nv * 4, (size_t)ctx->tally_nv * 4, (size_t)ctx->tally_nv * 4);
}

kp_status kp_get_tally(kp_ctx* ctx, double* out, size_t n) {
  if (!ctx) return KP_ERR_ARG;
  if (!ctx->have_tally) return fail(ctx, KP_ERR_STATE, "no tally: call kp_transport first");
  if (ctx->tally_views)
    return fail(ctx, KP_ERR_STATE, "tabulated grains tally the per-view source: use kp_get_view_tally");
  const size_t rows = (size_t)ctx->tally_lambda * ctx->ncell;
  const size_t need = rows * 9;
  if (!out || n != need) return fail(ctx, KP_ERR_ARG, "destination must hold %zu doubles", need);
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  return copy_tally_cells(ctx, out, 9, ctx->tally_ts, ctx->tally_nc);
}

kp_status kp_get_stats(kp_ctx* ctx, kp_stats* out) {
  if (!ctx) return KP_ERR_ARG;
  if (!out) return fail(ctx, KP_ERR_ARG, "output is NULL");
  *out = ctx->stats;
  return KP_OK;
}

kp_status kp_get_trace(kp_ctx* ctx, kp_packet_trace* out, size_t n) {
  if (!ctx) return KP_ERR_ARG;
  if (!out || n != ctx->traces_valid) return fail(ctx, KP_ERR_ARG, "destination must hold %zu traces", ctx->traces_valid);
  if (n == 0) return KP_OK;
  static_assert(sizeof(kp_packet_trace) == sizeof(TraceDev), "trace layout");
  KP_HIP(hipSetDevice(ctx->device), "hipSetDevice");
  KP_HIP(hipMemcpy(out, ctx->d_traces, n * sizeof(TraceDev), hipMemcpyDeviceToHost), "trace copy");
  return KP_OK;
}

}  // extern "C"
