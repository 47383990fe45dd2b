// kp_dn_api.cpp -- host side of the denoiser C ABI (include/polrad_denoiser.h):
// parameter layout, workspace carving, the forward and backward schedules of
// the network, Adam, timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <algorithm>
#include <vector>

#include "../../include/polrad_denoiser.h"
#include "kp_dn_internal.hpp"

using namespace kp::dn;

namespace {

constexpr int MAX_LEVELS = 6;

struct Layer {
  int cin_true = 0;  // input channels of the network layer
  int cin = 0;       // channels per tap in the GEMM (cin_true rounded up to 8)
  int cout = 0;
  int kp = 0;        // padded GEMM K of the forward weights
  int kpd = 0;       // padded GEMM K of the input-gradient weights (0: none)
  size_t w_off = 0, b_off = 0;          // offsets into the flat FP32 parameters
  size_t pk_off = 0, pkd_off = 0;       // offsets into the packed BF16 weights
};

// Workspace of one batch shape.  Level l (0 = full resolution) holds
// cap / 4^l pixels; widths c[l].  Encoder level l < L-1: block input (x0 at
// l = 0, pooled map otherwise), conv-a output, and the block output written
// into the skip part (channels c[l+1]..) of cat[l]; the bottleneck l = L-1:
// input pool, conv-a output, output; decoder level l: cat[l] (up(below) in
// channels 0..c[l+1]-1), conv-a output, output.  Gradients mirror them.
struct Work {
  size_t cap = 0;    // level-0 pixel capacity
  int bcap = 0;      // batch capacity
  void* mem = nullptr;
  size_t bytes = 0;
  uint16_t* x0 = nullptr;
  uint16_t *pool[MAX_LEVELS] = {}, *ea[MAX_LEVELS] = {}, *cat[MAX_LEVELS] = {}, *da[MAX_LEVELS] = {},
           *dout[MAX_LEVELS] = {};
  uint16_t *ma = nullptr, *mout = nullptr;
  uint16_t *gd[MAX_LEVELS] = {}, *gdb[MAX_LEVELS] = {}, *gcat[MAX_LEVELS] = {}, *ge[MAX_LEVELS] = {},
           *geb[MAX_LEVELS] = {}, *gpool[MAX_LEVELS] = {};
  uint16_t *gm = nullptr, *gmb = nullptr;
  float *xq, *ihat, *tgt, *out, *go;
  float* wpart = nullptr;  // partial weight-gradient blocks (k_wgrad_halo)
  double *sum, *loss;
  int32_t* aug;
};

constexpr int NEVENT = 512;  // 8 averaged passes of a 6-level network record 354

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

}  // namespace

struct kp_dn {
  int device = 0;
  std::string err;
  int L = 0;
  int runs = 1;  // independent Monte Carlo runs per input image (1 or 2)
  int c[MAX_LEVELS] = {};
  std::vector<Layer> layers;
  size_t head_w = 0, head_b = 0, n_params = 0;
  float* d_p = nullptr;  // params, grads, m, v: 4 x n_params
  float* d_g = nullptr;
  float* d_m = nullptr;
  float* d_v = nullptr;
  uint16_t* d_pk = nullptr;
  size_t pk_n = 0;
  bool packed = false;
  int step = 0;
  Work w;
  // timing
  hipEvent_t ev[NEVENT] = {};
  struct Mark { int a, b, cat; double flop; };
  std::vector<Mark> marks;
  int nev = 0;
  int ev_total0 = -1, ev_total1 = -1;
  // layer index of encoder block l, the bottleneck and decoder block l (conv a; b = +1)
  int E(int l) const { return 2 * l; }
  int M() const { return 2 * (L - 1); }
  int D(int l) const { return 2 * (L - 1) + 2 + 2 * (L - 2 - l); }
};

namespace {

kp_status fail(kp_dn* d, kp_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
kp_status fail(kp_dn* d, kp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (d) d->err = buf;
  return st;
}

kp_status hip_fail(kp_dn* d, hipError_t e, const char* what) {
  return fail(d, e == hipErrorOutOfMemory ? KP_ERR_OOM : KP_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define DN_HIP(call, what)                      \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return hip_fail(dn, e_, what); \
  } while (0)

// --- timing marks --------------------------------------------------------------
enum { CAT_CONV = 0, CAT_WGRAD = 1 };

int mark_begin(kp_dn* dn, hipStream_t s) {
  if (dn->nev + 2 > NEVENT) return -1;
  const int e = dn->nev;
  dn->nev += 2;
  (void)hipEventRecord(dn->ev[e], s);
  return e;
}
void mark_end(kp_dn* dn, int e, int cat, double flop, hipStream_t s) {
  if (e < 0) return;
  (void)hipEventRecord(dn->ev[e + 1], s);
  dn->marks.push_back({e, e + 1, cat, flop});
}
void marks_reset(kp_dn* dn) {
  dn->marks.clear();
  dn->nev = 0;
  dn->ev_total0 = dn->ev_total1 = -1;
}

// --- workspace -------------------------------------------------------------------
kp_status ensure_work(kp_dn* dn, size_t P1, int B) {
  Work& w = dn->w;
  if (P1 <= w.cap && B <= w.bcap) return KP_OK;
  const size_t cap = P1 > w.cap ? P1 : w.cap;
  const int bcap = B > w.bcap ? B : w.bcap;
  const int L = dn->L;
  size_t c[MAX_LEVELS];
  for (int l = 0; l < L; ++l) c[l] = (size_t)dn->c[l];
  auto Pl = [&](int l) { return cap >> (2 * l); };
  size_t off = 0;
  std::vector<std::pair<void**, size_t>> plan;  // (pointer, bytes)
  auto bf = [&](uint16_t** p, size_t elems) { plan.push_back({(void**)p, elems * 2}); };
  bf(&w.x0, cap * 8);
  for (int l = 0; l < L - 1; ++l) {
    if (l > 0) bf(&w.pool[l], Pl(l) * c[l - 1]);
    bf(&w.ea[l], Pl(l) * c[l]);
    bf(&w.cat[l], Pl(l) * (c[l + 1] + c[l]));
    bf(&w.da[l], Pl(l) * c[l]);
    bf(&w.dout[l], Pl(l) * c[l]);
    bf(&w.gd[l], Pl(l) * c[l]);
    bf(&w.gdb[l], Pl(l) * c[l]);
    bf(&w.gcat[l], Pl(l) * (c[l + 1] + c[l]));
    bf(&w.ge[l], Pl(l) * c[l]);
    bf(&w.geb[l], Pl(l) * c[l]);
    if (l > 0) bf(&w.gpool[l], Pl(l) * c[l - 1]);
  }
  bf(&w.pool[L - 1], Pl(L - 1) * c[L - 2]);
  bf(&w.ma, Pl(L - 1) * c[L - 1]);
  bf(&w.mout, Pl(L - 1) * c[L - 1]);
  bf(&w.gm, Pl(L - 1) * c[L - 1]);
  bf(&w.gmb, Pl(L - 1) * c[L - 1]);
  bf(&w.gpool[L - 1], Pl(L - 1) * c[L - 2]);
  plan.push_back({(void**)&w.xq, cap * 2 * 4});
  plan.push_back({(void**)&w.ihat, cap * 4});
  plan.push_back({(void**)&w.tgt, cap * 2 * 4});
  plan.push_back({(void**)&w.out, cap * 2 * 4});
  plan.push_back({(void**)&w.go, cap * 2 * 4});
  plan.push_back({(void**)&w.sum, (size_t)bcap * 16});
  plan.push_back({(void**)&w.loss, 8});
  plan.push_back({(void**)&w.aug, (size_t)bcap * 4});
  size_t part = 0;
  for (const Layer& y : dn->layers) part = std::max(part, wgrad_part_floats(y.cout, y.cin));
  plan.push_back({(void**)&w.wpart, part * 4});
  std::vector<size_t> offs;
  for (auto& e : plan) {
    offs.push_back(off);
    off += (e.second + 255) / 256 * 256;
  }
  size_t free_b = 0, total_b = 0;
  DN_HIP(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
  if (off > free_b + w.bytes)
    return fail(dn, KP_ERR_OOM, "denoiser workspace of %zu bytes exceeds free device memory (%zu)", off,
                free_b + w.bytes);
  DN_HIP(hipDeviceSynchronize(), "synchronise before workspace reallocation");
  if (w.mem) {
    (void)hipFree(w.mem);
    w.mem = nullptr;
    w.cap = 0;
    w.bcap = 0;
    w.bytes = 0;
  }
  DN_HIP(hipMalloc(&w.mem, off), "denoiser workspace allocation");
  for (size_t k = 0; k < plan.size(); ++k) *plan[k].first = (char*)w.mem + offs[k];
  w.cap = cap;
  w.bcap = bcap;
  w.bytes = off;
  return KP_OK;
}

kp_status ensure_packed(kp_dn* dn, hipStream_t s) {
  if (dn->packed) return KP_OK;
  for (const Layer& y : dn->layers)
    pack(dn->d_p + y.w_off, y.cout, y.cin, y.cin_true, y.kp, y.kpd, dn->d_pk + y.pk_off,
         y.kpd ? dn->d_pk + y.pkd_off : nullptr, s);
  DN_HIP(hipGetLastError(), "weight packing launch");
  dn->packed = true;
  return KP_OK;
}

kp_status check_maps(kp_dn* dn, const void* a, const void* b, int32_t B, int32_t H, int32_t W) {
  if (!a || !b) return fail(dn, KP_ERR_ARG, "map pointer is NULL");
  if (B < 1) return fail(dn, KP_ERR_ARG, "batch must be >= 1 (got %d)", B);
  const int m = 1 << (dn->L - 1);
  if (H < m || W < m || H % m || W % m)
    return fail(dn, KP_ERR_ARG, "height and width must be positive multiples of %d (got %d x %d)", m, H, W);
  if ((uint64_t)B * H * W > (1ull << 24))
    return fail(dn, KP_ERR_ARG, "batch * height * width = %llu exceeds 2^24",
                (unsigned long long)((uint64_t)B * H * W));
  return KP_OK;
}

// --- network schedule --------------------------------------------------------------
double conv_flop(const Layer& y, size_t P) { return 2.0 * (double)P * 9.0 * y.cin_true * y.cout; }

void conv_fwd(kp_dn* dn, int l, const uint16_t* x, int xs, uint16_t* y, int ys, int B, int H, int W, hipStream_t s) {
  const Layer& L = dn->layers[l];
  ConvArgs a{};
  a.x = x;
  a.xs = xs;
  a.cin = L.cin;
  a.w = dn->d_pk + L.pk_off;
  a.kp = L.kp;
  a.nout = L.cout;
  a.bias = dn->d_p + L.b_off;
  a.y = y;
  a.ys = ys;
  a.B = B;
  a.H = H;
  a.W = W;
  const int e = mark_begin(dn, s);
  conv3(a, CONV_RELU, s);
  mark_end(dn, e, CAT_CONV, conv_flop(L, (size_t)B * H * W), s);
}

// input gradient of layer l: gx (stride gxs) from gz (stride cout), zero where mask <= 0
void conv_dgrad(kp_dn* dn, int l, const uint16_t* gz, uint16_t* gx, int gxs, const uint16_t* mask, int ms, int B,
                int H, int W, hipStream_t s) {
  const Layer& L = dn->layers[l];
  ConvArgs a{};
  a.x = gz;
  a.xs = L.cout;
  a.cin = L.cout;
  a.w = dn->d_pk + L.pkd_off;
  a.kp = L.kpd;
  a.nout = L.cin_true;
  a.y = gx;
  a.ys = gxs;
  a.mask = mask;
  a.ms = ms;
  a.B = B;
  a.H = H;
  a.W = W;
  const int e = mark_begin(dn, s);
  conv3(a, CONV_MASK, s);
  mark_end(dn, e, CAT_CONV, conv_flop(L, (size_t)B * H * W), s);
}

void conv_wgrad(kp_dn* dn, int l, const uint16_t* gz, const uint16_t* x, int xs, int B, int H, int W, hipStream_t s) {
  const Layer& L = dn->layers[l];
  WgradArgs a{};
  a.gz = gz;
  a.gzs = L.cout;
  a.cout = L.cout;
  a.x = x;
  a.xs = xs;
  a.cin = L.cin;
  a.cin_true = L.cin_true;
  a.gw = dn->d_g + L.w_off;
  a.gb = dn->d_g + L.b_off;
  a.part = dn->w.wpart;
  a.B = B;
  a.H = H;
  a.W = W;
  const int e = mark_begin(dn, s);
  wgrad(a, s);
  mark_end(dn, e, CAT_WGRAD, conv_flop(L, (size_t)B * H * W), s);
}

// maps -> w.out (network output: predicted fractions q', u'); activations kept
// code_all >= 0: every image transformed by that dihedral element (test-time averaging)
kp_status forward(kp_dn* dn, const double* maps, const double* target, int B, int H, int W, bool use_aug,
                  hipStream_t s, int code_all = -1) {
  Work& w = dn->w;
  const int L = dn->L;
  const int* c = dn->c;
  const size_t P1 = (size_t)B * H * W;
  auto Hl = [&](int l) { return H >> l; };
  auto Wl = [&](int l) { return W >> l; };
  zero(w.sum, (size_t)B * 16, s);
  sums(maps, B, H * W, dn->runs, w.sum, s);
  prep(maps, target, w.sum, use_aug ? w.aug : nullptr, code_all, B, H, W, dn->runs, w.x0, w.xq, w.ihat, w.tgt, s);
  // encoder
  for (int l = 0; l < L - 1; ++l) {
    const uint16_t* in = l == 0 ? w.x0 : w.pool[l];
    const int ins = l == 0 ? 8 : c[l - 1];
    conv_fwd(dn, dn->E(l), in, ins, w.ea[l], c[l], B, Hl(l), Wl(l), s);
    conv_fwd(dn, dn->E(l) + 1, w.ea[l], c[l], w.cat[l] + c[l + 1], c[l + 1] + c[l], B, Hl(l), Wl(l), s);
    pool(w.cat[l] + c[l + 1], c[l + 1] + c[l], w.pool[l + 1], c[l], B, Hl(l), Wl(l), c[l], s);
  }
  // bottleneck
  conv_fwd(dn, dn->M(), w.pool[L - 1], c[L - 2], w.ma, c[L - 1], B, Hl(L - 1), Wl(L - 1), s);
  conv_fwd(dn, dn->M() + 1, w.ma, c[L - 1], w.mout, c[L - 1], B, Hl(L - 1), Wl(L - 1), s);
  // decoder
  const uint16_t* below = w.mout;
  int bs = c[L - 1];
  for (int l = L - 2; l >= 0; --l) {
    up(below, bs, w.cat[l], c[l + 1] + c[l], B, Hl(l), Wl(l), c[l + 1], s);
    conv_fwd(dn, dn->D(l), w.cat[l], c[l + 1] + c[l], w.da[l], c[l], B, Hl(l), Wl(l), s);
    conv_fwd(dn, dn->D(l) + 1, w.da[l], c[l], w.dout[l], c[l], B, Hl(l), Wl(l), s);
    below = w.dout[l];
    bs = c[l];
  }
  head(w.dout[0], c[0], dn->d_p + dn->head_w, dn->d_p + dn->head_b, w.xq, w.out, P1, s);
  DN_HIP(hipGetLastError(), "denoiser forward launch");
  return KP_OK;
}

kp_status backward(kp_dn* dn, int B, int H, int W, hipStream_t s) {
  Work& w = dn->w;
  const int L = dn->L;
  const int* c = dn->c;
  const size_t P1 = (size_t)B * H * W;
  auto Hl = [&](int l) { return H >> l; };
  auto Wl = [&](int l) { return W >> l; };
  zero(dn->d_g, dn->n_params * 4, s);
  zero(w.loss, 8, s);
  loss(w.out, w.tgt, w.ihat, w.sum, B, H * W, w.go, w.loss, s);
  head_bwd(w.go, w.dout[0], c[0], dn->d_p + dn->head_w, dn->d_g + dn->head_w, dn->d_g + dn->head_b, w.gd[0], P1,
           s);
  // decoder, finest level first
  for (int l = 0; l < L - 1; ++l) {
    const int cc = c[l + 1] + c[l];
    conv_wgrad(dn, dn->D(l) + 1, w.gd[l], w.da[l], c[l], B, Hl(l), Wl(l), s);
    conv_dgrad(dn, dn->D(l) + 1, w.gd[l], w.gdb[l], c[l], w.da[l], c[l], B, Hl(l), Wl(l), s);
    conv_wgrad(dn, dn->D(l), w.gdb[l], w.cat[l], cc, B, Hl(l), Wl(l), s);
    conv_dgrad(dn, dn->D(l), w.gdb[l], w.gcat[l], cc, nullptr, 0, B, Hl(l), Wl(l), s);
    // gradient of the block below's output: adjoint of up, masked by its relu
    if (l + 1 < L - 1) up_bwd(w.gcat[l], cc, w.gd[l + 1], c[l + 1], w.dout[l + 1], c[l + 1], B, Hl(l), Wl(l), c[l + 1], s);
    else up_bwd(w.gcat[l], cc, w.gm, c[L - 1], w.mout, c[L - 1], B, Hl(l), Wl(l), c[L - 1], s);
  }
  // bottleneck
  conv_wgrad(dn, dn->M() + 1, w.gm, w.ma, c[L - 1], B, Hl(L - 1), Wl(L - 1), s);
  conv_dgrad(dn, dn->M() + 1, w.gm, w.gmb, c[L - 1], w.ma, c[L - 1], B, Hl(L - 1), Wl(L - 1), s);
  conv_wgrad(dn, dn->M(), w.gmb, w.pool[L - 1], c[L - 2], B, Hl(L - 1), Wl(L - 1), s);
  conv_dgrad(dn, dn->M(), w.gmb, w.gpool[L - 1], c[L - 2], nullptr, 0, B, Hl(L - 1), Wl(L - 1), s);
  // encoder, coarsest level first: skip gradient plus the pooled path
  for (int l = L - 2; l >= 0; --l) {
    const int cc = c[l + 1] + c[l];
    pool_bwd_add(w.gcat[l] + c[l + 1], cc, w.gpool[l + 1], c[l], w.cat[l] + c[l + 1], cc, w.ge[l], c[l], B, Hl(l),
                 Wl(l), c[l], s);
    conv_wgrad(dn, dn->E(l) + 1, w.ge[l], w.ea[l], c[l], B, Hl(l), Wl(l), s);
    conv_dgrad(dn, dn->E(l) + 1, w.ge[l], w.geb[l], c[l], w.ea[l], c[l], B, Hl(l), Wl(l), s);
    if (l > 0) {
      conv_wgrad(dn, dn->E(l), w.geb[l], w.pool[l], c[l - 1], B, Hl(l), Wl(l), s);
      conv_dgrad(dn, dn->E(l), w.geb[l], w.gpool[l], c[l - 1], nullptr, 0, B, Hl(l), Wl(l), s);
    } else {
      conv_wgrad(dn, dn->E(0), w.geb[0], w.x0, 8, B, H, W, s);
    }
  }
  DN_HIP(hipGetLastError(), "denoiser backward launch");
  return KP_OK;
}

kp_status check_n(kp_dn* dn, size_t n) {
  if (n != dn->n_params) return fail(dn, KP_ERR_ARG, "n = %zu but the network has %zu parameters", n, dn->n_params);
  return KP_OK;
}

}  // namespace

extern "C" {

kp_status kp_dn_create(int device, const int32_t* widths, int32_t n_levels, kp_dn** out) {
  return kp_dn_create_runs(device, widths, n_levels, 1, out);
}

kp_status kp_dn_create_runs(int device, const int32_t* widths, int32_t n_levels, int32_t runs, kp_dn** out) {
  if (!out) return KP_ERR_ARG;
  *out = nullptr;
  if (!widths || n_levels < 2 || n_levels > MAX_LEVELS || (runs != 1 && runs != 2)) return KP_ERR_ARG;
  for (int l = 0; l < n_levels; ++l)
    if (widths[l] < 16 || widths[l] > 512 || widths[l] % 16) return KP_ERR_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return KP_ERR_DEVICE;
  kp_dn* dn = new (std::nothrow) kp_dn;
  if (!dn) return KP_ERR_OOM;
  dn->device = device;
  dn->L = n_levels;
  dn->runs = runs;
  for (int l = 0; l < n_levels; ++l) dn->c[l] = widths[l];
  const int L = n_levels;
  const int* c = dn->c;
  // (cin, cout) in parameter order: encoder blocks, bottleneck, decoder blocks
  std::vector<std::pair<int, int>> io;
  for (int l = 0; l < L - 1; ++l) {
    io.push_back({l == 0 ? 4 * runs : c[l - 1], c[l]});
    io.push_back({c[l], c[l]});
  }
  io.push_back({c[L - 2], c[L - 1]});
  io.push_back({c[L - 1], c[L - 1]});
  for (int l = L - 2; l >= 0; --l) {
    io.push_back({c[l + 1] + c[l], c[l]});
    io.push_back({c[l], c[l]});
  }
  size_t off = 0, pk = 0;
  dn->layers.resize(io.size());
  for (size_t l = 0; l < io.size(); ++l) {
    Layer& y = dn->layers[l];
    y.cin_true = io[l].first;
    y.cout = io[l].second;
    y.cin = round_up(y.cin_true, 8);
    y.kp = round_up(9 * y.cin, 32);
    y.kpd = l == 0 ? 0 : round_up(9 * y.cout, 32);  // the first layer needs no input gradient
    y.w_off = off;
    off += (size_t)y.cout * 9 * y.cin_true;
    y.b_off = off;
    off += y.cout;
    y.pk_off = pk;
    pk += (size_t)y.cout * y.kp;
    pk = (pk + 127) / 128 * 128;
    y.pkd_off = pk;
    pk += (size_t)y.cin_true * y.kpd;
    pk = (pk + 127) / 128 * 128;
  }
  dn->head_w = off;
  off += 2 * (size_t)c[0];
  dn->head_b = off;
  off += 2;
  dn->n_params = off;
  dn->pk_n = pk;
  const size_t np = (off + 63) / 64 * 64;
  if (hipSetDevice(device) != hipSuccess || hipMalloc(&dn->d_p, 4 * np * sizeof(float)) != hipSuccess ||
      hipMalloc(&dn->d_pk, pk * 2) != hipSuccess) {
    kp_dn_destroy(dn);
    return KP_ERR_OOM;
  }
  dn->d_g = dn->d_p + np;
  dn->d_m = dn->d_g + np;
  dn->d_v = dn->d_m + np;
  for (auto& e : dn->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      kp_dn_destroy(dn);
      return KP_ERR_DEVICE;
    }
  zero(dn->d_p, 4 * np * sizeof(float), nullptr);
  zero(dn->d_pk, pk * 2, nullptr);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    kp_dn_destroy(dn);
    return KP_ERR_DEVICE;
  }
  *out = dn;
  return KP_OK;
}

void kp_dn_destroy(kp_dn* dn) {
  if (!dn) return;
  (void)hipSetDevice(dn->device);
  (void)hipDeviceSynchronize();
  for (void* p : {(void*)dn->d_p, (void*)dn->d_pk, dn->w.mem})
    if (p) (void)hipFree(p);
  for (auto& e : dn->ev)
    if (e) (void)hipEventDestroy(e);
  delete dn;
}

const char* kp_dn_last_error(const kp_dn* dn) { return dn ? dn->err.c_str() : "null denoiser"; }

kp_status kp_dn_num_params(const kp_dn* dn, size_t* n) {
  if (!dn || !n) return KP_ERR_ARG;
  *n = dn->n_params;
  return KP_OK;
}

kp_status kp_dn_set_params(kp_dn* dn, const float* host, size_t n) {
  if (!dn) return KP_ERR_ARG;
  if (!host) return fail(dn, KP_ERR_ARG, "host_params is NULL");
  if (kp_status st = check_n(dn, n)) return st;
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(host[k]))
      return fail(dn, KP_ERR_ARG, "parameter %zu is not finite", k);
  DN_HIP(hipSetDevice(dn->device), "hipSetDevice");
  DN_HIP(hipDeviceSynchronize(), "synchronise");
  DN_HIP(hipMemcpy(dn->d_p, host, n * 4, hipMemcpyHostToDevice), "parameter upload");
  zero(dn->d_m, n * 4, nullptr);
  zero(dn->d_v, n * 4, nullptr);
  DN_HIP(hipGetLastError(), "fill launch");
  DN_HIP(hipDeviceSynchronize(), "synchronise");
  dn->step = 0;
  dn->packed = false;
  return KP_OK;
}

static kp_status copy_out(kp_dn* dn, float* host, const float* dev, size_t n, const char* what) {
  if (!host) return fail(dn, KP_ERR_ARG, "%s destination is NULL", what);
  if (kp_status st = check_n(dn, n)) return st;
  DN_HIP(hipSetDevice(dn->device), "hipSetDevice");
  DN_HIP(hipDeviceSynchronize(), "synchronise");
  DN_HIP(hipMemcpy(host, dev, n * 4, hipMemcpyDeviceToHost), what);
  return KP_OK;
}

kp_status kp_dn_get_params(kp_dn* dn, float* host, size_t n) {
  if (!dn) return KP_ERR_ARG;
  return copy_out(dn, host, dn->d_p, n, "parameter copy");
}

kp_status kp_dn_get_grads(kp_dn* dn, float* host, size_t n) {
  if (!dn) return KP_ERR_ARG;
  return copy_out(dn, host, dn->d_g, n, "gradient copy");
}

kp_status kp_dn_get_adam(kp_dn* dn, float* m, float* v, size_t n, int32_t* step) {
  if (!dn) return KP_ERR_ARG;
  if (!step) return fail(dn, KP_ERR_ARG, "step is NULL");
  if (kp_status st = copy_out(dn, m, dn->d_m, n, "first-moment copy")) return st;
  if (kp_status st = copy_out(dn, v, dn->d_v, n, "second-moment copy")) return st;
  *step = dn->step;
  return KP_OK;
}

kp_status kp_dn_set_adam(kp_dn* dn, const float* m, const float* v, size_t n, int32_t step) {
  if (!dn) return KP_ERR_ARG;
  if (!m || !v) return fail(dn, KP_ERR_ARG, "moment array is NULL");
  if (step < 0) return fail(dn, KP_ERR_ARG, "step must be >= 0 (got %d)", step);
  if (kp_status st = check_n(dn, n)) return st;
  for (size_t k = 0; k < n; ++k)
    if (!std::isfinite(m[k]) || !std::isfinite(v[k]) || v[k] < 0.0f)
      return fail(dn, KP_ERR_ARG, "moment %zu is not finite or the second moment is negative", k);
  DN_HIP(hipSetDevice(dn->device), "hipSetDevice");
  DN_HIP(hipDeviceSynchronize(), "synchronise");
  DN_HIP(hipMemcpy(dn->d_m, m, n * 4, hipMemcpyHostToDevice), "first-moment upload");
  DN_HIP(hipMemcpy(dn->d_v, v, n * 4, hipMemcpyHostToDevice), "second-moment upload");
  dn->step = step;
  return KP_OK;
}

kp_status kp_dn_infer(kp_dn* dn, const double* d_maps, double* d_out, int32_t B, int32_t H, int32_t W,
                      void* stream) {
  if (!dn) return KP_ERR_ARG;
  if (kp_status st = check_maps(dn, d_maps, d_out, B, H, W)) return st;
  if ((const void*)d_maps == (const void*)d_out) return fail(dn, KP_ERR_ARG, "d_out may not alias d_maps");
  hipStream_t s = (hipStream_t)stream;
  DN_HIP(hipSetDevice(dn->device), "hipSetDevice");
  if (kp_status st = ensure_work(dn, (size_t)B * H * W, B)) return st;
  marks_reset(dn);
  dn->ev_total0 = mark_begin(dn, s);
  if (kp_status st = ensure_packed(dn, s)) return st;
  if (kp_status st = forward(dn, d_maps, nullptr, B, H, W, false, s)) return st;
  output(d_maps, dn->w.out, B, H * W, dn->runs, 1.0, d_out, s);
  DN_HIP(hipGetLastError(), "output launch");
  if (dn->ev_total0 >= 0) {
    dn->ev_total1 = dn->ev_total0 + 1;
    DN_HIP(hipEventRecord(dn->ev[dn->ev_total1], s), "event record");
  }
  return KP_OK;
}

kp_status kp_dn_infer_tta(kp_dn* dn, const double* d_maps, double* d_out, int32_t B, int32_t H, int32_t W,
                          void* stream) {
  if (!dn) return KP_ERR_ARG;
  if (kp_status st = check_maps(dn, d_maps, d_out, B, H, W)) return st;
  if ((const void*)d_maps == (const void*)d_out) return fail(dn, KP_ERR_ARG, "d_out may not alias d_maps");
  hipStream_t s = (hipStream_t)stream;
  DN_HIP(hipSetDevice(dn->device), "hipSetDevice");
  if (kp_status st = ensure_work(dn, (size_t)B * H * W, B)) return st;
  marks_reset(dn);
  dn->ev_total0 = mark_begin(dn, s);
  if (kp_status st = ensure_packed(dn, s)) return st;
  // quarter turns need square images; otherwise the four elements without one
  const int step = H == W ? 1 : 2, n = 8 / step;
  // the loss gradient buffer (unused by inference) accumulates the fractions
  for (int code = 0; code < 8; code += step) {
    if (kp_status st = forward(dn, d_maps, nullptr, B, H, W, false, s, code)) return st;
    tta_acc(dn->w.out, B, H, W, code, code == 0, dn->w.go, s);
  }
  output(d_maps, dn->w.go, B, H * W, dn->runs, 1.0 / n, d_out, s);
  DN_HIP(hipGetLastError(), "output launch");
  if (dn->ev_total0 >= 0) {
    dn->ev_total1 = dn->ev_total0 + 1;
    DN_HIP(hipEventRecord(dn->ev[dn->ev_total1], s), "event record");
  }
  return KP_OK;
}

kp_status kp_dn_backward(kp_dn* dn, const double* d_low, const double* d_high, int32_t B, int32_t H, int32_t W,
                         const int32_t* host_aug, double* loss_out, void* stream) {
  if (!dn) return KP_ERR_ARG;
  if (kp_status st = check_maps(dn, d_low, d_high, B, H, W)) return st;
  if (!loss_out) return fail(dn, KP_ERR_ARG, "loss is NULL");
  if (host_aug)
    for (int b = 0; b < B; ++b) {
      if (host_aug[b] < 0 || host_aug[b] > 7)
        return fail(dn, KP_ERR_ARG, "aug[%d] = %d is outside 0..7", b, host_aug[b]);
      if ((host_aug[b] & 1) && H != W)
        return fail(dn, KP_ERR_ARG, "aug[%d] = %d rotates by a quarter turn but the maps are %d x %d", b,
                    host_aug[b], H, W);
    }
  hipStream_t s = (hipStream_t)stream;
  DN_HIP(hipSetDevice(dn->device), "hipSetDevice");
  if (kp_status st = ensure_work(dn, (size_t)B * H * W, B)) return st;
  if (host_aug)
    DN_HIP(hipMemcpyAsync(dn->w.aug, host_aug, (size_t)B * 4, hipMemcpyHostToDevice, s), "augmentation upload");
  marks_reset(dn);
  dn->ev_total0 = mark_begin(dn, s);
  if (kp_status st = ensure_packed(dn, s)) return st;
  if (kp_status st = forward(dn, d_low, d_high, B, H, W, host_aug != nullptr, s)) return st;
  if (kp_status st = backward(dn, B, H, W, s)) return st;
  if (dn->ev_total0 >= 0) {
    dn->ev_total1 = dn->ev_total0 + 1;
    DN_HIP(hipEventRecord(dn->ev[dn->ev_total1], s), "event record");
  }
  double l = 0.0;
  DN_HIP(hipMemcpyAsync(&l, dn->w.loss, 8, hipMemcpyDeviceToHost, s), "loss copy");
  DN_HIP(hipStreamSynchronize(s), "synchronise");
  *loss_out = l;
  return KP_OK;
}

kp_status kp_dn_adam_step(kp_dn* dn, float lr, void* stream) {
  if (!dn) return KP_ERR_ARG;
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(dn, KP_ERR_ARG, "lr must be finite and > 0");
  hipStream_t s = (hipStream_t)stream;
  DN_HIP(hipSetDevice(dn->device), "hipSetDevice");
  dn->step += 1;
  adam(dn->d_p, dn->d_g, dn->d_m, dn->d_v, dn->n_params, lr, dn->step, s);
  DN_HIP(hipGetLastError(), "Adam launch");
  dn->packed = false;
  return KP_OK;
}

kp_status kp_dn_train_step(kp_dn* dn, const double* d_low, const double* d_high, int32_t B, int32_t H, int32_t W,
                           const int32_t* host_aug, float lr, double* loss_out, void* stream) {
  if (!dn) return KP_ERR_ARG;
  if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(dn, KP_ERR_ARG, "lr must be finite and > 0");
  if (kp_status st = kp_dn_backward(dn, d_low, d_high, B, H, W, host_aug, loss_out, stream)) return st;
  return kp_dn_adam_step(dn, lr, stream);
}

kp_status kp_dn_get_timing(kp_dn* dn, kp_dn_timing* out) {
  if (!dn || !out) return KP_ERR_ARG;
  if (dn->ev_total1 < 0) return fail(dn, KP_ERR_STATE, "no timed denoiser call yet");
  DN_HIP(hipEventSynchronize(dn->ev[dn->ev_total1]), "event synchronise");
  kp_dn_timing t{};
  float ms = 0.f;
  DN_HIP(hipEventElapsedTime(&ms, dn->ev[dn->ev_total0], dn->ev[dn->ev_total1]), "event time");
  t.ms_total = ms;
  for (const auto& m : dn->marks) {
    DN_HIP(hipEventElapsedTime(&ms, dn->ev[m.a], dn->ev[m.b]), "event time");
    if (m.cat == CAT_CONV) {
      t.ms_conv += ms;
      t.conv_flop += m.flop;
    } else {
      t.ms_wgrad += ms;
      t.wgrad_flop += m.flop;
    }
  }
  t.ms_other = t.ms_total - t.ms_conv - t.ms_wgrad;
  *out = t;
  return KP_OK;
}

}  // extern "C"
