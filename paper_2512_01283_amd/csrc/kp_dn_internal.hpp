// kp_dn_internal.hpp -- launch interface between the denoiser's host code
// (kp_dn_api.cpp) and its kernels (kp_denoiser.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace kp {
namespace dn {

enum { CONV_RELU = 0, CONV_LINEAR = 1, CONV_MASK = 2 };

// pixel count from which convolutions use the LDS-tiled kernel (256 pixels per workgroup)
constexpr size_t CONV_TILED_MIN_PIXELS = 1024;  // from here on the LDS-staged kernel

// y[p][n] (stride ys) from x[p][c] (stride xs, cin channels per tap, cin % 8 == 0)
// and GEMM weights w[nout][kp] (kp % 32 == 0, kp >= 9 cin, nout % 16 == 0).
struct ConvArgs {
  const uint16_t* x;
  int xs, cin;
  const uint16_t* w;
  int kp, nout;
  const float* bias;     // CONV_RELU / CONV_LINEAR
  uint16_t* y;
  int ys;
  const uint16_t* mask;  // CONV_MASK: zero the output where mask[p][n] <= 0 (none if null)
  int ms;
  int B, H, W;
};

// gw[cout][9][cin_true] += gradient of a conv layer's weights from the
// gradient gz[p][co] (stride gzs) of its pre-activation output and its input
// x[p][c] (stride xs, cin channels per tap, cin % 8 == 0, cout % 16 == 0).
struct WgradArgs {
  const uint16_t* gz;
  int gzs, cout;
  const uint16_t* x;
  int xs, cin, cin_true;
  float* gw;  // weight gradient [cout][9][cin_true], accumulated
  float* gb;  // bias gradient [cout], accumulated
  float* part;  // k_wgrad_halo's partial blocks, wgrad_part_floats(cout, cin) floats
  int B, H, W;
  int chunk, nch, ktiles, mtiles;  // set by the launcher
};

// Weight-gradient work split: 64 x 64 (cout, 9 cin) tiles times nch pixel
// chunks of `chunk` pixels.
constexpr int WG_SLAB = 128;        // pixels per LDS slab
constexpr int WG_TARGET = 1024;     // workgroups per launch to aim for
constexpr int WG_MIN_CHUNK = 1024;  // fewest pixels per chunk
struct WgradPlan {
  int ktiles, mtiles, nch, chunk;
};
WgradPlan wgrad_plan(int cout, int cin, size_t P);
// k_wgrad_halo (cin >= 48): 64 x 64 (co, c) channel tiles times nch chunks of
// `chunk` pixel tiles of 8 x 16
WgradPlan wgrad_halo_plan(int cout, int cin, int B, int H, int W);
// scratch of the partial blocks k_wgrad_halo writes for a layer at any image
// size (0 where the layer keeps k_wgrad)
size_t wgrad_part_floats(int cout, int cin);

void conv3(const ConvArgs& a, int mode, hipStream_t s);
void wgrad(WgradArgs a, hipStream_t s);
void pool(const uint16_t* x, int xs, uint16_t* y, int ys, int B, int H, int W, int C, hipStream_t s);
void up(const uint16_t* x, int xs, uint16_t* y, int ys, int B, int H, int W, int C, hipStream_t s);
void up_bwd(const uint16_t* gy, int gys, uint16_t* gx, int gxs, const uint16_t* mask, int ms, int B, int H, int W,
            int C, hipStream_t s);
void pool_bwd_add(const uint16_t* a, int as, const uint16_t* g, int gs, const uint16_t* mask, int ms, uint16_t* dst,
                  int ds, int B, int H, int W, int C, hipStream_t s);
void sums(const double* maps, int B, int HW, int runs, double* sum, hipStream_t s);
void prep(const double* maps, const double* target, const double* sum, const int32_t* aug, int code_all, int B,
          int H, int W, int runs, uint16_t* x, float* xq, float* ihat, float* tgt, hipStream_t s);
void head(const uint16_t* d, int C, const float* hw, const float* hb, const float* xq, float* out, size_t P,
          hipStream_t s);
void loss(const float* out, const float* tgt, const float* ihat, const double* sum, int B, int HW, float* go,
          double* l, hipStream_t s);
void head_bwd(const float* go, const uint16_t* d, int C, const float* hw, float* ghw, float* ghb, uint16_t* gd,
              size_t P, hipStream_t s);
void tta_acc(const float* out, int B, int H, int W, int code, bool first, float* acc, hipStream_t s);
void output(const double* maps, const float* out, int B, int HW, int runs, double scale, double* dst,
            hipStream_t s);
void adam(float* p, const float* g, float* m, float* v, size_t n, float lr, int t, hipStream_t s);
void pack(const float* wf, int cout, int cin, int cin_true, int kp, int kpd, uint16_t* w, uint16_t* wd,
          hipStream_t s);
void zero(void* p, size_t bytes, hipStream_t s);

}  // namespace dn
}  // namespace kp
