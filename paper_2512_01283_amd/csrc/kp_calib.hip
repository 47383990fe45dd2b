// kp_calib.hip -- device calibration for the transport's roofline (not part
// of the method; loaded only by bench.py as libkpcalib.so).
//
// 64-byte-line FP64 atomics: the transport's tally flush adds six FP64
// values to the 64-byte block of a cell, wave-cooperatively (lane L adds
// component L % 6 of block L / 6).  This kernel does exactly that over the
// blocks of a [256^3][8] FP64 array in one of two orders: uniformly random
// (no locality at all) or consecutive (every line's neighbours follow it:
// the most locality the pattern can have, so its rate bounds the flush).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// splitmix64 finaliser: block index of line e (uniform over ncell)
__device__ __forceinline__ uint32_t line_of(uint64_t e, uint64_t ncell) {
  uint64_t z = e + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (uint32_t)(z % ncell);
}

// block of line e: pattern 0 uniformly random, 1 consecutive
__global__ void k_lines(uint32_t* idx, int64_t n, uint64_t ncell, int pattern) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    idx[e] = pattern ? (uint32_t)((uint64_t)e % ncell) : line_of((uint64_t)e, ncell);
}

__global__ void k_atomic_lines(double* __restrict__ t, const uint32_t* __restrict__ idx, int64_t n, int comps) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int g = 64 / comps;
  const int slot = lane / comps, k = lane - slot * comps;
  for (int64_t base = wave * g; base < n; base += nwaves * g) {
    const int64_t e = base + slot;
    if (slot < g && e < n) unsafeAtomicAdd(t + (size_t)idx[e] * 8 + k, 1.0);
  }
}

}  // namespace

extern "C" {

// Lines per second of the line atomic pattern above in order `pattern` (0
// uniformly random, 1 consecutive): `lines` (1 .. 2^28) blocks of `comps`
// (1..8) FP64 values each, best of `reps` (>= 1) launches timed with HIP
// events, on HIP device `device`.  Allocates and frees its own 1 GiB array.
// Returns 0 on success, 1 for an argument out of range, else a hipError_t.
int kpcal_atomic_lines_order(int device, int64_t lines, int comps, int reps, int pattern, double* lines_per_s) {
  if (lines < 1 || lines > (1ll << 28) || comps < 1 || comps > 8 || reps < 1 || !lines_per_s ||
      (pattern != 0 && pattern != 1))
    return 1;
  hipError_t e = hipSetDevice(device);
  if (e != hipSuccess) return (int)e;
  const uint64_t ncell = 256ull * 256ull * 256ull;
  double* t = nullptr;
  uint32_t* idx = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float best = -1.f;
  if ((e = hipMalloc(&t, ncell * 64)) != hipSuccess) goto done;
  if ((e = hipMalloc(&idx, (size_t)lines * 4)) != hipSuccess) goto done;
  if ((e = hipMemset(t, 0, ncell * 64)) != hipSuccess) goto done;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) goto done;
  hipLaunchKernelGGL(k_lines, dim3(4096), dim3(256), 0, 0, idx, lines, ncell, pattern);
  for (int r = 0; r < reps; ++r) {
    if ((e = hipEventRecord(e0, 0)) != hipSuccess) goto done;
    hipLaunchKernelGGL(k_atomic_lines, dim3(4096), dim3(256), 0, 0, t, idx, lines, comps);
    if ((e = hipEventRecord(e1, 0)) != hipSuccess) goto done;
    if ((e = hipEventSynchronize(e1)) != hipSuccess) goto done;
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) goto done;
    if (best < 0.f || ms < best) best = ms;
  }
  *lines_per_s = (double)lines / (best * 1e-3);
  e = hipSuccess;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (idx) (void)hipFree(idx);
  if (t) (void)hipFree(t);
  return (int)e;
}

// the uniformly random order
int kpcal_atomic_lines(int device, int64_t lines, int comps, int reps, double* lines_per_s) {
  return kpcal_atomic_lines_order(device, lines, comps, reps, 0, lines_per_s);
}

}  // extern "C"
