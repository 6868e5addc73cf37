// Mass assignment of a particle catalogue to one or two density grids.
//
// The paper does not specify the assignment; the estimator of its standard
// estimator section needs a density field delta(x) on a grid. This uses cloud-
// in-cell (CIC, weights prod_a (1 - d_a) or d_a to the 8 surrounding nodes)
// or nearest grid point (NGP), with an optional second grid built from the
// positions shifted by half a cell (interlacing).
//
// Positions are grid units in [0, N); a position outside that range or not
// finite sets bit 0 of the error word and is skipped.
#include "bsp_internal.h"

namespace bsp {

template <int WINDOW>
__global__ __launch_bounds__(256) void k_assign(const float* __restrict__ ux, const float* __restrict__ uy,
                                                const float* __restrict__ uz, const float* __restrict__ w,
                                                int64_t np, int n, int interlace, float* __restrict__ grids,
                                                double* __restrict__ wsum, int32_t* __restrict__ err) {
  const int64_t n3 = (int64_t)n * n * n;
  const float fn = (float)n;
  double acc = 0.0;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const float x = ux[i], y = uy[i], z = uz[i];
    const float wt = w ? w[i] : 1.0f;
    if (!(x >= 0.0f && x < fn && y >= 0.0f && y < fn && z >= 0.0f && z < fn && wt == wt)) {
      bad = 1;
      continue;
    }
    acc += (double)wt;
    for (int s = 0; s <= interlace; ++s) {
      float vx = x, vy = y, vz = z;
      if (s) {
        vx += 0.5f;
        vy += 0.5f;
        vz += 0.5f;
        if (vx >= fn) vx -= fn;
        if (vy >= fn) vy -= fn;
        if (vz >= fn) vz -= fn;
      }
      float* g = grids + (int64_t)s * n3;
      if constexpr (WINDOW == 0) {
        int ix = (int)floorf(vx + 0.5f), iy = (int)floorf(vy + 0.5f), iz = (int)floorf(vz + 0.5f);
        if (ix >= n) ix -= n;
        if (iy >= n) iy -= n;
        if (iz >= n) iz -= n;
        unsafeAtomicAdd(g + ((int64_t)ix * n + iy) * n + iz, wt);
      } else {
        const int ix = (int)floorf(vx), iy = (int)floorf(vy), iz = (int)floorf(vz);
        const float dx = vx - (float)ix, dy = vy - (float)iy, dz = vz - (float)iz;
        const int jx = (ix + 1 == n) ? 0 : ix + 1;
        const int jy = (iy + 1 == n) ? 0 : iy + 1;
        const int jz = (iz + 1 == n) ? 0 : iz + 1;
        const float wx[2] = {1.0f - dx, dx}, wy[2] = {1.0f - dy, dy}, wz[2] = {1.0f - dz, dz};
        const int64_t px[2] = {(int64_t)ix * n * n, (int64_t)jx * n * n};
        const int64_t py[2] = {(int64_t)iy * n, (int64_t)jy * n};
        const int pz[2] = {iz, jz};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const float wab = wt * wx[a] * wy[b];
#pragma unroll
            for (int c = 0; c < 2; ++c) unsafeAtomicAdd(g + px[a] + py[b] + pz[c], wab * wz[c]);
          }
      }
    }
  }
  // block reduction of the weight sum
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0.0) unsafeAtomicAdd(wsum, red[0]);
  if (bad) atomicOr(err, 1);
}

hipError_t launch_assign(const float* ux, const float* uy, const float* uz, const float* w, int64_t np,
                         int n, int window, int interlace, float* grids, double* wsum, int32_t* err,
                         hipStream_t s) {
  if (np <= 0) return hipSuccess;
  int64_t blocks = (np + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (window == 0)
    hipLaunchKernelGGL((k_assign<0>), dim3((unsigned)blocks), dim3(256), 0, s, ux, uy, uz, w, np, n,
                       interlace, grids, wsum, err);
  else
    hipLaunchKernelGGL((k_assign<1>), dim3((unsigned)blocks), dim3(256), 0, s, ux, uy, uz, w, np, n,
                       interlace, grids, wsum, err);
  return hipGetLastError();
}

}  // namespace bsp
