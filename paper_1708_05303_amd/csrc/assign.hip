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
//
// Reproducible sums: node sums and the weight sum are accumulated as 64-bit
// integers in units of 2^-S (fixed point), so their value does not depend on
// the order of the atomic additions. Each contribution w prod(weights) is
// formed in FP64 and rounded once to a multiple of 2^-S; S = min(36,
// 62 - e - l) with max|w| < 2^e and np < 2^l keeps every sum below 2^62. For
// unit weights and positions that are multiples of 2^-12 (as the catalogue
// generator writes them) every CIC weight product is a multiple of 2^-36, so
// the sums are exact and each grid value is the exact node sum rounded once
// to FP32.
#include "bsp_internal.h"

namespace bsp {

// Fixed-point scale exponent from the largest |w| (as FP32 bits; unit weights
// give 1.0) and the particle count.
__device__ __forceinline__ int fixed_shift(unsigned wmax_bits, int64_t np) {
  const float wmax = __uint_as_float(wmax_bits);
  int e = 0;
  if (wmax > 0.0f) (void)frexpf(wmax, &e);
  const int l = 64 - __clzll((unsigned long long)(np > 0 ? np : 1));
  const int sh = 62 - e - l;
  return sh < 36 ? sh : 36;
}

__device__ __forceinline__ long long to_fixed(double v, int sh) { return __double2ll_rn(ldexp(v, sh)); }

__device__ __forceinline__ void lds_add_fixed(long long* a, long long v) {
  atomicAdd(reinterpret_cast<unsigned long long*>(a), (unsigned long long)v);
}

// Fills n 32-bit words with v (used instead of hipMemsetAsync, so that the
// stream's work is kernels only and can be captured in a graph).
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

hipError_t launch_fill_u32(void* p, uint32_t v, int64_t words, hipStream_t s) {
  if (words <= 0) return hipSuccess;
  int64_t blocks = (words + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<uint32_t*>(p), v, words);
  return hipGetLastError();
}

// Fills n floats with values uniform in [-1, 1) from a counter hash of the
// index (the autotuner times the reduction on such fields: matrix units draw
// more power, and run at lower clocks, on varying operands than on constants).
__global__ __launch_bounds__(256) void k_fill_noise(float* __restrict__ p, int64_t n, uint32_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t h = (uint64_t)i * 0x9e3779b97f4a7c15ull + seed;
    h ^= h >> 31;
    h *= 0xbf58476d1ce4e5b9ull;
    h ^= h >> 29;
    p[i] = (float)(int32_t)(uint32_t)(h >> 32) * 4.656612873077393e-10f;
  }
}

hipError_t launch_fill_noise(float* p, int64_t n, uint32_t seed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_noise, dim3((unsigned)blocks), dim3(256), 0, s, p, n, seed);
  return hipGetLastError();
}

// wmax_bits[0] = max |w| over the finite weights, as FP32 bits (|w| >= 0, so the
// integer order of the bits is the order of the values).
__global__ __launch_bounds__(256) void k_weight_max(const float* __restrict__ w, const int64_t* __restrict__ npd,
                                                    unsigned* __restrict__ wmax_bits) {
  const int64_t np = *npd;
  unsigned m = 0u;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const float a = fabsf(w[i]);
    if (a == a && a <= 3.4e38f) m = max(m, __float_as_uint(a));
  }
  for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off));
  if ((threadIdx.x & 63) == 0 && m) atomicMax(wmax_bits, m);
}

// Global fixed-point assignment into int64 grids (zeroed by the caller) and
// a fixed-point weight sum wsum_fx[0].
template <int WINDOW>
__global__ __launch_bounds__(256) void k_assign_fixed(const float* __restrict__ ux, const float* __restrict__ uy,
                                                      const float* __restrict__ uz, const float* __restrict__ w,
                                                      const int64_t* __restrict__ npd, int n, int interlace,
                                                      const unsigned* __restrict__ wmax_bits,
                                                      unsigned long long* __restrict__ gfx,
                                                      unsigned long long* __restrict__ wsum_fx,
                                                      int32_t* __restrict__ err) {
  const int64_t np = *npd;
  const int64_t n3 = (int64_t)n * n * n;
  const float fn = (float)n;
  const int sh = fixed_shift(*wmax_bits, np);
  long long acc = 0;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const float x = ux[i], y = uy[i], z = uz[i];
    const float wt = w ? w[i] : 1.0f;
    if (!(x >= 0.0f && x < fn && y >= 0.0f && y < fn && z >= 0.0f && z < fn && wt == wt)) {
      bad = 1;
      continue;
    }
    acc += to_fixed((double)wt, sh);
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
      unsigned long long* g = gfx + (int64_t)s * n3;
      if constexpr (WINDOW == 0) {
        int ix = (int)floorf(vx + 0.5f), iy = (int)floorf(vy + 0.5f), iz = (int)floorf(vz + 0.5f);
        if (ix >= n) ix -= n;
        if (iy >= n) iy -= n;
        if (iz >= n) iz -= n;
        atomicAdd(g + ((int64_t)ix * n + iy) * n + iz, (unsigned long long)to_fixed((double)wt, sh));
      } else {
        const int ix = (int)floorf(vx), iy = (int)floorf(vy), iz = (int)floorf(vz);
        const float dx = vx - (float)ix, dy = vy - (float)iy, dz = vz - (float)iz;
        const int jx = (ix + 1 == n) ? 0 : ix + 1;
        const int jy = (iy + 1 == n) ? 0 : iy + 1;
        const int jz = (iz + 1 == n) ? 0 : iz + 1;
        const double wx[2] = {1.0 - (double)dx, (double)dx}, wy[2] = {1.0 - (double)dy, (double)dy},
                     wz[2] = {1.0 - (double)dz, (double)dz};
        const int64_t px[2] = {(int64_t)ix * n * n, (int64_t)jx * n * n};
        const int64_t py[2] = {(int64_t)iy * n, (int64_t)jy * n};
        const int pz[2] = {iz, jz};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) {
            const double wab = (double)wt * wx[a] * wy[b];
#pragma unroll
            for (int c = 0; c < 2; ++c)
              atomicAdd(g + px[a] + py[b] + pz[c], (unsigned long long)to_fixed(wab * wz[c], sh));
          }
      }
    }
  }
  __shared__ long long red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0) atomicAdd(wsum_fx, (unsigned long long)red[0]);
  if (bad) atomicOr(err, 1);
}

// grids[i] (+)= gfx[i] 2^-S rounded to FP32; block 0 also adds the weight sum.
__global__ __launch_bounds__(256) void k_fixed_to_float(const unsigned long long* __restrict__ gfx, int64_t count,
                                                        const int64_t* __restrict__ npd,
                                                        const unsigned* __restrict__ wmax_bits,
                                                        const unsigned long long* __restrict__ wsum_fx,
                                                        int accumulate, float* __restrict__ grids,
                                                        double* __restrict__ wsum) {
  const int64_t np = *npd;
  const int sh = fixed_shift(*wmax_bits, np);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = (float)ldexp((double)(long long)gfx[i], -sh);
    grids[i] = accumulate ? grids[i] + v : v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) wsum[0] += ldexp((double)(long long)wsum_fx[0], -sh);
}

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

// ---------------------------------------------------------------------------
// Tiled assignment without global atomics on the grids: particles are counted
// by the 8 x 8 x TZ tile of their node floor(x) (the count's atomic returns each
// particle's rank within its tile, kept for the scatter) and placed at their
// tile's offset plus that rank; one workgroup per tile gathers
// the particles of its own tile and of the 7 tiles below it (a CIC or NGP
// cloud, also on the grid shifted by half a cell, reaches at most two nodes
// past floor(x)), sums their weights into LDS and writes its nodes once.
// Needs N divisible by 8 and by TZ with at least two tiles along each axis.

constexpr int TXY = 8;

__device__ __forceinline__ bool valid_particle(float x, float y, float z, float wt, float fn) {
  return x >= 0.0f && x < fn && y >= 0.0f && y < fn && z >= 0.0f && z < fn && wt == wt;
}

__global__ __launch_bounds__(256) void k_tile_count(const float* __restrict__ ux, const float* __restrict__ uy,
                                                    const float* __restrict__ uz, const float* __restrict__ w,
                                                    const int64_t* __restrict__ npd, int n, int ntx, int ntz, int tz,
                                                    int32_t* __restrict__ count, int32_t* __restrict__ rank,
                                                    const unsigned* __restrict__ wmax_bits,
                                                    unsigned long long* __restrict__ wsum_fx,
                                                    int32_t* __restrict__ err) {
  const int64_t np = *npd;
  const float fn = (float)n;
  const int sh = fixed_shift(*wmax_bits, np);
  long long acc = 0;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const float x = ux[i], y = uy[i], z = uz[i];
    const float wt = w ? w[i] : 1.0f;
    if (!valid_particle(x, y, z, wt, fn)) {
      bad = 1;
      continue;
    }
    acc += to_fixed((double)wt, sh);
    const int key = (((int)x / TXY) * ntx + (int)y / TXY) * ntz + (int)z / tz;
    rank[i] = atomicAdd(count + key, 1);
  }
  __shared__ long long red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0) atomicAdd(wsum_fx, (unsigned long long)red[0]);
  if (bad) atomicOr(err, 1);
}

// The same count with the tile histogram of each workgroup in LDS, for grids
// of at most kPrivTiles tiles: a workgroup takes a contiguous range of `per`
// particles, ranks them in its LDS histogram, then adds each nonzero bin to
// the global count with one atomic that returns the bin's base, and a second
// pass adds that base to the ranks. Few workgroups touch a tile, so the global
// atomics do not queue on the busy tiles of small clustered catalogues.
constexpr int kPrivTiles = 16384;

__global__ __launch_bounds__(256) void k_tile_count_lds(const float* __restrict__ ux, const float* __restrict__ uy,
                                                        const float* __restrict__ uz, const float* __restrict__ w,
                                                        const int64_t* __restrict__ npd, int64_t per, int n, int ntx,
                                                        int ntz, int tz, int nt, int32_t* __restrict__ count,
                                                        int32_t* __restrict__ rank,
                                                        const unsigned* __restrict__ wmax_bits,
                                                        unsigned long long* __restrict__ wsum_fx,
                                                        int32_t* __restrict__ err) {
  extern __shared__ int32_t hist[];
  const int64_t np = *npd;
  const float fn = (float)n;
  const int sh = fixed_shift(*wmax_bits, np);
  for (int k = threadIdx.x; k < nt; k += blockDim.x) hist[k] = 0;
  __syncthreads();
  const int64_t i0 = (int64_t)blockIdx.x * per;
  const int64_t i1 = i0 + per < np ? i0 + per : np;
  long long acc = 0;
  int bad = 0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const float x = ux[i], y = uy[i], z = uz[i];
    const float wt = w ? w[i] : 1.0f;
    if (!valid_particle(x, y, z, wt, fn)) {
      bad = 1;
      continue;
    }
    acc += to_fixed((double)wt, sh);
    const int key = (((int)x / TXY) * ntx + (int)y / TXY) * ntz + (int)z / tz;
    rank[i] = atomicAdd(&hist[key], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nt; k += blockDim.x)
    if (hist[k] > 0) hist[k] = atomicAdd(count + k, hist[k]);
  __syncthreads();
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const float x = ux[i], y = uy[i], z = uz[i];
    const float wt = w ? w[i] : 1.0f;
    if (!valid_particle(x, y, z, wt, fn)) continue;
    const int key = (((int)x / TXY) * ntx + (int)y / TXY) * ntz + (int)z / tz;
    rank[i] += hist[key];
  }
  __shared__ long long red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] != 0) atomicAdd(wsum_fx, (unsigned long long)red[0]);
  if (bad) atomicOr(err, 1);
}

// Exclusive prefix sum of count[0..nt) into offs[0..nt], one workgroup of 1024
// threads, each scanning a contiguous run.
__global__ __launch_bounds__(1024) void k_tile_scan(const int32_t* __restrict__ count, int nt,
                                                     int32_t* __restrict__ offs) {
  __shared__ int32_t part[1024];
  const int t = threadIdx.x;
  const int per = (nt + 1023) / 1024;
  const int b = t * per, e = min(nt, b + per);
  int s = 0;
  for (int i = b; i < e; ++i) s += count[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = b; i < e; ++i) {
    offs[i] = run;
    run += count[i];
  }
  if (t == 1023) offs[nt] = part[1023];
}

__global__ __launch_bounds__(256) void k_tile_scatter(const float* __restrict__ ux, const float* __restrict__ uy,
                                                      const float* __restrict__ uz, const float* __restrict__ w,
                                                      const int64_t* __restrict__ npd, int n, int ntx, int ntz, int tz,
                                                      const int32_t* __restrict__ offs,
                                                      const int32_t* __restrict__ rank, float4* __restrict__ sorted) {
  const int64_t np = *npd;
  const float fn = (float)n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    const float x = ux[i], y = uy[i], z = uz[i];
    const float wt = w ? w[i] : 1.0f;
    if (!valid_particle(x, y, z, wt, fn)) continue;
    const int key = (((int)x / TXY) * ntx + (int)y / TXY) * ntz + (int)z / tz;
    sorted[offs[key] + rank[i]] = make_float4(x, y, z, wt);
  }
}

template <int WINDOW, int TZ>
__global__ __launch_bounds__(256) void k_assign_tiles(const float4* __restrict__ sorted,
                                                      const int32_t* __restrict__ offs, int n, int ntx, int ntz,
                                                      int interlace, int accumulate, const int64_t* __restrict__ npd,
                                                      const unsigned* __restrict__ wmax_bits,
                                                      const unsigned long long* __restrict__ wsum_fx,
                                                      float* __restrict__ grids, double* __restrict__ wsum) {
  constexpr int CELLS = TXY * TXY * TZ;
  __shared__ long long acc[2][CELLS];
  const int tile = blockIdx.x;
  const int tzi = tile % ntz, txy = tile / ntz, tyi = txy % ntx, txi = txy / ntx;
  const int x0 = txi * TXY, y0 = tyi * TXY, z0 = tzi * TZ;
  const int sh = fixed_shift(*wmax_bits, *npd);
  for (int i = threadIdx.x; i < 2 * CELLS; i += 256) (&acc[0][0])[i] = 0;
  __syncthreads();
  const float fn = (float)n;
  for (int nb = 0; nb < 8; ++nb) {
    const int lx = (nb >> 2) & 1, ly = (nb >> 1) & 1, lz = nb & 1;  // neighbour below along x / y / z
    const int ax = txi - lx, ay = tyi - ly, az = tzi - lz;
    const int axw = ax < 0 ? ax + ntx : ax, ayw = ay < 0 ? ay + ntx : ay, azw = az < 0 ? az + ntz : az;
    const int k = (axw * ntx + ayw) * ntz + azw;
    // A particle of a lower neighbour reaches this tile only from within 1.5
    // nodes of the shared face: an offset d < size - 1.5 in its tile puts
    // x + 0.5 below x0 - 1, so neither its CIC nodes floor(v), floor(v) + 1 nor
    // its NGP node reach x0 on either grid (and a shifted position that wraps
    // round the box has d >= size - 0.5).
    const float fx = (float)(axw * TXY), fy = (float)(ayw * TXY), fz = (float)(azw * TZ);
    const int e = offs[k + 1];
    for (int i = offs[k] + threadIdx.x; i < e; i += 256) {
      const float4 pt = sorted[i];
      if ((lx && pt.x - fx < TXY - 1.5f) || (ly && pt.y - fy < TXY - 1.5f) || (lz && pt.z - fz < TZ - 1.5f)) continue;
      for (int s = 0; s <= interlace; ++s) {
        float vx = pt.x, vy = pt.y, vz = pt.z;
        if (s) {
          vx += 0.5f;
          vy += 0.5f;
          vz += 0.5f;
          if (vx >= fn) vx -= fn;
          if (vy >= fn) vy -= fn;
          if (vz >= fn) vz -= fn;
        }
        if constexpr (WINDOW == 0) {
          int ix = (int)floorf(vx + 0.5f), iy = (int)floorf(vy + 0.5f), iz = (int)floorf(vz + 0.5f);
          if (ix >= n) ix -= n;
          if (iy >= n) iy -= n;
          if (iz >= n) iz -= n;
          const int lx = ix - x0, ly = iy - y0, lz = iz - z0;
          if ((unsigned)lx < (unsigned)TXY && (unsigned)ly < (unsigned)TXY && (unsigned)lz < (unsigned)TZ)
            lds_add_fixed(&acc[s][(lx * TXY + ly) * TZ + lz], to_fixed((double)pt.w, sh));
        } else {
          const int ix = (int)floorf(vx), iy = (int)floorf(vy), iz = (int)floorf(vz);
          const float dx = vx - (float)ix, dy = vy - (float)iy, dz = vz - (float)iz;
          const double wx[2] = {1.0 - (double)dx, (double)dx}, wy[2] = {1.0 - (double)dy, (double)dy},
                       wz[2] = {1.0 - (double)dz, (double)dz};
#pragma unroll
          for (int a = 0; a < 2; ++a) {
            int cx = ix + a;
            if (cx == n) cx = 0;
            const int lx = cx - x0;
            if ((unsigned)lx >= (unsigned)TXY) continue;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
              int cy = iy + b;
              if (cy == n) cy = 0;
              const int ly = cy - y0;
              if ((unsigned)ly >= (unsigned)TXY) continue;
              const double wab = (double)pt.w * wx[a] * wy[b];
#pragma unroll
              for (int c = 0; c < 2; ++c) {
                int cz = iz + c;
                if (cz == n) cz = 0;
                const int lz = cz - z0;
                if ((unsigned)lz < (unsigned)TZ)
                  lds_add_fixed(&acc[s][(lx * TXY + ly) * TZ + lz], to_fixed(wab * wz[c], sh));
              }
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // one float4 of a z row per thread
  const int64_t n3 = (int64_t)n * n * n;
  for (int s = 0; s <= interlace; ++s) {
    float* g = grids + (int64_t)s * n3;
    for (int v = threadIdx.x; v < CELLS / 4; v += 256) {
      const int c = v * 4;
      const int lz = c % TZ, ly = (c / TZ) % TXY, lx = c / (TZ * TXY);
      float4* dst = reinterpret_cast<float4*>(g + ((int64_t)(x0 + lx) * n + (y0 + ly)) * n + z0 + lz);
      float4 val = make_float4((float)ldexp((double)acc[s][c], -sh), (float)ldexp((double)acc[s][c + 1], -sh),
                               (float)ldexp((double)acc[s][c + 2], -sh), (float)ldexp((double)acc[s][c + 3], -sh));
      if (accumulate) {
        const float4 old = *dst;
        val.x += old.x;
        val.y += old.y;
        val.z += old.z;
        val.w += old.w;
      }
      typedef float F4 __attribute__((ext_vector_type(4)));
      __builtin_nontemporal_store(F4{val.x, val.y, val.z, val.w}, reinterpret_cast<F4*>(dst));
    }
  }
  // the count kernel, earlier on the stream, has finished the weight sum
  if (tile == 0 && threadIdx.x == 0) wsum[0] += ldexp((double)(long long)wsum_fx[0], -sh);
}

// Tile depth along z: 32 nodes keeps the two grids' int64 node sums of an
// 8 x 8 x 32 tile at 32 KB, so four workgroups share a CU (64-deep tiles left
// under two waves per SIMD to hide the gather's memory latency).
static int tile_tz(int n) {
  if (n % TXY != 0 || n / TXY < 2) return 0;
  for (int tz = 32; tz >= 8; tz >>= 1)
    if (n % tz == 0 && n / tz >= 2) return tz;
  return 0;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The tiled path runs one workgroup per tile: with fewer than 512 tiles
// (grids of 96 nodes a side or less) it cannot fill the GPU and the
// global-atomic kernel is faster.
bool assign_tiled_preferred(int n) {
  const int tz = tile_tz(n);
  return tz && (int64_t)(n / TXY) * (n / TXY) * (n / tz) >= 512;
}

// 256 bytes at the head of an assignment scratch: the largest |w| (FP32 bits)
// at byte 0, the fixed-point weight sum at byte 8 and the particle count the
// kernels read at byte 16 (unless the caller points them at its own).
constexpr size_t kHead = 256;

__global__ void k_set_i64(int64_t* __restrict__ p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_i64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

size_t assign_tiled_bytes(int64_t np, int n) {
  const int tz = tile_tz(n);
  if (!tz || np <= 0 || np > (int64_t)INT32_MAX) return 0;
  const int64_t nt = (int64_t)(n / TXY) * (n / TXY) * (n / tz);
  return kHead + align256((size_t)np * sizeof(float4)) + 2 * align256((size_t)(nt + 1) * sizeof(int32_t)) +
         align256((size_t)np * sizeof(int32_t));
}

size_t assign_fixed_bytes(int n, int interlace) { return kHead + (size_t)(1 + interlace) * n * n * n * 8; }

// Head of an assignment scratch: zero the weight sum and set the largest |w|
// (1.0 for unit weights, else from the weights). Kernels only.
// npd: the caller's device-side count, or null: np is stored at byte 16 of
// the head; returns through npd_out the pointer the kernels read.
static hipError_t fixed_head(const float* w, int64_t np, const int64_t* npd, unsigned* head,
                             const int64_t** npd_out, hipStream_t s) {
  hipError_t e = launch_fill_u32(head, 0u, kHead / 4, s);
  if (e != hipSuccess) return e;
  if (!npd) {
    int64_t* slot = reinterpret_cast<int64_t*>(reinterpret_cast<char*>(head) + 16);
    e = launch_set_i64(slot, np, s);
    if (e != hipSuccess) return e;
    npd = slot;
  }
  *npd_out = npd;
  if (!w) return launch_fill_u32(head, 0x3f800000u, 1, s);
  int64_t blocks = (np + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_weight_max, dim3((unsigned)blocks), dim3(256), 0, s, w, npd, head);
  return hipGetLastError();
}

hipError_t launch_assign_tiled(const float* ux, const float* uy, const float* uz, const float* w, int64_t np, int n,
                               int window, int interlace, int accumulate, float* grids, double* wsum, int32_t* err,
                               void* scratch, size_t scratch_bytes, hipStream_t s, const int64_t* npd) {
  const int tz = tile_tz(n);
  const size_t need = assign_tiled_bytes(np, n);
  if (!tz || need == 0 || need > scratch_bytes || !scratch || interlace < 0 || interlace > 1)
    return hipErrorInvalidValue;
  const int ntx = n / TXY, ntz = n / tz;
  const int nt = ntx * ntx * ntz;
  unsigned* head = reinterpret_cast<unsigned*>(scratch);
  unsigned long long* wsum_fx = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(scratch) + 8);
  char* base = reinterpret_cast<char*>(scratch) + kHead;
  float4* sorted = reinterpret_cast<float4*>(base);
  int32_t* count = reinterpret_cast<int32_t*>(base + align256((size_t)np * sizeof(float4)));
  int32_t* offs = count + align256((size_t)(nt + 1) * sizeof(int32_t)) / sizeof(int32_t);
  int32_t* rank = offs + align256((size_t)(nt + 1) * sizeof(int32_t)) / sizeof(int32_t);
  hipError_t e = launch_fill_u32(count, 0u, nt, s);
  if (e != hipSuccess) return e;
  const int64_t* np_dev = nullptr;
  e = fixed_head(w, np, npd, head, &np_dev, s);
  if (e != hipSuccess) return e;
  int64_t blocks = (np + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (nt <= kPrivTiles) {
    // about 8 particles per thread, and at most 1024 workgroups touching a tile
    int64_t per = 2048;
    while ((np + per - 1) / per > 1024) per *= 2;
    const int64_t cb = (np + per - 1) / per;
    hipLaunchKernelGGL(k_tile_count_lds, dim3((unsigned)cb), dim3(256), (size_t)nt * sizeof(int32_t), s, ux, uy, uz,
                       w, np_dev, per, n, ntx, ntz, tz, nt, count, rank, head, wsum_fx, err);
  } else {
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)blocks), dim3(256), 0, s, ux, uy, uz, w, np_dev, n, ntx, ntz, tz,
                       count, rank, head, wsum_fx, err);
  }
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, count, nt, offs);
  hipLaunchKernelGGL(k_tile_scatter, dim3((unsigned)blocks), dim3(256), 0, s, ux, uy, uz, w, np_dev, n, ntx, ntz, tz,
                     offs, rank, sorted);
#define TCASE(WIN, TZV)                                                                                         if (window == WIN && tz == TZV) {                                                                               hipLaunchKernelGGL((k_assign_tiles<WIN, TZV>), dim3((unsigned)nt), dim3(256), 0, s, sorted, offs, n, ntx,                        ntz, interlace, accumulate, np_dev, head, wsum_fx, grids, wsum);                                                        return hipGetLastError();                                                                                   }
  TCASE(0, 32) TCASE(0, 16) TCASE(0, 8) TCASE(1, 32) TCASE(1, 16) TCASE(1, 8)
#undef TCASE
  return hipErrorInvalidValue;
}

hipError_t launch_assign(const float* ux, const float* uy, const float* uz, const float* w, int64_t np,
                         int n, int window, int interlace, int accumulate, float* grids, double* wsum, int32_t* err,
                         void* scratch, size_t scratch_bytes, hipStream_t s, const int64_t* npd) {
  const int64_t count = (int64_t)(1 + interlace) * n * n * n;
  if (np <= 0) {
    if (accumulate) return hipSuccess;
    return launch_fill_u32(grids, 0u, count, s);
  }
  int64_t blocks = (np + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (scratch && scratch_bytes >= assign_fixed_bytes(n, interlace)) {
    // fixed point: int64 node sums, converted (and added) once
    unsigned* head = reinterpret_cast<unsigned*>(scratch);
    unsigned long long* wsum_fx = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(scratch) + 8);
    unsigned long long* gfx = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(scratch) + kHead);
    hipError_t e = launch_fill_u32(gfx, 0u, 2 * count, s);
    if (e != hipSuccess) return e;
    const int64_t* np_dev = nullptr;
    e = fixed_head(w, np, npd, head, &np_dev, s);
    if (e != hipSuccess) return e;
    if (window == 0)
      hipLaunchKernelGGL((k_assign_fixed<0>), dim3((unsigned)blocks), dim3(256), 0, s, ux, uy, uz, w, np_dev, n,
                         interlace, head, gfx, wsum_fx, err);
    else
      hipLaunchKernelGGL((k_assign_fixed<1>), dim3((unsigned)blocks), dim3(256), 0, s, ux, uy, uz, w, np_dev, n,
                         interlace, head, gfx, wsum_fx, err);
    int64_t cb = (count + 255) / 256;
    if (cb > 16384) cb = 16384;
    hipLaunchKernelGGL(k_fixed_to_float, dim3((unsigned)cb), dim3(256), 0, s, gfx, count, np_dev, head, wsum_fx,
                       accumulate, grids, wsum);
    return hipGetLastError();
  }
  // no scratch: FP32 atomics on the grids (summation order varies between runs)
  if (npd) return hipErrorInvalidValue;  // a device-side count needs the fixed-point path
  if (!accumulate) {
    hipError_t e = launch_fill_u32(grids, 0u, count, s);
    if (e != hipSuccess) return e;
  }
  if (window == 0)
    hipLaunchKernelGGL((k_assign<0>), dim3((unsigned)blocks), dim3(256), 0, s, ux, uy, uz, w, np, n,
                       interlace, grids, wsum, err);
  else
    hipLaunchKernelGGL((k_assign<1>), dim3((unsigned)blocks), dim3(256), 0, s, ux, uy, uz, w, np, n,
                       interlace, grids, wsum, err);
  return hipGetLastError();
}

}  // namespace bsp
