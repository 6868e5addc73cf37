// Integrated bispectrum multipoles (Sec. 3.4, eq. integBisp and the RSD
// estimator after it): the grid is cut into s^3 cubic sub-volumes of side
// M = N / s; each sub-volume's mean overdensity dbar_i and power-spectrum
// multipoles P^(l)_i(k) are formed from one batched real-to-complex transform
// of all sub-volumes, and iB^(l)(k) = (1/N_s) sum_i P^(l)_i(k) dbar_i.
//
// By default the line of sight inside a sub-volume is the single unit vector
// e_i from the observer to the sub-volume centre (z for plane-parallel plans),
// so P^(l)_i needs no line-of-sight weighted transforms:
//   P^(l)_i(k_b) = V_s sum_{n in b} (2l+1) L_l(nhat . e_i) |F_i(n) / W(n)|^2 / (M^6 N_b);
// on request the line of sight varies over the nodes (below).
#include "bsp_internal.h"

namespace bsp {

// out[i][x][y][z] (sub-volume i, local node) = delta of the grid at the
// sub-volume origin + (x, y, z); delta = rho N^3 / wsum - 1 when wsum is given.
__global__ __launch_bounds__(256) void k_gather_subvolumes(const float* __restrict__ grid,
                                                           const double* __restrict__ wsum, int n, int s, int m,
                                                           float* __restrict__ out) {
  const int64_t m3 = (int64_t)m * m * m;
  const int64_t total4 = (int64_t)s * s * s * m3 / 4;
  float scale = 1.0f, sub = 0.0f;
  if (wsum) {
    scale = (float)((double)n * (double)n * (double)n / wsum[0]);
    sub = 1.0f;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total4;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i * 4;
    const int64_t box = e / m3;
    const int64_t r = e % m3;
    const int lx = (int)(r / ((int64_t)m * m)), ly = (int)((r / m) % m), lz = (int)(r % m);
    const int bx = (int)(box / ((int64_t)s * s)), by = (int)((box / s) % s), bz = (int)(box % s);
    const float4 v = *reinterpret_cast<const float4*>(grid + ((int64_t)(bx * m + lx) * n + (by * m + ly)) * n +
                                                      bz * m + lz);
    *reinterpret_cast<float4*>(out + e) =
        make_float4(v.x * scale - sub, v.y * scale - sub, v.z * scale - sub, v.w * scale - sub);
  }
}

// Shell sums of one sub-volume per blockIdx.y over its half spectrum
// [m][m][h]; psum[i][l][b] += mult (2l+1) L_l(mu) |F / W|^2, dbar[i] = F(0) / m^3.
// Each thread walks whole k_z lines: |n|^2 grows along a line, so the current
// shell's sums stay in registers and go to the workgroup's LDS histogram only
// when the shell changes; the window factors come from a per-axis table.
__global__ __launch_bounds__(256) void k_subvolume_shells(const float2* __restrict__ F, int m, int s, int plane,
                                                          double ox, double oy, double oz, int window, int nl,
                                                          const int32_t* __restrict__ bin_of_n2, int n2max,
                                                          int nbins, double* __restrict__ psum,
                                                          double* __restrict__ dbar) {
  extern __shared__ double smem[];
  double* hist = smem;                     // [nl][nbins]
  double* wtab = smem + nl * nbins;        // [m / 2 + 1]: 1 / W of one axis at |a|
  const int h = m / 2 + 1;
  for (int b = threadIdx.x; b < nl * nbins; b += blockDim.x) hist[b] = 0.0;
  for (int a = threadIdx.x; a < h; a += blockDim.x) {
    double w = 1.0;
    if (window >= 0 && a > 0) {
      // assignment window at the sub-volume frequencies (same cell size)
      const double x = 3.14159265358979323846 * a / m;
      w = sin(x) / x;
      if (window == 1) w *= w;
    }
    wtab[a] = 1.0 / w;
  }
  const int box = blockIdx.y;
  // line of sight of this sub-volume: observer to its centre
  double ex = 0.0, ey = 0.0, ez = 1.0;
  if (!plane) {
    const int bx = box / (s * s), by = (box / s) % s, bz = box % s;
    const double half = 0.5 * (m - 1);
    ex = bx * (double)m + half - ox;
    ey = by * (double)m + half - oy;
    ez = bz * (double)m + half - oz;
    const double inv = 1.0 / sqrt(ex * ex + ey * ey + ez * ez);
    ex *= inv;
    ey *= inv;
    ez *= inv;
  }
  __syncthreads();
  const float2* Fi = F + (int64_t)box * m * m * h;
  double acc[3] = {0.0, 0.0, 0.0};
  int cur = -1;
  auto flush = [&]() {
    if (cur >= 0)
      for (int li = 0; li < nl; ++li) atomicAdd(&hist[li * nbins + cur], acc[li]);
    acc[0] = acc[1] = acc[2] = 0.0;
  };
  for (int line = blockIdx.x * blockDim.x + threadIdx.x; line < m * m; line += gridDim.x * blockDim.x) {
    const int iy = line % m, ix = line / m;
    const int nx = ix <= m / 2 ? ix : ix - m, ny = iy <= m / 2 ? iy : iy - m;
    const int nxy = nx * nx + ny * ny;
    const double wxy = wtab[nx < 0 ? -nx : nx] * wtab[ny < 0 ? -ny : ny];
    const float2* row = Fi + (int64_t)line * h;
    for (int kz = 0; kz < h; ++kz) {
      const int n2 = nxy + kz * kz;
      if (n2 > n2max) break;  // |n|^2 only grows along the line
      if (n2 == 0) {
        dbar[box] = (double)row[0].x / ((double)m * m * m);
        continue;
      }
      const int b = bin_of_n2[n2];
      if (b < 0) continue;
      if (b != cur) {
        flush();
        cur = b;
      }
      const float2 v = row[kz];
      const double wc = wxy * wtab[kz];
      const double p = ((double)v.x * v.x + (double)v.y * v.y) * wc * wc;
      const double mult = (kz == 0 || 2 * kz == m) ? 1.0 : 2.0;
      const double mu = (nx * ex + ny * ey + kz * ez) / sqrt((double)n2);
      const double mu2 = mu * mu;
      acc[0] += mult * p;
      if (nl > 1) acc[1] += mult * 5.0 * 0.5 * (3.0 * mu2 - 1.0) * p;
      if (nl > 2) acc[2] += mult * 9.0 * (35.0 * mu2 * mu2 - 30.0 * mu2 + 3.0) / 8.0 * p;
    }
  }
  flush();
  __syncthreads();
  for (int b = threadIdx.x; b < nl * nbins; b += blockDim.x)
    if (hist[b] != 0.0) unsafeAtomicAdd(&psum[(int64_t)box * nl * nbins + b], hist[b]);
}

// ---------------------------------------------------------------- local line of sight
// With the line of sight varying over the nodes of a sub-volume (eq.
// PowSpecMultipole inside each sub-volume), delta^(l)_i(n) =
// (2l+1) sum_m a_m h_m(n_hat) F_im(n), F_im the DFT of h_m(x_hat) delta over
// the sub-volume (the addition theorem of the main path's LOS moments), and
//   P^(l)_i(k_b) = V_s sum_{n in b} Re[delta^(l)_i(n) conj delta^(0)_i(n)] / (M^6 N_b)
//                = V_s (2l+1) sum_m a_m sum_{n in b} h_m(n_hat) Re[F_im(n) conj F_i0(n)] / (|W|^2 M^6 N_b),
// linear in each F_im: the harmonics are transformed and summed one at a time
// against the kept F_i0.

// h_m with m known only at run time (uniform over a launch).
__device__ __forceinline__ double harmonic_rt(int m, double x, double y, double z) {
  switch (m) {
    case 0: return los_harmonic<0, double>(x, y, z);
    case 1: return los_harmonic<1, double>(x, y, z);
    case 2: return los_harmonic<2, double>(x, y, z);
    case 3: return los_harmonic<3, double>(x, y, z);
    case 4: return los_harmonic<4, double>(x, y, z);
    case 5: return los_harmonic<5, double>(x, y, z);
    case 6: return los_harmonic<6, double>(x, y, z);
    case 7: return los_harmonic<7, double>(x, y, z);
    case 8: return los_harmonic<8, double>(x, y, z);
    case 9: return los_harmonic<9, double>(x, y, z);
    case 10: return los_harmonic<10, double>(x, y, z);
    case 11: return los_harmonic<11, double>(x, y, z);
    case 12: return los_harmonic<12, double>(x, y, z);
    case 13: return los_harmonic<13, double>(x, y, z);
    default: return los_harmonic<14, double>(x, y, z);
  }
}

// As k_gather_subvolumes, times h_m(x_hat) of each node: x_hat points from the
// observer (grid units) to the node's grid position.
__global__ __launch_bounds__(256) void k_gather_subvolumes_los(const float* __restrict__ grid,
                                                               const double* __restrict__ wsum, int n, int s, int m,
                                                               int harm, double ox, double oy, double oz,
                                                               float* __restrict__ out) {
  const int64_t m3 = (int64_t)m * m * m;
  const int64_t total4 = (int64_t)s * s * s * m3 / 4;
  float scale = 1.0f, sub = 0.0f;
  if (wsum) {
    scale = (float)((double)n * (double)n * (double)n / wsum[0]);
    sub = 1.0f;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total4;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i * 4;
    const int64_t box = e / m3;
    const int64_t r = e % m3;
    const int lx = (int)(r / ((int64_t)m * m)), ly = (int)((r / m) % m), lz = (int)(r % m);
    const int bx = (int)(box / ((int64_t)s * s)), by = (int)((box / s) % s), bz = (int)(box % s);
    const int gx = bx * m + lx, gy = by * m + ly, gz = bz * m + lz;
    const float4 v = *reinterpret_cast<const float4*>(grid + ((int64_t)gx * n + gy) * n + gz);
    const double rx = gx - ox, ry = gy - oy;
    float h[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double rz = (gz + q) - oz;
      const double inv = 1.0 / sqrt(rx * rx + ry * ry + rz * rz);
      h[q] = (float)harmonic_rt(harm, rx * inv, ry * inv, rz * inv);
    }
    *reinterpret_cast<float4*>(out + e) = make_float4(h[0] * (v.x * scale - sub), h[1] * (v.y * scale - sub),
                                                      h[2] * (v.z * scale - sub), h[3] * (v.w * scale - sub));
  }
}

// psum[i][l][b] += mult coef h_m(n_hat) Re[Fm(n) conj F0(n)] / W(n)^2 over the
// half spectrum of sub-volume i = blockIdx.y, coef = (2l+1) a_m; harm 0 also
// sets dbar[i] = F0(0) / M^3. Lines and the per-workgroup histogram as in
// k_subvolume_shells.
__global__ __launch_bounds__(256) void k_subvolume_cross(const float2* __restrict__ F0, const float2* __restrict__ Fm,
                                                         int m, int harm, int ell_slot, double coef, int window,
                                                         int nl, const int32_t* __restrict__ bin_of_n2, int n2max,
                                                         int nbins, double* __restrict__ psum,
                                                         double* __restrict__ dbar) {
  extern __shared__ double smem[];
  double* hist = smem;               // [nbins]
  double* wtab = smem + nbins;       // [m / 2 + 1]: 1 / W of one axis at |a|
  const int h = m / 2 + 1;
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) hist[b] = 0.0;
  for (int a = threadIdx.x; a < h; a += blockDim.x) {
    double w = 1.0;
    if (window >= 0 && a > 0) {
      const double x = 3.14159265358979323846 * a / m;
      w = sin(x) / x;
      if (window == 1) w *= w;
    }
    wtab[a] = 1.0 / w;
  }
  const int box = blockIdx.y;
  __syncthreads();
  const int64_t off = (int64_t)box * m * m * h;
  double acc = 0.0;
  int cur = -1;
  auto flush = [&]() {
    if (cur >= 0) atomicAdd(&hist[cur], acc);
    acc = 0.0;
  };
  for (int line = blockIdx.x * blockDim.x + threadIdx.x; line < m * m; line += gridDim.x * blockDim.x) {
    const int iy = line % m, ix = line / m;
    const int nx = ix <= m / 2 ? ix : ix - m, ny = iy <= m / 2 ? iy : iy - m;
    const int nxy = nx * nx + ny * ny;
    const double wxy = wtab[nx < 0 ? -nx : nx] * wtab[ny < 0 ? -ny : ny];
    const float2* r0 = F0 + off + (int64_t)line * h;
    const float2* rm = Fm + off + (int64_t)line * h;
    for (int kz = 0; kz < h; ++kz) {
      const int n2 = nxy + kz * kz;
      if (n2 > n2max) break;  // |n|^2 only grows along the line
      if (n2 == 0) {
        if (harm == 0) dbar[box] = (double)r0[0].x / ((double)m * m * m);
        continue;
      }
      const int b = bin_of_n2[n2];
      if (b < 0) continue;
      if (b != cur) {
        flush();
        cur = b;
      }
      const float2 a = r0[kz], c = rm[kz];
      const double wc = wxy * wtab[kz];
      const double inv = 1.0 / sqrt((double)n2);
      const double hk = harmonic_rt(harm, nx * inv, ny * inv, kz * inv);
      const double mult = (kz == 0 || 2 * kz == m) ? 1.0 : 2.0;
      acc += mult * hk * ((double)c.x * a.x + (double)c.y * a.y) * wc * wc;
    }
  }
  flush();
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x)
    if (hist[b] != 0.0) unsafeAtomicAdd(&psum[((int64_t)box * nl + ell_slot) * nbins + b], coef * hist[b]);
}

// iB[l][b] = (1/N_s) sum_i P[i][l][b] dbar[i], P = scale psum / N_b (optionally
// stored); one workgroup per (l, b) sums over the sub-volumes.
__global__ __launch_bounds__(256) void k_subvolume_finalize(const double* __restrict__ psum,
                                                            const double* __restrict__ dbar, int ns, int nl,
                                                            int nbins, const int64_t* __restrict__ nb_modes,
                                                            double scale, double* __restrict__ iB,
                                                            double* __restrict__ P) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  const int64_t nm = nb_modes[j % nbins];
  const double f = nm > 0 ? scale / (double)nm : 0.0;
  double acc = 0.0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    const double pv = f * psum[(int64_t)i * nl * nbins + j];
    if (P) P[(int64_t)i * nl * nbins + j] = pv;
    acc += pv * dbar[i];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) iB[j] = red[0] / ns;
}

hipError_t launch_gather_subvolumes(const float* grid, const double* wsum, int n, int s, float* out, hipStream_t st) {
  if (s < 1 || n % s != 0 || (n / s) % 4 != 0) return hipErrorInvalidValue;
  const int m = n / s;
  const int64_t total4 = (int64_t)n * n * n / 4;
  int64_t blocks = (total4 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_gather_subvolumes, dim3((unsigned)blocks), dim3(256), 0, st, grid, wsum, n, s, m, out);
  return hipGetLastError();
}

hipError_t launch_subvolume_shells(const float2* F, int m, int s, int plane, const double* obs, int window, int nl,
                                   const int32_t* bin_of_n2, int n2max, int nbins, double* psum, double* dbar,
                                   hipStream_t st) {
  const int ns = s * s * s;
  const size_t lds = ((size_t)nl * nbins + m / 2 + 1) * sizeof(double);
  if (ns > 65535 || nl < 1 || nl > 3 || lds > 64 * 1024) return hipErrorInvalidValue;
  // about 16 k_z lines per thread
  const int64_t lines = (int64_t)m * m;
  int64_t bx = (lines + 256 * 16 - 1) / (256 * 16);
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_subvolume_shells, dim3((unsigned)bx, (unsigned)ns), dim3(256), lds, st, F, m, s, plane,
                     obs[0], obs[1], obs[2], window, nl, bin_of_n2, n2max, nbins, psum, dbar);
  return hipGetLastError();
}

hipError_t launch_gather_subvolumes_los(const float* grid, const double* wsum, int n, int s, int harm,
                                       const double* obs, float* out, hipStream_t st) {
  if (s < 1 || n % s != 0 || (n / s) % 4 != 0 || harm < 0 || harm >= kLosFields) return hipErrorInvalidValue;
  const int m = n / s;
  const int64_t total4 = (int64_t)n * n * n / 4;
  int64_t blocks = (total4 + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_gather_subvolumes_los, dim3((unsigned)blocks), dim3(256), 0, st, grid, wsum, n, s, m, harm,
                     obs[0], obs[1], obs[2], out);
  return hipGetLastError();
}

hipError_t launch_subvolume_cross(const float2* F0, const float2* Fm, int m, int s, int harm, int ell_slot,
                                  double coef, int window, int nl, const int32_t* bin_of_n2, int n2max, int nbins,
                                  double* psum, double* dbar, hipStream_t st) {
  const int ns = s * s * s;
  const size_t lds = ((size_t)nbins + m / 2 + 1) * sizeof(double);
  if (ns > 65535 || nl < 1 || nl > 3 || ell_slot < 0 || ell_slot >= nl || harm < 0 || harm >= kLosFields ||
      lds > 64 * 1024)
    return hipErrorInvalidValue;
  const int64_t lines = (int64_t)m * m;
  int64_t bx = (lines + 256 * 16 - 1) / (256 * 16);
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(k_subvolume_cross, dim3((unsigned)bx, (unsigned)ns), dim3(256), lds, st, F0, Fm, m, harm,
                     ell_slot, coef, window, nl, bin_of_n2, n2max, nbins, psum, dbar);
  return hipGetLastError();
}

hipError_t launch_subvolume_finalize(const double* psum, const double* dbar, int ns, int nl, int nbins,
                                     const int64_t* nb_modes, double scale, double* iB, double* P, hipStream_t st) {
  hipLaunchKernelGGL(k_subvolume_finalize, dim3((unsigned)(nl * nbins)), dim3(256), 0, st, psum, dbar, ns, nl, nbins,
                     nb_modes, scale, iB, P);
  return hipGetLastError();
}

}  // namespace bsp
