// Line-of-sight Legendre moments delta^(l)(k), l = 0, 2, 4, from the transforms
// of the x-hat-weighted fields, and the shell sums of |delta^(0)|^2.
//
// The LOS moment field of the paper's power-spectrum section is
//   delta^(l)(k) = (2l+1) int d^3x e^{-ik.x} delta(x) L_l(k_hat . x_hat).
// By the addition theorem L_l(k_hat . x_hat) = sum_m a_m h_m(k_hat) h_m(x_hat)
// over the 2l+1 real solid harmonics h_m of degree l (their polynomials are
// listed with kLosPoly), so with F_m = FT[h_m(x_hat) delta]
//   delta^(l)(k) = (2l+1) sum_m a_m h_m(k_hat) F_m(k):
// 1 + 5 + 9 weighted transforms for l <= 4, each F_m a single multipole of
// the line of sight (no cancellation between the l = 0, 2, 4 parts, which the
// products of x-hat components would carry). Plane parallel: the one field F
// and delta^(l) = (2l+1) L_l(k_hat_z) F.
// The mass-assignment window is divided out (CIC: prod sinc^2(pi n_a / N)) and
// two interlaced grids are averaged after the half-cell phase
// exp(i pi (nx + ny + nz) / N) is applied to the shifted one.
#include "bsp_internal.h"

namespace bsp {

template <int M> __device__ __forceinline__ void add_harmonic(double2& acc, const double* kh, double2 f) {
  const double h = kLosCoef[M] * los_harmonic<M, double>(kh[0], kh[1], kh[2]);
  acc.x += h * f.x;
  acc.y += h * f.y;
}

__device__ __forceinline__ double sinc_pi(int n, int N) {
  if (n == 0) return 1.0;
  const double a = M_PI * (double)n / (double)N;
  return sin(a) / a;
}

// One mode per thread. NLOS weighted fields per grid (1, 6 or 15) and NG grids
// are template parameters so that all NG x NLOS loads of a mode are issued
// before its arithmetic.
template <typename T, int NLOS, int NG>
__global__ __launch_bounds__(256) void k_los_combine(const cplx_t<T>* __restrict__ X, cplx_t<T>* __restrict__ dl,
                                                     LosDesc d) {
  using V = cplx_t<T>;
  typedef T T2 __attribute__((ext_vector_type(2)));
  const int w = 2 * d.c + 1;
  const int64_t cube = (int64_t)w * w * d.cz;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= cube) return;
  const int nl = d.lmax / 2 + 1;
  const int kz = (int)(idx % d.cz);
  const int64_t rest = idx / d.cz;
  const int iy = (int)(rest % w), ix = (int)(rest / w);
  const int nx = ix - d.c, ny = iy - d.c, nz = kz;
  const int n2 = nx * nx + ny * ny + nz * nz;
  if (kz > d.c || n2 == 0 || n2 > d.n2max) {
    for (int l = 0; l < nl; ++l) dl[l * cube + idx] = V{(T)0, (T)0};
    return;
  }
  T2 xv[NG][NLOS];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int t = 0; t < NLOS; ++t)
      xv[g][t] = __builtin_nontemporal_load(reinterpret_cast<const T2*>(X + ((int64_t)g * NLOS + t) * cube + idx));
  double comp = 1.0;
  if (d.compensate) {
    double wv = sinc_pi(nx, d.n) * sinc_pi(ny, d.n) * sinc_pi(nz, d.n);
    if (d.window == 1) wv *= wv;
    comp = 1.0 / wv;
  }
  double2 fac[2];
  fac[0] = double2{comp / NG, 0.0};
  if constexpr (NG == 2) {
    const double ph = M_PI * (double)(nx + ny + nz) / (double)d.n;
    fac[1] = double2{comp / NG * cos(ph), comp / NG * sin(ph)};
  }
  auto F = [&](int t) -> double2 {
    double2 s{0.0, 0.0};
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      s.x += fac[g].x * (double)xv[g][t].x - fac[g].y * (double)xv[g][t].y;
      s.y += fac[g].x * (double)xv[g][t].y + fac[g].y * (double)xv[g][t].x;
    }
    return s;
  };
  const double inv = 1.0 / sqrt((double)n2);
  const double kh[3] = {nx * inv, ny * inv, nz * inv};
  const double2 F0 = F(0);
  dl[idx] = V{(T)F0.x, (T)F0.y};
  if (d.lmax < 2) return;
  double2 D2{0.0, 0.0}, D4{0.0, 0.0};
  if constexpr (NLOS == 1) {
    // plane parallel: mu = k_hat_z for every node
    const double m2 = kh[2] * kh[2];
    const double L2 = 0.5 * (3.0 * m2 - 1.0), L4 = (35.0 * m2 * m2 - 30.0 * m2 + 3.0) / 8.0;
    D2 = double2{5.0 * L2 * F0.x, 5.0 * L2 * F0.y};
    D4 = double2{9.0 * L4 * F0.x, 9.0 * L4 * F0.y};
  } else {
    add_harmonic<1>(D2, kh, F(1));
    add_harmonic<2>(D2, kh, F(2));
    add_harmonic<3>(D2, kh, F(3));
    add_harmonic<4>(D2, kh, F(4));
    add_harmonic<5>(D2, kh, F(5));
    D2 = double2{5.0 * D2.x, 5.0 * D2.y};
    if constexpr (NLOS == 15) {
      add_harmonic<6>(D4, kh, F(6));
      add_harmonic<7>(D4, kh, F(7));
      add_harmonic<8>(D4, kh, F(8));
      add_harmonic<9>(D4, kh, F(9));
      add_harmonic<10>(D4, kh, F(10));
      add_harmonic<11>(D4, kh, F(11));
      add_harmonic<12>(D4, kh, F(12));
      add_harmonic<13>(D4, kh, F(13));
      add_harmonic<14>(D4, kh, F(14));
      D4 = double2{9.0 * D4.x, 9.0 * D4.y};
    }
  }
  dl[cube + idx] = V{(T)D2.x, (T)D2.y};
  if (d.lmax < 4) return;
  dl[2 * cube + idx] = V{(T)D4.x, (T)D4.y};
}

// psum[b] += sum over the compact half cube of mult * |delta0|^2, mult = 2 for kz > 0
// (the conjugate partner at -n is not stored).
__global__ __launch_bounds__(256) void k_shell_power(const float2* __restrict__ d0, int c, int cz,
                                                     const int32_t* __restrict__ bin_of_n2, int n2max,
                                                     int nbins, double* __restrict__ psum) {
  extern __shared__ double hist[];
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) hist[b] = 0.0;
  __syncthreads();
  const int w = 2 * c + 1;
  const int64_t cube = (int64_t)w * w * cz;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < cube;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int kz = (int)(idx % cz);
    if (kz > c) continue;
    const int64_t rest = idx / cz;
    const int ny = (int)(rest % w) - c, nx = (int)(rest / w) - c;
    const int n2 = nx * nx + ny * ny + kz * kz;
    if (n2 > n2max) continue;
    const int b = bin_of_n2[n2];
    if (b < 0) continue;
    const float2 v = d0[idx];
    const double p = (double)v.x * v.x + (double)v.y * v.y;
    atomicAdd(&hist[b], kz == 0 ? p : 2.0 * p);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x)
    if (hist[b] != 0.0) unsafeAtomicAdd(&psum[b], hist[b]);
}

// Shell cross sums of the compact spectra: per shell b and moment l, the sum
// over the full lattice of Re[delta^(l)(n) conj(X(n))], with X = delta^(0) for
// the power-spectrum multipoles (Sec. 2, eq. PowSpecMultipole) or the transform
// of the squared monopole field for the skew spectra (Sec. 3.2). The compact
// cube holds n_z >= 0, so n_z > 0 entries stand for the pair n, -n.
__global__ __launch_bounds__(256) void k_shell_cross(const float2* __restrict__ dl, int64_t ell_stride, int nl,
                                                     const float2* __restrict__ partner, int c, int cz,
                                                     const int32_t* __restrict__ bin_of_n2, int n2max, int nbins,
                                                     double* __restrict__ psum) {
  extern __shared__ double hist[];  // [nl][nbins]
  for (int b = threadIdx.x; b < nl * nbins; b += blockDim.x) hist[b] = 0.0;
  __syncthreads();
  const int w = 2 * c + 1;
  const int64_t cube = (int64_t)w * w * cz;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < cube;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int kz = (int)(idx % cz);
    if (kz > c) continue;
    const int64_t rest = idx / cz;
    const int ny = (int)(rest % w) - c, nx = (int)(rest / w) - c;
    const int n2 = nx * nx + ny * ny + kz * kz;
    if (n2 > n2max) continue;
    const int b = bin_of_n2[n2];
    if (b < 0) continue;
    const double m = kz == 0 ? 1.0 : 2.0;
    const float2 x = partner[idx];
    for (int li = 0; li < nl; ++li) {
      const float2 v = dl[li * ell_stride + idx];
      atomicAdd(&hist[li * nbins + b], m * ((double)v.x * x.x + (double)v.y * x.y));
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nl * nbins; b += blockDim.x)
    if (hist[b] != 0.0) unsafeAtomicAdd(&psum[b], hist[b]);
}

// out[l][b] = scale * psum[l][b] / N_b.
__global__ void k_shell_finalize(const double* __restrict__ psum, int nl, int nbins,
                                 const int64_t* __restrict__ nb_modes, double scale, double* __restrict__ P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl * nbins) return;
  const int64_t nm = nb_modes[i % nbins];
  P[i] = nm > 0 ? scale * psum[i] / (double)nm : 0.0;
}

hipError_t launch_shell_cross(const float2* delta_l, int64_t ell_stride, int nl, const float2* partner, int c, int cz,
                              const int32_t* bin_of_n2, int n2max, int nbins, const int64_t* nb_modes, double scale,
                              double* psum, double* P, hipStream_t s) {
  if (nl < 1 || nbins < 1 || (size_t)nl * nbins * sizeof(double) > 64 * 1024) return hipErrorInvalidValue;
  hipError_t e = launch_fill_u32(psum, 0u, 2 * (int64_t)nl * nbins, s);
  if (e != hipSuccess) return e;
  const int64_t cube = (int64_t)(2 * c + 1) * (2 * c + 1) * cz;
  int64_t blocks = (cube + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_shell_cross, dim3((unsigned)blocks), dim3(256), (size_t)nl * nbins * sizeof(double), s,
                     delta_l, ell_stride, nl, partner, c, cz, bin_of_n2, n2max, nbins, psum);
  hipLaunchKernelGGL(k_shell_finalize, dim3((unsigned)((nl * nbins + 255) / 256)), dim3(256), 0, s, psum, nl, nbins,
                     nb_modes, scale, P);
  return hipGetLastError();
}

// x <- x^2 elementwise (the real-space product of the skew spectrum).
__global__ __launch_bounds__(256) void k_square(float4* __restrict__ x, int64_t n4) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    float4 v = x[i];
    v.x *= v.x;
    v.y *= v.y;
    v.z *= v.z;
    v.w *= v.w;
    x[i] = v;
  }
}

hipError_t launch_square(float* x, int64_t n, hipStream_t s) {
  if (n % 4 != 0 || (reinterpret_cast<uintptr_t>(x) & 15) != 0) return hipErrorInvalidValue;
  const int64_t n4 = n / 4;
  int64_t blocks = (n4 + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_square, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<float4*>(x), n4);
  return hipGetLastError();
}

// The field count must match the moments asked for: one field (lmax 0, or a
// plane-parallel line of sight), 6 (lmax 2) or 15 (lmax 4).
template <typename T>
static hipError_t los_combine_impl(const cplx_t<T>* X, cplx_t<T>* delta_l, const LosDesc& d, hipStream_t s) {
  if (d.ngrid < 1 || d.ngrid > 2 || d.lmax < 0 || d.lmax > 4) return hipErrorInvalidValue;
  const bool ok = d.nlos == 1 ? (d.plane || d.lmax == 0) : (d.nlos == 6 ? d.lmax <= 2 : d.nlos == 15);
  if (!ok) return hipErrorInvalidValue;
  const int64_t cube = (int64_t)(2 * d.c + 1) * (2 * d.c + 1) * d.cz;
  const dim3 grid((unsigned)((cube + 255) / 256));
#define LCASE(NL, G)                                                                                   \
  if (d.nlos == NL && d.ngrid == G) {                                                                  \
    hipLaunchKernelGGL((k_los_combine<T, NL, G>), grid, dim3(256), 0, s, X, delta_l, d);              \
    return hipGetLastError();                                                                          \
  }
  LCASE(1, 1) LCASE(1, 2) LCASE(6, 1) LCASE(6, 2) LCASE(15, 1) LCASE(15, 2)
#undef LCASE
  return hipErrorInvalidValue;
}

hipError_t launch_los_combine(const float2* X, float2* delta_l, const LosDesc& d, hipStream_t s) {
  return los_combine_impl<float>(X, delta_l, d, s);
}


hipError_t launch_shell_power(const float2* delta0, int c, int cz, const int32_t* bin_of_n2, int n2max,
                              int nbins, double* psum, hipStream_t s) {
  const int64_t cube = (int64_t)(2 * c + 1) * (2 * c + 1) * cz;
  int64_t blocks = (cube + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_shell_power, dim3((unsigned)blocks), dim3(256), nbins * sizeof(double), s, delta0, c, cz,
                     bin_of_n2, n2max, nbins, psum);
  return hipGetLastError();
}

}  // namespace bsp
