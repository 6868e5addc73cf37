// FP64 finishing kernels: normalisation of the binned multipoles and their
// shot noise, rounding of the triangle counts, assembly of the modal
// numerators and of the Gram matrix from triple sums, the Cholesky
// factorisation gamma = L L^T and the two triangular solves, and the sample
// covariance over a batch of mocks.
#include "bsp_internal.h"

namespace bsp {

// B^l_i = norm_b T^l_i / N_tri,i  (norm_b = V^2 / (N^9 N'^3)): the lattice form of
// (1/V_B) sum_closed delta delta delta / V of the standard estimator.
// Pbar_b = pnorm psum_b / N_b (pnorm = V / N^6); B0sub = B^0 - sum Pbar / nbar + 2 / nbar^2.
__global__ void k_binned_finalize(const double* __restrict__ T, const int32_t* __restrict__ tri_tidx, int ntri,
                                  int nl, const int64_t* __restrict__ counts, const double* __restrict__ psum,
                                  const int64_t* __restrict__ nb_modes, int nbins,
                                  const int32_t* __restrict__ tri_bins, double norm_b, double pnorm,
                                  const double* __restrict__ nbar_p, double* __restrict__ B,
                                  double* __restrict__ B0sub, double* __restrict__ Pbar) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (Pbar && i < nbins) Pbar[i] = nb_modes[i] > 0 ? pnorm * psum[i] / (double)nb_modes[i] : 0.0;
  if (i >= ntri) return;
  const double inv = 1.0 / (double)counts[i];
  for (int l = 0; l < nl; ++l) B[(int64_t)l * ntri + i] = norm_b * T[tri_tidx[(int64_t)l * ntri + i]] * inv;
  const double nbar = nbar_p ? nbar_p[0] : 0.0;
  if (B0sub && nbar > 0.0) {
    double ps = 0.0;
    for (int a = 0; a < 3; ++a) {
      const int b = tri_bins[3 * i + a];
      ps += nb_modes[b] > 0 ? pnorm * psum[b] / (double)nb_modes[b] : 0.0;
    }
    B0sub[i] = B[i] - ps / nbar + 2.0 / (nbar * nbar);
  }
}

// Poisson shot noise of B_l (the reading of the multipole estimator's
// coincidence terms): per triangle i and multipole l,
//   SN_0 = (P_0(b1) + P_0(b2) + P_0(b3)) / nbar - 2 / nbar^2,
//   SN_l = (P_l(b1) + W[l][i][0] P_l(b2) + W[l][i][1] P_l(b3)) / nbar  (l > 0),
// W the ring factors of the plan ([nl][ntri][2], row 0 unused).
__global__ void k_shot_noise(const double* __restrict__ Pl, int nbins, const int32_t* __restrict__ tri_bins, int ntri,
                             int nl, const double* __restrict__ ring, double nbar, double* __restrict__ SN) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntri) return;
  const int b1 = tri_bins[3 * i], b2 = tri_bins[3 * i + 1], b3 = tri_bins[3 * i + 2];
  SN[i] = (Pl[b1] + Pl[b2] + Pl[b3]) / nbar - 2.0 / (nbar * nbar);
  for (int l = 1; l < nl; ++l) {
    const double* P = Pl + (int64_t)l * nbins;
    const double* w = ring + ((int64_t)l * ntri + i) * 2;
    SN[(int64_t)l * ntri + i] = (P[b1] + w[0] * P[b2] + w[1] * P[b3]) / nbar;
  }
}

// counts_i = round(T_i / N'^3); bit 2 of err if any |T/N'^3 - round| >= 0.05
// (rounding is unambiguous below 0.5; FP64 sums of 1e8 terms of this dynamic
// range leave ~1e-3 on counts of 1e10).
// Counts round the FP64 sums; the residual from an integer must stay below
// 0.05 + rel |c| (rel: the FP64 transforms' relative error, proportional to the
// count), and that bound below 0.5, where the rounding is no longer certain.
__global__ void k_counts_finalize(const double* __restrict__ T, const int32_t* __restrict__ tidx, int ntri,
                                  double inv_k, double rel, int64_t* __restrict__ counts, double* __restrict__ raw,
                                  int32_t* __restrict__ err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ntri) return;
  const double c = T[tidx[i]] * inv_k;
  const double r = rint(c);
  counts[i] = (int64_t)r;
  raw[i] = c;
  const double tol = 0.05 + rel * fabs(c);
  if (!(tol < 0.5 && fabs(c - r) < tol)) atomicOr(err, 4);
}

// bnum[l][m] = scale sum_{j<6, combo >= 0} T[combo[l][m][j]]  (minus shot noise for l = 0)
__global__ void k_modal_assemble(const double* __restrict__ T, const int32_t* __restrict__ combo, int nmodes,
                                 int nl, double scale, const double* __restrict__ sn,
                                 const double* __restrict__ nbar_p, double* __restrict__ bnum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nl * nmodes) return;
  double s = 0.0;
  for (int j = 0; j < 6; ++j) {
    const int t = combo[6 * i + j];
    if (t >= 0) s += T[t];
  }
  s *= scale;
  const double nbar = nbar_p ? nbar_p[0] : 0.0;
  if (i < nmodes && sn && nbar > 0.0) s -= 3.0 / nbar * sn[i] - 2.0 / (nbar * nbar) * sn[nmodes + i];
  bnum[i] = s;
}

// gamma[n][m] = scale sum_{tau in S3} T[gidx[n][m][tau]]
__global__ void k_gram_assemble(const double* __restrict__ T, const int32_t* __restrict__ gidx, int nmodes,
                                double scale, double* __restrict__ gamma) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nmodes * nmodes) return;
  double s = 0.0;
  for (int j = 0; j < 6; ++j) s += T[gidx[6 * i + j]];
  gamma[i] = s * scale;
}

// sn[0][m] = scale (T[a] + T[b] + T[c]) / 3, sn[1][m] = scale T[d]
__global__ void k_sn_assemble(const double* __restrict__ T, const int32_t* __restrict__ sidx, int nmodes,
                              double scale, double* __restrict__ sn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nmodes) return;
  sn[i] = scale * (T[sidx[4 * i]] + T[sidx[4 * i + 1]] + T[sidx[4 * i + 2]]) / 3.0;
  sn[nmodes + i] = scale * T[sidx[4 * i + 3]];
}

// Cholesky factor of the Gram matrix with optional pivoting and truncation
// (Gram-Schmidt of the modes in the gamma inner product). tol <= 0: modes in
// table order, all kept, non-positive pivots latch error bit 8. tol > 0: the
// next mode is the one whose residual norm relative to its own,
// resid_j / gamma_jj, is largest (ties to the lower index); stop once it falls
// below tol (the rest are numerically dependent on the modes taken). One
// workgroup of 256 threads, n <= 128.
//   A: in gamma [n][n]; out L [n][n], row i = i-th kept mode, lower triangular,
//      rows >= rank zero.
//   W: scratch [n][n] (factor indexed by mode, step).
//   piv: out [n] kept modes in order taken, -1 past the rank; piv[n] = rank.
__global__ __launch_bounds__(256) void k_cholesky_pivoted(double* __restrict__ A, double* __restrict__ W, int n,
                                                          double tol, int32_t* __restrict__ piv,
                                                          int32_t* __restrict__ err) {
  __shared__ double resid[128], d0[128];
  __shared__ int taken[128];
  __shared__ double rv[256];
  __shared__ int ri[256];
  __shared__ int jstar, stop, fail;
  const int t = threadIdx.x;
  for (int i = t; i < n * n; i += blockDim.x) W[i] = 0.0;
  if (t < n) {
    resid[t] = A[(int64_t)t * n + t];
    d0[t] = resid[t];
    taken[t] = 0;
  }
  if (t == 0) {
    stop = 0;
    fail = 0;
  }
  __syncthreads();
  int k = 0;
  for (; k < n; ++k) {
    if (tol > 0.0) {
      // argmax of resid / d0 over the modes not taken, lower index on ties
      double v = -1.0;
      int vi = n;
      if (t < n && !taken[t]) {
        v = resid[t] / d0[t];
        vi = t;
      }
      rv[t] = v;
      ri[t] = vi;
      __syncthreads();
      for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
          const double a = rv[t], b = rv[t + off];
          const int ia = ri[t], ib = ri[t + off];
          if (b > a || (b == a && ib < ia)) {
            rv[t] = b;
            ri[t] = ib;
          }
        }
        __syncthreads();
      }
      if (t == 0) {
        jstar = ri[0];
        stop = !(rv[0] >= tol) || ri[0] >= n;
      }
    } else if (t == 0) {
      jstar = k;
      if (!(resid[k] > 0.0)) {
        fail = 1;
        resid[k] = 1.0;
      }
    }
    __syncthreads();
    if (stop) break;
    const int j0 = jstar;
    const double dk = sqrt(resid[j0]);
    if (t == 0) {
      piv[k] = j0;
      taken[j0] = 1;
      W[(int64_t)j0 * n + k] = dk;
    }
    __syncthreads();
    if (t < n && !taken[t]) {
      double sum = A[(int64_t)t * n + j0];
      for (int m = 0; m < k; ++m) sum -= W[(int64_t)t * n + m] * W[(int64_t)j0 * n + m];
      const double c = sum / dk;
      W[(int64_t)t * n + k] = c;
      resid[t] -= c * c;
    }
    __syncthreads();
  }
  const int rank = k;
  __syncthreads();
  for (int idx = t; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, m = idx % n;
    A[idx] = (i < rank && m <= i) ? W[(int64_t)piv[i] * n + m] : 0.0;
  }
  for (int i = rank + t; i < n; i += blockDim.x) piv[i] = -1;
  if (t == 0) {
    piv[n] = rank;
    if (fail) atomicOr(err, 8);
  }
}

// Inverse of the lower Cholesky factor of the kept modes (rank = piv[n] rows),
// once per geometry: thread j solves L x = e_j by forward substitution into
// column j of Linv. Entries outside the lower rank x rank block are zero.
__global__ __launch_bounds__(128) void k_tri_inverse(const double* __restrict__ L, const int32_t* __restrict__ piv,
                                                     int n, double* __restrict__ Linv) {
  const int rank = piv[n];
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) Linv[idx] = 0.0;
  __syncthreads();
  const int j = threadIdx.x;
  if (j >= rank) return;
  for (int i = j; i < rank; ++i) {
    double s = (i == j) ? 1.0 : 0.0;
    for (int k = j; k < i; ++k) s -= L[(int64_t)i * n + k] * Linv[(int64_t)k * n + j];
    Linv[(int64_t)i * n + j] = s / L[(int64_t)i * n + i];
  }
}

// Coefficients on the kept, orthonormalised modes for nrhs right-hand sides
// (one workgroup each), as products with the precomputed inverse factor:
// alpha_i = sum_k Linv_ik b_piv[k] for i < rank (0 past it), and on the kept
// modes beta_piv[i] = sum_k Linv_ki alpha_k (beta = L^-T alpha), 0 on the
// dropped ones. Every sum runs in a fixed order.
__global__ __launch_bounds__(128) void k_modal_solve(const double* __restrict__ Linv, const int32_t* __restrict__ piv,
                                                     int n, const double* __restrict__ b, double* __restrict__ alpha,
                                                     double* __restrict__ beta) {
  __shared__ double al[128];
  const int r = blockIdx.x;
  const int rank = piv[n];
  const double* bb = b + (int64_t)r * n;
  double* ao = alpha + (int64_t)r * n;
  double* bo = beta + (int64_t)r * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double a = 0.0;
    if (i < rank)
      for (int k = 0; k <= i; ++k) a += Linv[(int64_t)i * n + k] * bb[piv[k]];
    al[i] = a;
    ao[i] = a;
    bo[i] = 0.0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < rank; i += blockDim.x) {
    double v = 0.0;
    for (int k = i; k < rank; ++k) v += Linv[(int64_t)k * n + i] * al[k];
    bo[piv[i]] = v;
  }
}

// cov[i][j] = sum_m (x_mi - mean_i)(x_mj - mean_j) / (M - 1), x row major [M][D].
__global__ void k_covariance(const double* __restrict__ x, int m, int d, double* __restrict__ cov) {
  const int i = blockIdx.y * blockDim.y + threadIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d || j >= d) return;
  double mi = 0.0, mj = 0.0;
  for (int k = 0; k < m; ++k) {
    mi += x[(int64_t)k * d + i];
    mj += x[(int64_t)k * d + j];
  }
  mi /= m;
  mj /= m;
  double s = 0.0;
  for (int k = 0; k < m; ++k) s += (x[(int64_t)k * d + i] - mi) * (x[(int64_t)k * d + j] - mj);
  cov[(int64_t)i * d + j] = s / (double)(m - 1);
}

// nbar = wsum * scale (scale = 1/V), so no host round trip is needed.
__global__ void k_scale_scalar(const double* __restrict__ x, double scale, double* __restrict__ y) {
  if (threadIdx.x == 0 && blockIdx.x == 0) y[0] = x[0] * scale;
}

static unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_binned_finalize(const double* T, const int32_t* tri_tidx, int ntri, int nl, const int64_t* counts,
                                  const double* psum, const int64_t* nb_modes, int nbins, const int32_t* tri_bins,
                                  double norm_b, double pnorm, const double* nbar, double* B, double* B0sub,
                                  double* Pbar, hipStream_t s) {
  const int n = ntri > nbins ? ntri : nbins;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_binned_finalize, dim3(nblk(n, 256)), dim3(256), 0, s, T, tri_tidx, ntri, nl, counts, psum,
                     nb_modes, nbins, tri_bins, norm_b, pnorm, nbar, B, B0sub, Pbar);
  return hipGetLastError();
}

hipError_t launch_shot_noise(const double* Pl, int nbins, const int32_t* tri_bins, int ntri, int nl,
                             const double* ring, double nbar, double* SN, hipStream_t s) {
  if (ntri <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_shot_noise, dim3((unsigned)((ntri + 255) / 256)), dim3(256), 0, s, Pl, nbins, tri_bins, ntri,
                     nl, ring, nbar, SN);
  return hipGetLastError();
}

hipError_t launch_counts_finalize(const double* T, const int32_t* tidx, int ntri, double inv_k, double rel,
                                  int64_t* counts, double* raw, int32_t* err, hipStream_t s) {
  if (ntri <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_counts_finalize, dim3(nblk(ntri, 256)), dim3(256), 0, s, T, tidx, ntri, inv_k, rel, counts,
                     raw, err);
  return hipGetLastError();
}

hipError_t launch_modal_assemble(const double* T, const int32_t* combo, int nmodes, int nl, double scale,
                                 const double* sn, const double* nbar, double* bnum, hipStream_t s) {
  if (nmodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_modal_assemble, dim3(nblk((int64_t)nl * nmodes, 256)), dim3(256), 0, s, T, combo, nmodes,
                     nl, scale, sn, nbar, bnum);
  return hipGetLastError();
}

hipError_t launch_gram_assemble(const double* T, const int32_t* gidx, int nmodes, double scale, double* gamma,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_gram_assemble, dim3(nblk((int64_t)nmodes * nmodes, 256)), dim3(256), 0, s, T, gidx, nmodes,
                     scale, gamma);
  return hipGetLastError();
}

hipError_t launch_sn_assemble(const double* T, const int32_t* sidx, int nmodes, double scale, double* sn,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_sn_assemble, dim3(nblk(nmodes, 256)), dim3(256), 0, s, T, sidx, nmodes, scale, sn);
  return hipGetLastError();
}

hipError_t launch_cholesky(double* A, double* W, int n, double tol, int32_t* piv, int32_t* err, hipStream_t s) {
  if (n < 1 || n > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cholesky_pivoted, dim3(1), dim3(256), 0, s, A, W, n, tol, piv, err);
  return hipGetLastError();
}

hipError_t launch_tri_inverse(const double* L, const int32_t* piv, int n, double* Linv, hipStream_t s) {
  if (n < 1 || n > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tri_inverse, dim3(1), dim3(128), 0, s, L, piv, n, Linv);
  return hipGetLastError();
}

hipError_t launch_modal_solve(const double* Linv, const int32_t* piv, int n, int nrhs, const double* b, double* alpha,
                              double* beta, hipStream_t s) {
  if (nrhs <= 0) return hipSuccess;
  if (n < 1 || n > 128) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_modal_solve, dim3(nrhs), dim3(128), 0, s, Linv, piv, n, b, alpha, beta);
  return hipGetLastError();
}

hipError_t launch_scale_scalar(const double* x, double scale, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_scalar, dim3(1), dim3(64), 0, s, x, scale, y);
  return hipGetLastError();
}

hipError_t launch_covariance(const double* x, int m, int d, double* cov, hipStream_t s) {
  dim3 blk(16, 16);
  dim3 grid(nblk(d, 16), nblk(d, 16));
  hipLaunchKernelGGL(k_covariance, grid, blk, 0, s, x, m, d, cov);
  return hipGetLastError();
}

}  // namespace bsp
