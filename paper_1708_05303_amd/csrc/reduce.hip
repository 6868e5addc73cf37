// Triple reduction T[p, s] = sum_x F_a(p)(x) F_b(p)(x) F_s(x) written as a GEMM
// over the spatial points x (the K dimension): rows are pair products
// (F_a F_b)(x), columns are third fields F_s(x).
//
// This is the FFT form of the standard estimator (Sec. 3.1, also its
// multipole form with D^(l)_k) and the real-space sum of M M M of the modal
// estimator (Sec. 3.5, eq. (betaEst)).
//
// Structure: a workgroup (12 waves, three per SIMD) owns a chunk of K points and a group of
// row tiles; each wave owns up to MAXR row tiles of 16 pairs and every needed
// 16-wide column tile of thirds, with the accumulators resident in registers.
// Points stream through LDS in stages of 64 (double buffered, one
// barrier per stage). Tiles whose outputs no triangle needs are skipped (the
// output is block sparse: a pair (b2, b3) only meets thirds b1 >= b2 that close
// a triangle).
//
// Precision modes (rows x cols per MFMA, points per MFMA):
//   0 FP32 : v_mfma 16x16x4 f32, exact FP32 products
//   1 BF16X3: a = ah + al, b = bh + bl (bf16 round-to-nearest-even splits of the
//            FP32 values), T += ah bh + ah bl + al bh on 16x16x32 bf16 MFMA
//   2 FP16X3: the same with fp16 splits of fields scaled by powers of two
//   3 FP64 : v_mfma 16x16x4 f64 (geometry precompute)
//   4 BF16X1: T += ah bh only (error study: what the lo parts buy)
// Each workgroup writes its chunk's partial tiles; a second kernel sums the
// chunks in FP64.
#include "tile_mfma.h"

namespace bsp {

constexpr int WAVES = 12;
constexpr int NTHR = WAVES * 64;
// LDS bytes of one workgroup for KS points per stage (two stage buffers).
template <int PREC, int KS>
size_t reduce_lds_bytes(const ReduceDesc& d) {
  constexpr bool SPLIT = (PREC == 1 || PREC == 2 || PREC == 4);
  using L = LdsRows<typename RT<PREC>::T, KS>;
  const size_t nfull = (SPLIT ? d.npf : d.nfields) + 1;
  size_t b = nfull * L::RS;
  if (SPLIT) b += (size_t)(d.nfields + 1) * L::HS;
  return b;
}

template <int PREC, int MAXR, int MAXC, int KS>
__global__ __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_reduce(
    const typename RT<PREC>::T* __restrict__ fields, ReduceDesc d, typename RT<PREC>::T* __restrict__ partials) {
  using WT = WaveTiles<PREC, MAXR, MAXC, WAVES, KS>;
  using T = typename WT::T;
  using L = typename WT::L;
  constexpr bool SPLIT = WT::SPLIT;
  constexpr int EPV = 16 / (int)sizeof(T);         // elements per 16-byte vector
  using VEC = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  constexpr int MAXV = (128 * KS / EPV + NTHR - 1) / NTHR;  // vectors per thread per stage (<= 128 fields)

  extern __shared__ __align__(16) unsigned char smem_raw[];
  // full-precision rows: the pair factors (split precisions: thirds come from the
  // split rows) or every field; the last row stays zero
  const int nfull = SPLIT ? d.npf : d.nfields;
  unsigned char* lf = smem_raw;
  unsigned char* lh = smem_raw + (size_t)(nfull + 1) * L::RS;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = lane >> 4, r16 = lane & 15;
  const int chunk = blockIdx.x, group = blockIdx.y;
  const int set = chunk / d.chunks_per_set;
  fields += (int64_t)set * d.set_stride;
  const int64_t k0 = (int64_t)(chunk - set * d.chunks_per_set) * d.kchunk;
  int64_t k1 = k0 + d.kchunk;
  if (k1 > d.K) k1 = d.K;
  const int nst = (int)((k1 - k0 + KS - 1) / KS);

  WT wt;
  wt.init(d, group, wave, q, r16);

  // zero rows (both buffers)
  for (int i = threadIdx.x; i < L::RS / 4; i += NTHR)
    reinterpret_cast<uint32_t*>(lf + (size_t)nfull * L::RS)[i] = 0u;
  if constexpr (SPLIT) {
    for (int i = threadIdx.x; i < L::HS / 4; i += NTHR)
      reinterpret_cast<uint32_t*>(lh + (size_t)d.nfields * L::HS)[i] = 0u;
  }

  // Each thread stages the same MAXV vectors (field f, point offset e) of every
  // stage; f and e follow from the thread index. Split precisions keep the
  // full-precision row of f packed (8 bits per vector, row + 1, 0: none);
  // otherwise the row is f itself.
  constexpr int VPR = KS / EPV;  // vectors per field row and stage
  static_assert(!SPLIT || MAXV <= 4, "packed rows: at most four vectors per thread");
  const int nvec = d.nfields * VPR;
  uint32_t frow_packed = 0;
  if constexpr (SPLIT) {
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
      const int vi = threadIdx.x + v * NTHR;
      const int fr = vi < nvec ? d.pf_row[vi / VPR] : -1;
      frow_packed |= (uint32_t)(fr + 1) << (8 * v);
    }
  }
  // 16-byte loads only when every field row stays 16-byte aligned
  const bool aligned = (d.field_stride % EPV == 0) && (d.set_stride % EPV == 0);
  VEC stage_regs[MAXV];
  auto gload = [&](int st) {
    const int64_t kb = k0 + (int64_t)st * KS;
    const bool full = aligned && (kb + KS <= k1);
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
      const int vi = threadIdx.x + v * NTHR;
      VEC val{};
      if (vi < nvec) {
        const int f = vi / VPR, e = (vi % VPR) * EPV;
        const T* src = fields + (int64_t)f * d.field_stride + kb + e;
        if (full) {
          typedef T TV __attribute__((ext_vector_type(EPV)));
          const TV x = __builtin_nontemporal_load(reinterpret_cast<const TV*>(src));
          if constexpr (EPV == 4) val = VEC{x[0], x[1], x[2], x[3]};
          else val = VEC{x[0], x[1]};
        } else {
          T tmp[EPV];
#pragma unroll
          for (int j = 0; j < EPV; ++j) tmp[j] = (kb + e + j < k1) ? src[j] : (T)0;
          val = *reinterpret_cast<VEC*>(tmp);
        }
      }
      stage_regs[v] = val;
    }
  };
  auto sstore = [&](auto bufc) {
    constexpr int BUF = decltype(bufc)::value;
#pragma unroll
    for (int v = 0; v < MAXV; ++v) {
      const int vi = threadIdx.x + v * NTHR;
      if (vi >= nvec) continue;
      const int f = vi / VPR, e = (vi % VPR) * EPV;
      VEC val = stage_regs[v];
      if constexpr (PREC == 2) {
        // FP16 split: every staged value carries its field's power-of-two scale
        const float sc = d.scale ? d.scale[f] : 1.0f;
        val.x *= sc; val.y *= sc; val.z *= sc; val.w *= sc;
      }
      const int fr = SPLIT ? (int)((frow_packed >> (8 * v)) & 0xffu) - 1 : f;
      if (fr >= 0) *reinterpret_cast<VEC*>(lf + fr * L::RS + e * (int)sizeof(T) + L::full(BUF)) = val;
      if constexpr (SPLIT) {
        // round-to-nearest-even split x = hi + lo, once per workgroup
        const float x[4] = {val.x, val.y, val.z, val.w};
        int2 hi, lo;
        split4<typename WT::H2>(x, hi, lo);
        unsigned char* hrow = lh + f * L::HS + e * 2;
        *reinterpret_cast<int2*>(hrow + L::half(BUF, 0)) = hi;
        *reinterpret_cast<int2*>(hrow + L::half(BUF, 1)) = lo;
      }
    }
  };
  auto ksteps = [&](auto bufc) {
    constexpr int BUF = decltype(bufc)::value;
    if (!wt.colmask_any) return;
#pragma unroll 1
    for (int ks = 0; ks < WT::NKS; ++ks) wt.template kstep<BUF>(lf, lh, ks);
  };
  using B0 = std::integral_constant<int, 0>;
  using B1 = std::integral_constant<int, 1>;

  if (nst > 0) {
    gload(0);
    sstore(B0{});
  }
  __syncthreads();
  // stages alternate between the two buffers; the loop body covers two
  for (int st = 0; st < nst; st += 2) {
    if (st + 1 < nst) gload(st + 1);
    ksteps(B0{});
    if (st + 1 < nst) sstore(B1{});
    __syncthreads();
    if (st + 1 >= nst) break;
    if (st + 2 < nst) gload(st + 2);
    ksteps(B1{});
    if (st + 2 < nst) sstore(B0{});
    __syncthreads();
  }
  wt.store(d, partials, chunk, q, r16);
}

// Sum chunk partials in FP64 and write T[pair][third] (entries outside every
// tile are left as they are; the caller zeroes T). The sums run in a fixed
// order, so T does not change between runs: block (tile, y) adds its range of
// chunks [y cpb, end) in order; with one range per tile it writes T directly,
// otherwise it parks its 256 FP64 sums in the partial slots of its own first
// two chunks (which nobody reads again) and k_combine_ranges adds the ranges
// in order. Every range holds at least cpb >= 2 chunks except when there is
// a single range.
template <typename PT>
__device__ __forceinline__ double* park_slot(PT* partials, int c0, int ntiles, int tile, int e) {
  if constexpr (sizeof(PT) == 8) {
    return reinterpret_cast<double*>(partials + ((int64_t)c0 * ntiles + tile) * 256) + e;
  } else {
    const int c = c0 + (e >> 7);
    return reinterpret_cast<double*>(partials + ((int64_t)c * ntiles + tile) * 256) + (e & 127);
  }
}

template <typename PT>
__device__ __forceinline__ void write_t(double s, int tile, int e, const int32_t* __restrict__ tile_rc,
                                        const int32_t* __restrict__ slot_pair, int npairs,
                                        int nthirds, const int32_t* __restrict__ pair_a,
                                        const int32_t* __restrict__ pair_b, const int32_t* __restrict__ third,
                                        const float* __restrict__ scale, double tscale, int accumulate,
                                        double* __restrict__ T) {
  const int slot = tile_rc[2 * tile] * 16 + e / 16;
  const int th = tile_rc[2 * tile + 1] * 16 + e % 16;
  const int pr = slot_pair[slot];
  if (pr >= 0 && pr < npairs && th < nthirds) {
    double f = tscale;
    if (scale) f /= (double)scale[pair_a[slot]] * (double)scale[pair_b[slot]] * (double)scale[third[th]];
    double* t = T + (int64_t)pr * nthirds + th;
    *t = accumulate ? *t + s * f : s * f;
  }
}

template <typename PT>
__global__ __launch_bounds__(256) void k_combine(PT* __restrict__ partials, int nchunks, int ntiles, int cpb, int nranges,
                                                 const int32_t* __restrict__ tile_rc,
                                                 const int32_t* __restrict__ slot_pair, int npairs, int nthirds,
                                                 const int32_t* __restrict__ pair_a, const int32_t* __restrict__ pair_b,
                                                 const int32_t* __restrict__ third, const float* __restrict__ scale,
                                                 double tscale, int accumulate, double* __restrict__ T) {
  const int tile = blockIdx.x;
  const int e = threadIdx.x;
  const int y = blockIdx.y;
  const int c0 = y * cpb;
  const int c1 = (y == nranges - 1) ? nchunks : c0 + cpb;
  double s = 0.0;
  for (int c = c0; c < c1; ++c) s += (double)partials[((int64_t)c * ntiles + tile) * 256 + e];
  if (nranges == 1) {
    write_t<PT>(s, tile, e, tile_rc, slot_pair, npairs, nthirds, pair_a, pair_b, third, scale, tscale, accumulate, T);
    return;
  }
  __syncthreads();  // every thread has read its values before the slots are overwritten
  *park_slot(partials, c0, ntiles, tile, e) = s;
}

template <typename PT>
__global__ __launch_bounds__(256) void k_combine_ranges(PT* __restrict__ partials, int ntiles, int cpb, int nranges,
                                                        const int32_t* __restrict__ tile_rc,
                                                 const int32_t* __restrict__ slot_pair, int npairs, int nthirds,
                                                        const int32_t* __restrict__ pair_a,
                                                        const int32_t* __restrict__ pair_b,
                                                        const int32_t* __restrict__ third,
                                                        const float* __restrict__ scale, double tscale,
                                                        int accumulate, double* __restrict__ T) {
  const int tile = blockIdx.x;
  const int e = threadIdx.x;
  double s = 0.0;
  for (int y = 0; y < nranges; ++y) s += *park_slot(partials, y * cpb, ntiles, tile, e);
  write_t<PT>(s, tile, e, tile_rc, slot_pair, npairs, nthirds, pair_a, pair_b, third, scale, tscale, accumulate, T);
}

int reduce_waves_per_group() { return WAVES; }
// (rows, columns) per wave: 12 waves, three per SIMD, 168 registers per lane;
// the FP32 accumulators of rows x columns tiles take 4 registers each (FP64: 8).
int reduce_shapes(int prec, ReduceShape* out, int max_out) {
  static const ReduceShape f32[] = {{5, 1}, {6, 2}, {4, 4}, {3, 6}, {2, 8}};
  static const ReduceShape f64[] = {{4, 1}, {4, 2}, {2, 4}, {1, 8}};
  const ReduceShape* t = prec == 3 ? f64 : f32;
  const int n = prec == 3 ? 4 : 5;
  for (int i = 0; i < n && i < max_out; ++i) out[i] = t[i];
  return n;
}

template <int PREC, int KS>
static hipError_t reduce_dispatch_ks(const void* fields, const ReduceDesc& d, void* partials, hipStream_t s) {
  using T = typename RT<PREC>::T;
  const size_t lds = reduce_lds_bytes<PREC, KS>(d);
  dim3 grid((unsigned)d.nchunks, (unsigned)d.ngroups);
  const T* f = reinterpret_cast<const T*>(fields);
  T* p = reinterpret_cast<T*>(partials);
#define RCASE(R, C)                                                                       \
  if (d.maxr == R && d.maxcw == C) {                                                      \
    hipLaunchKernelGGL((k_reduce<PREC, R, C, KS>), grid, dim3(NTHR), lds, s, f, d, p);    \
    return hipGetLastError();                                                             \
  }
  if constexpr (PREC == 3) {
    RCASE(4, 1) RCASE(4, 2) RCASE(2, 4) RCASE(1, 8)
  } else {
    RCASE(5, 1) RCASE(6, 2) RCASE(4, 4) RCASE(3, 6) RCASE(2, 8)
  }
#undef RCASE
  return hipErrorInvalidValue;
}

constexpr size_t LDS_LIMIT = 160 * 1024;

template <int PREC>
static hipError_t reduce_dispatch(const void* fields, const ReduceDesc& d, void* partials, hipStream_t s) {
  // 96-point stages (fewer barriers) need more staging registers than the
  // 168-register budget of three waves per SIMD leaves: 64 points throughout
  if (reduce_lds_bytes<PREC, 64>(d) > LDS_LIMIT) return hipErrorInvalidValue;
  return reduce_dispatch_ks<PREC, 64>(fields, d, partials, s);
}

hipError_t launch_reduce(int prec, const float* fields, const ReduceDesc& d, float* partials, hipStream_t s) {
  if (d.nfields > 128) return hipErrorInvalidValue;
  switch (prec) {
    case 0: return reduce_dispatch<0>(fields, d, partials, s);
    case 1: return reduce_dispatch<1>(fields, d, partials, s);
    case 2: return reduce_dispatch<2>(fields, d, partials, s);
    case 4: return reduce_dispatch<4>(fields, d, partials, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_reduce_f64(const double* fields, const ReduceDesc& d, double* partials, hipStream_t s) {
  if (d.nfields > 128) return hipErrorInvalidValue;
  return reduce_dispatch<3>(fields, d, partials, s);
}

hipError_t launch_combine_partials(void* partials, int is_f64, const ReduceDesc& d, int npairs, int nthirds,
                                   double* T, double tscale, int accumulate, hipStream_t s) {
  const int cpb = 64;
  const int nranges = d.nchunks > cpb ? d.nchunks / cpb : 1;
  dim3 grid((unsigned)d.ntiles, (unsigned)nranges);
  if (is_f64) {
    double* pp = reinterpret_cast<double*>(partials);
    hipLaunchKernelGGL((k_combine<double>), grid, dim3(256), 0, s, pp, d.nchunks, d.ntiles, cpb, nranges, d.tile_rc, d.slot_pair,
                       npairs, nthirds, d.pair_a, d.pair_b, d.third, d.scale, tscale, accumulate, T);
    if (nranges > 1)
      hipLaunchKernelGGL((k_combine_ranges<double>), dim3((unsigned)d.ntiles), dim3(256), 0, s, pp, d.ntiles, cpb,
                         nranges, d.tile_rc, d.slot_pair, npairs, nthirds, d.pair_a, d.pair_b, d.third, d.scale, tscale, accumulate, T);
  } else {
    float* pp = reinterpret_cast<float*>(partials);
    hipLaunchKernelGGL((k_combine<float>), grid, dim3(256), 0, s, pp, d.nchunks, d.ntiles, cpb, nranges, d.tile_rc, d.slot_pair,
                       npairs, nthirds, d.pair_a, d.pair_b, d.third, d.scale, tscale, accumulate, T);
    if (nranges > 1)
      hipLaunchKernelGGL((k_combine_ranges<float>), dim3((unsigned)d.ntiles), dim3(256), 0, s, pp, d.ntiles, cpb,
                         nranges, d.tile_rc, d.slot_pair, npairs, nthirds, d.pair_a, d.pair_b, d.third, d.scale, tscale, accumulate, T);
  }
  return hipGetLastError();
}

}  // namespace bsp
