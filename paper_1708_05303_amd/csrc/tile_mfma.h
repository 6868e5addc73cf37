// Register-resident 16x16 output tiles of the triple-reduction GEMM and the
// MFMA k-step over one LDS stage of the reduction over materialised fields
// (reduce.hip).

//
// A wave owns up to MAXR row tiles (16 pair products each) and up to MAXC
// column tiles (16 third fields each) of its own; a row's needed columns are
// a bit mask over the wave's column slots.
#pragma once

#include "bsp_internal.h"

namespace bsp {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// Split eight floats into 16-bit high parts and the 16-bit rounding of their
// remainders, two values per conversion; each pair is kept as one 32-bit word
// (int vectors survive control flow without being split into 16-bit pieces).
template <typename H2>
__device__ __forceinline__ void split8(const float* x, i32x4& hi, i32x4& lo) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const f32x2 v{x[2 * j], x[2 * j + 1]};
    const H2 h = __builtin_convertvector(v, H2);
    const f32x2 hf = __builtin_convertvector(h, f32x2);
    const f32x2 rem{v.x - hf.x, v.y - hf.y};
    hi[j] = __builtin_bit_cast(int, h);
    lo[j] = __builtin_bit_cast(int, __builtin_convertvector(rem, H2));
  }
}

// PREC 0 FP32, 1 BF16 hi+lo, 2 FP16 hi+lo, 3 FP64, 4 BF16 hi only (error study).
template <int PREC> struct RT;
template <> struct RT<0> { using T = float; using acc = f32x4; static constexpr int KK = 8; };
template <> struct RT<1> { using T = float; using acc = f32x4; static constexpr int KK = 8; };
template <> struct RT<2> { using T = float; using acc = f32x4; static constexpr int KK = 8; };
template <> struct RT<3> { using T = double; using acc = f64x4; static constexpr int KK = 2; };
template <> struct RT<4> { using T = float; using acc = f32x4; static constexpr int KK = 8; };

// The same split for four floats (two packed words each).
template <typename H2>
__device__ __forceinline__ void split4(const float* x, int2& hi, int2& lo) {
  int h[2], l[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const f32x2 v{x[2 * j], x[2 * j + 1]};
    const H2 hv = __builtin_convertvector(v, H2);
    const f32x2 hf = __builtin_convertvector(hv, f32x2);
    const f32x2 rem{v.x - hf.x, v.y - hf.y};
    h[j] = __builtin_bit_cast(int, hv);
    l[j] = __builtin_bit_cast(int, __builtin_convertvector(rem, H2));
  }
  hi = int2{h[0], h[1]};
  lo = int2{l[0], l[1]};
}

template <typename V>
__device__ __forceinline__ V lds_ld(const unsigned char* p) {
  return *reinterpret_cast<const V*>(p);
}

// LDS layout of one stage pair (both double buffers interleaved in each row, so
// that every k-step reads at compile-time offsets from per-lane row addresses):
//   full-precision row  [buffer 0: KS values][buffer 1: KS values][16 bytes pad]
//   split row (16-bit)  [hi 0][lo 0][hi 1][lo 1] (KS halves each) [16 bytes pad]
// The 16-byte pad puts 16 consecutive rows on distinct 4-bank groups.
template <typename T, int KS> struct LdsRows {
  static constexpr int RS = 2 * KS * (int)sizeof(T) + 16;
  static constexpr int HS = 8 * KS + 16;
  static constexpr int full(int buf) { return buf * KS * (int)sizeof(T); }
  static constexpr int half(int buf, int lo) { return (2 * buf + lo) * KS * 2; }
};

template <int PREC, int MAXR, int MAXC, int WAVES, int KS> struct WaveTiles {
  using T = typename RT<PREC>::T;
  using ACC = typename RT<PREC>::acc;
  static constexpr bool SPLIT = (PREC == 1 || PREC == 2 || PREC == 4);
  using H = typename std::conditional<PREC == 2, _Float16, __bf16>::type;
  using H8 = typename std::conditional<PREC == 2, f16x8, bf16x8>::type;
  using H2 = typename std::conditional<PREC == 2, f16x2, bf16x2>::type;
  using L = LdsRows<T, KS>;
  static constexpr int KK = RT<PREC>::KK;
  static constexpr int KSTEP = 4 * KK;
  static constexpr int NKS = KS / KSTEP;

  int rows[MAXR], masks[MAXR], cols[MAXC];
  // per-lane byte offsets into the LDS rows: first and second pair factor of
  // each row slot, third of each column slot
  int oa[MAXR], ob[MAXR], oc[MAXC];
  int colmask_any;
  ACC acc[MAXR][MAXC];

  // The tile lists are wave-uniform: reading them through a uniform wave index
  // keeps them in scalar registers and the block-sparse skips scalar branches.
  __device__ __forceinline__ void init(const ReduceDesc& d, int group, int wave_in, int q, int r16) {
    const int wave = __builtin_amdgcn_readfirstlane(wave_in);
#pragma unroll
    for (int c = 0; c < MAXC; ++c) cols[c] = d.wave_cols[(group * WAVES + wave) * MAXC + c];
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
      rows[r] = d.wave_rows[(group * WAVES + wave) * MAXR + r];
      const int gm = rows[r] >= 0 ? d.row_mask[rows[r]] : 0;
      int m = 0;
#pragma unroll
      for (int c = 0; c < MAXC; ++c)
        if (cols[c] >= 0 && ((gm >> cols[c]) & 1)) m |= 1 << c;
      masks[r] = __builtin_amdgcn_readfirstlane(m);
    }
    // pair factors index the full-precision rows: only the pair-factor fields
    // (row npf stays zero) when SPLIT, every field (row nfields zero) otherwise
    const int32_t* ra = SPLIT ? d.pair_ra : d.pair_a;
    const int32_t* rb = SPLIT ? d.pair_rb : d.pair_b;
    const int zrow = SPLIT ? d.npf : d.nfields;
    const int lane_k = q * KK * (int)sizeof(T);
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
      const int pr = rows[r] * 16 + r16;
      const int a = rows[r] >= 0 ? ra[pr] : -1;
      const int b = rows[r] >= 0 ? rb[pr] : -1;
      oa[r] = (a >= 0 ? a : zrow) * L::RS + lane_k;
      ob[r] = (b >= 0 ? b : zrow) * L::RS + lane_k;
    }
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
      const int s = cols[c] >= 0 ? d.third[cols[c] * 16 + r16] : -1;
      const int srow = s >= 0 ? s : d.nfields;
      oc[c] = SPLIT ? srow * L::HS + q * KK * 2 : srow * L::RS + lane_k;
    }
    colmask_any = 0;
#pragma unroll
    for (int r = 0; r < MAXR; ++r) colmask_any |= masks[r];
#pragma unroll
    for (int r = 0; r < MAXR; ++r)
#pragma unroll
      for (int c = 0; c < MAXC; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[r][c][i] = (T)0;
  }

  // Pair products of row slot r at the KK points of this lane (byte offset
  // `ko` of the k-step inside the rows).
  __device__ __forceinline__ void products(const unsigned char* __restrict__ lf, int r, int ko, T* x) const {
    if constexpr (PREC == 3) {
      const double2 a0 = lds_ld<double2>(lf + oa[r] + ko);
      const double2 b0 = lds_ld<double2>(lf + ob[r] + ko);
      x[0] = a0.x * b0.x;
      x[1] = a0.y * b0.y;
    } else {
      const float4 a0 = lds_ld<float4>(lf + oa[r] + ko), a1 = lds_ld<float4>(lf + oa[r] + ko + 16);
      const float4 b0 = lds_ld<float4>(lf + ob[r] + ko), b1 = lds_ld<float4>(lf + ob[r] + ko + 16);
      x[0] = a0.x * b0.x;
      x[1] = a0.y * b0.y;
      x[2] = a0.z * b0.z;
      x[3] = a0.w * b0.w;
      x[4] = a1.x * b1.x;
      x[5] = a1.y * b1.y;
      x[6] = a1.z * b1.z;
      x[7] = a1.w * b1.w;
    }
  }

  // One k-step (KSTEP points) of stage buffer BUF: lf holds the full-precision
  // rows, lh the split rows (SPLIT only).
  template <int BUF>
  __device__ __forceinline__ void kstep(const unsigned char* __restrict__ lf, const unsigned char* __restrict__ lh,
                                        int ks) {
    const int ko = L::full(BUF) + ks * KSTEP * (int)sizeof(T);
    if constexpr (!SPLIT) {
      T av[MAXR][KK];
#pragma unroll
      for (int r = 0; r < MAXR; ++r) products(lf, r, ko, av[r]);
      auto load_col = [&](int c, T* dst) {
        if constexpr (PREC == 3) {
          const double2 b0 = lds_ld<double2>(lf + oc[c] + ko);
          dst[0] = b0.x;
          dst[1] = b0.y;
        } else {
          const float4 b0 = lds_ld<float4>(lf + oc[c] + ko), b1 = lds_ld<float4>(lf + oc[c] + ko + 16);
          dst[0] = b0.x; dst[1] = b0.y; dst[2] = b0.z; dst[3] = b0.w;
          dst[4] = b1.x; dst[5] = b1.y; dst[6] = b1.z; dst[7] = b1.w;
        }
      };
#pragma unroll
      for (int c = 0; c < MAXC; ++c) {
        if (!((colmask_any >> c) & 1)) continue;
        T b[KK];
        load_col(c, b);
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
          if (!((masks[r] >> c) & 1)) continue;
#pragma unroll
          for (int j = 0; j < KK; ++j) {
            if constexpr (PREC == 0)
              acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r][j], b[j], acc[r][c], 0, 0, 0);
            else
              acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r][j], b[j], acc[r][c], 0, 0, 0);
          }
        }
      }
    } else {
      const int ho = L::half(BUF, 0) + ks * KSTEP * 2, lo_o = L::half(BUF, 1) + ks * KSTEP * 2;
      i32x4 ah[MAXR], al[MAXR];
#pragma unroll
      for (int r = 0; r < MAXR; ++r) {
        // empty rows read the zero row: no branch, no value carried across steps
        float x[KK];
        products(lf, r, ko, x);
        split8<H2>(x, ah[r], al[r]);
      }
#pragma unroll
      for (int c = 0; c < MAXC; ++c) {
        if (!((colmask_any >> c) & 1)) continue;
        const H8 h = lds_ld<H8>(lh + oc[c] + ho);
        const H8 l = lds_ld<H8>(lh + oc[c] + lo_o);
#pragma unroll
        for (int r = 0; r < MAXR; ++r) {
          if (!((masks[r] >> c) & 1)) continue;
          const H8 a_h = __builtin_bit_cast(H8, ah[r]), a_l = __builtin_bit_cast(H8, al[r]);
          if constexpr (PREC == 1) {
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, h, acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, l, acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_l, h, acc[r][c], 0, 0, 0);
          } else if constexpr (PREC == 4) {
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a_h, h, acc[r][c], 0, 0, 0);
          } else {
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, h, acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_h, l, acc[r][c], 0, 0, 0);
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a_l, h, acc[r][c], 0, 0, 0);
          }
        }
      }
    }
  }

  // Partial tiles of one chunk, column r16 of each tile; the f32 16x16x4 and
  // 16x16x32 results hold rows 4q + i in lane group q, the f64 16x16x4 result
  // holds rows q + 4i.
  __device__ __forceinline__ void store(const ReduceDesc& d, T* __restrict__ partials, int chunk, int q, int r16) {
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
      if (masks[r] == 0) continue;
#pragma unroll
      for (int c = 0; c < MAXC; ++c) {
        if (!((masks[r] >> c) & 1)) continue;
        const int tile = d.tile_index[rows[r] * 8 + cols[c]];
        T* out = partials + ((int64_t)chunk * d.ntiles + tile) * 256;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = (PREC == 3) ? (q + 4 * i) : (4 * q + i);
          out[row * 16 + r16] = acc[r][c][i];
        }
      }
    }
  }
};

}  // namespace bsp
