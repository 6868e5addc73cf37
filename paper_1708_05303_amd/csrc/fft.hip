// Radix-2/3/4/8 Stockham FFTs staged in LDS, and the three kinds of passes a
// pruned 3-D transform is built from:
//
//   fwd_z : real lines along z -> half-complex, two real lines packed per
//           complex transform; optionally forms the density contrast and the
//           line-of-sight weights, so that one read of the grid feeds every
//           weighted field h_m(x_hat) delta(x) (the LOS moment field of the
//           power-spectrum section of the paper, expanded in the real solid
//           harmonics h_m of x_hat: 1 + 5 + 9 fields for l <= 4).
//   c2c   : a strided column pass along y or x; a workgroup owns W consecutive
//           inner columns (one 128-byte row segment) and all N rows, so every
//           global access is a coalesced row segment. Input and output rows may
//           be pruned to the band |n| <= c the estimator needs; the shell or
//           modal filter of the inverse transforms (the D^(l)_k and M^(l)_n
//           fields of the standard and modal estimators) can be applied while
//           loading.
//   inv_z : half-complex -> real lines along z, two fields per complex
//           transform (Hermitian fill of the missing half).
//
// Twiddles come from a per-length table exp(-2 pi i j / N) built on the host
// in double precision, in the order the butterfly passes read them, and
// staged through LDS.
// The z-line kernels address their line buffers through a bank swizzle
// (swz), which keeps the strided stores of the first passes conflict-free.
#include "bsp_internal.h"

namespace bsp {

constexpr int pick_radix(int m) {
  return (m % 8 == 0) ? 8 : (m % 4 == 0) ? 4 : (m % 2 == 0) ? 2 : (m % 3 == 0) ? 3 : 1;
}
constexpr int radix_at(int n, int s) {
  int m = n;
  for (int i = 0; i < s; ++i) m /= pick_radix(m);
  return pick_radix(m);
}
constexpr int nstages(int n) {
  int c = 0, m = n;
  while (m > 1) {
    m /= pick_radix(m);
    ++c;
  }
  return c;
}

// LDS twiddles are stored pass by pass: the pass with sub-length NS and radix R
// reads W_{NS R}^{r k} (r = 1 .. R-1, k < NS) at (NS - 1) + (r - 1) NS + k, so
// the lanes of a pass read consecutive entries; the host builds the table in
// this order (N - 1 entries).

// Bank swizzle of a line buffer: XOR of the low five index bits with bits
// 3..7. A permutation of [0, N) for every supported N (multiples of 32, or
// below 32), it spreads the stride-R stores of the early passes over distinct
// banks for 8- and 16-byte elements.
template <int SWZ> __device__ __forceinline__ int swz(int i) {
  if constexpr (SWZ) return i ^ ((i >> 3) & 31);
  else return i;
}

// Synchronisation between the LDS passes of one transform. When the NT = N/8
// threads of a z line divide 64 (power-of-two N), a line lives inside one wave;
// a wave's LDS instructions complete in order, so the passes only need the
// compiler kept from reordering them (WAVE = 1). Lines of N = 96, 192, 384
// straddle waves, and column tiles span the whole workgroup: both take a
// workgroup barrier.
template <int WAVE> __device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Line groups per workgroup of the z-line kernels: one twiddle staging serves
// LZ_GROUPS x (256 / (N/8)) lines.
constexpr int LZ_GROUPS = 8;
constexpr int FZ_GROUPS = 1;     // line groups per workgroup of the forward z pass
constexpr int FZ_WAVE_SYNC = 1;  // wave-level sync of the forward z pass (power-of-two N)
// 1 when the lines of a z-line kernel of length N never straddle waves.
constexpr int line_in_wave(int n) { return (64 % ((n >= 8) ? n / 8 : 1)) == 0 ? 1 : 0; }

// multiply by SIGN * i
template <int SIGN, typename V> __device__ __forceinline__ V mul_si(V a) {
  if constexpr (SIGN < 0) return V{a.y, -a.x};
  else return V{-a.y, a.x};
}

template <int R, int SIGN, typename V> __device__ __forceinline__ void butterfly(V* v) {
  using T = decltype(v[0].x);
  if constexpr (R == 2) {
    V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 3) {
    const T h = (T)0.86602540378443864676;  // sqrt(3)/2
    V t1 = cadd(v[1], v[2]);
    V t2 = V{v[0].x - (T)0.5 * t1.x, v[0].y - (T)0.5 * t1.y};
    V d = csub(v[1], v[2]);
    V t3 = mul_si<SIGN>(V{h * d.x, h * d.y});
    v[0] = cadd(v[0], t1);
    v[1] = cadd(t2, t3);
    v[2] = csub(t2, t3);
  } else if constexpr (R == 4) {
    V a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
    V a2 = cadd(v[1], v[3]), a3 = mul_si<SIGN>(csub(v[1], v[3]));
    v[0] = cadd(a0, a2);
    v[2] = csub(a0, a2);
    v[1] = cadd(a1, a3);
    v[3] = csub(a1, a3);
  } else if constexpr (R == 8) {
    const T r2 = (T)0.70710678118654752440;
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    butterfly<4, SIGN>(e);
    butterfly<4, SIGN>(o);
    // o[k] *= exp(SIGN i pi k / 4)
    V o1 = V{r2 * o[1].x, r2 * o[1].y};
    o1 = cadd(o1, mul_si<SIGN>(o1));
    V o2 = mul_si<SIGN>(o[2]);
    V o3 = mul_si<SIGN>(V{r2 * o[3].x, r2 * o[3].y});
    o3 = cadd(o3, mul_si<SIGN>(o3));
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
}

// One length-N transform held in buf[0..N) (LDS), computed by NT threads with
// thread index t. All threads of the block must call this (it synchronises).
// Stage s with sub-length NS: butterfly b reads b + r N/R, twiddles by
// W_{NS R}^{r (b mod NS)}, and writes (b/NS) NS R + (b mod NS) + r NS.
template <typename V, int N, int SIGN, int NT, int S, int NS, int SWZ, int WAVE, int SEND = nstages(N)>
__device__ __forceinline__ void fft_stages(V* __restrict__ buf, const V* __restrict__ tw, int t) {
  if constexpr (S < SEND) {
    constexpr int R = radix_at(N, S);
    constexpr int NB = N / R;
    constexpr int PER = (NB + NT - 1) / NT;
    V v[PER][R];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = t + i * NT;
      if ((NB % NT == 0) || b < NB) {
        const int k = b % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = buf[swz<SWZ>(b + r * NB)];
        if constexpr (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            V w = tw[(NS - 1) + (r - 1) * NS + k];
            if constexpr (SIGN > 0) w.y = -w.y;
            v[i][r] = cmul(v[i][r], w);
          }
        }
        butterfly<R, SIGN>(v[i]);
      }
    }
    lds_sync<WAVE>();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = t + i * NT;
      if ((NB % NT == 0) || b < NB) {
        const int k = b % NS;
        const int d = (b / NS) * NS * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[swz<SWZ>(d + r * NS)] = v[i][r];
      }
    }
    lds_sync<WAVE>();
    fft_stages<V, N, SIGN, NT, S + 1, NS * R, SWZ, WAVE, SEND>(buf, tw, t);
  }
}

// Register-held ends of a transform. Thread t holds elements t + NT e
// (e < N / NT). When N / R0 (R0 the first radix) is a multiple of NT, the
// first pass's butterflies read exactly those elements, so the pass takes its
// input from registers instead of an LDS round trip; when N / RL (RL the last
// radix) is a multiple of NT, the last pass's butterflies write exactly those
// elements, so its output stays in registers.
constexpr bool reg_in(int n, int nt) { return n % nt == 0 && nstages(n) >= 2 && (n / radix_at(n, 0)) % nt == 0; }
constexpr bool reg_out(int n, int nt) {
  return reg_in(n, nt) && (n / radix_at(n, nstages(n) - 1)) % nt == 0;
}

// Length-N transform of x (layout above) with buf as the exchange buffer
// between passes. OUT_REG: the result is left in x; otherwise in buf (natural
// order), as fft_stages leaves it. The caller synchronises before buf is
// written again.
template <typename V, int N, int SIGN, int NT, int SWZ, int WAVE, bool OUT_REG>
__device__ __forceinline__ void fft_reg(V* __restrict__ buf, const V* __restrict__ tw, int t, V* x) {
  static_assert(reg_in(N, NT) && (!OUT_REG || reg_out(N, NT)), "pass layout does not match the thread layout");
  constexpr int NSTG = nstages(N);
  constexpr int R0 = radix_at(N, 0);
  {
    constexpr int PER = N / R0 / NT;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      V v[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) v[r] = x[i + r * PER];
      butterfly<R0, SIGN>(v);
      const int b = t + i * NT;
#pragma unroll
      for (int r = 0; r < R0; ++r) buf[swz<SWZ>(b * R0 + r)] = v[r];
    }
  }
  lds_sync<WAVE>();
  if constexpr (!OUT_REG) {
    fft_stages<V, N, SIGN, NT, 1, R0, SWZ, WAVE>(buf, tw, t);
  } else {
    fft_stages<V, N, SIGN, NT, 1, R0, SWZ, WAVE, NSTG - 1>(buf, tw, t);
    constexpr int R = radix_at(N, NSTG - 1), NS = N / R, PER = NS / NT;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int b = t + i * NT;  // b < NS: the butterfly's twiddle index and output base
      V v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = buf[swz<SWZ>(b + r * NS)];
#pragma unroll
      for (int r = 1; r < R; ++r) {
        V w = tw[(NS - 1) + (r - 1) * NS + b];
        if constexpr (SIGN > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
      }
      butterfly<R, SIGN>(v);
#pragma unroll
      for (int r = 0; r < R; ++r) x[i + r * PER] = v[r];
    }
  }
}

// Streaming store of a complex value (written once, read by a later kernel).
template <typename V> __device__ __forceinline__ void nt_store(V* p, const V& v) {
  using E = decltype(v.x);
  typedef E E2 __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(E2{v.x, v.y}, reinterpret_cast<E2*>(p));
}

template <typename V> __device__ __forceinline__ V nt_load(const V* p) {
  using E = decltype(p->x);
  typedef E E2 __attribute__((ext_vector_type(2)));
  const E2 v = __builtin_nontemporal_load(reinterpret_cast<const E2*>(p));
  return V{v.x, v.y};
}

// Value of v in the lane whose byte address (4 x lane) is addr, within the
// wave (ds_bpermute per 32-bit word; every lane of the wave must execute it).
template <typename T> __device__ __forceinline__ T lane_read(int addr, T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, v)));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)u);
    const unsigned hi = (unsigned)__builtin_amdgcn_ds_bpermute(addr, (int)(unsigned)(u >> 32));
    return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
  }
}

// Weight of LOS field F at a node: the real solid harmonic h_F(x_hat) (see
// kLosPoly), evaluated in the transform's precision.
template <int F, typename T> __device__ __forceinline__ T los_weight(T hx, T hy, T hz) {
  return los_harmonic<F, T>(hx, hy, hz);
}

// One packed pair (F0, F0+1) of LOS fields for every line of the block, then
// the next pair; the field indices are compile-time so the weights unroll.
template <int F0, int NLOS, typename T, typename V, int N, int NT, int E, int PAD>
__device__ __forceinline__ void fwd_z_pairs(V* b, const V* tw, int t, const T* rv, T rx, T ry, T sh, T oz,
                                            const T* inv, bool plane, bool valid, V* out_g, int64_t nlines,
                                            int64_t line, int cout, int zs) {
  if constexpr (F0 < NLOS) {
    constexpr bool HAS1 = F0 + 1 < NLOS;
    constexpr int WS = FZ_WAVE_SYNC && line_in_wave(N);
    V x[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      T w0 = (T)1, w1 = (T)0;
      if (!plane) {
        // x_hat of node z = t + e NT, rebuilt from its 1 / |r| (fewer live registers)
        const T hx = rx * inv[e], hy = ry * inv[e], hz = ((T)(t + e * NT) - sh - oz) * inv[e];
        w0 = los_weight<F0>(hx, hy, hz);
        if constexpr (HAS1) w1 = los_weight<(HAS1 ? F0 + 1 : 0)>(hx, hy, hz);
      }
      x[e] = V{w0 * rv[e], w1 * rv[e]};
    }
    V* o0 = out_g + ((int64_t)F0 * nlines + line) * zs;
    V* o1 = out_g + ((int64_t)(F0 + 1) * nlines + line) * zs;
    // the two real fields packed as z = a + i b separate as
    // a_k = (z_k + conj z_{N-k}) / 2, b_k = (z_k - conj z_{N-k}) / (2i)
    auto split = [&](int k, const V& zk, const V& zm) {
      nt_store(o0 + k, V{(zk.x + zm.x) * (T)0.5, (zk.y - zm.y) * (T)0.5});
      if constexpr (HAS1) nt_store(o1 + k, V{(zk.y + zm.y) * (T)0.5, (zm.x - zk.x) * (T)0.5});
    };
    if constexpr (reg_out(N, NT) && line_in_wave(N) && E == 8) {
      // both ends in registers. Lane t holds z at t + NT e; the partner of
      // k = t + NT j is N - k = (NT - t) + NT (7 - j) for t > 0 (lane NT - t of
      // the same line, same wave) and NT (8 - j) mod N for t = 0 (own lane)
      fft_reg<V, N, -1, NT, 1, WS, true>(b, tw, t, x);
      const int lane = (int)(threadIdx.x & 63);
      const int src = (lane - t + ((NT - t) & (NT - 1))) * 4;
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        if (NT * j >= cout) break;  // uniform: cout <= N/2 + 1
        const V zr = V{lane_read(src, x[7 - j].x), lane_read(src, x[7 - j].y)};
        const V zm = t == 0 ? x[(8 - j) & 7] : zr;
        if (valid && t + NT * j < cout) split(t + NT * j, x[j], zm);
      }
    } else {
      if constexpr (reg_in(N, NT)) {
        // the first pass takes the weighted line from registers
        fft_reg<V, N, -1, NT, 1, WS, false>(b, tw, t, x);
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) b[swz<1>(t + e * NT)] = x[e];
        lds_sync<WS>();
        fft_stages<V, N, -1, NT, 0, 1, 1, WS>(b, tw, t);
      }
      if (valid)
        for (int k = t; k < cout; k += NT) split(k, b[swz<1>(k)], b[swz<1>((N - k) % N)]);
    }
    lds_sync<WS>();
    fwd_z_pairs<F0 + 2, NLOS, T, V, N, NT, E, PAD>(b, tw, t, rv, rx, ry, sh, oz, inv, plane, valid, out_g, nlines,
                                                   line, cout, zs);
  }
}

// Waves per SIMD the forward z pass is compiled for: FP32 power-of-two sizes
// keep both transform ends in registers and fit 128 registers (four waves);
// the others keep the compiler's choice.
constexpr int fz_waves(size_t tsize, int n) { return tsize == 4 && (n & (n - 1)) == 0 ? 4 : 1; }

// ---------------------------------------------------------------- fwd_z
// grid: blockIdx.x -> LZ_GROUPS consecutive groups of L lines (line = x*N + y), blockIdx.y -> input grid.
// FP32 power-of-two sizes are held to 128 registers (fz_waves).
template <typename T, int N, int NLOS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(fz_waves(sizeof(T), N))))
void k_fwd_z(const T* __restrict__ in, cplx_t<T>* __restrict__ out, FwdZDesc d, const cplx_t<T>* __restrict__ twg) {
  using V = cplx_t<T>;
  constexpr int NT = (N >= 8) ? N / 8 : 1;
  constexpr int L = 256 / NT;
  constexpr int PAD = N + 1;
  constexpr int E = N / NT;
  __shared__ V buf[L * PAD];
  __shared__ V tw[N];
  for (int i = threadIdx.x; i < N; i += L * NT) tw[i] = twg[i];
  const int ll = threadIdx.x / NT, t = threadIdx.x % NT;
  const int64_t nlines = (int64_t)N * N;
  const int g = blockIdx.y;
  T scale = (T)1, sub = (T)0;
  if (d.contrast) {
    scale = (T)((double)N * (double)N * (double)N / d.wsum[0]);
    sub = (T)1;
  }
  __syncthreads();  // twiddles staged
  V* b = buf + ll * PAD;
  V* out_g = out + (int64_t)g * NLOS * nlines * d.zs;
  for (int rep = 0; rep < FZ_GROUPS; ++rep) {
    const int64_t line = ((int64_t)blockIdx.x * FZ_GROUPS + rep) * L + ll;
    const bool valid = line < nlines;
    const int x = valid ? (int)(line / N) : 0, y = valid ? (int)(line % N) : 0;
    const T* src = in + (int64_t)g * N * N * N + (valid ? line : 0) * N;
    T rv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) rv[e] = valid ? src[t + e * NT] * scale - sub : (T)0;
    T inv[E];
    T rx = (T)0, ry = (T)0;
    const T sh = (T)d.shift[g], oz = (T)d.obs[2];
    if (!d.plane) {
      rx = (T)x - sh - (T)d.obs[0];
      ry = (T)y - sh - (T)d.obs[1];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const T rz = (T)(t + e * NT) - sh - oz;
        inv[e] = (T)1 / sqrt(rx * rx + ry * ry + rz * rz);
      }
    }
    fwd_z_pairs<0, NLOS, T, V, N, NT, E, PAD>(b, tw, t, rv, rx, ry, sh, oz, inv, d.plane != 0, valid, out_g, nlines,
                                              line, d.cout, d.zs);
  }
}

// ---------------------------------------------------------------- c2c
// grid: blockIdx.x -> column tile of W, blockIdx.y (+ gridDim.y * blockIdx.z) -> outer batch.
// Inner columns are runs of ncz: column col = jj * ncz + kz reads inner offset
// (jj + in_j0) * in_js + kz and writes jj * out_js + kz (a sub-block of a 2-D
// inner layout; 1-D when ncz >= ncols). Every global load of the tile is issued
// before the LDS writes, so each thread keeps N/NT loads in flight.
template <typename T, int N, int W, int SIGN, bool FILT, int BT>
__global__ __launch_bounds__(BT) void k_c2c(const cplx_t<T>* __restrict__ in, cplx_t<T>* __restrict__ out,
                                             PassDesc p, FilterDesc f, const cplx_t<T>* __restrict__ twg) {
  using V = cplx_t<T>;
  constexpr int NT = BT / W;
  constexpr int PAD = N + 1;
  constexpr int E = (N + NT - 1) / NT;
  __shared__ V buf[W * PAD];
  __shared__ V tw[N];
  for (int i = threadIdx.x; i < N; i += BT) tw[i] = twg[i];
  const int outer = blockIdx.y + gridDim.y * blockIdx.z;
  if (outer >= p.nouter) return;  // uniform per block
  const int c = threadIdx.x % W, j0 = threadIdx.x / W;
  const int col = blockIdx.x * W + c;
  const bool cv = col < p.ncols;
  const int jj = cv ? col / p.ncz : 0, kz = cv ? col % p.ncz : 0;
  const int64_t icol = (int64_t)(jj + p.in_j0) * p.in_js + kz;
  const int64_t ocol = (int64_t)jj * p.out_js + kz;
  const V* src;
  const T* tab = nullptr;
  int fny = 0, lo2 = 0, hi2 = 0, unit = 0;
  bool fz_ok = true;
  if constexpr (FILT) {
    const int field = f.field0 + outer;
    src = reinterpret_cast<const V*>(f.src) + (int64_t)f.field_ell[field] * f.src_ell_stride +
          (int64_t)f.row0 * p.in_row;
    const int row = f.field_table[field];
    tab = reinterpret_cast<const T*>(f.tables) + (int64_t)row * f.tablen;
    lo2 = f.row_range[3 * row];
    hi2 = f.row_range[3 * row + 1];
    unit = f.row_range[3 * row + 2];
    fny = jj + p.in_j0 - f.c;
    fz_ok = kz <= f.c;
  } else {
    src = in + (int64_t)outer * p.in_outer;
  }
  V* dst = out + (int64_t)outer * p.out_outer;
  if constexpr (FILT) {
    // a column with ny^2 + kz^2 >= hi (or kz beyond the cube) is zero after the
    // filter for every nx; a tile of such columns only writes its zeros
    const bool colnz = cv && fz_ok && fny * fny + kz * kz < hi2;
    if (!__syncthreads_or(colnz)) {
      if (cv)
        for (int r = j0; r < p.out_rows; r += NT) nt_store(dst + (int64_t)r * p.out_row + ocol, V{(T)0, (T)0});
      return;
    }
  }
  V v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int pos = j0 + e * NT;
    v[e] = V{(T)0, (T)0};
    if ((N % NT == 0 || pos < N) && cv) {
      const int r = (pos + p.in_off) % N;
      if (r < p.in_rows) {
        if constexpr (FILT) {
          // the range test needs no memory, so the spectrum and weight loads
          // issue together (the filter is zero outside [lo2, hi2))
          const int nx = r - p.in_off;
          const int n2 = nx * nx + fny * fny + kz * kz;
          if (fz_ok && n2 >= lo2 && n2 < hi2) {
            const V x = src[(int64_t)r * p.in_row + icol];
            const T wgt = unit ? (T)1 : tab[n2];
            v[e] = V{x.x * wgt, x.y * wgt};
          }
        } else {
          v[e] = nt_load(src + (int64_t)r * p.in_row + icol);
        }
      }
    }
  }
  if constexpr (reg_out(N, NT)) {
    // both ends of the transform in registers; element pos of the output
    // goes to row (pos + out_off) mod N when that row is kept (the first
    // barrier inside covers the twiddle staging)
    fft_reg<V, N, SIGN, NT, 0, 0, true>(buf + c * PAD, tw, j0, v);
    if (cv) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int r = (j0 + e * NT + p.out_off) % N;
        if (r < p.out_rows) nt_store(dst + (int64_t)r * p.out_row + ocol, v[e]);
      }
    }
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int pos = j0 + e * NT;
      if (N % NT == 0 || pos < N) buf[c * PAD + pos] = v[e];
    }
    __syncthreads();
    fft_stages<V, N, SIGN, NT, 0, 1, 0, 0>(buf + c * PAD, tw, j0);
    if (cv) {
#pragma unroll 4
      for (int r = j0; r < p.out_rows; r += NT) {
        const int pos = (r - p.out_off + N) % N;
        nt_store(dst + (int64_t)r * p.out_row + ocol, buf[c * PAD + pos]);
      }
    }
  }
}

// ---------------------------------------------------------------- inv_z
// grid: blockIdx.x -> LZ_GROUPS consecutive groups of L lines, blockIdx.y -> field pair.
// A field is nlines lines of zs inputs (N * N for a whole cube, fewer for an
// x-slab of it) and nlines * N real outputs.
template <typename T, int N>
__global__ __launch_bounds__(256) void k_inv_z(const cplx_t<T>* __restrict__ in, T* __restrict__ out, int nfields,
                                               int64_t nlines, int cin, int zs, int64_t in_field,
                                               int64_t out_field, const cplx_t<T>* __restrict__ twg) {
  using V = cplx_t<T>;
  constexpr int NT = (N >= 8) ? N / 8 : 1;
  constexpr int L = 256 / NT;
  constexpr int PAD = N + 1;
  constexpr int SW = 1;  // bank swizzle of the line buffers
  __shared__ V buf[L * PAD];
  __shared__ V tw[N];
  for (int i = threadIdx.x; i < N; i += L * NT) tw[i] = twg[i];
  const int ll = threadIdx.x / NT, t = threadIdx.x % NT;
  const int f0 = 2 * blockIdx.y, f1 = f0 + 1;
  const bool has1 = f1 < nfields;
  V* b = buf + ll * PAD;
  __syncthreads();  // twiddles staged
  for (int rep = 0; rep < LZ_GROUPS; ++rep) {
    const int64_t line = ((int64_t)blockIdx.x * LZ_GROUPS + rep) * L + ll;
    const bool valid = line < nlines;
    const V* a = in + (int64_t)f0 * in_field + (valid ? line : 0) * zs;
    const V* bb = in + (int64_t)f1 * in_field + (valid ? line : 0) * zs;
    // two fields packed as A + iB, each completed from its half spectrum
    auto packed = [&](int pos) {
      V z = V{(T)0, (T)0};
      if (valid) {
        if (pos < cin) {
          const V A = a[pos];
          const V B = has1 ? bb[pos] : V{(T)0, (T)0};
          if (pos == 0 || 2 * pos == N) z = V{A.x, B.x};
          else z = V{A.x - B.y, A.y + B.x};
        } else if (pos > N - cin) {
          const int k = N - pos;
          const V A = a[k];
          const V B = has1 ? bb[k] : V{(T)0, (T)0};
          z = V{A.x + B.y, B.x - A.y};
        }
      }
      return z;
    };
    T* o0 = out + (int64_t)f0 * out_field + line * N;
    T* o1 = out + (int64_t)f1 * out_field + line * N;
    if constexpr (reg_out(N, NT)) {
      // both ends of the transform in registers: the line passes through LDS
      // only between passes
      V x[N / NT];
#pragma unroll
      for (int e = 0; e < N / NT; ++e) x[e] = packed(t + e * NT);
      fft_reg<V, N, +1, NT, SW, line_in_wave(N), true>(b, tw, t, x);
      if (valid) {
#pragma unroll
        for (int e = 0; e < N / NT; ++e) {
          __builtin_nontemporal_store(x[e].x, o0 + t + e * NT);
          if (has1) __builtin_nontemporal_store(x[e].y, o1 + t + e * NT);
        }
      }
    } else {
      for (int pos = t; pos < N; pos += NT) b[swz<SW>(pos)] = packed(pos);
      lds_sync<line_in_wave(N)>();
      fft_stages<V, N, +1, NT, 0, 1, SW, line_in_wave(N)>(b, tw, t);
      if (valid) {
        for (int pos = t; pos < N; pos += NT) {
          const V v = b[swz<SW>(pos)];
          __builtin_nontemporal_store(v.x, o0 + pos);
          if (has1) __builtin_nontemporal_store(v.y, o1 + pos);
        }
      }
    }
    lds_sync<line_in_wave(N)>();  // the next line reuses the buffer
  }
}

// ---------------------------------------------------------------- launchers

bool fft_size_supported(int n) {
  switch (n) {
    case 16: case 32: case 64: case 96: case 128: case 192: case 256: case 384: case 512: case 1024:
      return true;
    default:
      return false;
  }
}

#define BSP_FOR_SIZES(X) X(16) X(32) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(1024)

template <typename T>
static hipError_t fwd_z_impl(int n, const T* in, cplx_t<T>* out, const FwdZDesc& d, const cplx_t<T>* tw,
                             hipStream_t s) {
#define CASE(NN)                                                                        \
  case NN: {                                                                            \
    constexpr int NT = (NN >= 8) ? NN / 8 : 1;                                          \
    constexpr int L = 256 / NT;                                                         \
    dim3 grid((unsigned)(((int64_t)NN * NN + L * FZ_GROUPS - 1) / (L * FZ_GROUPS)), (unsigned)d.ngrid); \
    if (d.nlos == 1) hipLaunchKernelGGL((k_fwd_z<T, NN, 1>), grid, dim3(L * NT), 0, s, in, out, d, tw);   \
    else if (d.nlos == 6) hipLaunchKernelGGL((k_fwd_z<T, NN, 6>), grid, dim3(L * NT), 0, s, in, out, d, tw); \
    else if (d.nlos == 15) hipLaunchKernelGGL((k_fwd_z<T, NN, 15>), grid, dim3(L * NT), 0, s, in, out, d, tw); \
    else return hipErrorInvalidValue;                                                   \
    return hipGetLastError();                                                           \
  }
  switch (n) { BSP_FOR_SIZES(CASE) }
#undef CASE
  return hipErrorInvalidValue;
}

template <typename T, int N, int W>
static hipError_t c2c_launch(int sign, const cplx_t<T>* in, cplx_t<T>* out, const PassDesc& p,
                             const FilterDesc* f, const cplx_t<T>* tw, hipStream_t s) {
  const unsigned tiles = (unsigned)((p.ncols + W - 1) / W);
  unsigned gy = (unsigned)p.nouter, gz = 1;
  while (gy > 65535) {
    gz *= 2;
    gy = (unsigned)((p.nouter + gz - 1) / gz);
  }
  dim3 grid(tiles, gy, gz);
  FilterDesc fd{};
  if (f) fd = *f;
  // 512 threads per FP32 workgroup (32 per column): the 16-column tile's 70 KB
  // of LDS allows two workgroups per CU, so this doubles the waves a CU keeps
  // in flight (FP64 tiles of 8 columns keep 256)
  constexpr int BT = sizeof(T) == 4 ? 512 : 256;
  if (sign < 0) {
    if (f) hipLaunchKernelGGL((k_c2c<T, N, W, -1, true, BT>), grid, dim3(BT), 0, s, in, out, p, fd, tw);
    else hipLaunchKernelGGL((k_c2c<T, N, W, -1, false, BT>), grid, dim3(BT), 0, s, in, out, p, fd, tw);
  } else {
    if (f) hipLaunchKernelGGL((k_c2c<T, N, W, +1, true, BT>), grid, dim3(BT), 0, s, in, out, p, fd, tw);
    else hipLaunchKernelGGL((k_c2c<T, N, W, +1, false, BT>), grid, dim3(BT), 0, s, in, out, p, fd, tw);
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t inv_z_impl(int n, const cplx_t<T>* in, T* out, int nfields, int64_t nlines, int cin, int zs,
                             int64_t in_field, int64_t out_field, const cplx_t<T>* tw, hipStream_t s) {
  if (nlines < 1 || nlines > (int64_t)n * n || nfields < 1) return hipErrorInvalidValue;
#define CASE(NN)                                                                                  \
  case NN: {                                                                                      \
    constexpr int NT = (NN >= 8) ? NN / 8 : 1;                                                    \
    constexpr int L = 256 / NT;                                                                   \
    dim3 grid((unsigned)((nlines + L * LZ_GROUPS - 1) / (L * LZ_GROUPS)), (unsigned)((nfields + 1) / 2)); \
    hipLaunchKernelGGL((k_inv_z<T, NN>), grid, dim3(L * NT), 0, s, in, out, nfields, nlines, cin, zs, \
                       in_field, out_field, tw);                                                  \
    return hipGetLastError();                                                                     \
  }
  switch (n) { BSP_FOR_SIZES(CASE) }
#undef CASE
  return hipErrorInvalidValue;
}

hipError_t launch_fwd_z_f32(int n, const float* in, float2* out, const FwdZDesc& d, const float2* tw,
                            hipStream_t s) {
  return fwd_z_impl<float>(n, in, out, d, tw, s);
}
hipError_t launch_fwd_z_f64(int n, const double* in, double2* out, const FwdZDesc& d, const double2* tw,
                            hipStream_t s) {
  return fwd_z_impl<double>(n, in, out, d, tw, s);
}

hipError_t launch_c2c_f32(int n, int sign, const float2* in, float2* out, const PassDesc& p,
                          const FilterDesc* f, const float2* tw, hipStream_t s) {
  // lines of at most 128 points: 64-column tiles (512-byte row pieces, 8 threads
  // per column) when the launch still has at least 2048 of them, else 16
  const bool wide = n <= 128 && (p.tiles == 2 || (p.tiles == 0 && (int64_t)((p.ncols + 63) / 64) * p.nouter >= 2048));
#define CASE(NN)                                                                                  \
  case NN:                                                                                        \
    if constexpr (NN <= 128)                                                                      \
      if (wide) return c2c_launch<float, NN, 64>(sign, in, out, p, f, tw, s);                     \
    return c2c_launch<float, NN, 16>(sign, in, out, p, f, tw, s);
  switch (n) { BSP_FOR_SIZES(CASE) }
#undef CASE
  return hipErrorInvalidValue;
}
hipError_t launch_c2c_f64(int n, int sign, const double2* in, double2* out, const PassDesc& p,
                          const FilterDesc* f, const double2* tw, hipStream_t s) {
#define CASE(NN) \
  case NN: return c2c_launch<double, NN, 8>(sign, in, out, p, f, tw, s);
  switch (n) { BSP_FOR_SIZES(CASE) }
#undef CASE
  return hipErrorInvalidValue;
}

hipError_t launch_inv_z_f32(int n, const float2* in, float* out, int nfields, int64_t nlines, int cin, int zs,
                            int64_t in_field, int64_t out_field, const float2* tw, hipStream_t s) {
  return inv_z_impl<float>(n, in, out, nfields, nlines, cin, zs, in_field, out_field, tw, s);
}
hipError_t launch_inv_z_f64(int n, const double2* in, double* out, int nfields, int64_t nlines, int cin, int zs,
                            int64_t in_field, int64_t out_field, const double2* tw, hipStream_t s) {
  return inv_z_impl<double>(n, in, out, nfields, nlines, cin, zs, in_field, out_field, tw, s);
}

}  // namespace bsp
