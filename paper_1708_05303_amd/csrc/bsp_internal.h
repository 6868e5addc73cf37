// Internal declarations shared by the HIP translation units of libbsp.
// Not part of the public C ABI (see include/bsp.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <string>
#include <vector>

namespace bsp {

// ---------------------------------------------------------------- complex
template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename T> using cplx_t = typename cplx_of<T>::type;

template <typename V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ __forceinline__ V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }
template <typename V, typename T> __device__ __forceinline__ V cscale(V a, T s) { return V{a.x * s, a.y * s}; }

// ---------------------------------------------------------------- LOS harmonics
// Weights of the line-of-sight fields: the field F_m = FT[h_m(x_hat) delta]
// with h_0 = 1, then the five l = 2 and the nine l = 4 real solid harmonics of
// the unit vector x_hat, as polynomials in its components (|x_hat| = 1 used
// to write them with lower-degree terms):
//   l = 2: zx, zy, x^2 - y^2, 2xy, 3z^2 - 1
//   l = 4: 35z^4 - 30z^2 + 3, (7z^2 - 3)zx, (7z^2 - 3)zy, (7z^2 - 1)(x^2 - y^2),
//          (7z^2 - 1)2xy, z(x^3 - 3xy^2), z(3x^2y - y^3), x^4 - 6x^2y^2 + y^4,
//          4x^3y - 4xy^3.
// The addition theorem L_l(k_hat . x_hat) = sum_m a_m h_m(k_hat) h_m(x_hat)
// (a_m: los.hip) gives delta^(l)(k) = (2l+1) sum_m a_m h_m(k_hat) F_m(k).
// Each weight is a sum of at most four terms coef x^ex y^ey z^ez.
struct LosTerm { int8_t c, ex, ey, ez; };
constexpr int kLosFields = 15;
constexpr LosTerm kLosPoly[kLosFields][4] = {
    {{1, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{1, 1, 0, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{1, 0, 1, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{1, 2, 0, 0}, {-1, 0, 2, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{2, 1, 1, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{3, 0, 0, 2}, {-1, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{35, 0, 0, 4}, {-30, 0, 0, 2}, {3, 0, 0, 0}, {0, 0, 0, 0}},
    {{7, 1, 0, 3}, {-3, 1, 0, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{7, 0, 1, 3}, {-3, 0, 1, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{7, 2, 0, 2}, {-7, 0, 2, 2}, {-1, 2, 0, 0}, {1, 0, 2, 0}},
    {{14, 1, 1, 2}, {-2, 1, 1, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{1, 3, 0, 1}, {-3, 1, 2, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{3, 2, 1, 1}, {-1, 0, 3, 1}, {0, 0, 0, 0}, {0, 0, 0, 0}},
    {{1, 4, 0, 0}, {-6, 2, 2, 0}, {1, 0, 4, 0}, {0, 0, 0, 0}},
    {{4, 3, 1, 0}, {-4, 1, 3, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}}};

// Addition-theorem coefficients a_m of the harmonics (kLosPoly order): l = 2
// (fields 1..5) and l = 4 (fields 6..14), from
// 2 (l-m)!/(l+m)! times the squared prefactors of the associated Legendre
// functions written as these polynomials.
constexpr double kLosCoef[kLosFields] = {1.0,
                                         3.0, 3.0, 0.75, 0.75, 0.25,
                                         1.0 / 64, 5.0 / 8, 5.0 / 8, 5.0 / 16, 5.0 / 16, 35.0 / 8, 35.0 / 8,
                                         35.0 / 64, 35.0 / 64};
// Degree l of each harmonic.
constexpr int kLosDegree[kLosFields] = {0, 2, 2, 2, 2, 2, 4, 4, 4, 4, 4, 4, 4, 4, 4};

template <int E, typename T> __device__ __forceinline__ T los_pow(T x) {
  if constexpr (E == 0) return (T)1;
  else if constexpr (E == 1) return x;
  else if constexpr (E == 2) return x * x;
  else if constexpr (E == 3) return x * x * x;
  else return (x * x) * (x * x);
}

// h_F(x, y, z), the field index and its terms resolved at compile time.
template <int F, typename T> __device__ __forceinline__ T los_harmonic(T x, T y, T z) {
  T v = (T)0;
  constexpr LosTerm a = kLosPoly[F][0], b = kLosPoly[F][1], c = kLosPoly[F][2], d = kLosPoly[F][3];
  v += (T)a.c * los_pow<a.ex>(x) * los_pow<a.ey>(y) * los_pow<a.ez>(z);
  if constexpr (b.c != 0) v += (T)b.c * los_pow<b.ex>(x) * los_pow<b.ey>(y) * los_pow<b.ez>(z);
  if constexpr (c.c != 0) v += (T)c.c * los_pow<c.ex>(x) * los_pow<c.ey>(y) * los_pow<c.ez>(z);
  if constexpr (d.c != 0) v += (T)d.c * los_pow<d.ex>(x) * los_pow<d.ey>(y) * los_pow<d.ez>(z);
  return v;
}

// ---------------------------------------------------------------- launch params

// Strided column pass of a 3-D transform (see fft.hip).
struct PassDesc {
  int64_t in_outer, out_outer;   // element stride between outer batches
  int64_t in_row, out_row;       // element stride between consecutive rows of the FFT axis
  int32_t ncols;                 // inner columns per row
  int32_t ncz;                   // columns are runs of ncz: col = jj * ncz + kz
  int32_t in_j0, in_js, out_js;  // input inner offset (jj + in_j0) * in_js + kz, output jj * out_js + kz
  int32_t in_rows, in_off;       // input row r holds FFT index (r - in_off) mod N
  int32_t out_rows, out_off;     // output row r receives FFT index (r - out_off) mod N
  int32_t nouter;
  int32_t tiles;                 // FP32 lines of <= 128 points: 0 automatic, 1 16-column, 2 64-column tiles
};

// Shell / modal filter applied while loading the first inverse pass.
struct FilterDesc {
  const void* src;               // compact delta_l cube(s)
  int64_t src_ell_stride;        // elements between ell cubes
  const int32_t* field_ell;      // [nfields] ell slot of each field
  const void* tables;            // [rows][tablen] weights by |n|^2 (float for FP32 passes, double for FP64)
  const int32_t* field_table;    // [nfields] table row of each field
  const int32_t* row_range;      // [rows][3]: lo, hi, unit: the row is zero outside lo <= |n|^2 < hi,
                                 // and exactly 1 inside when unit
  int32_t tablen;                // n2max + 1
  int32_t c;                     // half width of the compact cube
  int32_t row0;                  // first source row (the batch reads rows row0 .. row0 + in_rows - 1)
  int32_t cz;                    // padded kz extent
  int32_t field0;                // first field of this launch
};

// Forward z pass with line-of-sight weighting.
struct FwdZDesc {
  int32_t ngrid, nlos;           // grids (1 or 2), LOS fields per grid (1, 6, 15)
  int32_t contrast;              // 1: input is a density, form rho / rho_bar - 1
  const double* wsum;            // sum of weights (device), used when contrast
  double shift[2];               // node offset of each grid (0, 1/2)
  double obs[3];                 // observer, grid units
  int32_t plane;                 // 1: plane parallel (no weights)
  int32_t cout, zs;              // kz kept, kz stride of the output
};

struct ReduceDesc {
  int32_t nfields;               // fields in the stack (<= 128)
  int64_t K;                     // points per field
  int64_t field_stride;          // elements between fields
  int32_t kchunk;                // points per workgroup chunk (multiple of 64)
  int32_t nchunks;
  int32_t ngroups;               // row-tile groups (grid.y)
  int32_t nct;                   // column tiles of 16 thirds (<= 8)
  int32_t maxr, maxcw;           // row tiles and column tiles per wave of the schedule
  const int32_t* wave_rows;      // [ngroups][waves][maxr] row tile ids, -1 none
  const int32_t* wave_cols;      // [ngroups][waves][maxcw] column tile ids, -1 none
  const int32_t* row_mask;       // [nrt] bit c set: column tile c needed
  const int32_t* tile_index;     // [nrt][8] compact tile id, -1 if not needed
  const int32_t* tile_rc;        // [ntiles][2] row tile, column tile
  int32_t ntiles;
  const int32_t* pair_a;         // [nrt*16] field of the first pair factor (-1 pad)
  const int32_t* pair_b;         // [nrt*16]
  const int32_t* third;          // [nct*16] (-1 pad)
  const float* scale;            // [nfields] power-of-two scales (FP16 path) or null
  // pair factors: split precisions keep full-precision LDS rows for these only
  int32_t npf;                   // fields that appear as a pair factor
  const int32_t* pf_row;         // [nfields] full-precision row of each field, -1 if none
  const int32_t* pair_ra;        // [nrt*16] row of pair_a (-1 pad)
  const int32_t* pair_rb;        // [nrt*16] row of pair_b (-1 pad)
  // row slots: slot_pair[s] is the pair (row of T) that slot s computes, -1 pad
  const int32_t* slot_pair;      // [nrt*16]
  // several field stacks reduced by one launch (the same schedule on each):
  // chunk c works on stack c / chunks_per_set, elements set_stride apart;
  // chunks_per_set = nchunks for one stack
  int32_t chunks_per_set;
  int64_t set_stride;
};

// ---------------------------------------------------------------- launchers
// FFT passes (fft.hip). Return hipError_t of the launch.
hipError_t launch_fwd_z_f32(int n, const float* in, float2* out, const FwdZDesc& d,
                            const float2* tw, hipStream_t s);
hipError_t launch_fwd_z_f64(int n, const double* in, double2* out, const FwdZDesc& d,
                            const double2* tw, hipStream_t s);
hipError_t launch_c2c_f32(int n, int sign, const float2* in, float2* out, const PassDesc& p,
                          const FilterDesc* f, const float2* tw, hipStream_t s);
hipError_t launch_c2c_f64(int n, int sign, const double2* in, double2* out, const PassDesc& p,
                          const FilterDesc* f, const double2* tw, hipStream_t s);
// Last inverse pass (half complex along z to real), nlines lines per field.
hipError_t launch_inv_z_f32(int n, const float2* in, float* out, int nfields, int64_t nlines, int cin, int zs,
                            int64_t in_field, int64_t out_field, const float2* tw, hipStream_t s);
hipError_t launch_inv_z_f64(int n, const double2* in, double* out, int nfields, int64_t nlines, int cin, int zs,
                            int64_t in_field, int64_t out_field, const double2* tw, hipStream_t s);
bool fft_size_supported(int n);

// Assignment (assign.hip). Node and weight sums are order independent (64-bit
// fixed point) whenever scratch is given: at least assign_fixed_bytes for the
// global-atomic kernel, assign_tiled_bytes for the tiled one. Without scratch
// launch_assign falls back to FP32 atomics. accumulate = 0 overwrites the
// grids, 1 adds to them; wsum is always added to.
size_t assign_fixed_bytes(int n, int interlace);
// Fills `words` 32-bit words with v by a kernel (capturable, unlike a memset node).
hipError_t launch_fill_u32(void* p, uint32_t v, int64_t words, hipStream_t s);
hipError_t launch_fill_noise(float* p, int64_t n, uint32_t seed, hipStream_t s);
// npd (optional): a device-side particle count the kernels read instead of np
// (then np only bounds the launch grids and the scratch), so that a captured
// graph can be replayed on catalogues of other sizes.
hipError_t launch_assign(const float* ux, const float* uy, const float* uz, const float* w,
                         int64_t np, int n, int window, int interlace, int accumulate, float* grids,
                         double* wsum, int32_t* err, void* scratch, size_t scratch_bytes, hipStream_t s,
                         const int64_t* npd = nullptr);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);
// Tiled assignment (no global atomics on the grids): bytes of scratch it needs
// for np particles on an N^3 grid, 0 when N does not tile; accumulate = 0
// overwrites the grids, 1 adds to them. Returns hipErrorInvalidValue when N
// does not tile or the scratch is too small (nothing is launched then).
size_t assign_tiled_bytes(int64_t np, int n);
bool assign_tiled_preferred(int n);
hipError_t launch_assign_tiled(const float* ux, const float* uy, const float* uz, const float* w, int64_t np, int n,
                               int window, int interlace, int accumulate, float* grids, double* wsum, int32_t* err,
                               void* scratch, size_t scratch_bytes, hipStream_t s, const int64_t* npd = nullptr);

// LOS combination and shell sums (los.hip).
struct LosDesc {
  int32_t n, c, cz, ngrid, nlos, lmax, plane, window, compensate;
  int32_t n2max;
};
hipError_t launch_los_combine(const float2* X, float2* delta_l, const LosDesc& d, hipStream_t s);
hipError_t launch_shell_power(const float2* delta0, int c, int cz, const int32_t* bin_of_n2,
                              int n2max, int nbins, double* psum, hipStream_t s);
// Shell cross sums out[l][b] = scale * sum_{n in b} Re[delta^(l)(n) conj X(n)] / N_b over
// the full lattice, X a compact spectrum of the delta^(l) layout (psum: device
// scratch of nl * nbins doubles).
hipError_t launch_shell_cross(const float2* delta_l, int64_t ell_stride, int nl, const float2* partner, int c, int cz,
                              const int32_t* bin_of_n2, int n2max, int nbins, const int64_t* nb_modes, double scale,
                              double* psum, double* out, hipStream_t s);
// x <- x^2 over n floats (n a multiple of 4, x 16-byte aligned).
hipError_t launch_square(float* x, int64_t n, hipStream_t s);

// Integrated bispectrum (ib.hip): sub-volume gather (contrast when wsum),
// per-sub-volume shell sums with the local line of sight (window -1: none,
// 0: NGP, 1: CIC), and the average iB[l][b] = (1/N_s) sum_i P[i][l][b] dbar[i].
hipError_t launch_gather_subvolumes(const float* grid, const double* wsum, int n, int s, float* out, hipStream_t st);
hipError_t launch_subvolume_shells(const float2* F, int m, int s, int plane, const double* obs, int window, int nl,
                                   const int32_t* bin_of_n2, int n2max, int nbins, double* psum, double* dbar,
                                   hipStream_t st);
// Local line of sight: the sub-volumes times the harmonic h_harm(x_hat), x_hat
// from the observer obs (grid units) to each node; the cross sums
// psum[i][ell_slot][b] += coef sum_{n in b} mult h_harm(n_hat) Re[Fm conj F0] / W^2.
hipError_t launch_gather_subvolumes_los(const float* grid, const double* wsum, int n, int s, int harm,
                                       const double* obs, float* out, hipStream_t st);
hipError_t launch_subvolume_cross(const float2* F0, const float2* Fm, int m, int s, int harm, int ell_slot,
                                  double coef, int window, int nl, const int32_t* bin_of_n2, int n2max, int nbins,
                                  double* psum, double* dbar, hipStream_t st);
hipError_t launch_subvolume_finalize(const double* psum, const double* dbar, int ns, int nl, int nbins,
                                     const int64_t* nb_modes, double scale, double* iB, double* P, hipStream_t st);

// Triple reduction (reduce.hip).
hipError_t launch_reduce(int prec, const float* fields, const ReduceDesc& d, float* partials,
                         hipStream_t s);
hipError_t launch_reduce_f64(const double* fields, const ReduceDesc& d, double* partials,
                             hipStream_t s);
// Adds the chunk partials in a fixed order (reproducible T); overwrites part
// of the partials. accumulate = 1 adds the sums to T instead of storing them
// (the x-slabs of one reduction, each combined in turn).
hipError_t launch_combine_partials(void* partials, int is_f64, const ReduceDesc& d,
                                   int npairs, int nthirds, double* T, double tscale,
                                   int accumulate, hipStream_t s);
int reduce_waves_per_group();
// Register-budget shapes (rows, columns per wave) the kernel is instantiated for.
struct ReduceShape { int maxr, maxcw; };
int reduce_shapes(int prec, ReduceShape* out, int max_out);

// FP64 finishing kernels (fp64.hip).
hipError_t launch_binned_finalize(const double* T, const int32_t* tri_tidx, int ntri, int nl,
                                  const int64_t* counts, const double* psum, const int64_t* nb_modes,
                                  int nbins, const int32_t* tri_bins, double norm_b, double pnorm,
                                  const double* nbar, double* B, double* B0sub, double* Pbar, hipStream_t s);
hipError_t launch_shot_noise(const double* Pl, int nbins, const int32_t* tri_bins, int ntri, int nl,
                             const double* ring, double nbar, double* SN, hipStream_t s);
// counts = rint(T * inv_k); residual bound 0.05 + rel |count| (latched as error bit 4)
hipError_t launch_counts_finalize(const double* T, const int32_t* tidx, int ntri, double inv_k, double rel,
                                  int64_t* counts, double* raw, int32_t* err, hipStream_t s);
hipError_t launch_modal_assemble(const double* T, const int32_t* combo, int nmodes, int nl,
                                 double scale, const double* sn, const double* nbar, double* bnum,
                                 hipStream_t s);
hipError_t launch_gram_assemble(const double* T, const int32_t* gidx, int nmodes, double scale,
                                double* gamma, hipStream_t s);
hipError_t launch_sn_assemble(const double* T, const int32_t* sidx, int nmodes, double scale,
                              double* sn, hipStream_t s);
hipError_t launch_cholesky(double* A, double* W, int n, double tol, int32_t* piv, int32_t* err,
                           hipStream_t s);
hipError_t launch_tri_inverse(const double* L, const int32_t* piv, int n, double* Linv, hipStream_t s);
hipError_t launch_modal_solve(const double* Linv, const int32_t* piv, int n, int nrhs, const double* b,
                              double* alpha, double* beta, hipStream_t s);
hipError_t launch_covariance(const double* x, int m, int d, double* cov, hipStream_t s);
hipError_t launch_scale_scalar(const double* x, double scale, double* y, hipStream_t s);

// Batch journal (journal.hip): checksummed per-mock records, resumable.
uint64_t fnv1a64(const void* data, size_t n, uint64_t h = 0xcbf29ce484222325ull);
int64_t journal_payload_doubles(int nl, int ntri, int d, int has_beta);

struct JournalRecord {
  uint64_t key, hash;
  int64_t np;
  int nl, ntri, d, has_beta;
  int64_t offset;
};

class Journal {
 public:
  ~Journal();
  // Opens the file (create: read-write, created if absent, exclusive lock;
  // else read-only, shared lock) and indexes its valid records; with create a
  // torn or corrupt tail is truncated away.
  bool open(const std::string& path, bool create, std::string& err);
  void close();
  const JournalRecord* find(uint64_t key, uint64_t hash) const;
  bool read(const JournalRecord& r, double* B, double* alpha, double* beta, std::string& err) const;
  bool append(uint64_t key, uint64_t hash, int64_t np, int nl, int ntri, int d, const double* B,
              const double* alpha, const double* beta, bool sync, std::string& err);
  int64_t records() const { return (int64_t)recs_.size(); }
  int64_t valid_bytes() const { return valid_bytes_; }
  int64_t file_bytes() const { return file_bytes_; }

 private:
  int fd_ = -1;
  std::string path_;
  std::vector<JournalRecord> recs_;
  int64_t valid_bytes_ = 0, file_bytes_ = 0;
};

}  // namespace bsp
