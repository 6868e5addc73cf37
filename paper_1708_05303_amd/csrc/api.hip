// Host runtime of libbsp: plans (geometry, constant tables, reduction
// schedules), workspace carving, and the orchestration of the kernels behind
// the C ABI declared in include/bsp.h.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/bsp.h"
#include "bsp_internal.h"

using namespace bsp;

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

thread_local std::string g_create_error;

struct ReducePlan {
  int npairs = 0, nthirds = 0, nrt = 0, nct = 0, ngroups = 0, ntiles = 0, maxr = 0, maxcw = 0, nfields = 0;
  int64_t needed = 0;  // needed (pair, third) entries
  std::vector<int32_t> pair_a, pair_b, third, row_mask, tile_index, tile_rc, wave_rows, wave_cols;
  int npf = 0;                               // fields that are pair factors
  std::vector<int32_t> pf_row, pair_ra, pair_rb;  // their rows; pairs by row
  // device copies (plan-owned or workspace)
  int32_t* d = nullptr;  // one block holding every array
  size_t words = 0;
  int32_t *d_pair_a = nullptr, *d_pair_b = nullptr, *d_third = nullptr, *d_row_mask = nullptr,
          *d_tile_index = nullptr, *d_tile_rc = nullptr, *d_wave_rows = nullptr, *d_wave_cols = nullptr;
  int32_t *d_pf_row = nullptr, *d_pair_ra = nullptr, *d_pair_rb = nullptr;
  std::vector<int32_t> slot_pair;            // pair of each row slot (-1 pad)
  int32_t* d_slot_pair = nullptr;
  std::vector<int32_t> packed;
  int64_t kchunk_force = 0;  // points per workgroup chunk chosen by the autotuner (0: the rule)
};

// Greedy placement of one kind of row tiles on nw waves: each row goes to the
// least loaded wave that can still hold it. wrows / cm: per wave.
bool place_rows(const ReducePlan& rp, const std::vector<int>& rows, int maxr, int maxcw, int nw,
                std::vector<int>& wrows, std::vector<int>& cm) {
  std::vector<int> load(nw, 0), cnt(nw, 0);
  wrows.assign((size_t)nw * maxr, -1);
  cm.assign(nw, 0);
  for (int r : rows) {
    const int m = rp.row_mask[r];
    int best = -1, best_grow = 0;
    for (int w = 0; w < nw; ++w) {
      if (cnt[w] >= maxr || __builtin_popcount(cm[w] | m) > maxcw) continue;
      const int grow = __builtin_popcount((cm[w] | m) & ~cm[w]);
      if (best < 0 || load[w] < load[best] || (load[w] == load[best] && grow < best_grow)) {
        best = w;
        best_grow = grow;
      }
    }
    if (best < 0) return false;
    wrows[(size_t)best * maxr + cnt[best]++] = r;
    load[best] += __builtin_popcount(m);
    cm[best] |= m;
  }
  return true;
}

// Row tiles go to (group, wave) slots, heaviest first, each wave holding at
// most maxr row tiles whose needed column tiles number at most maxcw.
bool schedule_rows(ReducePlan& rp, const std::vector<int>& active, int maxr, int maxcw, int waves,
                   std::vector<int>& wrows, std::vector<int>& wcols, int& ngroups) {
  for (int r : active)
    if (__builtin_popcount(rp.row_mask[r]) > maxcw) return false;
  for (ngroups = std::max(1, (int)((active.size() + (size_t)waves * maxr - 1) / ((size_t)waves * maxr)));
       ngroups <= (int)active.size(); ++ngroups) {
    const int nw = ngroups * waves;
    std::vector<int> cm;
    if (!place_rows(rp, active, maxr, maxcw, nw, wrows, cm)) continue;
    wcols.assign((size_t)nw * maxcw, -1);
    for (int w = 0; w < nw; ++w) {
      int k = 0;
      for (int c = 0; c < 8; ++c)
        if ((cm[w] >> c) & 1) wcols[(size_t)w * maxcw + k++] = c;
    }
    return true;
  }
  return false;
}

// Row tiles of 16 pair slots: the pairs that meet a needed third, in their
// given order (a pair that meets none gets no slot; its row of T stays as the
// caller set it).
void tile_rows(const std::vector<std::array<int, 2>>& pairs, const std::vector<int>& pmask,
               std::vector<int32_t>& slot_pair, std::vector<int32_t>& pa, std::vector<int32_t>& pb) {
  slot_pair.clear();
  pa.clear();
  pb.clear();
  for (int i = 0; i < (int)pairs.size(); ++i) {
    if (!pmask[i]) continue;
    slot_pair.push_back(i);
    pa.push_back(pairs[i][0]);
    pb.push_back(pairs[i][1]);
  }
  while (slot_pair.size() % 16) {
    slot_pair.push_back(-1);
    pa.push_back(-1);
    pb.push_back(-1);
  }
}

// Tiles of 16 pair slots x 16 thirds; a tile is needed when any entry is. The
// register shape is the one that needs the fewest groups (each group reads
// every field once).
bool build_reduce(ReducePlan& rp, const std::vector<std::array<int, 2>>& pairs, const std::vector<int>& thirds,
                  const std::vector<uint8_t>& need, int nfields, int prec, int force_shape = -1) {
  rp = ReducePlan{};
  rp.npairs = (int)pairs.size();
  rp.nthirds = (int)thirds.size();
  rp.nfields = nfields;
  rp.nct = (rp.nthirds + 15) / 16;
  if (rp.nct > 8 || rp.nct == 0 || rp.npairs == 0) return false;
  for (int i = 0; i < rp.npairs; ++i)
    for (int k = 0; k < 2; ++k)
      if (pairs[i][k] < 0 || pairs[i][k] >= nfields) return false;
  // column tiles each pair needs (0: the pair meets no needed third and gets no slot)
  std::vector<int> pmask(rp.npairs, 0);
  for (int p = 0; p < rp.npairs; ++p)
    for (int t = 0; t < rp.nthirds; ++t)
      if (need.empty() || need[(size_t)p * rp.nthirds + t]) pmask[p] |= 1 << (t / 16);
  tile_rows(pairs, pmask, rp.slot_pair, rp.pair_a, rp.pair_b);
  rp.nrt = (int)rp.slot_pair.size() / 16;
  if (rp.nrt == 0) return false;
  rp.third.assign(rp.nct * 16, -1);
  for (int i = 0; i < rp.nthirds; ++i) rp.third[i] = thirds[i];
  // rows of the pair factors, in order of first use
  rp.pf_row.assign(std::max(nfields, 1), -1);
  rp.pair_ra.assign(rp.nrt * 16, -1);
  rp.pair_rb.assign(rp.nrt * 16, -1);
  rp.npf = 0;
  for (int i = 0; i < rp.nrt * 16; ++i)
    for (int k = 0; k < 2; ++k) {
      const int f = k ? rp.pair_b[i] : rp.pair_a[i];
      if (f < 0) continue;
      if (rp.pf_row[f] < 0) rp.pf_row[f] = rp.npf++;
      (k ? rp.pair_rb : rp.pair_ra)[i] = rp.pf_row[f];
    }
  rp.row_mask.assign(rp.nrt, 0);
  rp.tile_index.assign(rp.nrt * 8, -1);
  for (int sl = 0; sl < rp.nrt * 16; ++sl) {
    const int p = rp.slot_pair[sl];
    if (p < 0) continue;
    for (int t = 0; t < rp.nthirds; ++t)
      if (need.empty() || need[(size_t)p * rp.nthirds + t]) {
        rp.row_mask[sl / 16] |= 1 << (t / 16);
        rp.needed++;
      }
  }
  std::vector<int> active;
  for (int r = 0; r < rp.nrt; ++r)
    if (rp.row_mask[r]) {
      for (int c = 0; c < rp.nct; ++c)
        if ((rp.row_mask[r] >> c) & 1) {
          rp.tile_index[r * 8 + c] = rp.ntiles++;
          rp.tile_rc.push_back(r);
          rp.tile_rc.push_back(c);
        }
      active.push_back(r);
    }
  std::stable_sort(active.begin(), active.end(), [&](int a, int b) {
    return __builtin_popcount(rp.row_mask[a]) > __builtin_popcount(rp.row_mask[b]);
  });
  const int waves = reduce_waves_per_group();
  ReduceShape shapes[8];
  int best_groups = 1 << 30;
  const int ns = reduce_shapes(prec, shapes, 8);
  for (int i = 0; i < ns; ++i) {
    if (force_shape >= 0 && i != force_shape) continue;
    std::vector<int> wr, wc;
    int ng = 0;
    if (!schedule_rows(rp, active, shapes[i].maxr, shapes[i].maxcw, waves, wr, wc, ng)) continue;
    if (ng < best_groups) {
      best_groups = ng;
      rp.maxr = shapes[i].maxr;
      rp.maxcw = shapes[i].maxcw;
      rp.wave_rows = wr;
      rp.wave_cols = wc;
      rp.ngroups = ng;
    }
  }
  if (best_groups == (1 << 30)) return false;
  // pack for one upload
  rp.packed.clear();
  auto put = [&](const std::vector<int32_t>& v) {
    rp.packed.insert(rp.packed.end(), v.begin(), v.end());
    while (rp.packed.size() % 64) rp.packed.push_back(0);
  };
  put(rp.pair_a);
  put(rp.pair_b);
  put(rp.third);
  put(rp.row_mask);
  put(rp.tile_index);
  put(rp.tile_rc.empty() ? std::vector<int32_t>{0} : rp.tile_rc);
  put(rp.wave_rows);
  put(rp.wave_cols);
  put(rp.pf_row);
  put(rp.pair_ra);
  put(rp.pair_rb);
  put(rp.slot_pair);
  rp.words = rp.packed.size();
  return true;
}

void bind_reduce(ReducePlan& rp, int32_t* dev) {
  rp.d = dev;
  size_t off = 0;
  auto take = [&](size_t n) {
    int32_t* p = dev + off;
    off += n;
    while (off % 64) ++off;
    return p;
  };
  rp.d_pair_a = take(rp.pair_a.size());
  rp.d_pair_b = take(rp.pair_b.size());
  rp.d_third = take(rp.third.size());
  rp.d_row_mask = take(rp.row_mask.size());
  rp.d_tile_index = take(rp.tile_index.size());
  rp.d_tile_rc = take(rp.tile_rc.empty() ? 1 : rp.tile_rc.size());
  rp.d_wave_rows = take(rp.wave_rows.size());
  rp.d_wave_cols = take(rp.wave_cols.size());
  rp.d_pf_row = take(rp.pf_row.size());
  rp.d_pair_ra = take(rp.pair_ra.size());
  rp.d_pair_rb = take(rp.pair_rb.size());
  rp.d_slot_pair = take(rp.slot_pair.size());
}

// Points per workgroup chunk: about 2048 chunks, at least 1024 points, at most
// 16384 (FP32), 8192 (bf16 / fp16 hi+lo) or 65536 (FP64). The register
// accumulators of the 16-bit MFMAs lose accuracy with the number of k-steps
// they sum (measured at 512^3: 65536-point chunks leave about 1e-4 of the
// summed-term scale, 8192-point chunks 3e-5), so their chunks are short and
// the FP64 combination takes over. Independent of the schedule so that
// partial storage only grows with the number of tiles.
// Kernel precision code of a public precision: the kernels number FP64 3 (the
// geometry precompute), so the bf16 hi-only error-study mode is 4 there.
int kprec(bsp_precision prec) { return prec == BSP_BF16X1 ? 4 : (int)prec; }

int64_t kchunk_for(int prec, int64_t K, int /*ngroups*/) {
  const int64_t cap = (prec == 0) ? 16384 : (prec == 3 ? 65536 : 8192);
  const int64_t target_blocks = 2048;
  int64_t kc = (K + target_blocks - 1) / target_blocks;
  kc = (kc + 63) / 64 * 64;
  kc = std::max<int64_t>(kc, 1024);
  kc = std::min<int64_t>(kc, cap);
  return kc;
}

// kc_min: a longer chunk (multiple of 64) when the partials must fit a given space.
ReduceDesc make_desc(const ReducePlan& rp, int64_t K, int64_t field_stride, int prec, const float* scale,
                     int64_t kc_min = 0) {
  ReduceDesc d{};
  d.nfields = rp.nfields;
  d.K = K;
  d.field_stride = field_stride;
  d.kchunk = (int32_t)std::max<int64_t>(rp.kchunk_force > 0 ? rp.kchunk_force : kchunk_for(prec, K, rp.ngroups), kc_min);
  d.nchunks = (int32_t)((K + d.kchunk - 1) / d.kchunk);
  d.chunks_per_set = d.nchunks;
  d.set_stride = 0;
  d.ngroups = rp.ngroups;
  d.nct = rp.nct;
  d.maxr = rp.maxr;
  d.maxcw = rp.maxcw;
  d.wave_rows = rp.d_wave_rows;
  d.wave_cols = rp.d_wave_cols;
  d.row_mask = rp.d_row_mask;
  d.tile_index = rp.d_tile_index;
  d.tile_rc = rp.d_tile_rc;
  d.ntiles = rp.ntiles;
  d.pair_a = rp.d_pair_a;
  d.pair_b = rp.d_pair_b;
  d.third = rp.d_third;
  d.scale = scale;
  d.npf = rp.npf;
  d.pf_row = rp.d_pf_row;
  d.pair_ra = rp.d_pair_ra;
  d.pair_rb = rp.d_pair_rb;
  d.slot_pair = rp.d_slot_pair;
  return d;
}

size_t partial_bytes(const ReducePlan& rp, int64_t K, int prec, size_t elem) {
  const int64_t kc = rp.kchunk_force > 0 ? rp.kchunk_force : kchunk_for(prec, K, rp.ngroups);
  const int64_t nch = (K + kc - 1) / kc;
  return (size_t)nch * rp.ntiles * 256 * elem;
}

}  // namespace

struct bsp_plan_s {
  bsp_geom g{};
  hipStream_t stream = nullptr;
  std::string err;
  int N = 0, Nr = 0, c = 0, cz = 0, nl = 1, nlos = 1, ngrid = 1, n2max = 0, plane = 1;
  int nbins = 0;
  int64_t spec = 0;  // compact cube elements
  int64_t kept = 0;  // stored modes with 0 < n2 <= n2max (kz >= 0)
  double V = 0, kf = 0, kmin = 0, kmax = 0;
  // modal basis
  bool modal = false;
  int P = 0, nmodes = 0, nU = 0;
  std::vector<int32_t> modes;
  std::vector<double> pfid;
  // geometry
  std::vector<std::array<int, 3>> cand;
  std::vector<int64_t> nb_modes;
  std::vector<int32_t> bin_of_n2;
  // plan-owned device memory
  std::vector<void*> allocs;
  float2* tw32_N = nullptr;
  float2* tw32_Nr = nullptr;
  double2* tw64_Nr = nullptr;
  int32_t* d_bin_of_n2 = nullptr;
  int64_t* d_nb_modes = nullptr;
  float* d_tab32 = nullptr;   // rows: nbins shells, P modal weights
  double* d_tab64 = nullptr;  // rows: nbins shells, nU U_ab, P G_p, P G^P_p
  int32_t* d_rng32 = nullptr;  // [rows][3] nonzero |n|^2 range and unit flag of each tab32 row
  int32_t* d_rng64 = nullptr;  // the same for tab64
  int32_t* d_err = nullptr;
  int32_t* d_ints = nullptr;  // field_ell / field_tab for the main and precompute passes
  int F = 0;                  // fields of the main pipeline
  int slab = 0;               // x planes of N' per slab of the field stacks (N': whole cubes)
  std::vector<int> row_c;     // largest |n_a| kept by each filter table row (tab64 row numbering)
  // per tab32 row: modes of the compact half cube the filter keeps, and the
  // (n_y, n_z) columns it leaves nonzero (algorithmic bytes of the inverse passes)
  std::vector<int64_t> row_support32, row_cols32;
  std::vector<int32_t> field_row32;  // tab32 row of each main pipeline field
  int32_t band_row32 = 0;            // tab32 row of the union of the shells
  std::map<int, float2*> tw32_other;  // FP32 twiddles of other transform sizes, made on first use
  int32_t* d_band_meta = nullptr;    // {0, band_row32, 0, band_row32 + 1}: l slot and table row of the
                                     // monopole on the union of the shells, then on the ball
  std::vector<int> field_c;   // per main-pipeline field
  int32_t *d_field_ell = nullptr, *d_field_tab = nullptr;
  int32_t *d_ones_ell = nullptr, *d_pre_tab = nullptr;  // precompute: all ell 0, table row = index
  // precompute results
  bool pre_done = false;
  std::vector<std::array<int, 3>> tri;
  std::vector<int64_t> counts;
  std::vector<double> gamma_h, chol_h;
  double count_residual = -1.0;
  int64_t* d_counts = nullptr;
  int32_t* d_tri_bins = nullptr;
  double* d_ring = nullptr;  // ring factors of the l > 0 shot noise [nl][ntri][2]
  int32_t* d_tri_tidx = nullptr;
  int32_t* d_combo = nullptr;
  double* d_L = nullptr;
  double* d_Linv = nullptr;          // inverse of the kept modes' Cholesky factor
  int32_t* d_piv = nullptr;          // kept modes in the order orthonormalised, then the rank
  double drop_tol = 0.0;             // relative residual below which a mode is dropped (0: keep all)
  std::vector<int32_t> piv_h;
  int modal_rank = 0;
  double* d_sn = nullptr;
  // autotuned choices (bsp_autotune): register shape of the main reduction
  // (index into its shape list, -1 the fewest workgroup groups), its chunk
  // length (0 the rule) and the column tiles of short transform lines (0 the rule)
  int tune_shape = -1;
  int64_t tune_kchunk = 0;
  int tune_tiles = 0;
  ReducePlan main_rp, cnt_rp, gram_rp, sn_rp;
  ReducePlan full_rp;                // B^(l1 l2 l3): every (l2, l3) pair of shell fields, made on first use
  bool full_built = false;
  int32_t* d_full_tidx = nullptr;    // [nl^3][ntri] index of each output in T
  std::vector<int32_t> cnt_tidx, gidx, sidx, tri_tidx, tri_bins, combo;
  std::vector<double> ring_h;
  int32_t *d_cnt_tidx = nullptr, *d_gidx = nullptr, *d_sidx = nullptr, *d_urow = nullptr, *d_grow = nullptr;
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  // stage timers: event pairs recorded around launches while enabled
  bool timing = false;
  std::vector<std::array<hipEvent_t, 2>> ev_pool;
  std::vector<int> ev_stage;
  size_t ev_used = 0;
  double stage_ms[16] = {0};
  int64_t stage_n[16] = {0};
  double stage_amount[16] = {0};
  // generic triple_reduce staging
  ReducePlan call_rp;
  double host_scalar = 0.0;
  // batch replay: the whole path captured once in a graph over fixed input
  // and output slots, on a stream of the library's own
  struct BatchSlot {
    hipStream_t stream = nullptr;
    hipGraphExec_t exec = nullptr;
    int prec = -1, has_w = 0;
    int64_t cap = 0;
    float* in = nullptr;     // [3 or 4][cap]: ux, uy, uz (, w)
    int64_t* npd = nullptr;  // particle count of the mock being replayed
    double* out = nullptr;   // B [nl][ntri], alpha [nl][nmodes], beta [nl][nmodes]
    void release() {
      if (exec) (void)hipGraphExecDestroy(exec);
      if (in) (void)hipFree(in);
      if (npd) (void)hipFree(npd);
      if (out) (void)hipFree(out);
      exec = nullptr;
      in = nullptr;
      npd = nullptr;
      out = nullptr;
      prec = -1;
      cap = 0;
    }
  } bslot;

  ~bsp_plan_s() {
    bslot.release();
    if (bslot.stream) (void)hipStreamDestroy(bslot.stream);
    for (auto& e : ev_pool) {
      (void)hipEventDestroy(e[0]);
      (void)hipEventDestroy(e[1]);
    }
    for (void* p : allocs) (void)hipFree(p);
  }
};

namespace {

bsp_status fail(bsp_plan p, bsp_status s, const std::string& msg) {
  if (p) p->err = msg;
  else g_create_error = msg;
  return s;
}

#define HIPCHK(expr)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) return fail(p, BSP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Records an event pair around the launches of one stage when timing is on.
struct StageTimer {
  bsp_plan p;
  int stage;
  size_t slot = (size_t)-1;
  // amount: algorithmic bytes (or flops for the reduction) of the timed launch
  StageTimer(bsp_plan pp, int st, double amount = 0.0) : p(pp), stage(st) {
    if (!p->timing) return;
    p->stage_amount[st] += amount;
    if (p->ev_used == p->ev_pool.size()) {
      std::array<hipEvent_t, 2> e{};
      if (hipEventCreate(&e[0]) != hipSuccess || hipEventCreate(&e[1]) != hipSuccess) return;
      p->ev_pool.push_back(e);
      p->ev_stage.push_back(st);
    }
    slot = p->ev_used++;
    p->ev_stage[slot] = st;
    (void)hipEventRecord(p->ev_pool[slot][0], p->stream);
  }
  // records the end event now (once) instead of at scope exit
  void stop() {
    if (slot != (size_t)-1) (void)hipEventRecord(p->ev_pool[slot][1], p->stream);
    slot = (size_t)-1;
  }
  ~StageTimer() { stop(); }
};

template <typename T>
T* dalloc(bsp_plan p, size_t n) {
  void* q = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(&q, n * sizeof(T)) != hipSuccess) return nullptr;
  p->allocs.push_back(q);
  return reinterpret_cast<T*>(q);
}

template <typename T>
T* upload(bsp_plan p, const std::vector<T>& v) {
  T* d = dalloc<T>(p, v.size());
  if (!d) return nullptr;
  if (!v.empty() && hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return nullptr;
  return d;
}

// Twiddles of the length-n LDS transforms in the order the butterfly passes
// read them: the pass with sub-length ns and radix r (radices 8, 4, 2, 3 taken
// greedily, as the kernels do) holds W_{ns r}^{q k} = exp(-2 pi i q k n / (ns r) / n)
// for q = 1 .. r-1, k < ns at entry (ns - 1) + (q - 1) ns + k; n - 1 entries in all.
int twiddle_exponent(int n, int i) {
  int ns = 1, m = n;
  while (m > 1) {
    const int r = (m % 8 == 0) ? 8 : (m % 4 == 0) ? 4 : (m % 2 == 0) ? 2 : 3;
    if (i < ns * r - 1) {
      const int j = i - (ns - 1);
      return (j / ns + 1) * (j % ns) * (n / (ns * r));
    }
    ns *= r;
    m /= r;
  }
  return 0;
}

// exp(-2 pi i e(j) / n) for the pass-ordered exponents e(j), double precision
std::vector<double> twiddles(int n) {
  std::vector<double> t(2 * (size_t)n);
  for (int jj = 0; jj < n; ++jj) {
    const int j = twiddle_exponent(n, jj);
    // the exponent is an exact integer; one rounding of the angle
    const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)j / (long double)n;
    t[2 * jj] = (double)cosl(a);
    t[2 * jj + 1] = (double)sinl(a);
  }
  return t;
}

double legendre(int p, double t) {
  double p0 = 1.0, p1 = t;
  if (p == 0) return p0;
  for (int k = 1; k < p; ++k) {
    const double p2 = ((2.0 * k + 1.0) * t * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// workspace layout -------------------------------------------------------------
struct Layout {
  size_t dl, fields, T, small, scratch, total;  // main pipeline
  size_t s_grid, s_Z, s_Y;                     // forward scratch pieces
  int fb;                                      // inverse batch
  size_t xres;                                 // resident x-pass output (slabs only; 0 otherwise)
  int fb_res;                                  // inverse batch with the resident x pass
  size_t pre_ones, pre_fields, pre_T, pre_scratch, pre_total;
  int fb64;
};

// x planes per slab of the field stacks: all of N' when the FP32 main stack
// and the FP64 precompute stack each stay within kSlabCap bytes, else the
// largest power-of-two fraction of N' for which both do.
constexpr size_t kSlabCap = 64ull << 30;
int default_slab(const bsp_plan p) {
  const size_t plane = (size_t)p->Nr * p->Nr;
  const size_t nfp = std::max({p->nbins, p->modal ? p->nU : 0, p->modal ? 2 * p->P : 0});
  int S = p->Nr;
  while (S % 2 == 0 && S > 8 && ((size_t)p->F * S * plane * 4 > kSlabCap || nfp * S * plane * 8 > kSlabCap)) S /= 2;
  return S;
}

// Relative part of the triangle counts' residual bound. The counts are
// sum_x I_b1 I_b2 I_b3 / N'^3 with FP64 shell fields whose values near x = 0 are
// the coherent sums N_b; the product there is of the order of the count times
// N'^3, so the rounding of the FP64 transforms (about eps log2(N'^3) relative
// each) leaves an error proportional to the count. Measured: 0.11 on 2.9e12 at
// 1024^3 and about 1e-3 on 3e10 at 512^3, 10-11 eps log2(N'^3) |count|; the
// bound takes 32.
double count_rel_tol(int64_t K) { return 32.0 * std::ldexp(1.0, -53) * std::log2((double)K); }

// Scratch of the inverse passes of fb fields over an x-slab of S planes: the
// x pass output [fb][S][2c+1][cz] and the y pass output [fb][S][N'][cz].
size_t inv_scratch(const bsp_plan p, int fb, int S, size_t celem) {
  const size_t w = 2 * (size_t)p->c + 1;
  return align_up((size_t)fb * S * w * p->cz * celem) + align_up((size_t)fb * S * p->Nr * p->cz * celem);
}

std::vector<std::array<int, 2>> inverse_batches(int nf, int fb, int Nr, const std::vector<int>& cf);

// The resident x-pass output of the main fields, batches of at most fb fields:
// batch b holds [nb][N'][2 c_b + 1][cz_b] complex64 on its own band c_b (its
// widest filter). Returns the bytes; offsets (optional) of each batch.
size_t xres_bytes(const bsp_plan p, int fb, std::vector<size_t>* offsets = nullptr) {
  size_t total = 0;
  for (const auto& bt : inverse_batches(p->F, fb, p->Nr, p->field_c)) {
    int cb = 0;
    for (int f = bt[0]; f < bt[1]; ++f) cb = std::max(cb, p->field_c[f]);
    const size_t czb = (size_t)(cb + 1 + 15) / 16 * 16, wb = 2 * (size_t)cb + 1;
    if (offsets) offsets->push_back(total);
    total += align_up((size_t)(bt[1] - bt[0]) * p->Nr * wb * czb * sizeof(float2));
  }
  return total;
}

Layout layout(const bsp_plan p) {
  Layout L{};
  const size_t w = 2 * (size_t)p->c + 1;
  const size_t N = p->N, Nr = p->Nr;
  L.dl = align_up((size_t)p->nl * p->spec * sizeof(float2));
  const size_t S = p->slab;
  L.fields = align_up((size_t)p->F * S * Nr * Nr * sizeof(float));
  L.T = align_up(std::max<size_t>((size_t)p->main_rp.npairs * p->main_rp.nthirds, 1) * sizeof(double));
  L.small = align_up(4096 * sizeof(double) + (size_t)(p->F + 64) * sizeof(float));
  L.s_grid = align_up((size_t)p->ngrid * N * N * N * sizeof(float));
  L.s_Z = align_up((size_t)p->ngrid * p->nlos * N * N * p->cz * sizeof(float2));
  L.s_Y = align_up((size_t)p->ngrid * p->nlos * N * w * p->cz * sizeof(float2));
  const size_t fwd = L.s_grid + L.s_Z + L.s_Y;
  int fb = 2;
  while (fb + 2 <= std::max(p->F, 2) && inv_scratch(p, fb + 2, p->slab, sizeof(float2)) <= std::max<size_t>(fwd, 1ull << 31))
    fb += 2;
  L.fb = fb;
  size_t part = 0;
  if (p->main_rp.ntiles)
    for (int prec = 0; prec < 3; ++prec)
      part = std::max(part, partial_bytes(p->main_rp, (int64_t)S * Nr * Nr, prec, sizeof(float)));
  const size_t fullc2r = align_up((size_t)N * N * (N / 2 + 1) * sizeof(float2));
  // the grids plus the int64 node sums of the fixed-point assignment
  const size_t fixed = L.s_grid + align_up(assign_fixed_bytes(p->N, p->ngrid - 1));
  // With x-slabs the main pipeline's x pass runs once per mock into a resident
  // buffer (the forward scratch is dead by then), followed by the y-pass output
  // of one batch (at most 8 GiB) or the reduction partials.
  L.xres = 0;
  L.fb_res = fb;
  size_t res_need = 0;
  if (p->slab < p->Nr) {
    int fr = fb;
    while (fr > 2 && (size_t)fr * S * Nr * p->cz * sizeof(float2) > (8ull << 30)) fr -= 2;
    L.fb_res = fr;
    L.xres = xres_bytes(p, fr);
    res_need = L.xres + std::max(align_up((size_t)fr * S * Nr * p->cz * sizeof(float2)),
                                 align_up(part) + align_up(1 << 20));
  }
  // (two whole-cube fields: the single-field inverse of the skew spectra)
  L.scratch = std::max({fwd, inv_scratch(p, fb, p->slab, sizeof(float2)), inv_scratch(p, 2, p->Nr, sizeof(float2)),
                        align_up(part) + align_up(1 << 20), fullc2r, fixed, res_need});
  L.total = L.dl + L.fields + L.T + L.small + L.scratch;
  // FP64 precompute
  const int nfp = std::max({p->nbins, p->modal ? p->nU : 0, p->modal ? 2 * p->P : 0});
  L.pre_ones = align_up((size_t)p->spec * sizeof(double2));
  L.pre_fields = align_up((size_t)nfp * S * Nr * Nr * sizeof(double));
  L.pre_T = align_up((size_t)4096 * 128 * sizeof(double));
  int fb64 = 2;
  while (fb64 + 2 <= std::max(nfp, 2) && inv_scratch(p, fb64 + 2, p->slab, sizeof(double2)) <= std::max<size_t>(fwd, 1ull << 31))
    fb64 += 2;
  L.fb64 = fb64;
  const int64_t K = (int64_t)S * Nr * Nr;
  size_t part64 = partial_bytes(p->cnt_rp, K, 3, sizeof(double));
  if (p->modal)
    part64 = std::max({part64, partial_bytes(p->gram_rp, K, 3, sizeof(double)),
                       partial_bytes(p->sn_rp, K, 3, sizeof(double))});
  part64 = align_up(std::max<size_t>(part64, p->cand.size() * 2 * sizeof(int64_t) + ALIGN));
  L.pre_scratch = std::max(inv_scratch(p, fb64, p->slab, sizeof(double2)), part64 + align_up(1 << 20));
  L.pre_total = L.pre_ones + L.pre_fields + L.pre_T + L.pre_scratch;
  return L;
}

// Inner columns are one contiguous run (no 2-D sub-block).
void set1d(PassDesc& d) {
  d.ncz = d.ncols;
  d.in_j0 = 0;
  d.in_js = 0;
  d.out_js = 0;
}

bsp_status need_ws(bsp_plan p, size_t bytes) {
  if (!p->ws) return fail(p, BSP_ERR_WORKSPACE, "no workspace set");
  if (p->ws_bytes < bytes) return fail(p, BSP_ERR_WORKSPACE, "workspace smaller than required");
  return BSP_OK;
}

// ---------------------------------------------------------------- passes

// delta_l (compact) from the forward transforms of the LOS-weighted grids.
bsp_status forward_moments(bsp_plan p, const float* grids, int ngrid, int contrast, const double* wsum,
                           int compensate, float2* delta_l, char* scratch) {
  const Layout L = layout(p);
  const int N = p->N, c = p->c, cz = p->cz, w = 2 * c + 1;
  float2* Z = reinterpret_cast<float2*>(scratch);
  float2* Y = reinterpret_cast<float2*>(scratch + L.s_Z);
  FwdZDesc fz{};
  fz.ngrid = ngrid;
  fz.nlos = p->nlos;
  fz.contrast = contrast;
  fz.wsum = wsum;
  fz.shift[0] = 0.0;
  fz.shift[1] = 0.5;
  for (int a = 0; a < 3; ++a) fz.obs[a] = p->g.observer[a];
  fz.plane = p->plane;
  fz.cout = c + 1;
  fz.zs = cz;
  const double C1 = c + 1.0, W1 = w;
  {
    // reads the grids, writes c+1 kz modes per line of every LOS field
    StageTimer t(p, 1, (double)ngrid * N * N * N * 4.0 + (double)ngrid * p->nlos * N * N * C1 * 8.0);
    HIPCHK(launch_fwd_z_f32(N, grids, Z, fz, p->tw32_N, p->stream));
  }
  const int nb = ngrid * p->nlos;
  PassDesc py{};
  py.tiles = p->tune_tiles;
  py.nouter = nb * N;
  py.in_outer = (int64_t)N * cz;
  py.out_outer = (int64_t)w * cz;
  py.in_row = cz;
  py.out_row = cz;
  py.ncols = cz;
  py.in_rows = N;
  py.in_off = 0;
  py.out_rows = w;
  py.out_off = c;
  set1d(py);
  {
    StageTimer t(p, 2, (double)nb * N * C1 * 8.0 * (N + W1));
    HIPCHK(launch_c2c_f32(N, -1, Z, Y, py, nullptr, p->tw32_N, p->stream));
  }
  PassDesc px{};
  px.tiles = p->tune_tiles;
  px.nouter = nb;
  px.in_outer = (int64_t)N * w * cz;
  px.out_outer = (int64_t)w * w * cz;
  px.in_row = (int64_t)w * cz;
  px.out_row = (int64_t)w * cz;
  px.ncols = w * cz;
  px.in_rows = N;
  px.in_off = 0;
  px.out_rows = w;
  px.out_off = c;
  set1d(px);
  float2* X = Z;  // Z is dead once Y exists
  {
    StageTimer t(p, 3, (double)nb * W1 * C1 * 8.0 * (N + W1));
    HIPCHK(launch_c2c_f32(N, -1, Y, X, px, nullptr, p->tw32_N, p->stream));
  }
  LosDesc ld{};
  ld.n = N;
  ld.c = c;
  ld.cz = cz;
  ld.ngrid = ngrid;
  ld.nlos = p->nlos;
  ld.lmax = p->g.lmax;
  ld.plane = p->plane;
  ld.window = p->g.window;
  ld.compensate = compensate;
  ld.n2max = p->n2max;
  {
    // the weighted spectra are read only inside the sphere n2 <= n2max; the
    // moments are written over the compact box (zeros outside the sphere)
    StageTimer t(p, 4, 8.0 * ((double)p->kept * nb + W1 * W1 * C1 * p->nl));
    HIPCHK(launch_los_combine(X, delta_l, ld, p->stream));
  }
  return BSP_OK;
}

// Batches of consecutive fields for the inverse transforms: at most fb fields
// (the scratch bound), even sizes except the last (the z pass packs pairs).
// A batch runs on the band of its widest filter; the split minimises launch
// overhead plus, per field, the bytes its x and y passes write and the z pass
// reads on that band (dynamic programming over the boundaries).
std::vector<std::array<int, 2>> inverse_batches(int nf, int fb, int Nr, const std::vector<int>& cf) {
  auto band_bytes = [&](int cb) {
    const double czb = (double)((cb + 1 + 15) / 16 * 16), wb = 2.0 * cb + 1.0;
    return 16.0 * czb * ((double)Nr * Nr + (double)Nr * wb);
  };
  const double launch = 1.35e8;  // about 30 us of a 4.5 TB/s pass
  std::vector<double> best(nf + 1, 1e300);
  std::vector<int> from(nf + 1, -1);
  best[0] = 0.0;
  for (int j = 1; j <= nf; ++j)
    for (int i = std::max(0, j - fb); i < j; ++i) {
      if ((j - i) % 2 && j != nf) continue;
      int cb = 0;
      for (int f = i; f < j; ++f) cb = std::max(cb, cf[f]);
      const double cost = best[i] + launch + (j - i) * band_bytes(cb);
      if (cost < best[j]) {
        best[j] = cost;
        from[j] = i;
      }
    }
  std::vector<std::array<int, 2>> out;
  for (int j = nf; j > 0; j = from[j]) out.push_back({from[j], j});
  std::reverse(out.begin(), out.end());
  return out;
}

// Range of |n|^2 outside which a filter table row is zero, and whether it is
// exactly 1 inside (shell indicators): [rows][3] = lo, hi, unit.
template <typename T>
std::vector<int32_t> row_ranges(const std::vector<T>& tab, int tl) {
  const size_t rows = tab.size() / tl;
  std::vector<int32_t> r(rows * 3, 0);
  for (size_t row = 0; row < rows; ++row) {
    const T* t = tab.data() + row * tl;
    int lo = tl, hi = 0;
    for (int n2 = 0; n2 < tl; ++n2)
      if (t[n2] != (T)0) {
        lo = std::min(lo, n2);
        hi = n2 + 1;
      }
    if (hi == 0) lo = 0;
    int unit = hi > lo ? 1 : 0;
    for (int n2 = lo; n2 < hi; ++n2)
      if (t[n2] != (T)1) unit = 0;
    r[row * 3] = lo;
    r[row * 3 + 1] = hi;
    r[row * 3 + 2] = unit;
  }
  return r;
}

// Inverse transforms of filtered compact spectra to real fields on N'.
// field_ell / field_tab index the filter of each output field; cf[f] is the
// largest |n_a| the filter of field f keeps. A batch of fields is transformed
// on the band |n_a| <= c_b of its widest filter, so narrow shells move little data.
// Only the x-slab x0 <= x < x0 + S of each field is made (S = N': the whole
// cube): the x pass keeps the S output rows of the slab, the y and z passes
// run on those rows alone, and out holds [nf][S][N'][N'].
template <typename T>
bsp_status inverse_fields(bsp_plan p, const cplx_t<T>* src, int64_t src_ell_stride, int nf,
                          const int32_t* d_field_ell, const int32_t* d_field_tab, const T* tables,
                          const int32_t* row_range, T* out, char* scratch, int fb, const std::vector<int>& cf,
                          const int32_t* frow32 = nullptr, int x0 = 0, int S = 0, cplx_t<T>* xres_out = nullptr,
                          const cplx_t<T>* xres_in = nullptr) {
  const int Nr = p->Nr, c = p->c, cz = p->cz, w = 2 * c + 1;
  if (S == 0) S = Nr;
  if (S < 1 || x0 < 0 || x0 + S > Nr) return fail(p, BSP_ERR_ARG, "x-slab outside the grid");
  // resident x pass (FP32 main fields, batches as xres_bytes lays them out):
  // xres_out: only the x pass, all N' rows of every batch into the buffer;
  // xres_in: no x pass, the y pass reads the slab's rows of the buffer
  if (sizeof(T) != 4 && (xres_out || xres_in)) return fail(p, BSP_ERR_ARG, "resident x pass is FP32 only");
  if (xres_out) {
    x0 = 0;
    S = Nr;
  }
  using V = cplx_t<T>;
  V* Xb = reinterpret_cast<V*>(scratch);
  V* Yb = reinterpret_cast<V*>(xres_in ? scratch : scratch + align_up((size_t)fb * S * w * cz * sizeof(V)));
  size_t xoff = 0;  // offset (bytes) of the batch in the resident buffer
  for (const auto& bt : inverse_batches(nf, fb, Nr, cf)) {
    const int f0 = bt[0], nb = bt[1] - bt[0];
    int cb = 0;
    for (int f = f0; f < f0 + nb; ++f) cb = std::max(cb, cf[f]);
    const int czb = (cb + 1 + 15) / 16 * 16, wb = 2 * cb + 1;
    FilterDesc fd{};
    fd.src = src;
    fd.src_ell_stride = src_ell_stride;
    fd.field_ell = d_field_ell;
    fd.tables = tables;
    fd.field_table = d_field_tab;
    fd.row_range = row_range;
    fd.tablen = p->n2max + 1;
    fd.c = c;
    fd.row0 = c - cb;
    fd.cz = cz;
    fd.field0 = f0;
    PassDesc px{};
    px.tiles = p->tune_tiles;
    px.nouter = nb;
    px.in_outer = 0;
    px.out_outer = (int64_t)S * wb * czb;
    px.in_row = (int64_t)w * cz;
    px.out_row = (int64_t)wb * czb;
    px.ncols = wb * czb;
    px.ncz = czb;
    px.in_j0 = c - cb;
    px.in_js = cz;
    px.out_js = czb;
    px.in_rows = wb;
    px.in_off = cb;
    px.out_rows = S;              // output row r holds x = x0 + r
    px.out_off = (Nr - x0) % Nr;
    PassDesc py{};
    py.tiles = p->tune_tiles;
    py.nouter = nb * S;
    py.in_outer = (int64_t)wb * czb;
    py.out_outer = (int64_t)Nr * czb;
    py.in_row = czb;
    py.out_row = czb;
    py.ncols = czb;
    py.in_rows = wb;
    py.in_off = cb;
    py.out_rows = Nr;
    py.out_off = 0;
    set1d(py);
    if constexpr (sizeof(T) == 4) {
      // algorithmic bytes: the modes each field's filter keeps read once, the
      // (n_y, n_z) columns it leaves nonzero written by the x pass and read by the
      // y pass (the kernels also move the zero columns of the band), the y pass
      // output on the field's own band |n_z| <= c_f written once and read by the
      // z pass, and the real field written once (batching on the widest band of
      // a batch is the kernels' overhead, not part of the minimum)
      double a5 = 0.0, a6 = 0.0, a7 = 0.0;
      // (per slab: the modes read once per slab, the rest in proportion to S)
      for (int f = f0; f < f0 + nb; ++f) {
        const double c1 = cf[f] + 1.0, w1 = 2.0 * cf[f] + 1.0;
        double sup = w1 * w1 * c1, cols = w1 * c1;
        if (frow32) {
          sup = (double)p->row_support32[frow32[f]];
          cols = (double)p->row_cols32[frow32[f]];
        }
        a5 += (sup + (double)S * cols) * 8.0;
        a6 += ((double)S * cols + (double)S * Nr * c1) * 8.0;
        a7 += (double)S * Nr * c1 * 8.0 + (double)S * Nr * Nr * 4.0;
      }
      const size_t bbytes = align_up((size_t)nb * Nr * wb * czb * sizeof(V));
      if (xres_out) {
        StageTimer t(p, 5, a5);
        HIPCHK(launch_c2c_f32(Nr, +1, nullptr, reinterpret_cast<V*>(reinterpret_cast<char*>(xres_out) + xoff), px, &fd,
                              p->tw32_Nr, p->stream));
        xoff += bbytes;
        continue;
      }
      if (xres_in) {
        // one launch per field: its S rows x0.. are contiguous in [N'][wb][czb]
        StageTimer t(p, 6, a6);
        const V* xb = reinterpret_cast<const V*>(reinterpret_cast<const char*>(xres_in) + xoff);
        PassDesc pf = py;
        pf.nouter = S;
        for (int f = 0; f < nb; ++f)
          HIPCHK(launch_c2c_f32(Nr, +1, xb + ((int64_t)f * Nr + x0) * wb * czb, Yb + (int64_t)f * S * Nr * czb, pf,
                                nullptr, p->tw32_Nr, p->stream));
        xoff += bbytes;
      } else {
        {
          StageTimer t(p, 5, a5);
          HIPCHK(launch_c2c_f32(Nr, +1, nullptr, Xb, px, &fd, p->tw32_Nr, p->stream));
        }
        StageTimer t(p, 6, a6);
        HIPCHK(launch_c2c_f32(Nr, +1, Xb, Yb, py, nullptr, p->tw32_Nr, p->stream));
      }
      StageTimer t(p, 7, a7);
      HIPCHK(launch_inv_z_f32(Nr, Yb, out + (int64_t)f0 * S * Nr * Nr, nb, (int64_t)S * Nr, cb + 1, czb,
                              (int64_t)S * Nr * czb, (int64_t)S * Nr * Nr, p->tw32_Nr, p->stream));
    } else {
      HIPCHK(launch_c2c_f64(Nr, +1, nullptr, Xb, px, &fd, p->tw64_Nr, p->stream));
      HIPCHK(launch_c2c_f64(Nr, +1, Xb, Yb, py, nullptr, p->tw64_Nr, p->stream));
      HIPCHK(launch_inv_z_f64(Nr, Yb, out + (int64_t)f0 * S * Nr * Nr, nb, (int64_t)S * Nr, cb + 1, czb,
                              (int64_t)S * Nr * czb, (int64_t)S * Nr * Nr, p->tw64_Nr, p->stream));
    }
  }
  return BSP_OK;
}

// accumulate: add this reduction's T to Tout (the next x-slab of a field
// stack) instead of overwriting it.
template <typename T>
bsp_status run_reduce(bsp_plan p, const ReducePlan& rp, const T* fields, int64_t K, int prec, const float* scale,
                      double* Tout, char* scratch, size_t scratch_bytes, double tscale, int64_t kc_min = 0,
                      bool accumulate = false) {
  const ReduceDesc d = make_desc(rp, K, K, prec, scale, kc_min);
  const size_t need = (size_t)d.nchunks * d.ntiles * 256 * sizeof(T);
  if (need > scratch_bytes) return fail(p, BSP_ERR_WORKSPACE, "workspace too small for reduction partials");
  if (!accumulate) HIPCHK(launch_fill_u32(Tout, 0u, 2 * (int64_t)rp.npairs * rp.nthirds, p->stream));
  if (d.ntiles == 0) return BSP_OK;
  if constexpr (sizeof(T) == 4) {
    {
      // algorithmic flops: one multiply-add per needed (pair, third) entry per point, one multiply per pair
      StageTimer t(p, 8, (2.0 * rp.needed + rp.npairs) * (double)K);
      HIPCHK(launch_reduce(prec, fields, d, reinterpret_cast<float*>(scratch), p->stream));
    }
    StageTimer t(p, 9);
    HIPCHK(launch_combine_partials(scratch, 0, d, rp.npairs, rp.nthirds, Tout, tscale, accumulate, p->stream));
  } else {
    HIPCHK(launch_reduce_f64(fields, d, reinterpret_cast<double*>(scratch), p->stream));
    HIPCHK(launch_combine_partials(scratch, 1, d, rp.npairs, rp.nthirds, Tout, tscale, accumulate, p->stream));
  }
  return BSP_OK;
}

// Power-of-two scales so max |field| lies in (64, 128]: pair products stay
// below fp16's range and the lo parts stay normal.
__global__ void k_absmax(const float* __restrict__ f, int64_t K, unsigned* __restrict__ out) {
  const int fi = blockIdx.y;
  float m = 0.f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(f[(int64_t)fi * K + i]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(out + fi, __float_as_uint(m));
}
__global__ void k_pow2_scale(const unsigned* __restrict__ mx, int n, float* __restrict__ scale) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float m = __uint_as_float(mx[i]);
  int e = 0;
  if (m > 0.f) {
    frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
  }
  scale[i] = ldexpf(1.0f, 7 - e);
}

bsp_status field_scales(bsp_plan p, const float* fields, int nf, int64_t K, float* scale, unsigned* tmp) {
  HIPCHK(launch_fill_u32(tmp, 0u, nf, p->stream));
  hipLaunchKernelGGL(k_absmax, dim3(256, nf), dim3(256), 0, p->stream, fields, K, tmp);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_pow2_scale, dim3((nf + 63) / 64), dim3(64), 0, p->stream, tmp, nf, scale);
  HIPCHK(hipGetLastError());
  return BSP_OK;
}

// The filtered inverse transforms of nf fields and their triple reduction into
// T, one x-slab of p->slab planes at a time. The sum over x is additive, so
// each slab is made in the field stack, reduced, and added to T in slab order
// (a fixed order: T does not depend on timing); the stack holds slab / N' of
// the whole fields. With FP16 splits (scale given) the power-of-two scales are
// taken per slab and undone per slab in the combine.
template <typename T>
bsp_status slab_reduce(bsp_plan p, const ReducePlan& rp, const cplx_t<T>* src, int64_t src_ell_stride, int nf,
                       const int32_t* d_field_ell, const int32_t* d_field_tab, const T* tables,
                       const int32_t* row_range, const std::vector<int>& cf, const int32_t* frow32, int fb,
                       T* fields, int prec, float* scale, unsigned* tmpu, double* Tout, char* inv_scr,
                       char* red_scr, size_t red_bytes, int64_t kc_min = 0, cplx_t<T>* xres = nullptr) {
  const int Nr = p->Nr, S = p->slab;
  const int64_t K = (int64_t)S * Nr * Nr;
  if (xres) {
    // the x pass once, all rows, into the resident buffer (not repeated per slab)
    bsp_status s = inverse_fields<T>(p, src, src_ell_stride, nf, d_field_ell, d_field_tab, tables, row_range, fields,
                                     inv_scr, fb, cf, frow32, 0, Nr, xres, nullptr);
    if (s != BSP_OK) return s;
  }
  for (int x0 = 0; x0 < Nr; x0 += S) {
    bsp_status s = inverse_fields<T>(p, src, src_ell_stride, nf, d_field_ell, d_field_tab, tables, row_range, fields,
                                     inv_scr, fb, cf, frow32, x0, S, nullptr, xres);
    if (s != BSP_OK) return s;
    if constexpr (sizeof(T) == 4) {
      if (scale) {
        s = field_scales(p, fields, nf, K, scale, tmpu);
        if (s != BSP_OK) return s;
      }
    }
    s = run_reduce<T>(p, rp, fields, K, prec, scale, Tout, red_scr, red_bytes, 1.0, kc_min, x0 > 0);
    if (s != BSP_OK) return s;
  }
  return BSP_OK;
}

__global__ void k_fill_ones(double2* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = double2{1.0, 0.0};
}


bool upload_rp(bsp_plan p, ReducePlan& rp) {
  int32_t* dm = dalloc<int32_t>(p, rp.words);
  if (!dm) return false;
  if (hipMemcpy(dm, rp.packed.data(), rp.words * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) return false;
  bind_reduce(rp, dm);
  return true;
}

// T[(I_b2 I_b3)][I_b1] for every candidate b1 >= b2 >= b3
bool build_counts(bsp_plan p) {
  std::vector<std::array<int, 2>> pr;
  for (int b2 = 0; b2 < p->nbins; ++b2)
    for (int b3 = 0; b3 <= b2; ++b3) pr.push_back({b2, b3});
  std::vector<int> th(p->nbins);
  for (int b = 0; b < p->nbins; ++b) th[b] = b;
  std::vector<uint8_t> need(pr.size() * th.size(), 0);
  for (size_t i = 0; i < pr.size(); ++i)
    for (int b1 = 0; b1 < p->nbins; ++b1) need[i * th.size() + b1] = b1 >= pr[i][0];
  if (!build_reduce(p->cnt_rp, pr, th, need, p->nbins, 3)) return false;
  p->cnt_tidx.resize(p->cand.size());
  for (size_t i = 0; i < p->cand.size(); ++i) {
    const int b1 = p->cand[i][0], b2 = p->cand[i][1], b3 = p->cand[i][2];
    p->cnt_tidx[i] = (b2 * (b2 + 1) / 2 + b3) * p->nbins + b1;
  }
  return true;
}

// G(A,B,C) = sum_x U_A U_B U_C for the sorted U-index triples gamma needs
bool build_gram(bsp_plan p) {
  const int P = p->P, nm = p->nmodes, nU = p->nU;
  auto uidx = [&](int a, int b) {
    if (a > b) std::swap(a, b);
    return a * P - a * (a - 1) / 2 + (b - a);
  };
  std::vector<std::array<int, 2>> pr;
  std::vector<int> pidx((size_t)nU * nU, -1);
  for (int A = 0; A < nU; ++A)
    for (int B = A; B < nU; ++B) {
      pidx[(size_t)A * nU + B] = (int)pr.size();
      pr.push_back({A, B});
    }
  std::vector<int> th(nU);
  for (int u = 0; u < nU; ++u) th[u] = u;
  std::vector<uint8_t> need(pr.size() * nU, 0);
  p->gidx.assign((size_t)nm * nm * 6, 0);
  const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int i = 0; i < nm; ++i)
    for (int j = 0; j < nm; ++j)
      for (int t = 0; t < 6; ++t) {
        int tr[3];
        for (int a = 0; a < 3; ++a) tr[a] = uidx(p->modes[3 * i + a], p->modes[3 * j + perms[t][a]]);
        std::sort(tr, tr + 3);
        const int pi = pidx[(size_t)tr[0] * nU + tr[1]];
        need[(size_t)pi * nU + tr[2]] = 1;
        p->gidx[((size_t)i * nm + j) * 6 + t] = pi * nU + tr[2];
      }
  return build_reduce(p->gram_rp, pr, th, need, nU, 3);
}

// <G^P_p G_r G_s> (three placements) and <G_p G_r G_s> for every mode
bool build_sn(bsp_plan p) {
  const int P = p->P, nm = p->nmodes;
  std::vector<std::array<int, 2>> pr;
  std::vector<int> gp((size_t)P * P, -1);
  for (int a = 0; a < P; ++a)
    for (int b = a; b < P; ++b) {
      gp[(size_t)a * P + b] = gp[(size_t)b * P + a] = (int)pr.size();
      pr.push_back({a, b});
    }
  std::vector<int> th(2 * P);
  for (int a = 0; a < 2 * P; ++a) th[a] = a;
  std::vector<uint8_t> need(pr.size() * th.size(), 0);
  p->sidx.assign((size_t)nm * 4, 0);
  for (int i = 0; i < nm; ++i) {
    const int a = p->modes[3 * i], b = p->modes[3 * i + 1], cc = p->modes[3 * i + 2];
    const int e[4][2] = {{gp[(size_t)b * P + cc], P + a}, {gp[(size_t)a * P + cc], P + b},
                         {gp[(size_t)a * P + b], P + cc}, {gp[(size_t)b * P + cc], a}};
    for (int k = 0; k < 4; ++k) {
      need[(size_t)e[k][0] * th.size() + e[k][1]] = 1;
      p->sidx[4 * i + k] = e[k][0] * (int)th.size() + e[k][1];
    }
  }
  return build_reduce(p->sn_rp, pr, th, need, 2 * P, 3);
}

// Gauss-Legendre rule of n points on [-1, 1]: Newton's iteration on the
// Legendre polynomial P_n (three-term recurrence) from the first guesses
// cos(pi (i + 3/4) / (n + 1/2)).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        const double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
      }
      dp = n * (z * p0 - p1) / (z * z - 1.0);
      const double dz = p0 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// int_0^mu L_l(t) dt, l = 0, 2, 4.
double legendre_antiderivative(int l, double mu) {
  if (l == 2) return 0.5 * (mu * mu * mu - mu);
  if (l == 4) return (7.0 * std::pow(mu, 5) - 10.0 * mu * mu * mu + 3.0 * mu) / 8.0;
  return mu;
}

// Ring factor W_l(b1, b2 | b3) of the l > 0 shot noise: the mean of
// L_l(k1_hat . k2_hat) over the closed triangles with sides in the shells
// [c_i - dk/2, c_i + dk/2) (units of k_f), continuum density k1 k2 k3 dk1 dk2
// dk3 with k1_hat . k2_hat = (k3^2 - k1^2 - k2^2) / (2 k1 k2); the k3 integral
// in closed form (k3 dk3 = k1 k2 dmu), k1 and k2 by the 32-point rule.
double ring_factor(int l, double c1, double c2, double c3, double dk, const std::vector<double>& gx,
                   const std::vector<double>& gw) {
  const double lo = c3 - 0.5 * dk, hi = c3 + 0.5 * dk;
  double num = 0.0, den = 0.0;
  for (size_t a = 0; a < gx.size(); ++a) {
    const double k1 = c1 + 0.5 * dk * gx[a];
    for (size_t b = 0; b < gx.size(); ++b) {
      const double k2 = c2 + 0.5 * dk * gx[b];
      const double s = 2.0 * k1 * k2, q = k1 * k1 + k2 * k2;
      const double r_lo = std::max(lo, std::fabs(k1 - k2)), r_hi = std::min(hi, k1 + k2);
      const double m_lo = std::clamp((r_lo * r_lo - q) / s, -1.0, 1.0);
      const double m_hi = std::clamp(std::max((r_hi * r_hi - q) / s, m_lo), -1.0, 1.0);
      const double wt = gw[a] * gw[b] * (k1 * k2) * (k1 * k2);
      den += wt * (m_hi - m_lo);
      num += wt * (legendre_antiderivative(l, m_hi) - legendre_antiderivative(l, m_lo));
    }
  }
  return den > 0.0 ? num / den : 0.0;
}

// Ring factors of every triangle of the plan: [nl][ntri][2] = W_l(b1,b2|b3),
// W_l(b1,b3|b2) (row l = 0 unused, 1).
void build_ring(bsp_plan p) {
  const int ntri = (int)p->tri.size(), nl = p->nl;
  std::vector<double> gx, gw;
  gauss_legendre(32, gx, gw);
  p->ring_h.assign((size_t)nl * ntri * 2, 1.0);
  for (int li = 1; li < nl; ++li)
    for (int i = 0; i < ntri; ++i) {
      const double c1 = p->g.k0 + p->tri[i][0] * p->g.dk, c2 = p->g.k0 + p->tri[i][1] * p->g.dk,
                   c3 = p->g.k0 + p->tri[i][2] * p->g.dk;
      double* w = &p->ring_h[((size_t)li * ntri + i) * 2];
      w[0] = ring_factor(2 * li, c1, c2, c3, p->g.dk, gx, gw);
      w[1] = ring_factor(2 * li, c1, c3, c2, p->g.dk, gx, gw);
    }
}


// Main schedule: pairs (D0_b2 D0_b3, b2 >= b3), (M0_a M0_b), (M2_a M2_b);
// thirds D^l_b1 interleaved (b1, l), then M^l_s interleaved (s, l).
// exact: only triangles with nonzero counts; else every candidate.
bool build_main(bsp_plan p, bool exact) {
  const int nb = p->nbins, nl = p->nl, P = p->P;
  // field numbering: D^(l)_b = b * nl + l, M^(l)_a = nl * nb + a * nl + l
  std::vector<std::array<int, 2>> pr;
  std::vector<int> pbin((size_t)nb * nb, -1);
  for (int b2 = 0; b2 < nb; ++b2)
    for (int b3 = 0; b3 <= b2; ++b3) {
      pbin[(size_t)b2 * nb + b3] = (int)pr.size();
      pr.push_back({b2 * nl, b3 * nl});
    }
  std::vector<int> pm0((size_t)P * P, -1), pm2((size_t)P * P, -1);
  const int m0 = nl * nb;
  if (p->modal) {
    for (int a = 0; a < P; ++a)
      for (int b = a; b < P; ++b) {
        pm0[(size_t)a * P + b] = pm0[(size_t)b * P + a] = (int)pr.size();
        pr.push_back({m0 + a * nl, m0 + b * nl});
      }
    if (nl >= 3)
      for (int a = 0; a < P; ++a)
        for (int b = a; b < P; ++b) {
          pm2[(size_t)a * P + b] = pm2[(size_t)b * P + a] = (int)pr.size();
          pr.push_back({m0 + a * nl + 1, m0 + b * nl + 1});
        }
  }
  std::vector<int> th;
  for (int b1 = 0; b1 < nb; ++b1)
    for (int li = 0; li < nl; ++li) th.push_back(b1 * nl + li);
  if (p->modal)
    for (int a = 0; a < P; ++a)
      for (int li = 0; li < nl; ++li) th.push_back(m0 + a * nl + li);
  const int nth = (int)th.size();
  auto tb = [&](int b1, int li) { return b1 * nl + li; };
  auto tm = [&](int a, int li) { return nb * nl + a * nl + li; };
  std::vector<uint8_t> need(pr.size() * nth, 0);
  const std::vector<std::array<int, 3>>& tris = exact ? p->tri : p->cand;
  const int ntri = (int)tris.size();
  p->tri_tidx.assign((size_t)nl * ntri, 0);
  p->tri_bins.assign(3 * (size_t)ntri, 0);
  for (int i = 0; i < ntri; ++i) {
    const int b1 = tris[i][0], b2 = tris[i][1], b3 = tris[i][2];
    const int pi = pbin[(size_t)b2 * nb + b3];
    for (int li = 0; li < nl; ++li) {
      need[(size_t)pi * nth + tb(b1, li)] = 1;
      p->tri_tidx[(size_t)li * ntri + i] = pi * nth + tb(b1, li);
    }
    p->tri_bins[3 * i] = b1;
    p->tri_bins[3 * i + 1] = b2;
    p->tri_bins[3 * i + 2] = b3;
  }
  p->combo.clear();
  if (p->modal) {
    const int nm = p->nmodes;
    p->combo.assign((size_t)nl * nm * 6, -1);
    for (int i = 0; i < nm; ++i) {
      const int a = p->modes[3 * i], b = p->modes[3 * i + 1], cc = p->modes[3 * i + 2];
      auto put = [&](int li, int slot, int pair, int third) {
        need[(size_t)pair * nth + third] = 1;
        p->combo[((size_t)li * nm + i) * 6 + slot] = pair * nth + third;
      };
      put(0, 0, pm0[(size_t)a * P + b], tm(cc, 0));
      if (nl >= 2) {
        put(1, 0, pm0[(size_t)b * P + cc], tm(a, 1));
        put(1, 1, pm0[(size_t)a * P + cc], tm(b, 1));
        put(1, 2, pm0[(size_t)a * P + b], tm(cc, 1));
      }
      if (nl >= 3) {
        put(2, 0, pm0[(size_t)b * P + cc], tm(a, 2));
        put(2, 1, pm0[(size_t)a * P + cc], tm(b, 2));
        put(2, 2, pm0[(size_t)a * P + b], tm(cc, 2));
        put(2, 3, pm2[(size_t)b * P + cc], tm(a, 0));
        put(2, 4, pm2[(size_t)a * P + cc], tm(b, 0));
        put(2, 5, pm2[(size_t)a * P + b], tm(cc, 0));
      }
    }
  }
  if (!build_reduce(p->main_rp, pr, th, need, p->F, 1, p->tune_shape)) return false;
  p->main_rp.kchunk_force = p->tune_kchunk;
  return true;
}

}  // namespace

// =========================================================================== API

extern "C" {

const char* bsp_last_error(bsp_plan p) { return p ? p->err.c_str() : g_create_error.c_str(); }

bsp_status bsp_plan_create(bsp_plan* out, const bsp_geom* g, const bsp_modal_basis* m, void* stream) {
  bsp_plan p = nullptr;
  if (!out || !g) return fail(p, BSP_ERR_ARG, "null argument");
  *out = nullptr;
  const int Nr = g->n_reduce ? g->n_reduce : g->n;
  if (!fft_size_supported(g->n) || !fft_size_supported(Nr))
    return fail(p, BSP_ERR_SIZE, "unsupported grid size");
  if (g->lmax != 0 && g->lmax != 2 && g->lmax != 4) return fail(p, BSP_ERR_ARG, "lmax must be 0, 2 or 4");
  if (g->nbins < 1 || g->nbins > 64) return fail(p, BSP_ERR_ARG, "nbins must be in [1, 64]");
  if (!(g->box > 0) || !(g->dk > 0)) return fail(p, BSP_ERR_ARG, "box and dk must be positive");
  if (g->window != 0 && g->window != 1) return fail(p, BSP_ERR_ARG, "window must be 0 or 1");
  if (g->los != 0 && g->los != 1) return fail(p, BSP_ERR_ARG, "los must be 0 or 1");
  if (g->los == 1) {
    // x_hat is undefined at the observer: it must not sit on a node of either grid
    // (node j of the grid built at shift s represents the point j - s)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(g->observer[a])) return fail(p, BSP_ERR_ARG, "observer must be finite");
    for (int gi = 0; gi <= (g->interlace ? 1 : 0); ++gi) {
      bool on_node = true;
      for (int a = 0; a < 3; ++a) {
        const double j = g->observer[a] + 0.5 * gi;
        on_node = on_node && std::fabs(j - std::rint(j)) < 1e-9 && std::rint(j) >= 0 && std::rint(j) < g->n;
      }
      if (on_node) return fail(p, BSP_ERR_ARG, "observer on a grid node (its line of sight is undefined)");
    }
  }
  const double e0 = 2.0 * g->k0 - g->dk;
  if (std::fabs(2.0 * g->k0 - std::rint(2.0 * g->k0)) > 1e-9 || std::fabs(g->dk - std::rint(g->dk)) > 1e-9 || e0 <= 0)
    return fail(p, BSP_ERR_ARG, "2 k0 and dk must be integers with k0 > dk/2");
  p = new bsp_plan_s();
  p->g = *g;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  p->N = g->n;
  p->Nr = Nr;
  p->nbins = g->nbins;
  p->nl = g->lmax / 2 + 1;
  p->plane = g->los == 0 ? 1 : 0;
  p->nlos = p->plane ? 1 : (g->lmax == 0 ? 1 : (g->lmax == 2 ? 6 : 15));
  p->ngrid = g->interlace ? 2 : 1;
  p->V = g->box * g->box * g->box;
  p->kf = 2.0 * M_PI / g->box;
  p->kmin = g->k0 - 0.5 * g->dk;
  p->kmax = g->k0 + (g->nbins - 1) * g->dk + 0.5 * g->dk;
  // shells: (2 c_b - dk)^2 <= 4 n^2 < (2 c_b + dk)^2
  std::vector<int64_t> lo(g->nbins), hi(g->nbins);
  for (int b = 0; b < g->nbins; ++b) {
    const int64_t a = (int64_t)std::llround(2.0 * (g->k0 + b * g->dk) - g->dk);
    const int64_t z = (int64_t)std::llround(2.0 * (g->k0 + b * g->dk) + g->dk);
    lo[b] = a * a;
    hi[b] = z * z;
  }
  p->n2max = (int)((hi[g->nbins - 1] - 1) / 4);
  p->c = (int)std::floor(std::sqrt((double)p->n2max));
  while ((int64_t)(p->c + 1) * (p->c + 1) <= p->n2max) ++p->c;
  while ((int64_t)p->c * p->c > p->n2max) --p->c;
  if (3 * p->c >= Nr || 3 * p->c >= p->N) {
    delete p;
    return fail(nullptr, BSP_ERR_ALIAS, "3 c_max >= N': closed triangles would wrap");
  }
  p->cz = (p->c + 1 + 15) / 16 * 16;
  const int w = 2 * p->c + 1;
  p->spec = (int64_t)w * w * p->cz;
  p->kept = -1;  // the origin
  for (int nx = -p->c; nx <= p->c; ++nx)
    for (int ny = -p->c; ny <= p->c; ++ny) {
      const int64_t r = (int64_t)p->n2max - nx * nx - ny * ny;
      if (r < 0) continue;
      int kz = (int)std::sqrt((double)r);
      while ((int64_t)(kz + 1) * (kz + 1) <= r) ++kz;
      while ((int64_t)kz * kz > r) --kz;
      p->kept += std::min(kz, p->c) + 1;
    }
  p->bin_of_n2.assign(p->n2max + 1, -1);
  for (int n2 = 0; n2 <= p->n2max; ++n2)
    for (int b = 0; b < g->nbins; ++b)
      if (4 * (int64_t)n2 >= lo[b] && 4 * (int64_t)n2 < hi[b]) p->bin_of_n2[n2] = b;
  // modes per shell over the full lattice, and candidate triangles
  p->nb_modes.assign(g->nbins, 0);
  for (int x = -p->c; x <= p->c; ++x)
    for (int y = -p->c; y <= p->c; ++y)
      for (int z = -p->c; z <= p->c; ++z) {
        const int n2 = x * x + y * y + z * z;
        if (n2 <= p->n2max && p->bin_of_n2[n2] >= 0) p->nb_modes[p->bin_of_n2[n2]]++;
      }
  for (int b1 = 0; b1 < g->nbins; ++b1)
    for (int b2 = 0; b2 <= b1; ++b2)
      for (int b3 = 0; b3 <= b2; ++b3) p->cand.push_back({b1, b2, b3});
  // modal basis
  if (m && m->nmodes > 0) {
    if (m->P < 1 || m->P > 16 || !m->modes || !m->pfid) {
      delete p;
      return fail(nullptr, BSP_ERR_ARG, "bad modal basis");
    }
    if (m->pfid_len <= p->n2max) {
      delete p;
      return fail(nullptr, BSP_ERR_ARG, "pfid table shorter than the modal range");
    }
    p->modal = true;
    p->P = m->P;
    p->nmodes = m->nmodes;
    p->nU = m->P * (m->P + 1) / 2;
    p->modes.assign(m->modes, m->modes + 3 * (size_t)m->nmodes);
    for (int i = 0; i < m->nmodes; ++i) {
      const int a = p->modes[3 * i], b = p->modes[3 * i + 1], cc = p->modes[3 * i + 2];
      if (!(0 <= a && a <= b && b <= cc && cc < m->P)) {
        delete p;
        return fail(nullptr, BSP_ERR_ARG, "modes must satisfy 0 <= p <= r <= s < P");
      }
    }
    p->pfid.assign(m->pfid, m->pfid + m->pfid_len);
    if (!(m->drop_tol >= 0.0 && m->drop_tol < 1.0)) {
      delete p;
      return fail(nullptr, BSP_ERR_ARG, "drop_tol must be in [0, 1)");
    }
    p->drop_tol = m->drop_tol;
    for (int n2 = 1; n2 <= p->n2max; ++n2)
      if (p->bin_of_n2[n2] >= 0 && !(p->pfid[n2] > 0)) {
        delete p;
        return fail(nullptr, BSP_ERR_ARG, "pfid must be positive on the modal range");
      }
  }
  p->F = p->nl * p->nbins + (p->modal ? p->nl * p->P : 0);
  if (p->F > 128) {
    delete p;
    return fail(nullptr, BSP_ERR_ARG, "more than 128 shell and modal fields");
  }
  p->slab = default_slab(p);
  // ---- device tables
  auto tw = [&](int n, bool dbl) -> void* {
    std::vector<double> t = twiddles(n);
    if (dbl) return upload(p, t);
    std::vector<float> f(t.begin(), t.end());
    return upload(p, f);
  };
  p->tw32_N = reinterpret_cast<float2*>(tw(p->N, false));
  p->tw32_Nr = reinterpret_cast<float2*>(tw(p->Nr, false));
  p->tw64_Nr = reinterpret_cast<double2*>(tw(p->Nr, true));
  p->d_bin_of_n2 = upload(p, p->bin_of_n2);
  p->d_nb_modes = upload(p, p->nb_modes);
  const int tl = p->n2max + 1;
  // tab32 rows: nbins shells, P modal weights, the union of the shells, then
  // the ball 0 < |n|^2 <= n2max
  std::vector<float> tab32((size_t)(p->nbins + p->P + 2) * tl, 0.f);
  for (int n2 = 1; n2 < tl; ++n2) tab32[(size_t)(p->nbins + p->P + 1) * tl + n2] = 1.f;
  const int nrow64 = p->nbins + (p->modal ? p->nU + 2 * p->P : 0);
  std::vector<double> tab64((size_t)nrow64 * tl, 0.0);
  for (int n2 = 0; n2 < tl; ++n2) {
    const int b = p->bin_of_n2[n2];
    if (b >= 0) {
      tab32[(size_t)b * tl + n2] = 1.f;
      tab32[(size_t)(p->nbins + p->P) * tl + n2] = 1.f;
      tab64[(size_t)b * tl + n2] = 1.0;
    }
  }
  if (p->modal) {
    for (int n2 = 1; n2 < tl; ++n2) {
      if (p->bin_of_n2[n2] < 0) continue;  // the modal range is the union of the shells
      const double kn = std::sqrt((double)n2);
      const double k = p->kf * kn;
      const double t = (2.0 * kn - p->kmin - p->kmax) / (p->kmax - p->kmin);
      const double pf = p->pfid[n2];
      std::vector<double> q(p->P);
      for (int a = 0; a < p->P; ++a) q[a] = legendre(a, t);
      for (int a = 0; a < p->P; ++a) tab32[(size_t)(p->nbins + a) * tl + n2] = (float)(q[a] / std::sqrt(k * pf));
      int u = 0;
      for (int a = 0; a < p->P; ++a)
        for (int b = a; b < p->P; ++b, ++u) tab64[(size_t)(p->nbins + u) * tl + n2] = q[a] * q[b] / k;
      for (int a = 0; a < p->P; ++a) {
        tab64[(size_t)(p->nbins + p->nU + a) * tl + n2] = q[a] / std::sqrt(k * pf);
        tab64[(size_t)(p->nbins + p->nU + p->P + a) * tl + n2] = q[a] * std::sqrt(pf / k);
      }
    }
  }
  p->d_tab32 = upload(p, tab32);
  p->d_tab64 = upload(p, tab64);
  p->d_rng32 = upload(p, row_ranges(tab32, tl));
  p->d_rng64 = upload(p, row_ranges(tab64, tl));
  {
    // lattice points of the compact half cube (n_z >= 0) and of the (n_y, n_z)
    // column plane by |n|^2, summed over each row's nonzero range
    std::vector<int64_t> h3(tl, 0), h2(tl, 0);
    const int c = p->c;
    for (int ny = -c; ny <= c; ++ny)
      for (int nz = 0; nz <= c; ++nz) {
        const int64_t m = (int64_t)ny * ny + (int64_t)nz * nz;
        if (m < tl) h2[m]++;
        for (int nx = -c; nx <= c; ++nx) {
          const int64_t n2 = m + (int64_t)nx * nx;
          if (n2 < tl) h3[n2]++;
        }
      }
    const std::vector<int32_t> r32 = row_ranges(tab32, tl);
    const size_t rows = r32.size() / 3;
    p->row_support32.assign(rows, 0);
    p->row_cols32.assign(rows, 0);
    for (size_t row = 0; row < rows; ++row) {
      for (int n2 = r32[3 * row]; n2 < r32[3 * row + 1]; ++n2) p->row_support32[row] += h3[n2];
      for (int m = 0; m < r32[3 * row + 1]; ++m) p->row_cols32[row] += h2[m];
    }
  }
  // field metadata: main pipeline fields, then the precompute identity map
  // main fields: shell fields D^(l)_b at b * nl + l (so consecutive fields
  // widen with b), then modal fields M^(l)_a at nl * nbins + a * nl + l
  p->row_c.assign(nrow64, p->c);
  for (int b = 0; b < p->nbins; ++b) {
    int cb = 0;
    while ((int64_t)(cb + 1) * (cb + 1) * 4 < hi[b]) ++cb;  // largest integer with 4 cb^2 < (2 c_b + dk)^2
    p->row_c[b] = cb;
  }
  std::vector<int32_t> fe(p->F), ft(p->F);
  p->field_c.assign(p->F, p->c);
  for (int b = 0; b < p->nbins; ++b)
    for (int li = 0; li < p->nl; ++li) {
      fe[b * p->nl + li] = li;
      ft[b * p->nl + li] = b;
      p->field_c[b * p->nl + li] = p->row_c[b];
    }
  if (p->modal)
    for (int a = 0; a < p->P; ++a)
      for (int li = 0; li < p->nl; ++li) {
        fe[p->nl * p->nbins + a * p->nl + li] = li;
        ft[p->nl * p->nbins + a * p->nl + li] = p->nbins + a;
      }
  p->d_field_ell = upload(p, fe);
  p->d_field_tab = upload(p, ft);
  p->field_row32 = ft;
  p->band_row32 = p->nbins + p->P;
  p->d_band_meta = upload(p, std::vector<int32_t>{0, p->band_row32, 0, p->band_row32 + 1});
  std::vector<int32_t> zeros(std::max(nrow64, 1), 0), iota(std::max(nrow64, 1));
  for (int i = 0; i < (int)iota.size(); ++i) iota[i] = i;
  p->d_ones_ell = upload(p, zeros);
  p->d_pre_tab = upload(p, iota);
  p->d_err = dalloc<int32_t>(p, 1);
  bool ok = build_counts(p) && upload_rp(p, p->cnt_rp) && (p->d_cnt_tidx = upload(p, p->cnt_tidx)) != nullptr;
  if (ok && p->modal) {
    std::vector<int32_t> urow(p->nU), grow(2 * p->P);
    for (int u = 0; u < p->nU; ++u) urow[u] = p->nbins + u;
    for (int a = 0; a < 2 * p->P; ++a) grow[a] = p->nbins + p->nU + a;
    ok = build_gram(p) && upload_rp(p, p->gram_rp) && build_sn(p) && upload_rp(p, p->sn_rp) &&
         (p->d_gidx = upload(p, p->gidx)) && (p->d_sidx = upload(p, p->sidx)) && (p->d_urow = upload(p, urow)) &&
         (p->d_grow = upload(p, grow)) && (p->d_L = dalloc<double>(p, (size_t)p->nmodes * p->nmodes)) &&
         (p->d_piv = dalloc<int32_t>(p, (size_t)p->nmodes + 1)) &&
         (p->d_Linv = dalloc<double>(p, (size_t)p->nmodes * p->nmodes)) &&
         (p->d_sn = dalloc<double>(p, 2 * (size_t)p->nmodes));
  }
  ok = ok && build_main(p, false);  // candidate schedule: bounds the workspace before the counts exist
  if (!ok) {
    delete p;
    return fail(nullptr, BSP_ERR_ARG, "reduction schedule could not be built (too many fields or modes)");
  }
  if (!p->tw32_N || !p->tw32_Nr || !p->tw64_Nr || !p->d_bin_of_n2 || !p->d_tab32 || !p->d_tab64 || !p->d_rng32 ||
      !p->d_rng64 || !p->d_band_meta || !p->d_err ||
      !p->d_field_ell || !p->d_field_tab || !p->d_ones_ell || !p->d_pre_tab || !p->d_nb_modes) {
    delete p;
    return fail(nullptr, BSP_ERR_HIP, "device allocation of plan tables failed");
  }
  if (hipMemset(p->d_err, 0, sizeof(int32_t)) != hipSuccess) {
    delete p;
    return fail(nullptr, BSP_ERR_HIP, "hipMemset failed");
  }
  *out = p;
  return BSP_OK;
}

bsp_status bsp_plan_destroy(bsp_plan p) {
  if (!p) return BSP_ERR_ARG;
  (void)hipStreamSynchronize(p->stream);
  delete p;
  return BSP_OK;
}

bsp_status bsp_plan_info(bsp_plan p, bsp_info* info) {
  if (!p || !info) return fail(p, BSP_ERR_ARG, "null argument");
  info->c = p->c;
  info->cz = p->cz;
  info->nl = p->nl;
  info->nlos = p->nlos;
  info->ngrid = p->ngrid;
  info->n2max = p->n2max;
  info->ncand = (int32_t)p->cand.size();
  info->ntri = (int32_t)p->tri.size();
  info->nfields_binned = p->nl * p->nbins;
  info->nfields_modal = p->modal ? p->nl * p->P : 0;
  info->spec_elems = p->spec;
  info->count_residual = p->count_residual;
  const ReducePlan& m = p->main_rp;
  info->reduce_pairs = m.npairs;
  info->reduce_thirds = m.nthirds;
  info->reduce_tiles = m.ntiles;
  info->reduce_groups = m.ngroups;
  info->reduce_maxr = m.maxr;
  info->reduce_maxcw = m.maxcw;
  info->reduce_needed = m.needed;
  info->modal_rank = p->modal_rank;
  info->tune_shape = p->tune_shape;
  info->tune_tiles = p->tune_tiles;
  info->tune_kchunk = p->tune_kchunk;
  info->reduce_row_tiles = m.nrt;
  info->slab_planes = p->slab;
  return BSP_OK;
}

bsp_status bsp_workspace_size(bsp_plan p, size_t* bytes) {
  if (!p || !bytes) return fail(p, BSP_ERR_ARG, "null argument");
  // before bsp_precompute the main schedule covers every candidate triangle,
  // a superset of the final one, so this bound stays valid afterwards
  const Layout L = layout(p);
  *bytes = std::max(L.total, L.pre_total);
  return BSP_OK;
}

bsp_status bsp_set_slab(bsp_plan p, int32_t planes) {
  if (!p) return BSP_ERR_ARG;
  if (planes == 0) planes = default_slab(p);
  if (planes < 1 || planes > p->Nr || p->Nr % planes != 0)
    return fail(p, BSP_ERR_ARG, "slab planes must divide N'");
  if (planes != p->slab) {
    HIPCHK(hipStreamSynchronize(p->stream));
    if (p->bslot.stream) HIPCHK(hipStreamSynchronize(p->bslot.stream));
    p->bslot.release();  // a captured batch graph holds the launches of the old slabs
    p->slab = planes;
  }
  return BSP_OK;
}

bsp_status bsp_set_workspace(bsp_plan p, void* dev, size_t bytes) {
  if (!p) return BSP_ERR_ARG;
  if (dev && (reinterpret_cast<uintptr_t>(dev) % ALIGN)) return fail(p, BSP_ERR_ARG, "workspace must be 256-byte aligned");
  p->ws = reinterpret_cast<char*>(dev);
  p->ws_bytes = dev ? bytes : 0;
  return BSP_OK;
}

bsp_status bsp_sync(bsp_plan p) {
  if (!p) return BSP_ERR_ARG;
  HIPCHK(hipStreamSynchronize(p->stream));
  int32_t e = 0;
  HIPCHK(hipMemcpy(&e, p->d_err, sizeof(e), hipMemcpyDeviceToHost));
  if (e) {
    HIPCHK(hipMemset(p->d_err, 0, sizeof(int32_t)));
    if (e & 1) return fail(p, BSP_ERR_DEVICE, "particle outside [0, N) or not finite");
    if (e & 4) return fail(p, BSP_ERR_NUMERIC, "triangle count residual above 0.05 + rel |count| (or that bound >= 0.5)");
    if (e & 8) return fail(p, BSP_ERR_NUMERIC, "Gram matrix not positive definite");
    return fail(p, BSP_ERR_DEVICE, "device error");
  }
  return BSP_OK;
}

bsp_status bsp_grid_assign(bsp_plan p, const float* ux, const float* uy, const float* uz, const float* w, int64_t np,
                           float* grids, double* wsum) {
  if (!p || (np > 0 && (!ux || !uy || !uz)) || !grids || !wsum || np < 0) return fail(p, BSP_ERR_ARG, "null argument");
  // sorted, tiled accumulation when the grid tiles and the workspace holds the
  // sorted catalogue; otherwise fixed-point global atomics on int64 grids in the
  // workspace, or, without one, FP32 global atomics
  const size_t tb = assign_tiled_bytes(np, p->N);
  if (tb && p->ws && tb <= p->ws_bytes)
    HIPCHK(launch_assign_tiled(ux, uy, uz, w, np, p->N, p->g.window, p->g.interlace, 1, grids, wsum, p->d_err, p->ws,
                               p->ws_bytes, p->stream));
  else
    HIPCHK(launch_assign(ux, uy, uz, w, np, p->N, p->g.window, p->g.interlace, 1, grids, wsum, p->d_err, p->ws,
                         p->ws ? p->ws_bytes : 0, p->stream));
  return BSP_OK;
}

// ---------------------------------------------------------------- no-allocation assignment

extern "C++" {  // helpers keep C++ (internal) linkage inside the C block
namespace {

// Static device scratch of bsp_grid_assign_noalloc: the int64 node sums of the
// fixed-point assignment (up to 2^22 nodes over all grids) after a 256-byte
// head. Every GPU the library runs on holds its own copy until the process
// ends; host code must use the address returned by hipGetSymbolAddress for
// the current device, never the array's name.
constexpr size_t kNoAllocNodes = size_t(1) << 22;
constexpr size_t kNoAllocBytes = 256 + kNoAllocNodes * sizeof(int64_t);
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of `scratch` on the current device, looked up once per device.
hipError_t static_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // extern "C++"

bsp_status bsp_grid_assign_noalloc(bsp_plan p, const float* ux, const float* uy, const float* uz, const float* w,
                                   int64_t np, float* grids, double* wsum) {
  if (!p || (np > 0 && (!ux || !uy || !uz)) || !grids || !wsum || np < 0) return fail(p, BSP_ERR_ARG, "null argument");
  const size_t need = assign_fixed_bytes(p->N, p->g.interlace);
  if (need > kNoAllocBytes)
    return fail(p, BSP_ERR_SIZE, "bsp_grid_assign_noalloc: (1 + interlace) N^3 = " +
                                     std::to_string((need - 256) / sizeof(int64_t)) + " nodes exceed the static scratch of " +
                                     std::to_string(kNoAllocNodes) + " nodes");
  void* ptr = nullptr;
  const hipError_t e = static_scratch(&ptr);
  if (e != hipSuccess) return fail(p, BSP_ERR_HIP, std::string("static scratch: ") + hipGetErrorString(e));
  HIPCHK(launch_assign(ux, uy, uz, w, np, p->N, p->g.window, p->g.interlace, 1, grids, wsum, p->d_err, ptr,
                       kNoAllocBytes, p->stream));
  return BSP_OK;
}

// FP32 twiddles of a supported transform size (the plan's N and N' are built
// with the plan, other sizes on first use and kept with it).
static const float2* tw32_for(bsp_plan p, int n) {
  if (n == p->N) return p->tw32_N;
  if (n == p->Nr) return p->tw32_Nr;
  auto it = p->tw32_other.find(n);
  if (it != p->tw32_other.end()) return it->second;
  const std::vector<double> t = twiddles(n);
  std::vector<float> f(t.begin(), t.end());
  float2* d = reinterpret_cast<float2*>(upload(p, f));
  if (d) p->tw32_other[n] = d;
  return d;
}

// Unnormalised r2c of `batch` contiguous n^3 grids into [batch][n][n][n/2+1].
static bsp_status r2c_batch(bsp_plan p, int n, int batch, const float* in, float2* out, const float2* tw) {
  const int h = n / 2 + 1;
  // the tuned tile choice belongs to the plan's own grid sizes; other lengths
  // (the integrated bispectrum's sub-volumes) take the rule
  const int tiles = (n == p->N || n == p->Nr) ? p->tune_tiles : 0;
  FwdZDesc fz{};
  fz.ngrid = batch;
  fz.nlos = 1;
  fz.contrast = 0;
  fz.plane = 1;
  fz.cout = h;
  fz.zs = h;
  HIPCHK(launch_fwd_z_f32(n, in, out, fz, tw, p->stream));
  PassDesc py{};
  py.tiles = tiles;
  py.nouter = batch * n;
  py.in_outer = py.out_outer = (int64_t)n * h;
  py.in_row = py.out_row = h;
  py.ncols = h;
  py.in_rows = py.out_rows = n;
  set1d(py);
  HIPCHK(launch_c2c_f32(n, -1, out, out, py, nullptr, tw, p->stream));
  PassDesc px{};
  px.tiles = tiles;
  px.nouter = batch;
  px.in_outer = px.out_outer = (int64_t)n * n * h;
  px.in_row = px.out_row = (int64_t)n * h;
  px.ncols = n * h;
  px.in_rows = px.out_rows = n;
  set1d(px);
  HIPCHK(launch_c2c_f32(n, -1, out, out, px, nullptr, tw, p->stream));
  return BSP_OK;
}

bsp_status bsp_fft_r2c(bsp_plan p, int32_t n, int32_t batch, const float* in, void* out_c64) {
  if (!p || !in || !out_c64 || batch < 1 || batch > 65535) return fail(p, BSP_ERR_ARG, "bad argument");
  if (!fft_size_supported(n)) return fail(p, BSP_ERR_SIZE, "unsupported size");
  const float2* tw = (n == p->N) ? p->tw32_N : (n == p->Nr ? p->tw32_Nr : nullptr);
  if (!tw) return fail(p, BSP_ERR_SIZE, "size must be the plan's N or N'");
  return r2c_batch(p, n, batch, in, reinterpret_cast<float2*>(out_c64), tw);
}

bsp_status bsp_fft_c2r(bsp_plan p, int32_t n, int32_t batch, const void* in_c64, float* out) {
  if (!p || !in_c64 || !out || batch < 1) return fail(p, BSP_ERR_ARG, "bad argument");
  if (!fft_size_supported(n)) return fail(p, BSP_ERR_SIZE, "unsupported size");
  const float2* tw = (n == p->N) ? p->tw32_N : (n == p->Nr ? p->tw32_Nr : nullptr);
  if (!tw) return fail(p, BSP_ERR_SIZE, "size must be the plan's N or N'");
  const int h = n / 2 + 1;
  const size_t one = (size_t)n * n * h * sizeof(float2);
  bsp_status s = need_ws(p, one);
  if (s != BSP_OK) return s;
  const float2* in = reinterpret_cast<const float2*>(in_c64);
  float2* tmp = reinterpret_cast<float2*>(p->ws);
  for (int b = 0; b < batch; ++b) {
    PassDesc px{};
    px.tiles = p->tune_tiles;
    px.nouter = 1;
    px.in_outer = px.out_outer = 0;
    px.in_row = px.out_row = (int64_t)n * h;
    px.ncols = n * h;
    px.in_rows = px.out_rows = n;
    set1d(px);
    HIPCHK(launch_c2c_f32(n, +1, in + (size_t)b * n * n * h, tmp, px, nullptr, tw, p->stream));
    PassDesc py{};
    py.tiles = p->tune_tiles;
    py.nouter = n;
    py.in_outer = py.out_outer = (int64_t)n * h;
    py.in_row = py.out_row = h;
    py.ncols = h;
    py.in_rows = py.out_rows = n;
    set1d(py);
    HIPCHK(launch_c2c_f32(n, +1, tmp, tmp, py, nullptr, tw, p->stream));
    HIPCHK(launch_inv_z_f32(n, tmp, out + (size_t)b * n * n * n, 1, (int64_t)n * n, h, h, 0, 0, tw, p->stream));
  }
  return BSP_OK;
}

bsp_status bsp_los_moments(bsp_plan p, const float* grids, const double* wsum, void* delta_l) {
  if (!p || !grids || !wsum || !delta_l) return fail(p, BSP_ERR_ARG, "null argument");
  const Layout L = layout(p);
  bsp_status s = need_ws(p, L.s_grid + L.s_Z + L.s_Y);
  if (s != BSP_OK) return s;
  return forward_moments(p, grids, p->ngrid, 1, wsum, p->g.compensate, reinterpret_cast<float2*>(delta_l), p->ws);
}

bsp_status bsp_grid_entry(bsp_plan p, const float* delta, void* delta_l) {
  if (!p || !delta || !delta_l) return fail(p, BSP_ERR_ARG, "null argument");
  const Layout L = layout(p);
  bsp_status s = need_ws(p, L.s_Z + L.s_Y);
  if (s != BSP_OK) return s;
  return forward_moments(p, delta, 1, 0, nullptr, 0, reinterpret_cast<float2*>(delta_l), p->ws);
}

bsp_status bsp_filter_fields(bsp_plan p, const void* delta_l, int32_t nfilt, const int32_t* filt, float* fields) {
  if (!p || !delta_l || !filt || !fields || nfilt < 1) return fail(p, BSP_ERR_ARG, "bad argument");
  std::vector<int32_t> fe(nfilt), ft(nfilt);
  for (int i = 0; i < nfilt; ++i) {
    const int li = filt[3 * i], kind = filt[3 * i + 1], idx = filt[3 * i + 2];
    if (li < 0 || li >= p->nl) return fail(p, BSP_ERR_ARG, "ell index out of range");
    if (kind == 0) {
      if (idx < 0 || idx >= p->nbins) return fail(p, BSP_ERR_ARG, "bin index out of range");
      ft[i] = idx;
    } else if (kind == 1) {
      if (!p->modal || idx < 0 || idx >= p->P) return fail(p, BSP_ERR_ARG, "modal index out of range");
      ft[i] = p->nbins + idx;
    } else {
      return fail(p, BSP_ERR_ARG, "filter kind must be 0 or 1");
    }
    fe[i] = li;
  }
  // whole cubes into the caller's array (batches made smaller than the main
  // pipeline's when its field stacks are x-slabs and the workspace is short)
  const Layout L = layout(p);
  const size_t meta = align_up(2 * (size_t)nfilt * sizeof(int32_t));
  int fb = std::min(L.fb, (nfilt + 1) / 2 * 2);
  while (fb > 2 && meta + inv_scratch(p, fb, p->Nr, sizeof(float2)) > p->ws_bytes) fb -= 2;
  bsp_status s = need_ws(p, meta + inv_scratch(p, fb, p->Nr, sizeof(float2)));
  if (s != BSP_OK) return s;
  int32_t* dmeta = reinterpret_cast<int32_t*>(p->ws);
  std::vector<int32_t> both(fe);
  both.insert(both.end(), ft.begin(), ft.end());
  HIPCHK(hipMemcpyAsync(dmeta, both.data(), both.size() * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  std::vector<int> cf(nfilt);
  for (int i = 0; i < nfilt; ++i) cf[i] = p->row_c[ft[i]];
  return inverse_fields<float>(p, reinterpret_cast<const float2*>(delta_l), p->spec, nfilt, dmeta, dmeta + nfilt,
                               p->d_tab32, p->d_rng32, fields, p->ws + meta, fb, cf, ft.data());
}

bsp_status bsp_triple_reduce(bsp_plan p, const float* fields, int32_t nfields, int64_t K, const int32_t* pairs,
                             int32_t npairs, const int32_t* thirds, int32_t nthirds, const uint8_t* need,
                             bsp_precision prec, double* T) {
  if (!p || !fields || !pairs || !thirds || !T || nfields < 1 || nfields > 128 || npairs < 1 || nthirds < 1 ||
      nthirds > 128 || K < 1)
    return fail(p, BSP_ERR_ARG, "bad argument");
  if (prec < BSP_FP32 || prec > BSP_BF16X1) return fail(p, BSP_ERR_ARG, "bad precision");
  std::vector<std::array<int, 2>> pr(npairs);
  for (int i = 0; i < npairs; ++i) {
    pr[i] = {pairs[2 * i], pairs[2 * i + 1]};
    if (pr[i][0] < 0 || pr[i][0] >= nfields || pr[i][1] < 0 || pr[i][1] >= nfields)
      return fail(p, BSP_ERR_ARG, "pair field out of range");
  }
  std::vector<int> th(thirds, thirds + nthirds);
  for (int t : th)
    if (t < 0 || t >= nfields) return fail(p, BSP_ERR_ARG, "third field out of range");
  std::vector<uint8_t> nd;
  if (need) nd.assign(need, need + (size_t)npairs * nthirds);
  if (!build_reduce(p->call_rp, pr, th, nd, nfields, kprec(prec)))
    return fail(p, BSP_ERR_ARG, "reduction shape not supported");
  const size_t meta = align_up(p->call_rp.words * sizeof(int32_t));
  const size_t sc = align_up((size_t)nfields * sizeof(float)) * 2;
  const size_t part = partial_bytes(p->call_rp, K, kprec(prec), sizeof(float));
  bsp_status s = need_ws(p, meta + sc + part);
  if (s != BSP_OK) return s;
  int32_t* dm = reinterpret_cast<int32_t*>(p->ws);
  HIPCHK(hipMemcpyAsync(dm, p->call_rp.packed.data(), p->call_rp.words * sizeof(int32_t), hipMemcpyHostToDevice,
                        p->stream));
  bind_reduce(p->call_rp, dm);
  float* scale = nullptr;
  if (prec == BSP_FP16X3) {
    scale = reinterpret_cast<float*>(p->ws + meta);
    s = field_scales(p, fields, nfields, K, scale, reinterpret_cast<unsigned*>(p->ws + meta + sc / 2));
    if (s != BSP_OK) return s;
  }
  s = run_reduce<float>(p, p->call_rp, fields, K, kprec(prec), scale, T, p->ws + meta + sc, p->ws_bytes - meta - sc, 1.0);
  if (s != BSP_OK) return s;
  HIPCHK(hipStreamSynchronize(p->stream));  // host staging of the schedule stays valid until here
  return BSP_OK;
}

// ---------------------------------------------------------------- precompute

bsp_status bsp_precompute(bsp_plan p) {
  if (!p) return BSP_ERR_ARG;
  const Layout L = layout(p);
  bsp_status s = need_ws(p, L.pre_total);
  if (s != BSP_OK) return s;
  const int Nr = p->Nr;
  const int64_t K = (int64_t)Nr * Nr * Nr;
  char* ws = p->ws;
  double2* ones = reinterpret_cast<double2*>(ws);
  double* f64 = reinterpret_cast<double*>(ws + L.pre_ones);
  double* T64 = reinterpret_cast<double*>(ws + L.pre_ones + L.pre_fields);
  char* scr = ws + L.pre_ones + L.pre_fields + L.pre_T;
  const size_t scr_bytes = p->ws_bytes - (L.pre_ones + L.pre_fields + L.pre_T);
  hipLaunchKernelGGL(k_fill_ones, dim3((unsigned)((p->spec + 255) / 256)), dim3(256), 0, p->stream, ones, p->spec);
  HIPCHK(hipGetLastError());
  // --- triangle counts: I_b for every shell, T[(b2,b3)][b1] over the candidates
  s = slab_reduce<double>(p, p->cnt_rp, ones, 0, p->nbins, p->d_ones_ell, p->d_pre_tab, p->d_tab64, p->d_rng64,
                          std::vector<int>(p->row_c.begin(), p->row_c.begin() + p->nbins), nullptr, L.fb64, f64, 3,
                          nullptr, nullptr, T64, scr, scr, scr_bytes);
  if (s != BSP_OK) return s;
  int64_t* dc = reinterpret_cast<int64_t*>(scr);
  double* draw = reinterpret_cast<double*>(scr + align_up(p->cand.size() * sizeof(int64_t)));
  HIPCHK(launch_counts_finalize(T64, p->d_cnt_tidx, (int)p->cand.size(), 1.0 / (double)K, count_rel_tol(K), dc, draw,
                                p->d_err, p->stream));
  s = bsp_sync(p);
  if (s != BSP_OK) {
    // report the worst residual and its triangle
    std::vector<double> raw(p->cand.size());
    if (hipMemcpy(raw.data(), draw, raw.size() * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess) {
      size_t worst = 0;
      double wr = -1.0;
      for (size_t i = 0; i < raw.size(); ++i) {
        const double r = std::fabs(raw[i] - std::rint(raw[i]));
        if (r > wr) {
          wr = r;
          worst = i;
        }
      }
      p->err += " (max residual " + std::to_string(wr) + " at (" + std::to_string(p->cand[worst][0]) + "," +
                std::to_string(p->cand[worst][1]) + "," + std::to_string(p->cand[worst][2]) + "), value " +
                std::to_string(raw[worst]) + ")";
    }
    return s;
  }
  std::vector<int64_t> cc(p->cand.size());
  HIPCHK(hipMemcpy(cc.data(), dc, cc.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
  {
    std::vector<double> raw(p->cand.size());
    HIPCHK(hipMemcpy(raw.data(), draw, raw.size() * sizeof(double), hipMemcpyDeviceToHost));
    p->count_residual = 0.0;
    for (double v : raw) p->count_residual = std::max(p->count_residual, std::fabs(v - std::rint(v)));
  }
  p->tri.clear();
  p->counts.clear();
  for (size_t i = 0; i < cc.size(); ++i)
    if (cc[i] > 0) {
      p->tri.push_back(p->cand[i]);
      p->counts.push_back(cc[i]);
    }
  // --- modal geometry: Gram matrix, Cholesky factor, shot-noise integrals
  if (p->modal) {
    const int nm = p->nmodes;
    s = slab_reduce<double>(p, p->gram_rp, ones, 0, p->nU, p->d_ones_ell, p->d_urow, p->d_tab64, p->d_rng64,
                            std::vector<int>(p->nU, p->c), nullptr, L.fb64, f64, 3, nullptr, nullptr, T64, scr, scr,
                            scr_bytes);
    if (s != BSP_OK) return s;
    HIPCHK(launch_gram_assemble(T64, p->d_gidx, nm, 1.0 / (6.0 * p->V * p->V * (double)K), p->d_L, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    p->gamma_h.resize((size_t)nm * nm);
    HIPCHK(hipMemcpy(p->gamma_h.data(), p->d_L, p->gamma_h.size() * sizeof(double), hipMemcpyDeviceToHost));
    if ((size_t)nm * nm * sizeof(double) > scr_bytes) return fail(p, BSP_ERR_WORKSPACE, "workspace too small");
    HIPCHK(launch_cholesky(p->d_L, reinterpret_cast<double*>(scr), nm, p->drop_tol, p->d_piv, p->d_err, p->stream));
    s = bsp_sync(p);
    if (s != BSP_OK) return s;
    p->chol_h.resize((size_t)nm * nm);
    HIPCHK(hipMemcpy(p->chol_h.data(), p->d_L, p->chol_h.size() * sizeof(double), hipMemcpyDeviceToHost));
    p->piv_h.resize((size_t)nm + 1);
    HIPCHK(hipMemcpy(p->piv_h.data(), p->d_piv, p->piv_h.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    p->modal_rank = p->piv_h[nm];
    HIPCHK(launch_tri_inverse(p->d_L, p->d_piv, nm, p->d_Linv, p->stream));
    s = slab_reduce<double>(p, p->sn_rp, ones, 0, 2 * p->P, p->d_ones_ell, p->d_grow, p->d_tab64, p->d_rng64,
                            std::vector<int>(2 * p->P, p->c), nullptr, L.fb64, f64, 3, nullptr, nullptr, T64, scr, scr,
                            scr_bytes);
    if (s != BSP_OK) return s;
    HIPCHK(launch_sn_assemble(T64, p->d_sidx, nm, 1.0 / (p->V * p->V * (double)K), p->d_sn, p->stream));
    s = bsp_sync(p);
    if (s != BSP_OK) return s;
  }
  // --- main reduction schedule restricted to triangles with nonzero counts
  if (!build_main(p, true)) return fail(p, BSP_ERR_ARG, "main reduction shape not supported");
  if (!upload_rp(p, p->main_rp)) return fail(p, BSP_ERR_HIP, "allocation failed");
  p->d_counts = upload(p, p->counts);
  p->d_tri_tidx = upload(p, p->tri_tidx);
  p->d_tri_bins = upload(p, p->tri_bins);
  if (p->modal) p->d_combo = upload(p, p->combo);
  build_ring(p);
  if (!p->ring_h.empty()) p->d_ring = upload(p, p->ring_h);
  if (!p->d_counts || !p->d_tri_tidx || !p->d_tri_bins || (p->modal && !p->d_combo) ||
      (!p->ring_h.empty() && !p->d_ring))
    return fail(p, BSP_ERR_HIP, "allocation failed");
  p->pre_done = true;
  return BSP_OK;
}

bsp_status bsp_geometry(bsp_plan p, int32_t* tri, int64_t* counts, double* gamma, double* chol, int32_t* kept) {
  if (!p) return BSP_ERR_ARG;
  if (!p->pre_done) return fail(p, BSP_ERR_STATE, "bsp_precompute has not run");
  for (size_t i = 0; i < p->tri.size(); ++i) {
    if (tri)
      for (int a = 0; a < 3; ++a) tri[3 * i + a] = p->tri[i][a];
    if (counts) counts[i] = p->counts[i];
  }
  if (gamma && p->modal) std::memcpy(gamma, p->gamma_h.data(), p->gamma_h.size() * sizeof(double));
  if (chol && p->modal) std::memcpy(chol, p->chol_h.data(), p->chol_h.size() * sizeof(double));
  if (kept && p->modal) std::memcpy(kept, p->piv_h.data(), (size_t)p->nmodes * sizeof(int32_t));
  return BSP_OK;
}

// ---------------------------------------------------------------- autotuning

extern "C++" {  // helpers keep C++ (internal) linkage inside the C block
namespace {

std::string tune_key(const bsp_plan p, bsp_precision prec) {
  char buf[256];
  std::snprintf(buf, sizeof buf, "N%d_Nr%d_nb%d_k0%g_dk%g_l%d_w%d_i%d_los%d_P%d_m%d_kept%d_prec%d", p->N, p->Nr,
                p->nbins, p->g.k0, p->g.dk, p->g.lmax, p->g.window, p->g.interlace, p->g.los, p->modal ? p->P : 0,
                p->modal ? p->nmodes : 0, p->modal_rank, (int)prec);
  return buf;
}

struct TuneEntry {
  int shape = -1, tiles = 0;
  long long kchunk = 0;
  double reduce_ms = 0.0, inverse_ms = 0.0;
};

// The database is a JSON object with one entry per line:
//   "<key>": {"shape": 3, "kchunk": 8192, "tiles": 0, "reduce_ms": 26.1, "inverse_ms": 29.5},
// closed by the sentinel line  "_": {}.
bool tune_lookup(const std::string& path, const std::string& key, TuneEntry& e) {
  std::FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  const std::string pre = "\"" + key + "\": {";
  while (std::fgets(line, sizeof line, f)) {
    const std::string l(line);
    const size_t at = l.find(pre);
    if (at == std::string::npos) continue;
    found = std::sscanf(l.c_str() + at + pre.size(),
                        "\"shape\": %d, \"kchunk\": %lld, \"tiles\": %d, \"reduce_ms\": %lf, \"inverse_ms\": %lf",
                        &e.shape, &e.kchunk, &e.tiles, &e.reduce_ms, &e.inverse_ms) == 5;
    break;
  }
  std::fclose(f);
  return found;
}

bool tune_store(const std::string& path, const std::string& key, const TuneEntry& e) {
  std::vector<std::string> keep;
  if (std::FILE* f = std::fopen(path.c_str(), "r")) {
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
      std::string l(line);
      while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
      if (l.size() > 1 && l[0] == '"' && l.compare(0, 4, "\"_\":") != 0 && l.find("\"" + key + "\":") != 0)
        keep.push_back(l);
    }
    std::fclose(f);
  }
  char buf[512];
  std::snprintf(buf, sizeof buf,
                "\"%s\": {\"shape\": %d, \"kchunk\": %lld, \"tiles\": %d, \"reduce_ms\": %.4f, \"inverse_ms\": %.4f},",
                key.c_str(), e.shape, e.kchunk, e.tiles, e.reduce_ms, e.inverse_ms);
  keep.push_back(buf);
  const std::string tmp = path + ".tmp";
  std::FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fputs("{\n", f);
  for (const auto& l : keep) {
    std::fputs(l.c_str(), f);
    std::fputs("\n", f);
  }
  std::fputs("\"_\": {}\n}\n", f);
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path.c_str()) == 0;
}

// Applies a shape / chunk choice to the main reduction schedule.
bool apply_reduce_choice(bsp_plan p, int shape, int64_t kchunk) {
  p->tune_shape = shape;
  p->tune_kchunk = kchunk;
  return build_main(p, true) && upload_rp(p, p->main_rp);
}

// Milliseconds of the fastest of `reps` timed runs of f on the plan's stream.
double time_min(bsp_plan p, int reps, const std::function<bsp_status()>& f, bsp_status& st) {
  hipEvent_t a, b;
  st = BSP_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    st = BSP_ERR_HIP;
    return 0.0;
  }
  double best = 1e300;
  for (int r = 0; r < reps && st == BSP_OK; ++r) {
    (void)hipEventRecord(a, p->stream);
    st = f();
    (void)hipEventRecord(b, p->stream);
    if (st == BSP_OK && hipEventSynchronize(b) == hipSuccess) {
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, a, b);
      best = std::min(best, (double)ms);
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

}  // namespace
}  // extern "C++"

bsp_status bsp_autotune(bsp_plan p, bsp_precision prec, const char* db_path, int32_t flags) {
  if (!p) return BSP_ERR_ARG;
  if (!p->pre_done) return fail(p, BSP_ERR_STATE, "bsp_precompute has not run");
  if (prec < BSP_FP32 || prec > BSP_BF16X1) return fail(p, BSP_ERR_ARG, "bad precision");
  const Layout L = layout(p);
  bsp_status s = need_ws(p, L.total);
  if (s != BSP_OK) return s;
  const std::string key = tune_key(p, prec);
  TuneEntry e;
  const std::string path = db_path ? db_path : "";
  if (!path.empty() && !(flags & BSP_TUNE_FORCE) && tune_lookup(path, key, e)) {
    p->tune_tiles = e.tiles;
    if (!apply_reduce_choice(p, e.shape, e.kchunk))
      return fail(p, BSP_ERR_ARG, "tuned reduction shape not supported");
    return BSP_OK;
  }
  s = bsp_sync(p);
  if (s != BSP_OK) return s;
  const bool timing = p->timing;
  p->timing = false;
  const int Nr = p->Nr;
  // one x-slab of the field stack (every slab costs the same)
  const int64_t K = (int64_t)p->slab * Nr * Nr;
  char* ws = p->ws;
  float2* dl = reinterpret_cast<float2*>(ws);
  float* fields = reinterpret_cast<float*>(ws + L.dl);
  double* T = reinterpret_cast<double*>(ws + L.dl + L.fields);
  char* scr = ws + L.dl + L.fields + L.T + L.small;
  const size_t scr_bytes = p->ws_bytes - (L.dl + L.fields + L.T + L.small);
  // defined inputs: a unit spectrum (the transforms' timing does not depend on
  // the values) and noise fields (the reduction's does, through the clocks)
  HIPCHK(launch_fill_u32(dl, 0x3f800000u, 2 * (int64_t)p->nl * p->spec, p->stream));
  // 1. transform tiles of short lines: the inverse passes of the main pipeline
  TuneEntry best;
  best.inverse_ms = 1e300;
  for (int tiles : {1, 2}) {
    if (tiles == 2 && Nr > 128) break;  // only lines of <= 128 points have 64-column tiles
    p->tune_tiles = tiles;
    bsp_status st;
    const double ms = time_min(p, 3, [&]() {
      return inverse_fields<float>(p, dl, p->spec, p->F, p->d_field_ell, p->d_field_tab, p->d_tab32, p->d_rng32,
                                   fields, scr, L.fb, p->field_c, p->field_row32.data(), 0, p->slab);
    }, st);
    if (st != BSP_OK) {
      p->timing = timing;
      return st;
    }
    if (ms < best.inverse_ms) {
      best.inverse_ms = ms;
      best.tiles = tiles;
    }
  }
  p->tune_tiles = best.tiles;
  HIPCHK(launch_fill_noise(fields, (int64_t)p->F * K, 12345u, p->stream));
  // 2. register shape and chunk length of the main reduction
  ReduceShape shapes[8];
  const int ns = reduce_shapes(1, shapes, 8);
  const int64_t cap = (prec == BSP_FP32) ? 16384 : 8192;
  best.reduce_ms = 1e300;
  for (int si = 0; si < ns; ++si) {
    for (int64_t kc : {cap / 4, cap / 2, cap}) {
      if (kc < 1024 || kc > K) continue;
      if (!apply_reduce_choice(p, si, kc)) continue;  // shape cannot hold the schedule
      if (partial_bytes(p->main_rp, K, kprec(prec), sizeof(float)) > scr_bytes) continue;
      bsp_status st;
      const double ms = time_min(p, 3, [&]() {
        return run_reduce<float>(p, p->main_rp, fields, K, kprec(prec), nullptr, T, scr, scr_bytes, 1.0);
      }, st);
      if (st != BSP_OK) continue;
      if (ms < best.reduce_ms) {
        best.reduce_ms = ms;
        best.shape = si;
        best.kchunk = kc;
      }
    }
  }
  p->timing = timing;
  if (best.reduce_ms == 1e300) return fail(p, BSP_ERR_ARG, "no reduction shape could be timed");
  if (!apply_reduce_choice(p, best.shape, best.kchunk)) return fail(p, BSP_ERR_HIP, "reduction schedule upload");
  if (!path.empty() && !tune_store(path, key, best))
    return fail(p, BSP_ERR_ARG, "cannot write the tuning database " + path);
  return bsp_sync(p);
}

// ---------------------------------------------------------------- estimators

extern "C++" {  // helpers keep C++ (internal) linkage inside the C block
namespace {

// fields -> T -> B, Pbar, modal numerators and coefficients (everything after delta_l)
bsp_status estimate_from_spectrum(bsp_plan p, const float2* dl, bsp_precision prec, const double* nbar_dev,
                                  double* B, double* B0sub, double* Pbar, double* bnum, double* alpha, double* beta,
                                  bool binned, bool modal_out) {
  const Layout L = layout(p);
  const int Nr = p->Nr;
  const int64_t K = (int64_t)Nr * Nr * Nr;
  char* ws = p->ws;
  float* fields = reinterpret_cast<float*>(ws + L.dl);
  double* T = reinterpret_cast<double*>(ws + L.dl + L.fields);
  double* small = reinterpret_cast<double*>(ws + L.dl + L.fields + L.T);
  double* psum = small;               // [64]
  double* bn_tmp = small + 64;        // [3 * 128]
  double* al_tmp = small + 64 + 384;  // [3 * 128]
  double* be_tmp = small + 64 + 768;  // [3 * 128]
  float* scale = reinterpret_cast<float*>(small + 2048);
  unsigned* tmpu = reinterpret_cast<unsigned*>(small + 3072);
  char* scr = ws + L.dl + L.fields + L.T + L.small;
  const size_t scr_bytes = p->ws_bytes - (L.dl + L.fields + L.T + L.small);
  // with x-slabs the x pass is resident at the start of the scratch (the
  // forward scratch is dead here), the y-pass batches and the partials after it
  float2* xres = L.xres ? reinterpret_cast<float2*>(scr) : nullptr;
  char* after = scr + L.xres;
  bsp_status s = slab_reduce<float>(p, p->main_rp, dl, p->spec, p->F, p->d_field_ell, p->d_field_tab, p->d_tab32,
                                    p->d_rng32, p->field_c, p->field_row32.data(), L.xres ? L.fb_res : L.fb, fields,
                                    kprec(prec), prec == BSP_FP16X3 ? scale : nullptr, tmpu, T, after, after,
                                    scr_bytes - L.xres, 0, xres);
  if (s != BSP_OK) return s;
  HIPCHK(launch_fill_u32(psum, 0u, 2 * 64, p->stream));
  HIPCHK(launch_shell_power(dl, p->c, p->cz, p->d_bin_of_n2, p->n2max, p->nbins, psum, p->stream));
  const double N = p->N;
  if (binned && B) {
    const double norm_b = p->V * p->V / (std::pow(N, 9) * (double)K);
    const double pnorm = p->V / std::pow(N, 6);
    HIPCHK(launch_binned_finalize(T, p->d_tri_tidx, (int)p->tri.size(), p->nl, p->d_counts, psum, p->d_nb_modes,
                                  p->nbins, p->d_tri_bins, norm_b, pnorm, nbar_dev, B, B0sub, Pbar, p->stream));
  } else if (Pbar) {
    const double pnorm = p->V / std::pow(N, 6);
    HIPCHK(launch_binned_finalize(T, p->d_tri_tidx, 0, p->nl, p->d_counts, psum, p->d_nb_modes, p->nbins,
                                  p->d_tri_bins, 0.0, pnorm, nullptr, B, nullptr, Pbar, p->stream));
  }
  if (modal_out && p->modal) {
    const int nm = p->nmodes;
    double* bo = bnum ? bnum : bn_tmp;
    double* ao = alpha ? alpha : al_tmp;
    double* beo = beta ? beta : be_tmp;
    if (nm > 128) return fail(p, BSP_ERR_ARG, "more than 128 modes");
    const double scale_b = 1.0 / ((double)K * std::pow(N, 9));
    HIPCHK(launch_modal_assemble(T, p->d_combo, nm, p->nl, scale_b, p->d_sn, nbar_dev, bo, p->stream));
    HIPCHK(launch_modal_solve(p->d_Linv, p->d_piv, nm, p->nl, bo, ao, beo, p->stream));
  }
  return BSP_OK;
}

}  // namespace
}  // extern "C++"

bsp_status bsp_modal_coeffs(bsp_plan p, const void* delta_l, bsp_precision prec, double nbar, double* bnum,
                            double* alpha, double* beta) {
  if (!p || !delta_l) return fail(p, BSP_ERR_ARG, "null argument");
  if (!p->modal) return fail(p, BSP_ERR_STATE, "plan has no modal basis");
  if (!p->pre_done) return fail(p, BSP_ERR_STATE, "bsp_precompute has not run");
  if (prec < BSP_FP32 || prec > BSP_BF16X1) return fail(p, BSP_ERR_ARG, "bad precision");
  const Layout L = layout(p);
  bsp_status s = need_ws(p, L.total);
  if (s != BSP_OK) return s;
  double* nb = reinterpret_cast<double*>(p->ws + L.dl + L.fields + L.T) + 4000;
  p->host_scalar = nbar;
  HIPCHK(hipMemcpyAsync(nb, &p->host_scalar, sizeof(double), hipMemcpyHostToDevice, p->stream));
  return estimate_from_spectrum(p, reinterpret_cast<const float2*>(delta_l), prec, nbar > 0 ? nb : nullptr, nullptr,
                                nullptr, nullptr, bnum, alpha, beta, false, true);
}

extern "C++" {  // helpers keep C++ (internal) linkage inside the C block
namespace {

// The whole path on the plan's stream, kernels only (no host synchronisation,
// no memset or host-copy nodes), so that it can be captured in a graph. npd:
// optional device-side particle count read by the assignment kernels (np then
// bounds it).
bsp_status whole_path(bsp_plan p, const float* ux, const float* uy, const float* uz, const float* w, int64_t np,
                      const int64_t* npd, bsp_precision prec, double* B, double* B0sub, double* Pbar, double* bnum,
                      double* alpha, double* beta) {
  const Layout L = layout(p);
  bsp_status s = need_ws(p, L.total);
  if (s != BSP_OK) return s;
  char* scr = p->ws + L.dl + L.fields + L.T + L.small;
  double* small = reinterpret_cast<double*>(p->ws + L.dl + L.fields + L.T);
  double* wsum = small + 4000;
  double* nbar = small + 4001;
  float* grids = reinterpret_cast<float*>(scr);
  float2* dl = reinterpret_cast<float2*>(p->ws);
  HIPCHK(launch_fill_u32(wsum, 0u, 2, p->stream));
  {
    // algorithmic minimum: the catalogue read once, each grid node written once
    StageTimer t(p, 0, (double)np * (w ? 16.0 : 12.0) + (double)p->ngrid * p->N * p->N * p->N * 4.0);
    const size_t tb = assign_tiled_bytes(np, p->N);
    if (tb && tb <= L.scratch - L.s_grid && assign_tiled_preferred(p->N)) {
      HIPCHK(launch_assign_tiled(ux, uy, uz, w, np, p->N, p->g.window, p->g.interlace, 0, grids, wsum, p->d_err,
                                 scr + L.s_grid, L.scratch - L.s_grid, p->stream, npd));
    } else {
      HIPCHK(launch_assign(ux, uy, uz, w, np, p->N, p->g.window, p->g.interlace, 0, grids, wsum, p->d_err,
                           scr + L.s_grid, L.scratch - L.s_grid, p->stream, npd));
    }
  }
  HIPCHK(launch_scale_scalar(wsum, 1.0 / p->V, nbar, p->stream));
  s = forward_moments(p, grids, p->ngrid, 1, wsum, p->g.compensate, dl, scr + L.s_grid);
  if (s != BSP_OK) return s;
  return estimate_from_spectrum(p, dl, prec, nbar, B, B0sub, Pbar, bnum, alpha, beta, true, true);
}

}  // namespace
}  // extern "C++"

bsp_status bsp_bispectrum_multipoles(bsp_plan p, const float* ux, const float* uy, const float* uz, const float* w,
                                     int64_t np, bsp_precision prec, double* B, double* B0sub, double* Pbar,
                                     double* bnum, double* alpha, double* beta) {
  if (!p || !ux || !uy || !uz || !B || np < 1) return fail(p, BSP_ERR_ARG, "bad argument");
  if (!p->pre_done) return fail(p, BSP_ERR_STATE, "bsp_precompute has not run");
  if (prec < BSP_FP32 || prec > BSP_BF16X1) return fail(p, BSP_ERR_ARG, "bad precision");
  const bsp_status s = need_ws(p, layout(p).total);
  if (s != BSP_OK) return s;
  return whole_path(p, ux, uy, uz, w, np, nullptr, prec, B, B0sub, Pbar, bnum, alpha, beta);
}

bsp_status bsp_bispectrum_field(bsp_plan p, const float* delta, bsp_precision prec, double* B, double* Pbar,
                                double* bnum, double* alpha, double* beta) {
  if (!p || !delta || !B) return fail(p, BSP_ERR_ARG, "bad argument");
  if (!p->pre_done) return fail(p, BSP_ERR_STATE, "bsp_precompute has not run");
  if (prec < BSP_FP32 || prec > BSP_BF16X1) return fail(p, BSP_ERR_ARG, "bad precision");
  const Layout L = layout(p);
  bsp_status s = need_ws(p, L.total);
  if (s != BSP_OK) return s;
  char* scr = p->ws + L.dl + L.fields + L.T + L.small;
  float2* dl = reinterpret_cast<float2*>(p->ws);
  s = forward_moments(p, delta, 1, 0, nullptr, 0, dl, scr);
  if (s != BSP_OK) return s;
  return estimate_from_spectrum(p, dl, prec, nullptr, B, nullptr, Pbar, bnum, alpha, beta, true, true);
}

bsp_status bsp_set_timing(bsp_plan p, int32_t enable) {
  if (!p) return BSP_ERR_ARG;
  HIPCHK(hipStreamSynchronize(p->stream));
  p->timing = enable != 0;
  p->ev_used = 0;
  for (int i = 0; i < 16; ++i) {
    p->stage_ms[i] = 0.0;
    p->stage_n[i] = 0;
    p->stage_amount[i] = 0.0;
  }
  return BSP_OK;
}

bsp_status bsp_power_multipoles(bsp_plan p, const void* delta_l, double* P) {
  if (!p || !delta_l || !P) return fail(p, BSP_ERR_ARG, "null argument");
  bsp_status s = need_ws(p, align_up((size_t)p->nl * p->nbins * sizeof(double)));
  if (s != BSP_OK) return s;
  double* psum = reinterpret_cast<double*>(p->ws);
  // algorithmic bytes: every moment's spectrum read once at the shell modes
  double modes = 0.0;
  for (int b = 0; b < p->nbins; ++b) modes += (double)p->row_support32[b];
  StageTimer t(p, 10, modes * p->nl * 8.0);
  const float2* dl = reinterpret_cast<const float2*>(delta_l);
  HIPCHK(launch_shell_cross(dl, p->spec, p->nl, dl, p->c, p->cz, p->d_bin_of_n2, p->n2max, p->nbins, p->d_nb_modes,
                            p->V / std::pow((double)p->N, 6), psum, P, p->stream));
  return BSP_OK;
}

bsp_status bsp_shot_noise_multipoles(bsp_plan p, const double* Pl, double nbar, double* SN) {
  if (!p || !Pl || !SN || !(nbar > 0.0)) return fail(p, BSP_ERR_ARG, "null argument or nbar <= 0");
  if (!p->pre_done) return fail(p, BSP_ERR_STATE, "bsp_precompute has not run");
  HIPCHK(launch_shot_noise(Pl, p->nbins, p->d_tri_bins, (int)p->tri.size(), p->nl, p->d_ring, nbar, SN, p->stream));
  return BSP_OK;
}

bsp_status bsp_skew_spectra(bsp_plan p, const void* delta_l, double* S, int32_t flags) {
  if (!p || !delta_l || !S || (flags & ~BSP_SKEW_BALL)) return fail(p, BSP_ERR_ARG, "null argument or bad flags");
  const int brow = p->band_row32 + ((flags & BSP_SKEW_BALL) ? 1 : 0);  // table row of the squared monopole's range
  const int32_t* meta = p->d_band_meta + ((flags & BSP_SKEW_BALL) ? 2 : 0);
  const int Nr = p->Nr, c = p->c, cz = p->cz, w = 2 * c + 1;
  const size_t dbytes = align_up((size_t)Nr * Nr * Nr * sizeof(float));
  const size_t zb = align_up((size_t)Nr * Nr * cz * sizeof(float2)), yb = align_up((size_t)Nr * w * cz * sizeof(float2));
  const size_t scr = std::max(inv_scratch(p, 2, Nr, sizeof(float2)), zb + yb);
  const size_t acc = align_up((size_t)p->nl * p->nbins * sizeof(double));
  bsp_status s = need_ws(p, dbytes + scr + acc);
  if (s != BSP_OK) return s;
  float* d = reinterpret_cast<float*>(p->ws);
  char* sc = p->ws + dbytes;
  double* psum = reinterpret_cast<double*>(p->ws + dbytes + scr);
  const float2* dl = reinterpret_cast<const float2*>(delta_l);
  // algorithmic bytes of the passes: the band-limited monopole's inverse
  // transform (its modes read, nonzero columns, y output, real field written),
  // the square (read + write), the pruned forward transform of the square to
  // the compact cube, and the shell sums (nl moments and the partner spectrum)
  const double C1 = c + 1.0, W1 = w, R = Nr, sup = (double)p->row_support32[brow],
               cols = (double)p->row_cols32[brow];
  const double amount = (sup + 2.0 * R * cols + 2.0 * R * R * C1) * 8.0 + R * R * R * 4.0 + R * R * R * 8.0 +
                        R * R * R * 4.0 + R * R * C1 * 8.0 + R * C1 * 8.0 * (R + W1) + W1 * C1 * 8.0 * (R + W1) +
                        (p->nl + 1.0) * sup * 8.0;
  StageTimer t(p, 11, amount);
  // d(x): unnormalised inverse DFT at N' of delta^(0) kept on the union of the shells (or the ball)
  const std::vector<int> cf{c};
  s = inverse_fields<float>(p, dl, p->spec, 1, meta, meta + 1, p->d_tab32, p->d_rng32, d, sc, 2, cf, &brow);
  if (s != BSP_OK) return s;
  HIPCHK(launch_square(d, (int64_t)Nr * Nr * Nr, p->stream));
  // Q = DFT[d^2] at N', pruned to the compact cube |n_a| <= c
  float2* Z = reinterpret_cast<float2*>(sc);
  float2* Y = reinterpret_cast<float2*>(sc + zb);
  FwdZDesc fz{};
  fz.ngrid = 1;
  fz.nlos = 1;
  fz.contrast = 0;
  fz.plane = 1;
  fz.cout = c + 1;
  fz.zs = cz;
  HIPCHK(launch_fwd_z_f32(Nr, d, Z, fz, p->tw32_Nr, p->stream));
  PassDesc py{};
  py.tiles = p->tune_tiles;
  py.nouter = Nr;
  py.in_outer = (int64_t)Nr * cz;
  py.out_outer = (int64_t)w * cz;
  py.in_row = cz;
  py.out_row = cz;
  py.ncols = cz;
  py.in_rows = Nr;
  py.in_off = 0;
  py.out_rows = w;
  py.out_off = c;
  set1d(py);
  HIPCHK(launch_c2c_f32(Nr, -1, Z, Y, py, nullptr, p->tw32_Nr, p->stream));
  PassDesc px{};
  px.tiles = p->tune_tiles;
  px.nouter = 1;
  px.in_outer = (int64_t)Nr * w * cz;
  px.out_outer = (int64_t)w * w * cz;
  px.in_row = (int64_t)w * cz;
  px.out_row = (int64_t)w * cz;
  px.ncols = w * cz;
  px.in_rows = Nr;
  px.in_off = 0;
  px.out_rows = w;
  px.out_off = c;
  set1d(px);
  float2* X = Z;  // Z is dead once Y exists
  HIPCHK(launch_c2c_f32(Nr, -1, Y, X, px, nullptr, p->tw32_Nr, p->stream));
  // S^l_b = V sum_{n in b} Re[delta^(l) conj Q] / (N^9 N'^3 N_b)
  HIPCHK(launch_shell_cross(dl, p->spec, p->nl, X, c, cz, p->d_bin_of_n2, p->n2max, p->nbins, p->d_nb_modes,
                            p->V / (std::pow((double)p->N, 9) * std::pow((double)Nr, 3)), psum, S, p->stream));
  return BSP_OK;
}

bsp_status bsp_integrated_bispectrum(bsp_plan p, const float* grid, const double* wsum, int32_t s, double k0,
                                     double dk, int32_t nbins, double* iB, double* Psub, double* dbar, int32_t flags) {
  if (!p || !grid || !iB || s < 1 || nbins < 1 || !(dk > 0.0) || !(k0 > 0.0) || (flags & ~BSP_IB_LOCAL_LOS))
    return fail(p, BSP_ERR_ARG, "bad argument");
  // the local line of sight differs from the one per sub-volume only when it varies
  const bool local = (flags & BSP_IB_LOCAL_LOS) && !p->plane;
  const int N = p->N;
  if (N % s != 0) return fail(p, BSP_ERR_SIZE, "s must divide N");
  const int m = N / s, ns = s * s * s;
  if (!fft_size_supported(m) || m % 4 != 0) return fail(p, BSP_ERR_SIZE, "unsupported sub-volume size N / s");
  if (!p->plane && !(flags & BSP_IB_LOCAL_LOS)) {
    // the one line of sight of a sub-volume points at its centre, origin + (M - 1)/2
    bool at_centre = true;
    for (int a = 0; a < 3; ++a) {
      const double u = (p->g.observer[a] - 0.5 * (m - 1)) / m;
      at_centre = at_centre && std::fabs(u - std::rint(u)) < 1e-12 && std::rint(u) >= 0 && std::rint(u) < s;
    }
    if (at_centre) return fail(p, BSP_ERR_ARG, "observer at a sub-volume centre (its line of sight is undefined)");
  }
  if (ns > 65535) return fail(p, BSP_ERR_SIZE, "too many sub-volumes");
  // sub-volume shells (units of 2 pi s / L): (2 c_b - dk)^2 <= 4 n^2 < (2 c_b + dk)^2, 2 k0 and dk integers
  std::vector<int64_t> lo(nbins), hi(nbins);
  for (int b = 0; b < nbins; ++b) {
    const double a = 2.0 * (k0 + b * dk) - dk, z = 2.0 * (k0 + b * dk) + dk;
    if (std::fabs(a - std::round(a)) > 1e-9 || std::fabs(z - std::round(z)) > 1e-9 || a < 0)
      return fail(p, BSP_ERR_ARG, "2 k0 and dk must be integers");
    lo[b] = (int64_t)std::llround(a) * std::llround(a);
    hi[b] = (int64_t)std::llround(z) * std::llround(z);
  }
  const int n2max = (int)((hi[nbins - 1] - 1) / 4);
  if ((int64_t)4 * n2max >= (int64_t)m * m) return fail(p, BSP_ERR_SIZE, "sub-volume shells reach |n| >= M / 2");
  std::vector<int32_t> bin(n2max + 1, -1);
  for (int n2 = 0; n2 <= n2max; ++n2)
    for (int b = 0; b < nbins; ++b)
      if (4 * (int64_t)n2 >= lo[b] && 4 * (int64_t)n2 < hi[b]) bin[n2] = b;
  // modes per shell over the full lattice of the sub-volume
  std::vector<int64_t> nbm(nbins, 0);
  int cm = 0;
  while ((int64_t)(cm + 1) * (cm + 1) <= n2max) ++cm;
  for (int x = -cm; x <= cm; ++x)
    for (int y = -cm; y <= cm; ++y)
      for (int z = -cm; z <= cm; ++z) {
        const int64_t n2 = (int64_t)x * x + (int64_t)y * y + (int64_t)z * z;
        if (n2 <= n2max && bin[n2] >= 0) nbm[bin[n2]]++;
      }
  const int nl = p->nl;
  const int h = m / 2 + 1;
  const size_t gbytes = align_up((size_t)N * N * N * sizeof(float));
  const size_t fbytes = align_up((size_t)ns * m * m * h * sizeof(float2));
  const size_t pbytes = align_up((size_t)ns * nl * nbins * sizeof(double));
  const size_t dbytes = align_up((size_t)ns * sizeof(double));
  const size_t tbytes = align_up(bin.size() * sizeof(int32_t)) + align_up(nbm.size() * sizeof(int64_t));
  const size_t f2bytes = local ? fbytes : 0;  // the kept F_i0 beside each harmonic's spectra
  bsp_status st = need_ws(p, gbytes + fbytes + pbytes + dbytes + tbytes + f2bytes);
  if (st != BSP_OK) return st;
  const float2* tw = tw32_for(p, m);
  if (!tw) return fail(p, BSP_ERR_HIP, "twiddle table allocation failed");
  float* sub = reinterpret_cast<float*>(p->ws);
  float2* F = reinterpret_cast<float2*>(p->ws + gbytes);
  double* psum = reinterpret_cast<double*>(p->ws + gbytes + fbytes);
  double* db = dbar ? dbar : reinterpret_cast<double*>(p->ws + gbytes + fbytes + pbytes);
  int32_t* dbin = reinterpret_cast<int32_t*>(p->ws + gbytes + fbytes + pbytes + dbytes);
  int64_t* dnb = reinterpret_cast<int64_t*>(p->ws + gbytes + fbytes + pbytes + dbytes + align_up(bin.size() * 4));
  HIPCHK(hipMemcpyAsync(dbin, bin.data(), bin.size() * sizeof(int32_t), hipMemcpyHostToDevice, p->stream));
  HIPCHK(hipMemcpyAsync(dnb, nbm.data(), nbm.size() * sizeof(int64_t), hipMemcpyHostToDevice, p->stream));
  HIPCHK(launch_fill_u32(psum, 0u, 2 * (int64_t)ns * nl * nbins, p->stream));
  // algorithmic bytes: the grid read once, each transform pass's input and
  // output once, the sub-volume spectra read once by the shell sums
  const double R = (double)N * N * N, H = (double)ns * m * m * h * 8.0;
  const int window = p->g.compensate ? p->g.window : -1;
  // with the local line of sight, one pass per harmonic h_m of degree <= lmax
  const int nh = local ? (nl == 1 ? 1 : (nl == 2 ? 6 : 15)) : 1;
  StageTimer t(p, 12, local ? nh * (R * 4.0 + R * 4.0 * 2.0 + H * 6.0 + 2.0 * H) : R * 4.0 + R * 4.0 * 2.0 + H * 7.0);
  if (local) {
    // each harmonic's spectra are summed against the kept F_i0
    float2* Fm = reinterpret_cast<float2*>(p->ws + gbytes + fbytes + pbytes + dbytes + tbytes);
    for (int hm = 0; hm < nh; ++hm) {
      float2* dst = hm == 0 ? F : Fm;
      HIPCHK(launch_gather_subvolumes_los(grid, wsum, N, s, hm, p->g.observer, sub, p->stream));
      st = r2c_batch(p, m, ns, sub, dst, tw);
      if (st != BSP_OK) return st;
      const int l = kLosDegree[hm];
      HIPCHK(launch_subvolume_cross(F, dst, m, s, hm, l / 2, (2.0 * l + 1.0) * kLosCoef[hm], window, nl, dbin, n2max,
                                    nbins, psum, db, p->stream));
    }
  } else {
    HIPCHK(launch_gather_subvolumes(grid, wsum, N, s, sub, p->stream));
    st = r2c_batch(p, m, ns, sub, F, tw);
    if (st != BSP_OK) return st;
    HIPCHK(launch_subvolume_shells(F, m, s, p->plane, p->g.observer, window, nl, dbin, n2max, nbins, psum, db,
                                   p->stream));
  }
  const double Vs = p->V / ((double)s * s * s);
  HIPCHK(launch_subvolume_finalize(psum, db, ns, nl, nbins, dnb, Vs / std::pow((double)m, 6), iB, Psub, p->stream));
  t.stop();
  HIPCHK(hipStreamSynchronize(p->stream));  // the host tables above are read by the copies
  return BSP_OK;
}

// Reduction schedule of B^(l1 l2 l3) over the shell fields D^l_b (field b nl + l):
// pairs (D^l2_b2 D^l3_b3, b2 >= b3; for b2 = b3 only l2 <= l3, the other order
// is the same product) in b2-major order, thirds D^l1_b1, every combination of
// each triangle with a nonzero count.
static bool build_full(bsp_plan p) {
  const int nb = p->nbins, nl = p->nl, nsh = nb * nl;
  std::vector<std::array<int, 2>> pr;
  std::vector<int> pidx((size_t)nsh * nsh, -1);
  for (int b2 = 0; b2 < nb; ++b2)
    for (int b3 = 0; b3 <= b2; ++b3)
      for (int l2 = 0; l2 < nl; ++l2)
        for (int l3 = 0; l3 < nl; ++l3) {
          if (b2 == b3 && l3 < l2) continue;
          const int f2 = b2 * nl + l2, f3 = b3 * nl + l3;
          pidx[(size_t)f2 * nsh + f3] = pidx[(size_t)f3 * nsh + f2] = (int)pr.size();
          pr.push_back({f2, f3});
        }
  std::vector<int> th(nsh);
  for (int f = 0; f < nsh; ++f) th[f] = f;
  const int ntri = (int)p->tri.size();
  std::vector<uint8_t> need(pr.size() * nsh, 0);
  std::vector<int32_t> tidx((size_t)nl * nl * nl * ntri, 0);
  for (int i = 0; i < ntri; ++i) {
    const int b1 = p->tri[i][0], b2 = p->tri[i][1], b3 = p->tri[i][2];
    for (int l1 = 0; l1 < nl; ++l1)
      for (int l2 = 0; l2 < nl; ++l2)
        for (int l3 = 0; l3 < nl; ++l3) {
          const int pair = pidx[(size_t)(b2 * nl + l2) * nsh + (b3 * nl + l3)];
          const int third = b1 * nl + l1;
          if (pair < 0) return false;
          need[(size_t)pair * nsh + third] = 1;
          tidx[((size_t)(l1 * nl + l2) * nl + l3) * ntri + i] = pair * nsh + third;
        }
  }
  if (!build_reduce(p->full_rp, pr, th, need, nsh, 1)) return false;
  if (!upload_rp(p, p->full_rp)) return false;
  p->d_full_tidx = upload(p, tidx);
  if (!p->d_full_tidx) return false;
  p->full_built = true;
  return true;
}

bsp_status bsp_bispectrum_full(bsp_plan p, const void* delta_l, bsp_precision prec, double* B) {
  if (!p || !delta_l || !B) return fail(p, BSP_ERR_ARG, "null argument");
  if (!p->pre_done) return fail(p, BSP_ERR_STATE, "bsp_precompute has not run");
  if (prec < BSP_FP32 || prec > BSP_BF16X1) return fail(p, BSP_ERR_ARG, "bad precision");
  if (!p->full_built && !build_full(p)) return fail(p, BSP_ERR_ARG, "full multipole reduction shape not supported");
  const Layout L = layout(p);
  bsp_status s = need_ws(p, L.total);
  if (s != BSP_OK) return s;
  const int Nr = p->Nr, nl = p->nl, nsh = p->nbins * nl;
  const int64_t K = (int64_t)Nr * Nr * Nr;
  const int64_t Ks = (int64_t)p->slab * Nr * Nr;  // points of one x-slab
  char* ws = p->ws;
  float* fields = reinterpret_cast<float*>(ws + L.dl);
  double* small = reinterpret_cast<double*>(ws + L.dl + L.fields + L.T);
  float* scale = reinterpret_cast<float*>(small + 2048);
  unsigned* tmpu = reinterpret_cast<unsigned*>(small + 3072);
  char* scr = ws + L.dl + L.fields + L.T + L.small;
  const size_t scr_bytes = p->ws_bytes - (L.dl + L.fields + L.T + L.small);
  const ReducePlan& rp = p->full_rp;
  // T first in the scratch, the reduction partials after it. With one slab
  // the inverse passes may use the whole scratch (T is zeroed after them);
  // with several, T accumulates over the slabs and the inverse passes use the
  // rest, in batches small enough to fit (the batching does not change a value)
  double* T = reinterpret_cast<double*>(scr);
  const size_t tb = align_up((size_t)rp.npairs * rp.nthirds * sizeof(double));
  const bool one_slab = p->slab == Nr;
  int fb = L.fb;
  while (!one_slab && fb > 2 && tb + inv_scratch(p, fb, p->slab, sizeof(float2)) >= scr_bytes) fb -= 2;
  if (scr_bytes <= tb || (!one_slab && scr_bytes <= tb + inv_scratch(p, fb, p->slab, sizeof(float2))))
    return fail(p, BSP_ERR_WORKSPACE, "workspace too small for the full multipoles");
  // chunks long enough for the partials of every tile to fit the scratch
  const size_t avail = scr_bytes - tb;
  const int64_t per_chunk = (int64_t)rp.ntiles * 256 * (int64_t)sizeof(float);
  const int64_t max_chunks = std::max<int64_t>(1, (int64_t)(avail / std::max<int64_t>(per_chunk, 1)));
  int64_t kc_min = (Ks + max_chunks - 1) / max_chunks;
  kc_min = (kc_min + 63) / 64 * 64;
  // the shell fields D^l_b (the first nbins nl fields of the main numbering)
  s = slab_reduce<float>(p, rp, reinterpret_cast<const float2*>(delta_l), p->spec, nsh, p->d_field_ell,
                         p->d_field_tab, p->d_tab32, p->d_rng32, p->field_c, p->field_row32.data(), fb, fields,
                         kprec(prec), prec == BSP_FP16X3 ? scale : nullptr, tmpu, T, one_slab ? scr : scr + tb,
                         scr + tb, avail, kc_min);
  if (s != BSP_OK) return s;
  const double N = p->N;
  const double norm_b = p->V * p->V / (std::pow(N, 9) * (double)K);
  HIPCHK(launch_binned_finalize(T, p->d_full_tidx, (int)p->tri.size(), nl * nl * nl, p->d_counts, nullptr,
                                p->d_nb_modes, p->nbins, p->d_tri_bins, norm_b, 0.0, nullptr, B, nullptr, nullptr,
                                p->stream));
  return BSP_OK;
}

bsp_status bsp_stage_times(bsp_plan p, double* ms, int64_t* launches, double* amount) {
  if (!p || !ms) return fail(p, BSP_ERR_ARG, "null argument");
  HIPCHK(hipStreamSynchronize(p->stream));
  for (size_t i = 0; i < p->ev_used; ++i) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, p->ev_pool[i][0], p->ev_pool[i][1]));
    p->stage_ms[p->ev_stage[i]] += t;
    p->stage_n[p->ev_stage[i]] += 1;
  }
  p->ev_used = 0;
  for (int i = 0; i < 16; ++i) {
    ms[i] = p->stage_ms[i];
    if (launches) launches[i] = p->stage_n[i];
    if (amount) amount[i] = p->stage_amount[i];
  }
  return BSP_OK;
}

extern "C++" {  // helpers keep C++ (internal) linkage inside the C block
namespace {

// (Re)captures the whole path of plan q into q's batch graph for catalogues of
// up to cap particles at precision prec; the graph reads its catalogue from
// q->bslot.in and its count from q->bslot.npd and writes q->bslot.out.
bsp_status batch_graph(bsp_plan q, bsp_precision prec, int64_t cap, int has_w) {
  auto& b = q->bslot;
  if (b.exec && b.prec == (int)prec && b.cap >= cap && b.has_w == has_w) return BSP_OK;
  b.release();
  bsp_plan p = q;  // for HIPCHK
  if (!b.stream) HIPCHK(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
  const size_t nout = (size_t)q->nl * (q->tri.size() + 2 * (size_t)q->nmodes);
  HIPCHK(hipMalloc(&b.in, (size_t)(3 + has_w) * cap * sizeof(float)));
  HIPCHK(hipMalloc(&b.npd, sizeof(int64_t)));
  HIPCHK(hipMalloc(&b.out, nout * sizeof(double)));
  b.prec = (int)prec;
  b.cap = cap;
  b.has_w = has_w;
  double* oB = b.out;
  double* oA = oB + (size_t)q->nl * q->tri.size();
  double* oBe = oA + (size_t)q->nl * q->nmodes;
  // capture on the batch stream: the path enqueues on q->stream, pointed there
  // for the capture, with stage timing off
  const hipStream_t keep = q->stream;
  const bool timing = q->timing;
  q->stream = b.stream;
  q->timing = false;
  hipGraph_t graph = nullptr;
  bsp_status s = BSP_OK;
  hipError_t e = hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    s = whole_path(q, b.in, b.in + cap, b.in + 2 * cap, has_w ? b.in + 3 * cap : nullptr, cap, b.npd, prec, oB,
                   nullptr, nullptr, nullptr, oA, oBe);
    e = hipStreamEndCapture(b.stream, &graph);
  }
  q->stream = keep;
  q->timing = timing;
  if (s != BSP_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    b.release();
    return s;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b.exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    b.release();
    return fail(q, BSP_ERR_HIP, std::string("graph capture of the whole path: ") + hipGetErrorString(e));
  }
  return BSP_OK;
}

}  // namespace
}  // extern "C++"

extern "C++" {  // helpers keep C++ (internal) linkage inside the C block
namespace {

// Content hash of everything that fixes a mock's outputs apart from its
// catalogue: the geometry, the modal basis and the modes the
// orthonormalisation kept, the triangles, the precision and the journal
// format. Journal records are matched on (mock key, this hash).
uint64_t config_hash(const bsp_plan p, bsp_precision prec) {
  uint64_t h = fnv1a64("libbsp batch journal v1", 23);
  auto mix = [&h](const void* d, size_t n) { h = fnv1a64(d, n, h); };
  auto mixi = [&mix](int64_t v) { mix(&v, sizeof v); };
  auto mixd = [&mix](double v) { mix(&v, sizeof v); };
  mixi(p->N);
  mixi(p->Nr);
  mixd(p->g.box);
  mixi(p->g.window);
  mixi(p->g.compensate);
  mixi(p->g.interlace);
  mixi(p->g.los);
  for (double o : p->g.observer) mixd(p->g.los ? o : 0.0);
  mixi(p->g.lmax);
  mixi(p->g.nbins);
  mixd(p->g.k0);
  mixd(p->g.dk);
  mixi(p->modal ? 1 : 0);
  mixi(p->P);
  mixi(p->nmodes);
  mix(p->modes.data(), p->modes.size() * sizeof(int32_t));
  mix(p->pfid.data(), p->pfid.size() * sizeof(double));
  mixd(p->drop_tol);
  mix(p->piv_h.data(), p->piv_h.size() * sizeof(int32_t));
  for (const auto& t : p->tri) mix(t.data(), 3 * sizeof(int));
  mixi((int)prec);
  if (p->slab != p->Nr) mixi(p->slab);  // the slabs add T in another order (whole cubes keep their hash)
  return h;
}

// Pinned staging of finished mocks' outputs on their way to the journal: two
// slots, each [B | alpha | beta | error word]; the host writes mock k's record
// while mock k+1 runs. Released only after every stream that copies into it
// has drained.
struct JournalStage {
  double* h = nullptr;
  int64_t slot = 0;  // doubles per slot
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<hipStream_t> streams;
  ~JournalStage() {
    for (hipStream_t s : streams) (void)hipStreamSynchronize(s);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (h) (void)hipHostFree(h);
  }
};

bsp_status batch_impl(const bsp_plan* plans, int32_t nplans, const int32_t* mock_plan, int32_t nmocks,
                      const uint64_t* mock_key, const float* const* ux, const float* const* uy,
                      const float* const* uz, const float* const* w, const int64_t* np, bsp_precision prec,
                      double* B_all, double* alpha_all, double* beta_all, double* cov, int32_t flags,
                      const char* journal_path, int32_t* nresumed) {
  if (!plans || nplans < 1 || !mock_plan || nmocks < 2 || !ux || !uy || !uz || !np || !B_all || !alpha_all || !cov)
    return fail(nullptr, BSP_ERR_ARG, "bad argument");
  bsp_plan p0 = plans[0];
  if (!p0) return fail(nullptr, BSP_ERR_ARG, "null plan");
  if (prec < BSP_FP32 || prec > BSP_BF16X1) return fail(p0, BSP_ERR_ARG, "bad precision");
  const bool journaled = journal_path != nullptr;
  if (journaled && (!mock_key || !*journal_path)) return fail(p0, BSP_ERR_ARG, "journal without mock keys or path");
  // every plan must produce outputs of the same shape: nl, triangles and modes
  for (int i = 0; i < nplans; ++i) {
    bsp_plan q = plans[i];
    if (!q) return fail(p0, BSP_ERR_ARG, "null plan");
    if (!q->pre_done) return fail(p0, BSP_ERR_STATE, "bsp_precompute has not run on every plan");
    if (!q->modal || q->nl != p0->nl || q->nmodes != p0->nmodes || q->tri.size() != p0->tri.size())
      return fail(p0, BSP_ERR_ARG, "plans differ in multipoles, triangles or modes (or have no modal basis)");
    // alpha is a coefficient vector on the same orthonormal modes only when
    // every plan kept the same modes in the same order
    if (q->piv_h != p0->piv_h) return fail(p0, BSP_ERR_ARG, "plans kept different modes in their orthonormalisation");
    const bsp_status s = need_ws(q, layout(q).total);
    if (s != BSP_OK) {
      if (q != p0) p0->err = q->err;
      return s;
    }
  }
  for (int m = 0; m < nmocks; ++m) {
    if (mock_plan[m] < 0 || mock_plan[m] >= nplans) return fail(p0, BSP_ERR_ARG, "mock plan index out of range");
    if (np[m] < 1 || !ux[m] || !uy[m] || !uz[m]) return fail(p0, BSP_ERR_ARG, "empty or null mock catalogue");
  }
  const int64_t ntri = (int64_t)p0->tri.size();
  const int64_t nB = (int64_t)p0->nl * ntri;
  const int64_t D = (int64_t)p0->nl * p0->nmodes;
  const bool graphs = (flags & BSP_BATCH_GRAPH) != 0;
  if (nresumed) *nresumed = 0;

  // journal: which mocks are already recorded under their plan's configuration
  Journal jn;
  std::vector<uint64_t> hashes(nplans, 0);
  // records of the mocks taken from the journal (copies: appends may move the index)
  std::vector<JournalRecord> recv(nmocks);
  std::vector<char> rec(nmocks, 0);
  int64_t nres = 0;
  if (journaled) {
    std::string err;
    if (!jn.open(journal_path, true, err)) return fail(p0, BSP_ERR_IO, err);
    for (int i = 0; i < nplans; ++i) hashes[i] = config_hash(plans[i], prec);
    std::vector<std::pair<uint64_t, uint64_t>> seen;
    for (int m = 0; m < nmocks; ++m) {
      const uint64_t hm = hashes[mock_plan[m]];
      seen.emplace_back(mock_key[m], hm);
      const JournalRecord* r = jn.find(mock_key[m], hm);
      if (!r) continue;
      if (r->np != np[m] || r->nl != p0->nl || r->ntri != ntri || r->d != D)
        return fail(p0, BSP_ERR_ARG, "journal record of mock key " + std::to_string(mock_key[m]) +
                                         " has another particle count or output shape");
      if (beta_all && !r->has_beta) continue;  // recorded without beta: run it again
      recv[m] = *r;
      rec[m] = 1;
      ++nres;
    }
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
      return fail(p0, BSP_ERR_ARG, "two mocks share a key on the same configuration");
  }

  if (graphs) {
    // one graph per plan, sized for the largest catalogue the plan runs
    std::vector<int64_t> cap(nplans, 0);
    std::vector<int> hw(nplans, 0);
    for (int m = 0; m < nmocks; ++m) {
      if (rec[m]) continue;
      cap[mock_plan[m]] = std::max(cap[mock_plan[m]], np[m]);
      if (w && w[m]) hw[mock_plan[m]] = 1;
    }
    for (int i = 0; i < nplans; ++i) {
      if (cap[i] == 0) continue;
      // the plan's earlier work (and the caller's) finishes before its batch stream starts
      bsp_status s = bsp_sync(plans[i]);
      if (s == BSP_OK) s = batch_graph(plans[i], prec, cap[i], hw[i]);
      if (s != BSP_OK) {
        if (plans[i] != p0) p0->err = plans[i]->err;
        return s;
      }
    }
  }

  JournalStage st;
  if (journaled) {
    bsp_plan p = p0;  // for HIPCHK
    st.slot = nB + 2 * D + 1;
    for (int i = 0; i < nplans; ++i) {
      st.streams.push_back(plans[i]->stream);
      if (graphs && plans[i]->bslot.stream) st.streams.push_back(plans[i]->bslot.stream);
    }
    HIPCHK(hipHostMalloc((void**)&st.h, (size_t)(2 + nres) * st.slot * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&st.ev[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&st.ev[1], hipEventDisableTiming));
    // recorded mocks: their outputs go back to the device from the journal
    int64_t k = 0;
    for (int m = 0; m < nmocks; ++m) {
      if (!rec[m]) continue;
      double* hb = st.h + (2 + k++) * st.slot;
      std::string err;
      if (!jn.read(recv[m], hb, hb + nB, hb + nB + D, err)) return fail(p0, BSP_ERR_IO, err);
      HIPCHK(hipMemcpyAsync(B_all + m * nB, hb, nB * sizeof(double), hipMemcpyHostToDevice, p0->stream));
      HIPCHK(hipMemcpyAsync(alpha_all + m * D, hb + nB, D * sizeof(double), hipMemcpyHostToDevice, p0->stream));
      if (beta_all)
        HIPCHK(hipMemcpyAsync(beta_all + m * D, hb + nB + D, D * sizeof(double), hipMemcpyHostToDevice,
                              p0->stream));
    }
  }

  // record of the k-th mock run in this call, once its copies have landed;
  // a kernel error latched on its plan stops the journal there
  std::vector<int> run_mock;
  auto flush = [&](int64_t k) -> bsp_status {
    const int m = run_mock[k];
    bsp_plan p = p0;  // for HIPCHK
    HIPCHK(hipEventSynchronize(st.ev[k & 1]));
    const double* hb = st.h + (k & 1) * st.slot;
    int32_t e = 0;
    std::memcpy(&e, hb + nB + 2 * D, sizeof e);
    if (e) {
      // drain every stream, then report (and clear) the latched error
      for (hipStream_t s : st.streams) (void)hipStreamSynchronize(s);
      bsp_plan q = plans[mock_plan[m]];
      const bsp_status s = bsp_sync(q);
      if (q != p0) p0->err = q->err;
      return s != BSP_OK ? s : fail(p0, BSP_ERR_DEVICE, "device error");
    }
    std::string err;
    if (!jn.append(mock_key[m], hashes[mock_plan[m]], np[m], (int)p0->nl, (int)ntri, (int)D, hb, hb + nB,
                   beta_all ? hb + nB + D : nullptr, (flags & BSP_BATCH_FSYNC) != 0, err))
      return fail(p0, BSP_ERR_IO, err);
    return BSP_OK;
  };

  for (int m = 0; m < nmocks; ++m) {
    if (rec[m]) continue;
    bsp_plan q = plans[mock_plan[m]];
    bsp_plan p = p0;  // for HIPCHK: errors are reported on the first plan
    hipStream_t ms = q->stream;
    if (!graphs) {
      const bsp_status s = bsp_bispectrum_multipoles(q, ux[m], uy[m], uz[m], w ? w[m] : nullptr, np[m], prec,
                                                     B_all + m * nB, nullptr, nullptr, nullptr, alpha_all + m * D,
                                                     beta_all ? beta_all + m * D : nullptr);
      if (s != BSP_OK) {
        if (q != p0) p0->err = q->err;
        return s;
      }
    } else {
      auto& b = q->bslot;
      ms = b.stream;
      const size_t nb = (size_t)np[m] * sizeof(float);
      HIPCHK(hipMemcpyAsync(b.in, ux[m], nb, hipMemcpyDeviceToDevice, b.stream));
      HIPCHK(hipMemcpyAsync(b.in + b.cap, uy[m], nb, hipMemcpyDeviceToDevice, b.stream));
      HIPCHK(hipMemcpyAsync(b.in + 2 * b.cap, uz[m], nb, hipMemcpyDeviceToDevice, b.stream));
      if (b.has_w) {
        if (w && w[m]) HIPCHK(hipMemcpyAsync(b.in + 3 * b.cap, w[m], nb, hipMemcpyDeviceToDevice, b.stream));
        else HIPCHK(launch_fill_u32(b.in + 3 * b.cap, 0x3f800000u, np[m], b.stream));
      }
      HIPCHK(launch_set_i64(b.npd, np[m], b.stream));
      HIPCHK(hipGraphLaunch(b.exec, b.stream));
      const double* oB = b.out;
      const double* oA = oB + nB;
      HIPCHK(hipMemcpyAsync(B_all + m * nB, oB, nB * sizeof(double), hipMemcpyDeviceToDevice, b.stream));
      HIPCHK(hipMemcpyAsync(alpha_all + m * D, oA, D * sizeof(double), hipMemcpyDeviceToDevice, b.stream));
      if (beta_all)
        HIPCHK(hipMemcpyAsync(beta_all + m * D, oA + D, D * sizeof(double), hipMemcpyDeviceToDevice, b.stream));
    }
    if (!journaled) continue;
    // stage this mock's outputs and its plan's error word for the journal
    const int64_t k = (int64_t)run_mock.size();
    run_mock.push_back(m);
    double* hb = st.h + (k & 1) * st.slot;
    hb[nB + 2 * D] = 0.0;
    HIPCHK(hipMemcpyAsync(hb, B_all + m * nB, nB * sizeof(double), hipMemcpyDeviceToHost, ms));
    HIPCHK(hipMemcpyAsync(hb + nB, alpha_all + m * D, D * sizeof(double), hipMemcpyDeviceToHost, ms));
    if (beta_all) HIPCHK(hipMemcpyAsync(hb + nB + D, beta_all + m * D, D * sizeof(double), hipMemcpyDeviceToHost, ms));
    HIPCHK(hipMemcpyAsync(hb + nB + 2 * D, q->d_err, sizeof(int32_t), hipMemcpyDeviceToHost, ms));
    HIPCHK(hipEventRecord(st.ev[k & 1], ms));
    if (k > 0) {
      const bsp_status s = flush(k - 1);
      if (s != BSP_OK) return s;
    }
  }
  if (!run_mock.empty()) {
    const bsp_status s = flush((int64_t)run_mock.size() - 1);
    if (s != BSP_OK) return s;
  }
  if (nresumed) *nresumed = (int32_t)nres;

  // the covariance runs on the first plan's stream once every mock is done
  for (int i = 0; i < nplans; ++i) {
    bsp_plan p = plans[i];  // for HIPCHK
    if (graphs && p->bslot.stream) HIPCHK(hipStreamSynchronize(p->bslot.stream));
    const bsp_status s = bsp_sync(plans[i]);
    if (s != BSP_OK) {
      if (plans[i] != p0) p0->err = plans[i]->err;
      return s;
    }
  }
  st.streams.clear();  // drained above
  bsp_plan p = p0;
  HIPCHK(launch_covariance(alpha_all, nmocks, (int)D, cov, p0->stream));
  return BSP_OK;
}

}  // namespace
}  // extern "C++"

bsp_status bsp_batch_run(const bsp_plan* plans, int32_t nplans, const int32_t* mock_plan, int32_t nmocks,
                         const float* const* ux, const float* const* uy, const float* const* uz,
                         const float* const* w, const int64_t* np, bsp_precision prec, double* B_all,
                         double* alpha_all, double* beta_all, double* cov, int32_t flags) {
  return batch_impl(plans, nplans, mock_plan, nmocks, nullptr, ux, uy, uz, w, np, prec, B_all, alpha_all, beta_all,
                    cov, flags, nullptr, nullptr);
}

bsp_status bsp_batch_run_journal(const bsp_plan* plans, int32_t nplans, const int32_t* mock_plan, int32_t nmocks,
                                 const uint64_t* mock_key, const float* const* ux, const float* const* uy,
                                 const float* const* uz, const float* const* w, const int64_t* np,
                                 bsp_precision prec, double* B_all, double* alpha_all, double* beta_all,
                                 double* cov, int32_t flags, const char* journal, int32_t* nresumed) {
  if (!journal) return fail(plans ? plans[0] : nullptr, BSP_ERR_ARG, "null journal path");
  return batch_impl(plans, nplans, mock_plan, nmocks, mock_key, ux, uy, uz, w, np, prec, B_all, alpha_all, beta_all,
                    cov, flags, journal, nresumed);
}

bsp_status bsp_config_hash(bsp_plan p, bsp_precision prec, uint64_t* hash) {
  if (!p || !hash) return fail(p, BSP_ERR_ARG, "null argument");
  if (!p->pre_done) return fail(p, BSP_ERR_STATE, "bsp_precompute has not run");
  if (prec < BSP_FP32 || prec > BSP_BF16X1) return fail(p, BSP_ERR_ARG, "bad precision");
  *hash = config_hash(p, prec);
  return BSP_OK;
}

bsp_status bsp_journal_scan(const char* journal, int64_t* nrecords, int64_t* valid_bytes, int64_t* file_bytes) {
  if (!journal || !nrecords) return fail(nullptr, BSP_ERR_ARG, "null argument");
  Journal jn;
  std::string err;
  if (!jn.open(journal, false, err)) return fail(nullptr, BSP_ERR_IO, err);
  *nrecords = jn.records();
  if (valid_bytes) *valid_bytes = jn.valid_bytes();
  if (file_bytes) *file_bytes = jn.file_bytes();
  return BSP_OK;
}

bsp_status bsp_journal_append(const char* journal, uint64_t key, uint64_t config_hash, int64_t np, int32_t nl,
                              int32_t ntri, int32_t d, const double* B, const double* alpha, const double* beta) {
  if (!journal || !B || !alpha || np < 1 || nl < 1 || nl > 3 || ntri < 0 || d < 0 || d > 3 * 128)
    return fail(nullptr, BSP_ERR_ARG, "bad argument");
  Journal jn;
  std::string err;
  if (!jn.open(journal, true, err)) return fail(nullptr, BSP_ERR_IO, err);
  if (jn.find(key, config_hash)) return fail(nullptr, BSP_ERR_ARG, "key already recorded for this configuration");
  if (!jn.append(key, config_hash, np, nl, ntri, d, B, alpha, beta, false, err)) return fail(nullptr, BSP_ERR_IO, err);
  return BSP_OK;
}

bsp_status bsp_journal_lookup(const char* journal, uint64_t key, uint64_t config_hash, int64_t np, int32_t nl,
                              int32_t ntri, int32_t d, double* B, double* alpha, double* beta, int32_t* found) {
  if (!journal || !B || !alpha || !found) return fail(nullptr, BSP_ERR_ARG, "null argument");
  *found = 0;
  Journal jn;
  std::string err;
  if (!jn.open(journal, false, err)) return fail(nullptr, BSP_ERR_IO, err);
  const JournalRecord* r = jn.find(key, config_hash);
  if (!r) return BSP_OK;
  if (r->np != np || r->nl != nl || r->ntri != ntri || r->d != d)
    return fail(nullptr, BSP_ERR_ARG, "record has another particle count or output shape");
  if (beta && !r->has_beta) return BSP_OK;
  if (!jn.read(*r, B, alpha, beta, err)) return fail(nullptr, BSP_ERR_IO, err);
  *found = 1;
  return BSP_OK;
}

bsp_status bsp_batch_covariance(const double* x, int32_t m, int32_t d, double* cov, void* stream) {
  bsp_plan p = nullptr;
  if (!x || !cov || m < 2 || d < 1) return fail(p, BSP_ERR_ARG, "bad argument");
  HIPCHK(launch_covariance(x, m, d, cov, reinterpret_cast<hipStream_t>(stream)));
  return BSP_OK;
}

}  // extern "C"
