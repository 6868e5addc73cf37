/*
 * bsp.h -- C ABI of libbsp, an MI355X (gfx950) implementation of the FFT
 * bispectrum-multipole and modal estimators of
 *   D. Regan, "An Inventory of Bispectrum Estimators for Redshift Space
 *   Distortions", arXiv:1708.05303.
 *
 * Conventions shared by every call
 * --------------------------------
 * Ownership: every array argument is caller-owned. Pointers documented as
 *   "device" must point to device memory of the plan's GPU; "host" pointers to
 *   host memory. The library keeps no reference to any argument after a call
 *   returns, except the workspace given to bsp_set_workspace.
 * Asynchrony: compute calls are enqueued on the plan's stream and return at
 *   once; results are valid after bsp_sync. Host arguments are consumed before
 *   the call returns.
 * Errors: argument errors are returned synchronously; the message is available
 *   from bsp_last_error. Errors found by kernels (particle out of range, count
 *   residual, Cholesky failure) are latched on the device and returned by the
 *   next bsp_sync.
 * Threading: a plan is not thread safe; use one plan per stream.
 * Memory: bsp_plan_create allocates the plan's small constant tables
 *   (twiddles, shell and modal filter tables, reduction schedules; a few MB),
 *   and the first bsp_bispectrum_full or bsp_integrated_bispectrum call adds
 *   its own (the full-multipole schedule, sub-volume twiddles; kept with the
 *   plan); all large scratch comes from the caller's workspace
 *   (bsp_workspace_size). Calls that synchronise say so.
 *
 * Lattice conventions
 * -------------------
 * Wavevector k = k_f n with integer n, k_f = 2 pi / L, V = L^3.
 * Forward DFT X(n) = sum_j x(j) exp(-2 pi i n.j / N); inverse
 * x(j) = sum_n X(n) exp(+2 pi i n.j / N); both unnormalised.
 * Real grids are [N][N][N] float, z fastest. Standard half spectra are
 * [N][N][N/2+1] interleaved complex (re, im).
 * Shell b (b = 0 .. nbins-1) has centre c_b = k0 + b dk in units of k_f and holds
 * the n with (2 c_b - dk)^2 <= 4 |n|^2 < (2 c_b + dk)^2 (the "q in [k +- dk/2]"
 * shells of the standard estimator, Sec. 3.1); 2 k0 and dk must be integers.
 * c = floor(sqrt(n2max)) is the largest |n_a| in any shell; every estimator
 * output is exact on an N' grid when 3 c < N' (closed triangles never wrap).
 *
 * Compact spectra ("delta_l" arguments): the band |n_x|, |n_y| <= c,
 * 0 <= n_z <= c of a half spectrum, stored complex64 as
 * [nl][2c+1][2c+1][cz] with index (n_x + c, n_y + c, n_z) and cz = c + 1 rounded
 * up to a multiple of 16 (entries n_z > c are zero). nl = lmax/2 + 1.
 */
#ifndef BSP_H
#define BSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bsp_plan_s* bsp_plan;

typedef enum {
  BSP_OK = 0,
  BSP_ERR_ARG = 1,       /* null or inconsistent argument */
  BSP_ERR_SIZE = 2,      /* grid size without a transform kernel (supported: 16,32,64,96,128,192,256,384,512,1024) */
  BSP_ERR_ALIAS = 3,     /* 3 c >= N': closed triangles would wrap on the N' grid */
  BSP_ERR_WORKSPACE = 4, /* no workspace, or smaller than bsp_workspace_size */
  BSP_ERR_HIP = 5,       /* HIP runtime error (message in bsp_last_error) */
  BSP_ERR_DEVICE = 6,    /* latched by a kernel: particle outside [0,N) or not finite */
  BSP_ERR_NUMERIC = 7,   /* latched: triangle count residual above its bound (see bsp_precompute), or Cholesky failure */
  BSP_ERR_STATE = 8,     /* call out of order */
  BSP_ERR_IO = 9         /* batch journal could not be opened, read, locked or written */
} bsp_status;

typedef enum {
  BSP_FP32 = 0,   /* FP32 fields, FP32 MFMA products and accumulation */
  BSP_BF16X3 = 1, /* FP32 fields split hi+lo into bf16; ah*bh + ah*bl + al*bh on bf16 MFMA, FP32 accumulate */
  BSP_FP16X3 = 2, /* as BF16X3 with fp16 splits of power-of-two scaled fields */
  BSP_BF16X1 = 3  /* error study only: one bf16 MFMA per tile, ah*bh (no lo parts), FP32 accumulate */
} bsp_precision;

/* Geometry of one estimator run. */
typedef struct {
  int32_t n;           /* assignment / forward-transform grid N */
  int32_t n_reduce;    /* N' of the inverse transforms and triple sums; 0 means N */
  double box;          /* side L of the periodic box, Mpc/h */
  int32_t window;      /* 0 NGP, 1 CIC mass assignment */
  int32_t compensate;  /* 1: divide by the assignment window prod sinc^p(pi n_a / N) */
  int32_t interlace;   /* 1: second grid at u + 1/2, combined with phase exp(i pi (nx+ny+nz)/N) */
  int32_t los;         /* 0: plane parallel along +z; 1: varying, x_hat from the observer */
  double observer[3];  /* observer position in grid units (los = 1) */
  int32_t lmax;        /* 0, 2 or 4 */
  int32_t nbins;       /* number of k shells (<= 64) */
  double k0, dk;       /* first shell centre and width, units of k_f */
} bsp_geom;

/* Separable modal basis (Sec. 3.5): q_p(k) = Legendre P_p(t),
 * t = (2k - kmin - kmax)/(kmax - kmin) on kmin <= k < kmax, the union of the
 * shells; weight 1/sqrt(k P_fid(k)).
 * The modes are orthonormalised through the Gram matrix gamma (eq. betaCalc)
 * by Gram-Schmidt, i.e. a Cholesky factor. drop_tol = 0: in table order, every
 * mode kept (gamma must be positive definite). drop_tol in (0, 1): pivoted, the
 * next mode being the one with the largest residual norm relative to its own
 * after the modes already taken are projected out; modes whose relative
 * residual is below drop_tol are dropped as numerically dependent within the
 * tetrapyd (a separable polynomial basis has near-null directions there, and
 * the coefficients along them amplify any rounding of the numerators). */
typedef struct {
  int32_t P;             /* number of 1-D functions q_p, p < P */
  int32_t nmodes;        /* number of 3-D modes Q_n (<= 128) */
  const int32_t* modes;  /* host [nmodes][3]: (p, r, s), p <= r <= s < P */
  const double* pfid;    /* host [pfid_len]: P_fid at k = k_f sqrt(m), m = |n|^2, (Mpc/h)^3 */
  int32_t pfid_len;      /* must exceed the largest |n|^2 in the modal range */
  double drop_tol;       /* relative residual norm^2 below which a mode is dropped; 0 keeps all */
} bsp_modal_basis;

/* Sizes derived at plan creation. */
typedef struct {
  int32_t c, cz, nl, nlos, ngrid, n2max;
  int32_t ncand;          /* candidate triangles b1 >= b2 >= b3 */
  int32_t ntri;           /* triangles with nonzero count (valid after bsp_precompute) */
  int32_t nfields_binned; /* nl * nbins shell fields D^(l)_b */
  int32_t nfields_modal;  /* nl * P modal fields M^(l)_p */
  int64_t spec_elems;     /* complex elements of one compact cube: (2c+1)^2 cz */
  double count_residual;  /* max |sum I I I / N'^3 - N_tri| over candidates (after bsp_precompute) */
  /* schedule of the main triple reduction (16 x 16 tiles of pair products x
     third fields; after bsp_precompute it covers the nonzero triangles only) */
  int32_t reduce_pairs;   /* pair products F_a F_b */
  int32_t reduce_thirds;  /* third fields */
  int32_t reduce_tiles;   /* needed 16 x 16 tiles */
  int32_t reduce_groups;  /* workgroups per point chunk */
  int32_t reduce_maxr, reduce_maxcw; /* row tiles, column tiles per wave */
  int64_t reduce_needed;  /* (pair, third) entries the estimators use */
  int32_t modal_rank;     /* modes kept by the orthonormalisation (after bsp_precompute) */
  int32_t tune_shape;     /* main reduction register shape chosen by bsp_autotune (-1: the rule) */
  int32_t tune_tiles;     /* short-line transform tiles (0: the rule, 1: 16, 2: 64 columns) */
  int64_t tune_kchunk;    /* main reduction chunk length (0: the rule) */
  int32_t reduce_row_tiles; /* row tiles of 16 pair slots (pairs that meet a needed third) */
  int32_t slab_planes;    /* x planes of N' per slab of the field stacks (N': whole cubes; bsp_set_slab) */
} bsp_info;

/* ---------------------------------------------------------------- plans */

/* Validates the geometry (BSP_ERR_ARG, BSP_ERR_SIZE, BSP_ERR_ALIAS) and builds
 * the constant tables. basis may be NULL (no modal output). stream is a
 * hipStream_t (NULL: default stream). With los = 1 the observer must be finite
 * and must not sit on a node of either grid (node j of the grid at shift s is
 * the point j - s), where x_hat is undefined: BSP_ERR_ARG, before any device
 * work. */
bsp_status bsp_plan_create(bsp_plan* plan, const bsp_geom* geom, const bsp_modal_basis* basis, void* stream);
bsp_status bsp_plan_destroy(bsp_plan plan);
bsp_status bsp_plan_info(bsp_plan plan, bsp_info* info /*host*/);
/* Message of the last error on this plan (plan may be NULL for bsp_plan_create errors). */
const char* bsp_last_error(bsp_plan plan);
/* Bytes of device workspace every call of this plan may use. */
bsp_status bsp_workspace_size(bsp_plan plan, size_t* bytes /*host*/);
/* Workspace: device pointer, 256-byte aligned, at least bsp_workspace_size bytes. */
bsp_status bsp_set_workspace(bsp_plan plan, void* dev, size_t bytes);
/* Field stacks in x-slabs. The triple sum over x is additive, so the
 * estimators (and bsp_precompute) make the filtered real fields of one slab of
 * `planes` x planes at a time, reduce it, and add its sums to T in slab order:
 * the stacks need planes / N' of the whole fields' memory (at 1024^3 the 114
 * FP32 fields of three multipoles, 30 shells and 8 modal functions take 490 GB
 * whole, 61 GB in slabs of 128 planes). The estimators' first inverse pass
 * (along x) runs once per call into a resident buffer in the workspace (each
 * batch of fields on its own band; 103 GB at 1024^3), whose rows the slabs'
 * y passes read; the FP64 precompute repeats its x pass per slab instead.
 * planes must divide N'; 0 restores the plan's default, chosen at
 * bsp_plan_create: N' when the FP32 main stack and the FP64 precompute stack
 * each fit in 64 GiB, else the largest power-of-two fraction of N' for which
 * both do. The results agree with whole cubes to the
 * rounding of the FP64 sums of T (the slabs add in another order). Changes
 * bsp_workspace_size; call it between runs (it waits for the plan's streams
 * and drops a captured batch graph). */
bsp_status bsp_set_slab(bsp_plan plan, int32_t planes);
/* Waits for the plan's stream; returns the first latched device error. */
bsp_status bsp_sync(bsp_plan plan);

/* Geometry-only FP64 precompute on the GPU (once per plan): triangle counts
 * V_B(k1,k2,k3) of the standard estimator as round(sum_x I I I / N'^3) with
 * I_b the inverse DFT of the shell indicator (the residual from an integer must
 * stay below 0.05 + 32 eps log2(N'^3) |count|, eps = 2^-53, the FP64 transforms'
 * rounding, and that bound below 0.5; else BSP_ERR_NUMERIC), and, with a
 * modal basis, the lattice Gram matrix gamma_nm = <<Q_n|Q_m>> of eqs.
 * (betaCalc, innerProduct), its Cholesky factor, and the Poisson shot-noise
 * integrals of the modal numerators. Needs the workspace. Synchronises. */
bsp_status bsp_precompute(bsp_plan plan);
/* Host copies of the precompute results (after bsp_precompute); any pointer
 * may be NULL: tri [ntri][3] (b1 >= b2 >= b3, lexicographic), counts [ntri],
 * gamma [nmodes][nmodes]; kept [nmodes]: the kept modes in the order they were
 * orthonormalised, -1 past the rank; chol [nmodes][nmodes]: the lower Cholesky
 * factor of gamma restricted to the kept modes in that order (rows and
 * columns past the rank zero). */
bsp_status bsp_geometry(bsp_plan plan, int32_t* tri, int64_t* counts, double* gamma, double* chol, int32_t* kept);

/* Autotuning (after bsp_precompute, with the workspace): times, on the plan's
 * own geometry and unit data, (1) the column tiles of the transform passes
 * over lines of at most 128 points (16 or 64 columns per workgroup) on the
 * inverse passes of the whole path, and (2) every register shape of the main
 * triple reduction that holds its schedule, each with three chunk lengths (a
 * quarter, half and all of the accuracy cap: 16384 points FP32, 8192 split
 * precisions), and keeps the fastest for this plan. db_path (may be NULL):
 * a JSON file, one object per plan key (sizes, shells, multipoles, modes,
 * precision); an entry found there is applied without timing unless flags has
 * BSP_TUNE_FORCE; a timed choice is written back (the file is rewritten
 * whole). Synchronises. Outputs are unchanged up to the rounding of the
 * chunked FP32 sums. */
#define BSP_TUNE_FORCE 1
bsp_status bsp_autotune(bsp_plan plan, bsp_precision prec, const char* db_path, int32_t flags);

/* ---------------------------------------------------------------- steps */

/* Mass assignment (the paper is silent on it). ux, uy, uz, w: device [np]
 * positions in grid units in [0, N) (w NULL: unit weights). grids: device
 * [1+interlace][N^3], accumulated into (the caller zeroes them). wsum: device
 * double[1], accumulated sum of weights. Out-of-range or non-finite positions
 * are skipped and latch BSP_ERR_DEVICE.
 * Kernels: when the workspace holds the sorted catalogue (20 bytes per
 * particle plus the tile offsets and 256 bytes) the particles are sorted by
 * node tile and each tile is summed in LDS; else, when it holds
 * (1+interlace) N^3 int64 node sums plus 256 bytes, each contribution is a
 * global 64-bit atomic; without a workspace, a global FP32 atomic.
 * Reproducibility: the first two sum node values and weights as 64-bit
 * integers in units of 2^-S (S = min(36, 62 - e - l), max|w| < 2^e,
 * np < 2^l), each contribution rounded once, so their result does not depend
 * on the order of the atomics: the grids are bit-identical between runs, and
 * for unit weights and positions on multiples of 2^-12 the node sums are exact
 * (each grid value is the exact sum rounded once to FP32). The FP32-atomic
 * fallback sums in an unspecified order. */
bsp_status bsp_grid_assign(bsp_plan plan, const float* ux, const float* uy, const float* uz, const float* w,
                           int64_t np, float* grids, double* wsum);

/* bsp_grid_assign without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the same fixed-point global-atomic assignment, with
 * the same arguments, results and error behaviour, its int64 node sums held in
 * a static device array of the library (256 bytes plus 2^22 int64 nodes,
 * 32 MiB + 256 B, held by each GPU it runs on until the process ends) instead
 * of the workspace; the plan needs no workspace. (1 + interlace) N^3 above
 * 2^22 nodes (for example 128^3 interlaced is the largest interlaced grid)
 * returns BSP_ERR_SIZE before anything is launched. Every call on a GPU shares
 * that GPU's array, which keeps the last call's contents: each call clears
 * the sums it uses with a kernel first, and calls that overlap in time on one
 * GPU (different streams or host threads) race. Calls no hipMalloc or hipFree;
 * the first call on a device looks up the array's address there. */
bsp_status bsp_grid_assign_noalloc(bsp_plan plan, const float* ux, const float* uy, const float* uz, const float* w,
                                   int64_t np, float* grids, double* wsum);

/* Full unnormalised 3-D transforms in the standard layouts (forward e^{-i},
 * inverse e^{+i}), batch of independent grids of size n (any supported size).
 * in/out: device. c2r expects Hermitian input and uses the workspace. */
bsp_status bsp_fft_r2c(bsp_plan plan, int32_t n, int32_t batch, const float* in, void* out_c64);
bsp_status bsp_fft_c2r(bsp_plan plan, int32_t n, int32_t batch, const void* in_c64, float* out);

/* Line-of-sight Legendre moments delta^(l)(n), l = 0, 2, ..., lmax (the LOS
 * moment field defined with the power-spectrum multipoles, Sec. 2, evaluated
 * through x-hat-weighted fields so the line of sight may vary): density
 * contrast rho/rho_bar - 1 of each grid (rho_bar = wsum / N^3), weighting by
 * the real solid harmonics h_m(x_hat) of degree l (polynomials in the
 * components of x_hat; 1 + 5 + 9 fields for lmax = 4) at the nodes, forward
 * transforms, window compensation, interlacing, and the addition theorem
 * delta^(l) = (2l+1) sum_m a_m h_m(k_hat) F_m; delta^(l)(0) = 0.
 * grids: device [1+interlace][N^3] densities from bsp_grid_assign; wsum: device
 * double[1]; delta_l: device compact spectra (see top). Uses the workspace. */
bsp_status bsp_los_moments(bsp_plan plan, const float* grids, const double* wsum, void* delta_l);

/* Same for a caller-made contrast field delta(x) (device [N^3]): no assignment
 * window is divided out and no interlacing is applied. */
bsp_status bsp_grid_entry(bsp_plan plan, const float* delta, void* delta_l);

/* Filtered fields on the N' grid: for each filter f, the unnormalised inverse
 * DFT of (weight * delta^(l)) where filt[f] = {l_index, kind, index}:
 *   kind 0: shell indicator of bin `index` -> D^(l)_k(x) of eq. (Standard_ell_Estim);
 *   kind 1: modal weight q_index(k)/sqrt(k P_fid) -> N^3 M^(l)_n(x) of eq. (betaEst).
 * filt: host [nfilt][3]; fields: device [nfilt][N'^3] float. Uses the workspace;
 * synchronises once (after copying the filter list to the device). */
bsp_status bsp_filter_fields(bsp_plan plan, const void* delta_l, int32_t nfilt, const int32_t* filt, float* fields);

/* Triple reduction T[p][s] = sum_x F_{a_p}(x) F_{b_p}(x) F_{t_s}(x) over K points,
 * the sum over products of three transformed fields of the standard and modal
 * estimators. fields: device [nfields][K] float (nfields <= 128); pairs: host
 * [npairs][2]; thirds: host [nthirds] (<= 128); need: host [npairs][nthirds]
 * uint8 or NULL (all). The reduction works on tiles of 16 pairs x 16 thirds:
 * every entry of a tile holding a needed entry is computed, entries of other
 * tiles are 0. T: device double [npairs][nthirds]. Chunks of K are
 * accumulated in FP32 and combined in FP64. Uses the workspace. */
bsp_status bsp_triple_reduce(bsp_plan plan, const float* fields, int32_t nfields, int64_t K, const int32_t* pairs,
                             int32_t npairs, const int32_t* thirds, int32_t nthirds, const uint8_t* need,
                             bsp_precision prec, double* T);

/* Modal coefficients beta^l_n = sum_m gamma^-1_nm b^l_m (eqs. betaCalc, betaEst and
 * the multipole modal coefficients with the even compositions of eqs.
 * (Bisp_ell, Bisp_ell2)): b^0 = <M0 M0 M0>, b^2 the three (2,0,0) placements,
 * b^4 the three (4,0,0) and three (0,2,2) placements, <XYZ> = N'^-3 sum_x.
 * nbar > 0 subtracts the Poisson shot noise of b^0. With S the kept modes
 * in the order orthonormalised (see bsp_modal_basis) and L the Cholesky factor
 * of gamma_SS: alpha = L^-1 b_S, the coefficients on the orthonormal modes
 * L^-1 Q_S (entries past the rank are 0); beta_S = L^-T alpha and beta = 0 on
 * dropped modes (beta = gamma^-1 b when every mode is kept). bnum, alpha,
 * beta: device double [nl][nmodes]. Requires bsp_precompute and a modal basis. */
bsp_status bsp_modal_coeffs(bsp_plan plan, const void* delta_l, bsp_precision prec, double nbar, double* bnum,
                            double* alpha, double* beta);

/* The whole hot path for one catalogue: assignment (the sorted, tiled kernels
 * when the grid has at least 512 tiles of 8 x 8 x tz nodes, that is 128 nodes a
 * side and up; the fixed-point global-atomic kernel below), LOS moments, shell
 * and modal fields, one triple reduction, FP64 normalisation. B, bnum, alpha
 * and beta are bit-identical between runs on the same inputs (fixed-point
 * assignment, reduction partials combined in a fixed order); the shell power
 * (Pbar, and through it B0sub) adds FP64 partial sums in an unspecified order,
 * which can change its last bits.
 *   B: device double [nl][ntri], B^l = V^2 T^l / (N^9 N'^3 N_tri) (multipole on b1);
 *   B0sub: device double [ntri] or NULL, B^0 - sum_i Pbar_bi / nbar + 2/nbar^2;
 *   Pbar: device double [nbins] or NULL, shell power V sum |delta0|^2 / (N^6 N_b);
 *   bnum, alpha, beta: device double [nl][nmodes] or NULL (need a modal basis).
 * nbar = wsum / V is used for the shot noise; the catalogue is as in
 * bsp_grid_assign. Requires bsp_precompute. */
bsp_status bsp_bispectrum_multipoles(bsp_plan plan, const float* ux, const float* uy, const float* uz,
                                     const float* w, int64_t np, bsp_precision prec, double* B, double* B0sub,
                                     double* Pbar, double* bnum, double* alpha, double* beta);

/* The same from a caller-made contrast field delta(x) (device [N^3]); no shot
 * noise subtraction (B0sub, nbar unused). */
bsp_status bsp_bispectrum_field(bsp_plan plan, const float* delta, bsp_precision prec, double* B, double* Pbar,
                                double* bnum, double* alpha, double* beta);

/* ---------------------------------------------------------------- tracing */

/* Power-spectrum multipoles (Sec. 2, eq. PowSpecMultipole): the shell average
 * over directions of delta^(l)(k) delta^(0)(-k) / V, on the lattice
 *   P[l][b] = V sum_{n in shell b} Re[delta^(l)(n) conj(delta^(0)(n))] / (N^6 N_b)
 * over the full lattice (N_b modes in shell b; the n_z > 0 half of the compact
 * spectrum stands for the pairs n, -n). delta_l: device, the compact spectrum
 * [nl][spec] that bsp_los_moments writes. P: device double [nl][nbins]. Raw: no
 * shot-noise term (the paper gives none; P[0] equals the Pbar output of
 * bsp_bispectrum_multipoles). Uses nl * nbins doubles of the workspace. */
bsp_status bsp_power_multipoles(bsp_plan plan, const void* delta_l, double* P);

/* Poisson shot noise of the multipoles B_l of bsp_bispectrum_multipoles (the
 * paper gives no shot-noise model; this one is derived from the estimator of
 * Sec. 3.1, eq. Standard_ell_Estim, with the Legendre weight on the first
 * leg). For Poisson points the particle triple sum holds, beside the distinct
 * triples, the triples with two or three particles alike; shell-averaged they
 * give, for triangle i = (b1, b2, b3),
 *   SN[0][i] = (P[0][b1] + P[0][b2] + P[0][b3]) / nbar - 2 / nbar^2,
 *   SN[l][i] = (P[l][b1] + W_l(b1,b2|b3) P[l][b2] + W_l(b1,b3|b2) P[l][b3]) / nbar,
 * with W_l(b1,b2|b3) the mean of L_l(k1_hat . k2_hat) over the closed triangles
 * of the bin (continuum triangle density k1 k2 k3; computed once per plan by
 * bsp_precompute) and the triple-coincidence term of l > 0 dropped (zero for
 * l = 2 over the cubic-symmetric triangle set, a lattice-anisotropy term for
 * l = 4). Against the exact coincidence terms of unit particles on the nodes
 * the model holds to about 0.4%, 0.7% and 13% for l = 0, 2, 4 at k = 14-26
 * k_f; SN[0] equals B_l[0] - B0sub of bsp_bispectrum_multipoles.
 * P: device double [nl][nbins], the raw shell power multipoles
 * (bsp_power_multipoles; P[0] = Pbar). nbar > 0: number density in (length
 * unit)^-3. SN: device double [nl][ntri], triangles in the order of
 * bsp_geometry. BSP_ERR_STATE before bsp_precompute. Asynchronous on the
 * plan's stream; no workspace. */
bsp_status bsp_shot_noise_multipoles(bsp_plan plan, const double* P, double nbar, double* SN);

/* Skew-spectrum multipoles (Sec. 3.2, the estimator after eq. skewspecQ with
 * the convolution as quadratic form): the shell average over directions of
 * [delta^(0) * delta^(0)](-k) delta^(l)(k) / V. The monopole kept on the union
 * of the shells is transformed to real space at N' (unnormalised, as the
 * bispectrum fields), squared, and transformed back to the compact cube
 * (no wrap-around while 3 c < N'):
 *   S[l][b] = V sum_{n in shell b} Re[delta^(l)(n) conj(Q(n))] / (N^9 N'^3 N_b),
 *   Q = DFT_N'[d^2], d = IDFT_N'[delta^(0) on the shells].
 * The 1/V (absent from the printed estimator, present in its defining relation
 * and in the power-spectrum estimator) and the band are readings; with them
 * S[l][b] N_b = V / (N^9 N'^3) sum over all (b2, b3) of the triple sums
 * sum_x D^l_b D^0_b2 D^0_b3. delta_l: device, the compact spectrum [nl][spec]
 * of bsp_los_moments. S: device double [nl][nbins]. Uses the workspace.
 * flags: 0, or BSP_SKEW_BALL: d keeps delta^(0) on every mode
 * 0 < |n|^2 <= n2max (the modes below the first shell too), the widest range
 * that stays free of wrap-around, closer to squaring the whole density field
 * (the sum rule above then does not hold). Other bits: BSP_ERR_ARG. */
#define BSP_SKEW_BALL 1
bsp_status bsp_skew_spectra(bsp_plan plan, const void* delta_l, double* S, int32_t flags);

/* Integrated bispectrum multipoles (Sec. 3.4, eq. integBisp and the RSD
 * estimator after it): the N^3 grid is cut into s^3 cubic sub-volumes of side
 * M = N / s (M a supported transform size); for each, dbar_i = its mean
 * overdensity and P^(l)_i(k) = its power-spectrum multipoles with a single
 * line of sight e_i, the unit vector from the observer to the sub-volume
 * centre (z for plane-parallel plans; a reading: inside a small sub-volume the
 * plane-parallel form applies):
 *   P[i][l][b] = V_s sum_{n in b} (2l+1) L_l(nhat . e_i) |F_i(n) / W(n)|^2 / (M^6 N_b),
 * F_i the unnormalised DFT of the sub-volume's contrast, W the plan's
 * assignment window at the sub-volume frequencies (when the plan compensates),
 * V_s = V / s^3, and iB[l][b] = (1/s^3) sum_i P[i][l][b] dbar[i]. Shells
 * (2 c_b - dk)^2 <= 4 |n|^2 < (2 c_b + dk)^2, c_b = k0 + b dk, in units of the
 * sub-volume fundamental 2 pi s / L (2 k0 and dk integers; every shell below
 * |n| = M / 2). grid: device [N^3], the plan's first grid (interlacing is not
 * used); wsum: device double[1]: the grid is a density rho and
 * delta = rho N^3 / wsum - 1, or NULL: the grid is already a contrast.
 * iB: device double [nl][nbins]; Psub: device double [s^3][nl][nbins] or NULL;
 * dbar: device double [s^3] or NULL. Sub-volume i has origin
 * M (i / s^2, (i / s) mod s, i mod s). Uses the workspace (about 3 N^3 floats);
 * synchronises.
 * flags: 0, or BSP_IB_LOCAL_LOS: the line of sight varies over the nodes of
 * each sub-volume as in eq. (PowSpecMultipole) (x_hat from the observer to the
 * node; the grid's first node set, no shift):
 *   P[i][l][b] = V_s sum_{n in b} Re[delta^(l)_i(n) conj delta^(0)_i(n)] / (M^6 N_b),
 *   delta^(l)_i(n) = (2l+1) sum_x e^{-2 pi i n.x / M} delta(x) L_l(nhat . xhat) / W(n)
 * over the sub-volume's nodes, computed per real solid harmonic of x_hat
 * (1, 6 or 15 batched transforms of all sub-volumes, one after another) by
 * the addition theorem; about one more N^3 floats of workspace. For
 * plane-parallel plans both readings are the same and the flag is ignored.
 * Any other flag bit: BSP_ERR_ARG; so is an observer at the centre of a
 * sub-volume with the one-LOS reading (its direction is undefined). */
#define BSP_IB_LOCAL_LOS 1
bsp_status bsp_integrated_bispectrum(bsp_plan plan, const float* grid, const double* wsum, int32_t s, double k0,
                                     double dk, int32_t nbins, double* iB, double* Psub, double* dbar,
                                     int32_t flags);

/* Full bispectrum multipoles B^(l1 l2 l3) (Sec. 3, the general Legendre
 * decomposition with one multipole per side) in the FFT form of eq.
 * (Standard_ell_Estim): each side's field D^(l_i)_{b_i} comes from its own LOS
 * moment delta^(l_i), T = sum_x D^l1_b1 D^l2_b2 D^l3_b3 and
 * B = V^2 T / (N^9 N'^3 N_tri) over the plan's triangles b1 >= b2 >= b3 (so
 * B^(l00) is the B^l of bsp_bispectrum_multipoles). delta_l: device compact
 * spectrum [nl][spec] of bsp_los_moments; B: device double [nl^3][ntri] with
 * combination (l1 nl + l2) nl + l3 (l = 0, 2, ...). After bsp_precompute; the
 * first call builds the schedule; the reduction's chunks are lengthened until
 * its partial sums fit the workspace. Uses the workspace. */
bsp_status bsp_bispectrum_full(bsp_plan plan, const void* delta_l, bsp_precision prec, double* B);

/* Stage timers: while enabled, each compute call records a pair of HIP events
 * on the plan's stream around the launches of every stage:
 *   0 assignment, 1 forward z pass (r2c + LOS weights), 2 forward y pass,
 *   3 forward x pass, 4 LOS combination, 5 inverse x pass (shell/modal filter),
 *   6 inverse y pass, 7 inverse z pass (c2r), 8 triple reduction,
 *   9 FP64 combination of the reduction partials, 10 power-spectrum multipoles,
 *   11 skew spectra (the whole call; its transforms also count in stages 5-7),
 *   12 integrated bispectrum (the whole call).
 * bsp_set_timing(plan, 1) resets and starts, 0 stops (it synchronises).
 * bsp_stage_times synchronises and returns, per stage, the summed event
 * milliseconds since the reset (ms: host double[16]), the number of timed
 * launches (launches: host int64[16], may be NULL) and the summed algorithmic
 * amount of the timed launches (amount: host double[16], may be NULL): bytes
 * each pass must read and write once on the band it keeps (stages 0-7, 10-12), or
 * flops of the needed triple products (stage 8: two per needed entry per
 * point plus one per pair per point). */
bsp_status bsp_set_timing(bsp_plan plan, int32_t enable);
bsp_status bsp_stage_times(bsp_plan plan, double* ms, int64_t* launches, double* amount);

/* A batch of mocks for covariance estimates (Sec. 3.5, closing remark: the
 * modal coefficients of many realisations give the covariance of the
 * estimator). Mock m runs the whole path of bsp_bispectrum_multipoles on
 * plans[mock_plan[m]]: plans of different assignment grids N share one
 * reduction geometry (N', shells, modal basis), so every mock yields outputs
 * of the same shape, and keep the same modes in their orthonormalisation.
 * Outputs: B_all device [nmocks][nl][ntri]; alpha_all device [nmocks][nl*nmodes]
 * (shot-noise-subtracted alpha^l on the orthonormalised kept modes, l-major, as
 * in bsp_bispectrum_multipoles); beta_all likewise or NULL; cov device [D][D],
 * D = nl*nmodes, the FP64 sample covariance of the alpha_all rows (rows and
 * columns past each l's rank are 0). mock_plan, np: host [nmocks];
 * ux, uy, uz, w (w nullable, entries nullable): host arrays [nmocks] of device
 * pointers to the catalogues. Every plan needs bsp_precompute, a modal basis
 * and its own workspace (plans sharing a workspace must share a stream).
 * flags: BSP_BATCH_GRAPH replays, for each plan, its whole path captured once
 * in a HIP graph (kernels only) over input and output slots the library
 * allocates for the plan's largest catalogue and keeps with the plan (3 or 4
 * floats per particle and the outputs of one mock); each mock is then its
 * catalogue copied into the slot, its count written on the device, one graph
 * launch and the outputs copied out, on a stream of the plan's own. The
 * graph is kept and captured again only when the precision, the presence of
 * weights or a larger catalogue require it. 0: the mocks call
 * bsp_bispectrum_multipoles one after another on their plans' streams.
 * Either way the outputs are bit-identical. The call synchronises every
 * plan (and its batch stream) before enqueueing the covariance on plans[0]'s
 * stream (valid after bsp_sync(plans[0])). Errors: BSP_ERR_ARG if the plans' output shapes or
 * kept modes differ, nmocks < 2 or an index is out of range; the first failing mock's
 * status otherwise (its message via bsp_last_error(plans[0])). */
#define BSP_BATCH_GRAPH 1
bsp_status bsp_batch_run(const bsp_plan* plans, int32_t nplans, const int32_t* mock_plan, int32_t nmocks,
                         const float* const* ux, const float* const* uy, const float* const* uz,
                         const float* const* w, const int64_t* np, bsp_precision prec, double* B_all,
                         double* alpha_all, double* beta_all, double* cov, int32_t flags);

/* Checkpoint and resume of a batch (the covariance runs of Sec. 3.5 are
 * hundreds of independent mocks; a stopped batch should not redo the finished
 * ones). As bsp_batch_run, with a journal file of one record per finished
 * mock: the caller's key of the mock (mock_key host [nmocks], e.g. the seed
 * of its catalogue), the configuration hash of its plan (bsp_config_hash),
 * its particle count and its B, alpha and (when beta_all is given) beta,
 * closed by a 64-bit FNV-1a checksum. A mock whose (key, hash) is recorded
 * with the same particle count is not run: its outputs are copied from the
 * record into B_all, alpha_all and beta_all (a record without beta serves
 * only calls without beta_all; otherwise the mock runs again and its new
 * record, appended later, supersedes the old one: the last record of a key
 * and configuration wins). Every other mock runs and is
 * appended to the journal as soon as its outputs are on the host (the host
 * writes mock k while mock k+1 runs, through pinned host staging that the call
 * allocates for two mocks' outputs plus those of the recorded mocks and frees
 * before it returns), unless a kernel error is latched on its plan, which
 * ends the call with that error. A process killed at any point
 * leaves a journal whose valid prefix holds whole records only: a torn last
 * record fails its length or checksum test and is cut off by the next call.
 * The file is created if absent and locked exclusively (flock) for the call.
 * Outputs are bit-identical to one uninterrupted bsp_batch_run: the records
 * hold the FP64 outputs exactly, and the covariance is computed over all
 * mocks at the end. nresumed (host, nullable): mocks taken from the journal.
 * flags: BSP_BATCH_GRAPH as bsp_batch_run; BSP_BATCH_FSYNC also makes each
 * record durable (fdatasync) before the next is written. Errors: those of
 * bsp_batch_run; BSP_ERR_ARG if mock_key is NULL, two mocks share a key on the
 * same configuration, or a record of the same key and configuration has
 * another particle count; BSP_ERR_IO if the journal cannot be opened, is not
 * a journal, is locked by another process, or cannot be read or written. */
#define BSP_BATCH_FSYNC 2
bsp_status bsp_batch_run_journal(const bsp_plan* plans, int32_t nplans, const int32_t* mock_plan, int32_t nmocks,
                                 const uint64_t* mock_key, const float* const* ux, const float* const* uy,
                                 const float* const* uz, const float* const* w, const int64_t* np,
                                 bsp_precision prec, double* B_all, double* alpha_all, double* beta_all,
                                 double* cov, int32_t flags, const char* journal, int32_t* nresumed);

/* Configuration hash under which the journal records a mock of this plan at
 * precision prec: a 64-bit FNV-1a hash of the geometry, the modal basis
 * (functions, modes, P_fid, drop tolerance), the kept modes, the triangles,
 * the precision, the slab planes when they are not all of N' (bsp_set_slab)
 * and the journal format. Host output. Needs bsp_precompute
 * (BSP_ERR_STATE). Plans of different N hash differently. */
bsp_status bsp_config_hash(bsp_plan plan, bsp_precision prec, uint64_t* hash /*host*/);

/* Host-only journal access (no GPU call; errors via bsp_last_error(NULL)).
 * scan: opens read-only and counts the whole, checksummed records of the valid
 * prefix (valid_bytes) of a file of file_bytes (a torn tail is the
 * difference); the file is not changed. append: appends one record (host
 * arrays B [nl][ntri], alpha [d], beta [d] or NULL), cutting a torn tail off
 * first; BSP_ERR_ARG if the key is already recorded for config_hash. lookup:
 * found = 1 and the record copied to B, alpha, beta (beta nullable) if a
 * record of (key, config_hash) with these sizes exists and holds beta when
 * asked for; found = 0 otherwise; BSP_ERR_ARG if it exists with other sizes.
 * All three return BSP_ERR_IO for a file that cannot be opened or locked or
 * is not a journal of this format. */
bsp_status bsp_journal_scan(const char* journal, int64_t* nrecords /*host*/, int64_t* valid_bytes /*host*/,
                            int64_t* file_bytes /*host*/);
bsp_status bsp_journal_append(const char* journal, uint64_t key, uint64_t config_hash, int64_t np, int32_t nl,
                              int32_t ntri, int32_t d, const double* B, const double* alpha, const double* beta);
bsp_status bsp_journal_lookup(const char* journal, uint64_t key, uint64_t config_hash, int64_t np, int32_t nl,
                              int32_t ntri, int32_t d, double* B, double* alpha, double* beta, int32_t* found);

/* Sample covariance of a batch of coefficient vectors (FP64):
 * cov = (1/(M-1)) sum_m (x_m - mean)(x_m - mean)^T. x: device [m][d], cov:
 * device [d][d]. stream: hipStream_t or NULL. */
bsp_status bsp_batch_covariance(const double* x, int32_t m, int32_t d, double* cov, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* BSP_H */
