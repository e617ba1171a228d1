/*
 * aidg.h -- C ABI of the MI355X (gfx950) A-term image-domain gridding library.
 *
 * The library implements the hot path of image-domain gridding (IDG) with
 * direction-, time- and baseline-dependent 2x2 Jones A-terms (Hodgson 2025,
 * "That pesky A-term", arXiv:2502.17789, Sec. 2 and Sec. 3):
 *
 *   gridding   (Sec. 2.5, imaging steps 1-2):  for every subgrid p
 *       S(x,y)  = sum_k V_k exp(+2 pi i phi_k(x,y))            (Sec. 2.4, Eq. withw)
 *       S'(x,y) = T(x,y) A_p(x,y)^H S(x,y) A_q(x,y)            (Sec. 3.3, deferred A-term)
 *       G_w[window of p] += centred forward DFT of S'          (Sec. 2.3, Eq. shiftback)
 *   degridding (Sec. 2.5, prediction step 3), the exact adjoint:
 *       S  = centred inverse DFT of G_w[window of p]           (splitter + inverse FFT)
 *       S' = T A_p S A_q^H
 *       V_k = sum_{x,y} S'(x,y) exp(-2 pi i phi_k(x,y))        (Eq. degridder)
 *   phi_k(x,y) = (u_k - u0) l_x + (v_k - v0) m_y + (w_k - w0) (n - 1)   [turns]
 *
 * Geometry and conventions:
 *   grid cell (gu, gv), 0 <= gu, gv < N, sits at u = (gu - N/2) du, du = 1/(N dl).
 *   subgrid centre (U0, V0) is an integer cell; its window covers cells
 *   U0 - L/2 .. U0 + L/2 - 1 (same for v) and must lie on the grid.
 *   subgrid image pixel (x, y) sits at l = (x - L/2) N dl / L.
 *   Visibility k = (baseline b = (p, q), timestep t, channel c):
 *   u_k = uvw_m[b][t][0] f_c / c (metres to wavelengths), likewise v, w.
 *   Polarisations are the 2x2 row-major Jones layout [[XX, XY], [YX, YY]];
 *   V_pq = A_p B A_q^H.  Gridding applies A^H (the adjoint of degridding); for
 *   unitary A (phase screens) this equals the paper's A^-1 of Eq. withw, which
 *   the geometry's aterm_mode = 1 selects for any A (normalised, Sec. 3.3).
 *   The taper is the separable Kaiser-Bessel window of Sec. 4.2,
 *   T(x,y) = t(x) t(y), t(x) = I0(beta sqrt(1 - (2 (x - L/2)/L)^2)) / I0(beta).
 *   Subgrid DFTs are unnormalised; all image-domain scaling is left to the caller.
 *
 * Array layouts (all C order; "c64" = interleaved float re/im, "c128" = double):
 *   baselines  host   int32  [nbl][2]                  stations (p, q) of each baseline
 *   uvw_m      host   double [nbl][nt][3]              metres
 *   freqs_hz   host   double [nc]                      strictly increasing
 *   aterms     device c64|c128 [n_int][n_st][L][L][4]  n_int = ceil(nt / aterm_interval),
 *                                                      pixel [y][x], Jones row-major
 *   vis        device c64|c128 [nbl][nt][nc][4]
 *   grid       device c64|c128 [W][P][N][N]            W w-layers, u (gu) fastest; P = 4
 *                                                      planes (XX, XY, YX, YY), 1 with stokes_i
 * c64 with precision AIDG_FP32, c128 with AIDG_FP64.
 *
 * Ownership: host arrays are read during the call that receives them and may be
 * freed afterwards.  Device buffers passed to aidg_grid / aidg_degrid belong to
 * the caller and must stay alive until the work queued on the given HIP stream
 * has completed.  A plan owns its own device copies of the A-terms and its
 * metadata, taper and workspace; aidg_plan_destroy frees them.
 *
 * Errors: every call returns an aidg_status; nothing throws across the ABI.
 * aidg_last_error() returns a thread-local message describing the last non-OK
 * status.  aidg_grid / aidg_degrid never allocate memory and never synchronise
 * the host; they queue kernels on the given stream.  A plan must not be used by
 * two host threads at once (AIDG_E_BUSY).
 */
#ifndef AIDG_H
#define AIDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AIDG_ABI_VERSION 8

typedef enum {
  AIDG_OK = 0,
  AIDG_E_INVALID = 1,     /* bad argument or geometry */
  AIDG_E_NOMEM = 2,       /* host or device allocation failed */
  AIDG_E_DEVICE = 3,      /* a HIP call failed */
  AIDG_E_UNSUPPORTED = 4, /* valid request the GPU path does not implement (e.g. L) */
  AIDG_E_RANGE = 5,       /* strict_range set and a visibility cannot be placed */
  AIDG_E_BUSY = 6         /* plan already in use by another thread */
} aidg_status;

enum { AIDG_FP32 = 0, AIDG_FP64 = 1 };

/* Imaging geometry and numerics of a plan.  80 bytes. */
typedef struct {
  int32_t grid_size;       /* N: even, >= subgrid_size */
  int32_t subgrid_size;    /* L: 32, 64 or 96 */
  int32_t kernel_support;  /* K: even, 0 <= K < L; cells reserved for taper/w/A spread, both sides */
  int32_t aterm_interval;  /* timesteps per A-term interval (Sec. 3.3), >= 1 */
  double pixel_scale;      /* dl: image pixel size in direction cosines; FOV = N dl, FOV/sqrt(2) < 1 */
  double w_step;           /* w-layer spacing in wavelengths (Sec. 2.4): > 0 explicit,
                              0 automatic (2 w_max with w_max = K / (4 FOV rho),
                              rho = max |grad n| over the lattice; one layer when K = 0),
                              < 0 a single layer at w0 = 0 */
  double taper_beta;       /* Kaiser-Bessel beta; 0 selects pi K / 4 */
  int32_t precision;       /* AIDG_FP32 (FP32 phasors/accumulation, FP64 phase origins) or AIDG_FP64 */
  int32_t reseed_channels; /* R: each row's channels form runs of at most R (rounded down to
                              even; R = 1: every channel alone) whose phasors are seeded
                              from FP64 at the run's centre and stepped outward in FP32;
                              0 = 32 */
  int32_t strict_range;    /* 0: unplaceable visibilities are excluded (grid ignores them,
                              degrid writes 0); 1: plan creation fails with AIDG_E_RANGE */
  int32_t max_subgrid_vis; /* cap on visibilities per subgrid, 0 = 1024, at most 2048
                              (they are staged in LDS: AIDG_E_INVALID above); larger caller
                              sub-tables are split in time */
  int32_t center_lattice;  /* the library's partitioner puts subgrid centres on cells
                              N/2 + k * center_lattice (Sec. 2.2: a centre snaps to a grid
                              cell); 0 = automatic (largest power of two <= 2(L-K)/3), 1 = any cell.
                              Subgrids with the same centre and w-layer share one subgrid FFT
                              and one add to the grid (and one split + inverse FFT) */
  int32_t w_fold;          /* 1: fold rows with w < 0 to (-u, -v, -w) by the Hermitian
                              symmetry V(-u,-v,-w) = V(u,v,w)^H (Sec. 2.4 footnote): their
                              visibilities are gridded conjugate-transposed with the two
                              stations' A-terms swapped, and degridding returns the
                              conjugate transpose of what it predicts there.  All layers
                              are then at w >= 0, at odd multiples of w_step / 2
                              (w0 = (j + 1/2) w_step, the paper's {w_max, 3 w_max, ...}).
                              Degridding of a fold-mode plan is exact for Hermitian
                              brightness (any physical sky); the image of a fold-mode grid
                              has the right Hermitian part.  0: no fold (default) */
  int32_t aterm_mode;      /* A-term of gridding (Sec. 3.3, A-term application).
                              0 (default): A_p^H S A_q, the exact adjoint of degridding.
                              1 (inverse): the paper's A^-1 of Eq. withw, normalised:
                              S' = T f A_p^-1 S A_q^-H with f = 1 / ||A_p^-1 A_q^-H||_F
                              per pixel (f = 0 where an A-term is singular), and
                              aidg_invert divides the image by the bilinear interpolation
                              (periodic over the field) of the weighted-average map
                              M(x, y) = sum_s nvis_s f_s(x, y) / sum_s nvis_s over the
                              plan's subgrids (0 where M interpolates to 0).  Degridding
                              and aidg_predict are the same in both modes, so in mode 1
                              gridding is not the adjoint of degridding */
  int32_t stokes_i;        /* 1: Stokes-I grids, one complex value per cell (Sec. 5.5: the
                              master grid of Stokes-I imaging holds one complex value per
                              pixel, that of IQUV imaging four).  Gridding
                              adds I = (S'_XX + S'_YY) / 2 of each A-term-corrected subgrid
                              image; degridding reads I and predicts the visibilities of the
                              unpolarised brightness B = I [[1, 0], [0, 1]].  Grids are
                              [W][1][N][N] and images [1][N][N].  Gridding is then the
                              adjoint of degridding up to a factor 2:
                              <grid(V), G> = <V, degrid(G)> / 2.  0: four planes (default) */
  int32_t degrid_form;     /* degridder design per subgrid (Sec. 3.2, Degridder: a kernel
                              design chosen by subgrid occupancy); the forms agree to
                              rounding.  AIDG_DEGRID_AUTO (0): per subgrid, the form of
                              least modelled cost (the direct form for rows of a few
                              channels, the recurrence for longer ones).
                              AIDG_DEGRID_RECURRENCE (1): lanes own subgrid pixels, the
                              phasors step outward from the centre of each run of
                              reseed_channels (FP64-seeded there) and each pair of
                              visibilities is a cross-lane reduction; sub-tables without a
                              common channel spacing take the direct form.
                              AIDG_DEGRID_PER_VIS (2): lanes own visibilities, every
                              (visibility, pixel) phase is formed in FP64, for sub-tables
                              of at most 256 visibilities, the recurrence for larger ones
                              (the paper's "natural" thread-per-visibility design).
                              AIDG_DEGRID_DIRECT (3): lanes own subgrid pixels and every
                              visibility's phasor is seeded from FP64 (no recurrence) */
  int32_t reserved;        /* 0 */
  int64_t workspace_bytes; /* device budget for the group images of one batch
                              (4 L^2 complex each); 0 = 2 GiB */
} aidg_geometry;
enum { AIDG_DEGRID_AUTO = 0, AIDG_DEGRID_RECURRENCE = 1, AIDG_DEGRID_PER_VIS = 2, AIDG_DEGRID_DIRECT = 3 };

/* One subgrid: the rectangular sub-table [t0, t0+nt) x [c0, c0+nc) of one
 * baseline's visibility table (Sec. 3.1), its integer centre cell, its w-layer
 * and its A-term interval.  64 bytes. */
typedef struct {
  int32_t bl, st1, st2;   /* baseline index and its stations (p, q) */
  int32_t t0, nt, c0, nc; /* sub-table */
  int32_t U0, V0;         /* centre cell */
  int32_t wlayer;         /* index into the plan's w-layers, 0 .. W-1 */
  int32_t aint;           /* A-term interval = t0 / aterm_interval */
  int32_t folded;         /* 1: the sub-table's rows are folded to -uvw (w_fold plans
                             only); its U0, V0, w0 refer to the folded coordinates */
  double w0;              /* w of the layer, wavelengths */
  int64_t vis_offset;     /* flat index of visibility (bl, t0, c0) */
} aidg_subgrid;

typedef struct {
  int64_t n_subgrids;      /* after splitting at max_subgrid_vis */
  int64_t n_vis;           /* nbl * nt * nc */
  int64_t n_excluded;      /* visibilities in no subgrid */
  int32_t n_wlayers;       /* W */
  int32_t subgrid_size;    /* L */
  double w_step;           /* layer spacing used (0 for a single layer) */
  int64_t device_bytes;    /* everything the plan holds on the device */
  int64_t workspace_bytes; /* group image stack of one batch */
  int64_t grid_bytes;      /* size of one grid for this plan, W * 4 * N * N * complex */
  int64_t vis_bytes;       /* size of one visibility array */
  int64_t n_batches;       /* kernel batches per aidg_grid / aidg_degrid call: runs of
                              whole groups, as many as the workspace holds images */
  int64_t max_subgrid_vis; /* largest sub-table */
  int64_t n_groups;        /* runs of subgrids with one w-layer and centre that share one
                              subgrid FFT; a centre holding more than 8x the mean
                              visibilities per centre is split into several */
  int64_t n_subgrids_pervis; /* subgrids the degridder takes in its per-visibility form
                              (geometry degrid_form) */
  int64_t n_subgrids_direct; /* subgrids the degridder takes in its direct form */
} aidg_plan_info;

typedef struct aidg_plan aidg_plan;

/* Partition only (host, no device use): the library's sub-table partitioner of
 * Sec. 3.1.  Each baseline's rows of one A-term interval are split at their first
 * timestep into channel runs whose uv span comfortably fits (3/4 of L - K), and
 * each run is then extended in time while every visibility stays within
 * (L - K)/2 cells of a centre cell (on the centre lattice where one fits), in one
 * w-layer, and under max_subgrid_vis.
 * Writes up to cap records to out (may be NULL with cap 0), the count to *n_out
 * and the layer spacing used to *w_step_out.  AIDG_E_INVALID if cap is too small
 * (*n_out still receives the count). */
aidg_status aidg_partition(const aidg_geometry* geo, int32_t n_stations, int32_t n_baselines,
                           int32_t n_times, int32_t n_chans, const int32_t* baselines,
                           const double* uvw_m, const double* freqs_hz, aidg_subgrid* out,
                           int64_t cap, int64_t* n_out, double* w_step_out);

/* Build a plan: validate the geometry, partition (or take the caller's table),
 * upload metadata, taper and a copy of the A-terms on hip_stream, and allocate
 * the workspace.  table/n_table: optional caller partition (NULL/0 to use the
 * library's own); it must cover each visibility at most once and keep every
 * window on the grid, and its wlayer indices must map to one w0 each.  The
 * call synchronises hip_stream before returning. */
aidg_status aidg_plan_create(const aidg_geometry* geo, int32_t n_stations, int32_t n_baselines,
                             int32_t n_times, int32_t n_chans, const int32_t* baselines,
                             const double* uvw_m, const double* freqs_hz, const void* aterms,
                             const aidg_subgrid* table, int64_t n_table, void* hip_stream,
                             aidg_plan** out);

aidg_status aidg_plan_info_get(const aidg_plan* plan, aidg_plan_info* info);

/* Copy the plan's subgrid table (after splitting) to host memory; cap records at most. */
aidg_status aidg_plan_subgrids(const aidg_plan* plan, aidg_subgrid* out, int64_t cap);

/* Copy the w of each layer (cap entries at most) to host memory. */
aidg_status aidg_plan_wlayers(const aidg_plan* plan, double* w0, int32_t cap);

/* Replace the plan's A-terms (device buffer, same layout and precision).  In the
 * inverse A-term mode this also recomputes the inverse planes and the normalisation
 * map on hip_stream. */
aidg_status aidg_plan_set_aterms(aidg_plan* plan, const void* aterms, void* hip_stream);

/* Inverse A-term mode: copy the weighted-average normalisation map M [L][L] (y major,
 * FP64, see aterm_mode) to host memory; cap entries at most.  Waits for the plan's
 * queued work.  AIDG_E_INVALID for a plan in the adjoint mode. */
aidg_status aidg_plan_aterm_norm(aidg_plan* plan, double* out, int64_t cap);

/* Gridding (Sec. 2.5, imaging steps 1-2): for every subgrid of the plan, the direct
 * sum of its visibilities times exp(+2 pi i phi_k(x,y)) (Sec. 2.4, Eq. withw), the
 * A-term and taper correction (Sec. 3.3; A_p^H S A_q, or the normalised inverse of
 * aterm_mode = 1), the centred forward DFT (Sec. 2.3) and the add onto its window of
 * its w-layer (Eq. shiftback).  vis: device [nbl][nt][nc][4]; grid: device
 * [W][P][N][N], ACCUMULATED into (zero it for a fresh grid).  Visibilities in no
 * subgrid are ignored.  Never allocates or synchronises the host; AIDG_E_INVALID for
 * NULL buffers, AIDG_E_BUSY if the plan is in use, AIDG_E_DEVICE if a launch fails. */
aidg_status aidg_grid(aidg_plan* plan, const void* vis, void* grid, void* hip_stream);

/* Degridding (Sec. 2.5, prediction step 3), the adjoint chain: for every subgrid the
 * window of its w-layer (the splitter), the centred inverse DFT, the A-term and taper
 * (T A_p S A_q^H) and the direct sum over the subgrid's pixels times exp(-2 pi i phi_k)
 * for each of its visibilities (Eq. degridder).  grid: device [W][P][N][N]; vis_out:
 * device [nbl][nt][nc][4], OVERWRITTEN; visibilities that belong to no subgrid are set
 * to zero.  Deterministic: the same grid gives bitwise the same visibilities.  Errors
 * as aidg_grid. */
aidg_status aidg_degrid(aidg_plan* plan, const void* grid, void* vis_out, void* hip_stream);

/* The exact adjoints of the pair above, for differentiation (reverse mode needs the
 * adjoint of each forward map).  aidg_grid_adjoint ACCUMULATES D^H(vis) into grid, where
 * D is aidg_degrid; aidg_degrid_adjoint OVERWRITES vis_out with G^H(grid), where G is
 * aidg_grid (visibilities in no subgrid are set to zero).  With four grid planes they
 * are aidg_grid and aidg_degrid themselves (the gridder applies A_p^H . A_q, the forward
 * FFT and exp(+2 pi i phi) where the degridder applies A_p . A_q^H, the inverse FFT and
 * exp(-2 pi i phi)).  On a stokes_i plan the reduction I = (XX + YY) / 2 has the adjoint
 * I -> diag(I, I) / 2, so these two differ from aidg_grid / aidg_degrid by a factor 2
 * and 1/2, applied inside the kernels.  A plan in the inverse A-term mode
 * (aterm_mode = 1) has no such pair: AIDG_E_INVALID. */
aidg_status aidg_grid_adjoint(aidg_plan* plan, const void* vis, void* grid, void* hip_stream);
aidg_status aidg_degrid_adjoint(aidg_plan* plan, const void* grid, void* vis_out, void* hip_stream);

/* Device memory a plan and its data would take, estimated on the host without building
 * the plan or partitioning (for admission by device footprint).  n_wlayers is exact
 * for the library's own partition: the layers of the visibilities that can be placed
 * on the grid at the layer spacing the plan would use (geometry's w_step, or the
 * automatic one).  plan_bytes estimates everything aidg_plan_create allocates: the
 * A-term copy (two plane sets in the inverse A-term mode), uvw and channel tables, the
 * subgrid records (their count estimated from each row's uv extent over the channels,
 * its gaps and layer changes), the excluded-visibility list, the batch workspace
 * (workspace_bytes, capped at one group image per estimated same-centre group: the
 * distinct (layer, lattice centre) pairs of the rows' channel runs, plus a quarter for
 * groups the plan splits and centres the sample misses) and the image-level
 * tables.  All host arrays as in aidg_plan_create; nothing is allocated on the device. */
typedef struct {
  int32_t n_wlayers;      /* layers of the plan's grid */
  int32_t n_pol;          /* grid planes: 4, or 1 with stokes_i */
  double w_step;          /* layer spacing the plan would use (0: one layer) */
  int64_t n_subgrids;     /* estimate */
  int64_t n_excluded;     /* visibilities no subgrid can hold (outside the grid) */
  int64_t grid_bytes;     /* one grid, n_wlayers x n_pol x N x N complex */
  int64_t vis_bytes;      /* one visibility array */
  int64_t aterm_bytes;    /* the plan's A-term planes */
  int64_t plan_bytes;     /* estimate of the plan's own device memory (A-terms included) */
  int64_t n_groups;       /* estimate of the same-centre groups (subgrid images per batch) */
} aidg_footprint;
aidg_status aidg_footprint_estimate(const aidg_geometry* geo, int32_t n_stations, int32_t n_baselines,
                                    int32_t n_times, int32_t n_chans, const double* uvw_m,
                                    const double* freqs_hz, aidg_footprint* out);

/* Per-kernel device timing (the paper's per-subroutine breakdown, Sec. 5.4).
 * Kernel classes: 0 gridder DFT + Jones/taper epilogue, 1 FFT + adder,
 * 2 splitter + inverse FFT, 3 degridder DFT with Jones/taper prologue,
 * 4 zeroing of excluded visibilities, 5 image-level row FFTs (aidg_invert /
 * aidg_predict), 6 image-level transposes and w-stacking passes. */
#define AIDG_KERNEL_CLASSES 7
typedef struct {
  double ms[AIDG_KERNEL_CLASSES];            /* summed device time of the class */
  int64_t launches[AIDG_KERNEL_CLASSES];     /* kernel launches timed */
  int64_t vis_pixels[AIDG_KERNEL_CLASSES];   /* sum of (visibilities x L^2) over the
                                                subgrids the launches processed */
  int64_t subgrids[AIDG_KERNEL_CLASSES];     /* subgrids the launches processed */
} aidg_kernel_times;

/* Enable (1) or disable (0) timing: while enabled, aidg_grid / aidg_degrid record
 * a HIP event on their stream before and after every kernel (events come from a
 * pool created here; up to 8192 launches are timed between two reads). */
aidg_status aidg_plan_set_profiling(aidg_plan* plan, int32_t enable);

/* Wait for the recorded events, return the sums since the last read, and reset. */
aidg_status aidg_plan_kernel_times(aidg_plan* plan, aidg_kernel_times* out);

void aidg_plan_destroy(aidg_plan* plan);

/* ---- Image level: w-stacking (Sec. 2.4, Eq. wstack; Sec. 2.5 imaging step 3) and
 * its inverse for prediction (Eq. wunstack, prediction step 2).
 * Image pixel (X, Y), 0 <= X, Y < N, sits at l = (X - N/2) dl, m = (Y - N/2) dl,
 * with n1 = sqrt(1 - l^2 - m^2) - 1.  Image layout: device [4][N][N] (pol, Y, X), X
 * fastest, c64 / c128 as the plan's precision; [1][N][N] for a stokes_i plan, whose grids
 * are [W][1][N][N].
 *   aidg_invert:  I[p](X, Y) = 1 / (L^2 T(X, Y)) sum_w exp(+2 pi i w0_w n1)
 *                              sum_{gu, gv} G_w[p][gv][gu] exp(+2 pi i (u l + v m))
 *   aidg_predict: G_w[p][gv][gu] = sum_{X, Y} I[p](X, Y) exp(-2 pi i w0_w n1)
 *                              exp(-2 pi i (u l + v m)) / (L^2 T(X, Y))
 * with u l + v m = [(gu - N/2)(X - N/2) + (gv - N/2)(Y - N/2)] / N, w0_w the plan's
 * layers and T(X, Y) = t(X) t(Y) the plan's Kaiser-Bessel taper sampled at image
 * resolution, t(X) = I0(beta sqrt(1 - (2 (X - N/2)/N)^2)) / I0(beta).  The 1/L^2
 * undoes the unnormalised subgrid transforms: at image pixels on the subgrid lattice
 * (X - N/2 = (x - L/2) N / L) invert of gridded visibilities is the direct A-term
 * image of those visibilities, and prediction of point sources at such pixels
 * degrids to their direct visibilities.  aidg_predict is the exact adjoint of
 * aidg_invert; the taper divides in both (the degridder multiplies by T, unlike
 * the paper's Eq. degridder, which divides by it).
 * Both OVERWRITE their output (the whole image / every layer of the grid).
 * Supported: N = 2^a 3^b 5^c, N <= 8192 with a row of N complex values within 64 KB
 * (N <= 8192 in FP32, N <= 4096 in FP64); otherwise AIDG_E_UNSUPPORTED.  The
 * workspace is caller-owned device memory of aidg_image_workspace_bytes (two N x N
 * planes), AIDG_E_INVALID when smaller.  Neither call allocates or synchronises the
 * host; both queue kernels on hip_stream after the plan's earlier work. */
aidg_status aidg_image_workspace_bytes(const aidg_plan* plan, int64_t* bytes);
aidg_status aidg_invert(aidg_plan* plan, const void* grid, void* image, void* workspace,
                        int64_t workspace_bytes, void* hip_stream);
aidg_status aidg_predict(aidg_plan* plan, const void* image, void* grid, void* workspace,
                         int64_t workspace_bytes, void* hip_stream);

/* ---- Serving: grouped execution of work from many plans (continuous batching).
 * Gridding and degridding decompose into independent subgrids (Sec. 2.2: the
 * full grid is a sum over subgrids, and each visibility belongs to one), so a
 * range of one job's subgrids can share a kernel launch with ranges of other
 * jobs.  An executor owns a subgrid workspace on the device; aidg_execute packs
 * the given ranges into launches of at most 16 ranges each, grouped by
 * direction, subgrid size and precision. */
enum { AIDG_DIR_GRID = 0, AIDG_DIR_DEGRID = 1 };

typedef struct aidg_executor aidg_executor;

typedef struct {
  aidg_plan* plan;
  int32_t direction;   /* AIDG_DIR_GRID: accumulate vis `in` into grid `out`;
                          AIDG_DIR_DEGRID: write the visibilities of the range from grid `in`
                          into vis `out` (a range starting at 0 also zeroes the plan's
                          excluded visibilities) */
  int32_t reserved;    /* 0 */
  const void* in;      /* device buffer, layout as in aidg_grid / aidg_degrid */
  void* out;           /* device buffer */
  int64_t sg_begin;    /* range of the plan's subgrid table (aidg_plan_subgrids order) */
  int64_t sg_end;
} aidg_work;

/* Create an executor with a workspace of workspace_bytes (0 = 2 GiB) on the current device. */
aidg_status aidg_executor_create(int64_t workspace_bytes, aidg_executor** out);

/* Queue the work items on hip_stream.  Ranges of one plan within a call must not
 * overlap.  Every plan named waits for its earlier work (on any stream) first; the
 * executor's workspace makes calls on one executor run one after another.  The call
 * never allocates and never synchronises the host.  AIDG_E_BUSY if a plan or the
 * executor is in use by another host thread. */
aidg_status aidg_execute(aidg_executor* ex, const aidg_work* items, int32_t n_items, void* hip_stream);

void aidg_executor_destroy(aidg_executor* ex);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): aidg_execute without an executor.
 * The group images live in a library-owned static device array of
 * AIDG_STATIC_WORKSPACE_BYTES (128 MiB), one per device the library runs on, held
 * until the process ends; its address is looked up on the first call on a device.
 * workspace_bytes: how much of it the call may use (0 = all of it; a smaller budget
 * makes more, smaller launches); AIDG_E_INVALID beyond AIDG_STATIC_WORKSPACE_BYTES.
 * Items, ranges, ordering and errors as aidg_execute (every named plan waits for its
 * earlier work, AIDG_E_BUSY if a plan is in use by another host thread).  The call
 * allocates nothing and never synchronises the host.  All calls on one device share
 * the array: calls whose work overlaps on the device race (queue them on one stream,
 * or order them by events); no call needs the array cleared. */
#define AIDG_STATIC_WORKSPACE_BYTES ((int64_t)128 << 20)
aidg_status aidg_execute_static(const aidg_work* items, int32_t n_items, int64_t workspace_bytes,
                                void* hip_stream);

/* Thread-local description of the last non-OK status ("" if none). */
const char* aidg_last_error(void);

int32_t aidg_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* AIDG_H */
