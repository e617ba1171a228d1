// Internal declarations shared by the host plan code and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/aidg.h"

namespace aidg {

constexpr double kSpeedOfLight = 299792458.0;
constexpr int kMaxSubgridVisDefault = 1024;
// The (de)gridder stages one subgrid's visibilities (8 values each) in LDS:
// 2048 of them take 64 KB in FP32 and 128 KB in FP64, within the 160 KB of a CU.
constexpr int kMaxSubgridVisLimit = 2048;
constexpr int kReseedDefault = 32;
constexpr int64_t kWorkspaceDefault = int64_t(2) << 30;
// Size of the static subgrid workspace of aidg_execute_static (AIDG_STATIC_WORKSPACE_BYTES).
constexpr int64_t kStaticWorkspaceBytes = int64_t(128) << 20;
// A group of same-centre subgrids holds at most this many times the mean
// visibilities per centre (and at least one subgrid).
constexpr int64_t kGroupVisFactor = 8;

// Per-subgrid record the kernels read (device copy of the partition).
struct alignas(16) SubgridDev {
  int32_t t0, nt, c0, nc;      // sub-table
  int32_t U0, V0, wlayer, R;   // centre cell, layer, reseed interval (1: every channel)
  int32_t ap, aq, bl, group;   // A-term plane index (aint * n_st + station) of the left and
                               // right station (swapped for a folded sub-table); baseline;
                               // (layer, centre) group in the plan's order
  int64_t vis0;                // flat visibility index of (bl, t0, c0)
  int64_t uvw0;                // flat uvw row index of (bl, t0); folded sub-tables index the
                               // negated copy that follows the table
  double dfc;                  // channel spacing / c (s/m * Hz ... i.e. 1/m) for the recurrence
  double w0;                   // layer w, wavelengths
  int32_t fold;                // 1: visibilities enter and leave conjugate-transposed
  int32_t kind;                // degridder form: kDegridRecur, kDegridDirect or kDegridPerVis
  int32_t pad2, pad3;
};
// Degridder forms, chosen per subgrid by the plan (degrid_form).
constexpr int32_t kDegridRecur = 0;   // lanes own pixels; phasors step along each row's channels
constexpr int32_t kDegridDirect = 1;  // lanes own pixels; every visibility's phasor seeded directly
constexpr int32_t kDegridPerVis = 2;  // lanes own visibilities
static_assert(sizeof(SubgridDev) == 96, "SubgridDev layout");

// Geometry after validation, with derived quantities.
struct Geometry {
  int N, L, K, aterm_interval, precision, R, strict, max_sg_vis, lattice, fold, amode;
  int degrid_form;  // AIDG_DEGRID_AUTO, AIDG_DEGRID_COOPERATIVE or AIDG_DEGRID_PER_VIS
  int npol;  // grid planes: 4, or 1 for Stokes-I grids
  double dl, fov, du, beta, w_step;
  int64_t workspace;
};

// Host-side partition (library's own algorithm); table entries are aidg_subgrid.
struct PartitionResult {
  std::vector<aidg_subgrid> table;
  std::vector<int64_t> excluded;  // flat visibility indices
  double w_step = 0.0;            // 0: single layer
  int64_t jmin = 0, jmax = 0;
};

aidg_status validate_geometry(const aidg_geometry* g, Geometry* out, std::string* err);
double auto_w_step(const Geometry& g);
aidg_status partition(const Geometry& g, int n_st, int nbl, int nt, int nc, const int32_t* baselines,
                      const double* uvw, const double* freqs, PartitionResult* out, std::string* err);
// Host estimate of a partition's shape without building it: the w-layer range of the
// placeable visibilities, the unplaceable count, and an estimate of the number of
// subgrids (per row: the channel runs its uv extent needs, plus one per gap or layer
// change, plus the splits at max_sg_vis), and of the number of same-centre groups (the
// distinct (layer, lattice centre) pairs of the runs' midpoints, plus a quarter).
struct ShapeEstimate {
  int64_t jmin = 0, jmax = 0, n_excluded = 0, n_subgrids = 0, n_groups = 0;
};
void estimate_shape(const Geometry& g, int nbl, int nt, int nc, const double* uvw, const double* freqs,
                    ShapeEstimate* out);
aidg_status adopt_table(const Geometry& g, int n_st, int nbl, int nt, int nc,
                        const int32_t* baselines, const aidg_subgrid* table, int64_t n_table,
                        PartitionResult* out, std::string* err);
std::vector<aidg_subgrid> split_large(const std::vector<aidg_subgrid>& t, int max_vis, int nt_total,
                                      int nc_total);
void kaiser_bessel_taper(int L, double beta, std::vector<double>* T);

// Launch parameters of one plan; the plan keeps a device copy that kernels read.
struct KernelArgs {
  const SubgridDev* sg;     // device subgrid table
  const double* uvw;        // device [nbl][nt][3] metres
  const double* fc;         // device [nc] f / c
  const void* aterms;       // device [n_int][n_st][L][L][4]
  const void* ainvh;        // device (A^-1)^H planes of the inverse A-term mode, else null
  const void* taper;        // device [L][L] taper times (-1)^(x+y)
  const void* twiddle;      // device [L] exp(-2 pi i k / L)
  const int64_t* grp_begin; // device [n_groups + 1]: first subgrid of each (layer, centre) group
  int nt_total, nc_total, N;
  int npol;                 // grid planes: 4 (XX, XY, YX, YY) or 1 (Stokes I)
  double du;                // uv cell size, wavelengths
  double lstep;             // FOV / L, subgrid lattice spacing in direction cosines
};

// A grouped launch: consecutive ranges of subgrids from up to kMaxGroup plans
// share one kernel launch.  A plan's table is ordered so that subgrids with the
// same w-layer and centre are consecutive (a "group"); the gridder, FFT/adder and
// splitter/inverse FFT run one workgroup slot per group (slots gslot_begin..), the
// degridder one slot per subgrid (slots slot_begin..).  Group g of a range owns
// scratch slot gslot_begin + (g - g_first): its subgrid image sum, [4][L][L].
constexpr int kMaxGroup = 16;
struct JobRef {
  const KernelArgs* args;   // device copy of the plan's parameters
  const void* in;           // visibilities (gridder) or grid (splitter)
  void* out;                // grid (adder) or visibilities (degridder)
  int64_t sg_begin, sg_end; // range of the plan's table
  int64_t g_first;          // group of subgrid sg_begin
  int64_t slot_begin;       // first per-subgrid slot of the range in this launch
  int64_t gslot_begin;      // first per-group slot of the range in this launch
  int32_t adjoint;          // 1: the exact adjoint of the other direction (Stokes-I plans
                            // grid XX + YY and split into diag(I, I) / 2)
  int32_t pad;
};
struct Group {
  int32_t n, pad;
  int64_t total_sg;         // per-subgrid slots in the launch
  int64_t total_grp;        // per-group slots (scratch images) in the launch
  void* scratch;            // [total_grp][4][L][L] subgrid images
  JobRef job[kMaxGroup];
};

// Kernel classes, in the order of aidg_kernel_times.
enum KernelClass {
  kGridDft = 0, kFftAdd = 1, kSplitIfft = 2, kDegridDft = 3, kZeroVis = 4,
  kImageFft = 5,      // image-level row FFTs (invert / predict)
  kImageWstack = 6    // image-level transposes and w-stacking passes
};

// Degridder form of a sub-table of nt rows and nc channels (kernels.hip), `uniform`
// when its channels have a common spacing: the geometry's choice, or (automatic) the
// form of least modelled cost.  The recurrence needs a common spacing (else the
// direct form), and only sub-tables of at most the workgroup's lane count can take the
// per-visibility form (else the recurrence).
int32_t degrid_form(const Geometry& g, int nt, int nc, bool uniform);

// Launch one kernel class over a group (kernels.hip).  max_nv: the largest
// sub-table of the group (degridder LDS).  Returns a hipError_t as int.
int launch_group(KernelClass k, int L, int precision, const Group& g, void* stream, int max_nv);
int launch_zero_vis(int precision, const int64_t* idx, int64_t n, void* vis, void* stream);

// Image level (image.hip).  A row of N complex values is transformed in LDS: N must
// factor into radices 4, 2, 3 and 5 and a row must fit in 64 KB.
constexpr int kMaxImageN = 8192;
constexpr int kMaxImageRowBytes = 65536;
constexpr int kMaxImageRadices = 16;
struct ImageRadices {
  int32_t n;                     // number of Stockham passes
  int32_t r[kMaxImageRadices];   // radix of each pass
};
// Factorisation of N in pass order (5s, 3s, then 4s and a 2); false when N is not
// supported.
bool image_radices(int N, int elem_bytes, ImageRadices* out);
void kaiser_bessel_axis(int n, double beta, std::vector<double>* t);
int launch_image_fft_rows(int precision, int dir, bool predict, const void* src, void* dst, int N,
                          const ImageRadices& fr, const void* tw, const double* itaper, double dl,
                          double w0, double inv_l2, void* stream);
int launch_image_transpose(int precision, const void* src, void* dst, int N, void* stream);
int launch_image_wstack(int precision, const void* B, void* img, int N, const double* itaper, double dl,
                        double w0, double inv_l2, int assign, const double* nmap, int L, void* stream);

// Device address of the static workspace (kStaticWorkspaceBytes) on `device`, which
// must be the current device; looked up on the first call per device, then cached.
// Null with a message in *err on failure (static_workspace.hip).
void* static_workspace(int device, std::string* err);

// Inverse A-term mode (aterm.hip): (A^-1)^H of n 2x2 matrices, and the weighted-average
// normalisation map [L2] from (A_p plane, A_q plane) pairs [n_pairs][2] with their
// visibility counts, summed in n_chunks chunks of chunk_len pairs through partial
// [n_chunks][L2].
int launch_aterm_inverse_h(int precision, const void* A, void* B, int64_t n, void* stream);
int launch_aterm_norm(int precision, const void* B, const int32_t* pairs, const double* count, int64_t n_pairs,
                      int n_chunks, int64_t chunk_len, int L2, double inv_total, double* partial, double* map,
                      void* stream);

}  // namespace aidg
