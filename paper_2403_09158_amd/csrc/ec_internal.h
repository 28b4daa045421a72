// ec_internal.h - shared definitions of the HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "ec.h"

namespace ec {

constexpr int QSUB = 1024;  // coordinate quantisation steps per voxel edge (q = h/1024)

// Eigenstrain components are int64 fixed point with 56 fractional bits
// (|component| < 64 per defect): the contributions of overlapping defects add
// exactly and in any order, so the field is deterministic and an incremental
// move restores untouched voxels bit for bit.
//
// The field itself is not stored densely.  Every voxel keeps a link own[v]:
//   -1        no defect covers the voxel;
//   d >= 0    defect d (and nothing further);
//   -2 - e    membership entry e (its position in the footprint-id buffer),
//             whose record lnk[e] = {defect, link} continues with a link of the
//             same three forms.
// The first defect to reach a voxel stores itself with one compare-and-swap;
// later ones push an entry with an exchange.  A chain holds each defect at most
// once, so it is never longer than the defect count.
__host__ __device__ constexpr int32_t entry_link(int64_t e) { return (int32_t)(-2 - e); }

constexpr double FIX_SCALE = 72057594037927936.0;  // 2^56
constexpr double FIX_INV = 1.0 / 72057594037927936.0;

// Eigenstrain of one voxel: the exact sum of its owners' fixed-point
// components, rounded once to double.  Each component is split as
// f = hi 2^32 + lo (hi = f >> 32, lo in [0, 2^32)) and the halves are summed
// separately, so no number of owners can overflow (up to 2^21 owners the two
// sums stay exact in double); the result is hi 2^-24 + lo 2^-56 with a single
// rounding, the same value as (double)f * 2^-56 for a single owner.  The walk
// stops after max_links links (the defect count) whatever the data.
template <class Defs>
__device__ __forceinline__ void decode_voxel(int32_t link, const int2* __restrict__ lnk, const Defs& defs,
                                             double* e, int max_links) {
  if (link >= 0) {  // one owner (the common case): its converted value, three 16-byte loads
    const double2* f = reinterpret_cast<const double2*>(defs[link].efd);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double2 v = f[c];
      e[2 * c] = v.x;
      e[2 * c + 1] = v.y;
    }
    return;
  }
  int64_t hi[6] = {0, 0, 0, 0, 0, 0}, lo[6] = {0, 0, 0, 0, 0, 0};
  for (int guard = 0; guard < max_links && link != -1; ++guard) {
    int d;
    if (link >= 0) {
      d = link;
      link = -1;
    } else {
      const int2 L = lnk[-2 - link];
      d = L.x;
      link = L.y;
    }
    const int64_t* f = defs[d].efix;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      hi[c] += f[c] >> 32;
      lo[c] += (int64_t)(uint32_t)f[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = (double)hi[c] * 0x1p-24 + (double)lo[c] * 0x1p-56;
}

// 1 GPa nm^3 in eV (1e-18 J / elementary charge).
constexpr double GPA_NM3_EV = 1.0e-18 / 1.602176634e-19;

// Tensor-component weights of the double contraction A:B in 6-vector form.
__host__ __device__ constexpr double ddot_w(int a) { return a < 3 ? 1.0 : 2.0; }

// One quantised defect as the kernels see it (computed on the host).
struct DevDefect {
  int32_t kind;   // 0 loop, 1 sphere
  int32_t cq[3];  // centre in q units, [0, 1024 n)
  int32_t m[3];   // integer habit normal (loops)
  int32_t mm;     // m.m
  int32_t eq;     // slab thickness in q units
  int32_t lo[3];  // bounding-box first voxel index per axis, in [0, n)
  int32_t w[3];   // bounding-box widths per axis, <= n
  int32_t cls;    // eigenstrain direction class (-1: none)
  int32_t d0[3];  // unwrapped offset (q units) of the box's first voxel centre from the centre
  int32_t pad_;
  int64_t R2q;    // radius^2 in q^2 units
  int64_t slot;   // first element of this defect's footprint slot in the id buffer
  int64_t efix[6];
  double E[6];    // eigenstrain, tensor components xx yy zz yz xz xy
  double s;       // E = s * class direction (when cls >= 0)
  int32_t rt[3];  // run direction: a small lattice vector in the habit plane (loops) or x (spheres)
  int32_t rcls;   // run class (class and run direction) of the self-term tables, -1: none
  alignas(16) double efd[6];  // (double)efix * 2^-56: the eigenstrain of a voxel this defect alone covers
};

// The double form of a record's fixed-point eigenstrain (set with efix).
__host__ __device__ inline void set_efd(DevDefect& d) {
  for (int c = 0; c < 6; ++c) d.efd[c] = (double)d.efix[c] * 1.3877787807814457e-17;  // 2^-56
}

// Voxel-centre membership, exact integer arithmetic (loops: half-open slab
// along the lattice normal m, closed disk; spheres: closed ball).  d is the
// minimum-image offset of the voxel centre from the defect centre, q units.
__host__ __device__ inline bool member(const DevDefect& d, int n, int x, int y, int z) {
  const int32_t Lq = QSUB * n, half = Lq / 2;
  const int v[3] = {x, y, z};
  int32_t dd[3];
  for (int k = 0; k < 3; ++k) {
    int32_t t = QSUB * v[k] + QSUB / 2 - d.cq[k];  // in (-Lq, Lq)
    t += (t < -half) ? Lq : 0;
    t -= (t >= half) ? Lq : 0;
    dd[k] = t;
  }
  const int64_t d2 = (int64_t)dd[0] * dd[0] + (int64_t)dd[1] * dd[1] + (int64_t)dd[2] * dd[2];
  if (d.kind == 1) return d2 <= d.R2q;
  const int64_t t = (int64_t)d.m[0] * dd[0] + (int64_t)d.m[1] * dd[1] + (int64_t)d.m[2] * dd[2];
  const int64_t lim = (int64_t)d.eq * d.eq * d.mm;
  const bool slab = (t >= 0) ? (4 * t * t < lim) : (4 * t * t <= lim);
  return slab && ((int64_t)d.mm * d2 - t * t <= (int64_t)d.mm * d.R2q);
}

// Box enumeration order: per axis, the w voxels starting at lo (mod n) listed
// ascending, so (z, y, x)-lexicographic enumeration yields ascending linear ids.
__host__ __device__ inline int box_axis(int lo, int w, int n, int i) {
  const int wl = lo + w - n;  // voxels that wrap to the low end
  if (wl <= 0) return lo + i;
  return i < wl ? i : lo + (i - wl);
}

// Conservative range [u0, u1] of box x-indices (0 <= u < w[0]) that can hold
// members in the box row (iy, iz); the exact test is member().  Returns false if
// the row cannot hold any.  Bounds come from the geometry in floating point with
// a two-voxel margin: the slab fixes x within (e/2 |m|)/|m_x| of the plane when
// m_x != 0, and |d| <= sqrt(R^2 + e^2/4) bounds every member.
__host__ __device__ inline bool row_range(const DevDefect& d, int n, int y, int z, int& u0, int& u1) {
  if (d.w[0] >= n) {  // the box spans the whole x axis: no pruning
    u0 = 0;
    u1 = n - 1;
    return true;
  }
  const int32_t Lq = QSUB * n, hq = Lq / 2;
  int32_t ty = QSUB * y + QSUB / 2 - d.cq[1], tz = QSUB * z + QSUB / 2 - d.cq[2];
  ty += (ty < -hq) ? Lq : 0;
  ty -= (ty >= hq) ? Lq : 0;
  tz += (tz < -hq) ? Lq : 0;
  tz -= (tz >= hq) ? Lq : 0;
  const double dy = ty, dz = tz;
  const double dx0 = (double)d.d0[0];
  const double margin = 8.0;  // q units; covers rounding of the few operations below
  double lo, hi;
  if (d.kind == 1) {
    const double rem = (double)d.R2q - dy * dy - dz * dz;
    if (rem < -margin * margin) return false;
    const double r = sqrt(rem > 0.0 ? rem : 0.0) + margin;
    lo = -r;
    hi = r;
  } else {
    const double half = 0.5 * d.eq * sqrt((double)d.mm);  // slab half-width along m, in q * |m| units
    const double tyz = (double)d.m[1] * dy + (double)d.m[2] * dz;
    const double rem = (double)d.R2q + 0.25 * (double)d.eq * d.eq - dy * dy - dz * dz;
    if (rem < -margin * margin) return false;
    const double r = sqrt(rem > 0.0 ? rem : 0.0) + margin;
    lo = -r;
    hi = r;
    if (d.m[0] != 0) {
      double a = (-half - tyz) / d.m[0], b = (half - tyz) / d.m[0];
      if (a > b) {
        const double t = a;
        a = b;
        b = t;
      }
      lo = lo > a - margin ? lo : a - margin;
      hi = hi < b + margin ? hi : b + margin;
    } else if (fabs(tyz) > half + margin) {
      return false;
    }
  }
  const double a = ceil((lo - dx0) / QSUB), b = floor((hi - dx0) / QSUB);
  u0 = a < 0.0 ? 0 : (int)a;
  u1 = b > (double)(d.w[0] - 1) ? d.w[0] - 1 : (int)b;
  return u0 <= u1;
}

// Storage helpers
__device__ __forceinline__ double2 ld2(const float2* p) {
  float2 v = *p;
  return make_double2((double)v.x, (double)v.y);
}
__device__ __forceinline__ double2 ld2(const double2* p) { return *p; }
__device__ __forceinline__ void st2(float2* p, double2 v) { *p = make_float2((float)v.x, (float)v.y); }
__device__ __forceinline__ void st2(double2* p, double2 v) { *p = v; }

template <typename S>
struct Cplx;
template <>
struct Cplx<float> {
  using T = float2;
};
template <>
struct Cplx<double> {
  using T = double2;
};

// Cubic stiffness passed to kernels.  frm, when not null, points to the
// frame of a rotated crystal in device memory (FRAME_LEN doubles): [0, 36) the
// map of the six tensor components (xx yy zz yz xz xy) from the cell axes to
// the cube axes, [36, 72) the map back, [72, 81) the matrix A whose rows are
// the cell axes in cube coordinates (a cell vector v has cube components A^T v).
constexpr int FRAME_LEN = 81;
struct Cubic {
  double C11, C12, C44;
  const double* frm = nullptr;
};

// out = M in for a 6x6 row-major M (tensor components); in and out distinct.
template <typename V>
__host__ __device__ inline void rot6(const double* M, const V* in, V* out);
template <>
__host__ __device__ inline void rot6<double>(const double* M, const double* in, double* out) {
  for (int r = 0; r < 6; ++r) {
    double v = 0.0;
    for (int c = 0; c < 6; ++c) v += M[6 * r + c] * in[c];
    out[r] = v;
  }
}
template <>
__host__ __device__ inline void rot6<double2>(const double* M, const double2* in, double2* out) {
  for (int r = 0; r < 6; ++r) {
    double2 v = make_double2(0.0, 0.0);
    for (int c = 0; c < 6; ++c) {
      v.x += M[6 * r + c] * in[c].x;
      v.y += M[6 * r + c] * in[c].y;
    }
    out[r] = v;
  }
}

// A straight dislocation line along a cell axis: (u1, u2) its position in grid
// index units (voxel centres at integers) along the other two axes in
// increasing order, b its Burgers vector (nm), t its unit direction.
struct DevLine {
  double u1, u2;
  double b[3];
  double t[3];
};

// One piece of a dislocation path (a segment cut into pieces no longer than h):
// the grid cell holding its midpoint (f, integer grid indices reduced mod n),
// the midpoint's offset in that cell (fr in [0, 1) per axis) and the Nye
// tensor it carries, M_il = b_i dl_l / h^3.
struct DevPiece {
  int32_t f[3];
  int32_t pad_;
  double fr[3];
  double M[9];
};

// Profiling families (see ec_profile_read).
enum ProfFam { PF_RASTER = 0, PF_XF = 1, PF_Y = 2, PF_Z = 3, PF_XI = 4, PF_REDUCE = 5, PF_SELF = 6, PF_OTHER = 7 };

// One whole-voxel hop of a batch (device-resident table): every kernel of a
// batched hop update reads its replica's buffers and pruning from it, so one
// launch per pass serves the whole batch and the launch sequence does not
// depend on which replicas are in it (it can be captured in a graph once and
// replayed with new tables).  All replicas of a batch share one shape (n,
// precision, stiffness, frame).
constexpr int MAXBATCH = 16;
struct HopJob {
  void* spec;       // half spectrum
  double* sig;      // resident stress (voxel-major)
  int32_t* own;     // owner links
  int32_t* ids;     // footprint ids
  int2* lnk;        // membership entries
  int32_t* cnt;     // footprint counts
  DevDefect* tab;   // defect table
  const double* B;  // self terms
  double* S6;       // footprint stress sums
  double* E;        // the state's energies
  double* Eout;     // the caller's device output, or nullptr
  int64_t slot;     // first footprint entry of the moved defect
  int32_t idx, ndef;
  int32_t sx, sy, sz;
  int32_t ylo, ylen, zlo, zlen;
  int32_t xitems;   // row blocks of its sparse x-forward pass
  int32_t pad_;
  double h3c;
  double E12[12];   // eigenstrain removed from the old footprint, added on the new one
  DevDefect rec;    // the moved record
};

// ---- launch interfaces implemented in k_fft.hip ------------------------------

// Half spectrum layout: [kz][ky][kx][component], kx < n/2 + 1 padded to a
// row pitch of P, so element (c, kz, ky, kx) sits at ((kz n + ky) P + kx) 6 + c.
// The six components of a bin are adjacent: a tile of a few kx columns reads
// and writes contiguous runs of 6 x (columns) values in every pass.
__host__ __device__ inline size_t spec_at(int kz, int ky, int kx, int c, int n, int P) {
  return (((size_t)kz * n + ky) * P + kx) * 6 + c;
}

// Row pitch P of the half spectrum: n/2 + 1 bins rounded up to 16 with FP32
// storage (128-byte rows of float2) or to 8 with FP64 storage.
__host__ __device__ constexpr int spec_pitch(int n, bool fp64) {
  return fp64 ? ((n / 2 + 1 + 7) / 8) * 8 : ((n / 2 + 1 + 15) / 16) * 16;
}

// Rows per workgroup of the x passes: the most (a divisor of n) whose three
// pair transforms per row fit 1536 points.
__host__ __device__ constexpr int x_rows(int N) {
  int best = 1;
  for (int r = 1; r <= N; ++r)
    if (N % r == 0 && 3 * r * N <= 1536) best = r;
  return best;
}

struct SpecGeom {
  int n;
  int P;  // row pitch (complex elements) of the half spectrum, >= n/2 + 1
};

// Pruning of the pencil passes (incremental updates): only positions
// [lo, lo + len) (cyclic) of the transform axis carry data, and for the y pass
// only z planes [zlo, zlo + zlen) are transformed.  len = n / zlen = n: no pruning.
struct Prune {
  int in_lo, in_len;
  int z_lo, z_len;
};

bool fft_supported(int n);
int pencil_width(int n, bool fp64);

// Tile counters of the persistent passes (eight per pass, one per XCD; the
// y, z and y-inverse passes of a solve or update use counters 0-7, 8-15 and
// 16-23).  The x-forward pass that starts a solve or update zeroes them; a
// pass given no counters walks its tiles in a fixed order.
constexpr int NTILECTR = 24;

// Owner-list input (own/lnk/defs) or, when dense != nullptr, a dense FP64
// [6][n^3] field (kernel-level tests).  zero_ctr: NTILECTR counters to zero,
// or nullptr.
hipError_t launch_x_forward(bool fp64, const int32_t* own, const int2* lnk, const DevDefect* defs, int ndef,
                            const double* dense, void* spec, SpecGeom g, const double2* tw, uint32_t* zero_ctr,
                            hipStream_t s);
// Energies of a stored defect type at up to TYPE_NP translated positions per
// launch (Sec. 3.3): sig, te, ts are the half spectra of the field, of the
// type's eigenstrain and of its stress; tab/nyq the phase tables of the np
// positions and, in entry np, of the excluded mover; partial holds
// type_energy_grid(n) x TYPE_NP doubles; E[p] = scale * sum.
constexpr int TYPE_NP = 16;
int type_energy_grid(int n);
hipError_t launch_type_energies(bool fp64, const void* sig, const void* te, const void* ts, SpecGeom g,
                                const double2* tab, const double2* nyq, int np, bool excl, double* partial,
                                double scale, double* E, hipStream_t s);
// Dense voxel-major FP64 input [n^3][6] (the resident stress).
hipError_t launch_x_forward_vm(bool fp64, const double* vm, void* spec, SpecGeom g, const double2* tw, hipStream_t s);
// E: 12 doubles, the old eigenstrain (on old_ids) then the new one (on the new ids).
hipError_t launch_x_forward_sparse(bool fp64, const int32_t* old_ids, const int32_t* old_cnt, const int32_t* new_ids,
                                   int new_cnt,
                                   int shift_x, int shift_y, int shift_z, const double* E, void* spec, SpecGeom g,
                                   int y_lo, int y_len, int z_lo, int z_len, const double2* tw, uint32_t* zero_ctr,
                                   hipStream_t s);
// ctr: eight zeroed tile counters for this launch, or nullptr
hipError_t launch_pencil(bool fp64, bool inv, int axis, void* spec, SpecGeom g, Prune pr, const double2* tw,
                         uint32_t* ctr, hipStream_t s);
// Stress of straight dislocation lines along cell axis `axis` (Sec. 3.1, field
// dislocation mechanics): the spectrum on the plane k_axis = 0 (Nye tensor of
// the spread lines, incompatible plastic distortion, Green step; spec and tmp
// hold 6 n^2 complex values), then its inverse 2-D transform into plane
// ([n^2][6] FP64, index i2 * n + i1 over the other two axes).
hipError_t launch_disl_plane(const DevLine* lines, int nl, int axis, int n, double L, Cubic C, double2* spec,
                             double2* tmp, double* plane, hipStream_t s);
// sig (voxel-major [n^3][6]) += sgn * the planes of the axes in mask
// (planes: three [n^2][6] blocks).
hipError_t launch_bg_add(double* sig, const double* planes, int mask, int n, double sgn, hipStream_t s);
// sigma_hat of dislocation pieces (Sec. 3.1) over the whole half spectrum
// (xi = 0 left at zero), written into spec in the state's storage precision.
hipError_t launch_path_spectrum(bool fp64, const DevPiece* pieces, int np, SpecGeom g, double L, Cubic C,
                                const double2* tw, void* spec, hipStream_t s);
// sig[v][c] += sgn * bg3[v][c] over n^3 voxels (a 3-D background stress).
hipError_t launch_bg3_add(double* sig, const double* bg3, int64_t n3, double sgn, hipStream_t s);
hipError_t launch_green(bool fp64, void* spec, SpecGeom g, Cubic C, hipStream_t s);
hipError_t launch_z_green(bool fp64, void* spec, SpecGeom g, Cubic C, Prune pr, const double2* tw, uint32_t* ctr,
                          hipStream_t s);
// bg / bg_mask: stress planes of dislocation lines added to sigma (not with accum).
// add3: a stress field [n^3][6] (FP64) added to sigma (not with accum).
// own: the owner map; when given, sigma is stored only at voxels some defect
// covers (not with accum), or with all at every voxel by the same code, so
// that both give a covered voxel the same bits.
hipError_t launch_x_inverse(bool fp64, bool accum, const void* spec, double* sig, SpecGeom g, const double* mean6,
                            const double2* tw, hipStream_t s, const double* bg = nullptr, int bg_mask = 0,
                            const double* add3 = nullptr, const int32_t* own = nullptr, bool all = false);
// The Fourier passes of a batch of hops (jobs: njob device records, see
// HopJob; ctr: NTILECTR tile counters, zeroed by the first pass): sparse x
// forward, pruned y forward, fused z pass, y inverse, accumulating x inverse
// (the hop's mean-stress change is zero).
hipError_t launch_hop_batch_fft(bool fp64, const HopJob* jobs, int njob, SpecGeom g, Cubic C, const double2* tw,
                                uint32_t* ctr, const double* zero6, hipStream_t s);
// The lists, records and energies of a batch of hops (after the passes).
hipError_t launch_hop_batch_lists(const HopJob* jobs, int njob, int n, hipStream_t s);
hipError_t launch_hop_batch_energies(const HopJob* jobs, int njob, hipStream_t s);

// ---- k_raster.hip / k_energy.hip -----------------------------------------------

hipError_t launch_raster_fill(const DevDefect* d, int ndef, int n, int32_t* ids, int2* lnk, int32_t* counts,
                              int32_t* own, hipStream_t s);
// Empty the membership lists of every voxel of every listed footprint.
hipError_t launch_unraster(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids, int32_t* own,
                           hipStream_t s);
// One defect moved: unlink its old entries [slot, slot + *cnt_old), then link
// the new ones (new voxel = old shifted by whole voxels when new_ids ==
// nullptr, else new_ids[0 .. cnt_new) copied into [new_slot, ...)).
hipError_t launch_move_lists(int def, int ndef, const int32_t* cnt_old, int64_t old_slot, const int32_t* new_ids,
                             int cnt_new, int64_t new_slot, int shift_x, int shift_y, int shift_z, int n, int32_t* ids,
                             int2* lnk, int32_t* own, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s);
hipError_t launch_mean_stress(const DevDefect* d, const int32_t* counts, int ndef, int64_t n3, Cubic C, int bc,
                              double* add6, hipStream_t s);
hipError_t launch_scan(const int32_t* counts, int ndef, int64_t* offsets, hipStream_t s);
hipError_t launch_fill_i64(int64_t* p, int64_t count, int64_t v, hipStream_t s);
// sig: the resident stress, voxel-major [n^3][6]
hipError_t launch_reduce(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids, const double* sig,
                         const double* B, double h3c, double* S6, double* E, hipStream_t s);
hipError_t launch_window_crop(const double* sig, int n, int D, int b, double* K, hipStream_t s);
hipError_t launch_class_windows(const double* K, int D, const double* dirs, int ncls, double* g, hipStream_t s);
// Self-term work item: rows [p0, p1) of defect `def`'s pair triangle.
struct SelfWork {
  int32_t def, p0, p1, pad;
};
// Runs of one footprint held in LDS by the self-term run path at most; the host
// gives a defect a run class only when a bound on its run count stays below.
constexpr int SELF_RUN_MAX = 8192;

// Run tables of the self terms: for run class r (class c, run direction t),
// ff[r W^3 + point] holds the double prefix sum of the class window g_c along
// t over the window of half-width D (W = 2 D + 1; see k_run_tables);
// info[r] = {c, tx, ty, tz}.  D is the state's own window need, so the tables
// (and the self terms) do not depend on how wide the shared kernel window has
// grown for other states.
struct RunTables {
  const double* ff = nullptr;
  const int4* info = nullptr;
  int nrun = 0;
  int D = 0;
  int max_runs = 0;  // largest run bound of a defect on the run path (LDS of the run kernel)
};
// Builds the work list on the device in one workgroup (scratch: wbeg[ndef + 1])
// and runs it on a fixed grid; no host synchronisation.  Defects with a run
// class whose box fits the window take the run path instead (scratch:
// runsum[ndef]).
hipError_t launch_self_terms(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids, int n,
                             const double* K, const double* gcls, int D, RunTables rt, SelfWork* work,
                             int64_t work_cap, int64_t* wbeg, double* partial, double* runsum, double h3c, double* B,
                             hipStream_t s);
// The run tables of nrun run classes on the half-width Drun <= Dg from the
// class windows g ((2 Dg + 1)^3 per class).
hipError_t launch_run_tables(const double* g, int Dg, int Drun, const int4* info, int nrun, double* ff,
                             hipStream_t s);
// Jump probes: dE[i nj + j] for jump jumps[3 (i nj + j) ..] of defect i (see
// k_energy.hip); S0 = the footprint sums of the last reduction, B the self
// terms; scratch as for the self terms, t1[ndef nj], wbeg[ndef nj + 1].
hipError_t launch_jump_energies(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids,
                                const double* sig, int n, const int32_t* jumps, int nj, const double* S0,
                                const double* K, const double* gcls, int D, SelfWork* work, int64_t work_cap,
                                int64_t* wbeg, double* partial, double* t1, const double* B, double h3c, double* xc,
                                bool xc_valid, double* dE, hipStream_t s);
// Dipole-tensor energies: Edip[i] = -h^3 c m_i E_i : (sigma - sigma_i) at the
// voxel holding the defect centre (sig voxel-major; window as for the self terms).
hipError_t launch_dipole(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids, const double* sig,
                         int n, const double* K, const double* gcls, int D, double h3c, double* Edip, hipStream_t s);
// The table of the chosen whole-voxel jumps: dst[i] = src[i] with its centre
// and box moved by jumps[(i * nj + choice[i]) * 3 ..] voxels (choice < 0: as is).
hipError_t launch_apply_jumps(const DevDefect* src, DevDefect* dst, int ndef, const int32_t* choice,
                              const int32_t* jumps, int nj, int n, hipStream_t s);
// Biased jump frequencies and the frequency-line choice (nu, choice may be null).
hipError_t launch_jump_select(const double* dE, int ndef, int nj, const double* Em, double nu0, double kT,
                              const double* xi, const double* u, double dt, double* nu, int32_t* choice,
                              hipStream_t s);
// Eigenstrain direction class of a defect (index into the class windows, -1
// for the generic path) and its scale s (E = s e).
struct ClassTag {
  double s;
  int32_t cls, rcls;
};
// Writes tags[i] into defs[i].cls / defs[i].s / defs[i].rcls.
hipError_t launch_set_class(DevDefect* d, int ndef, const ClassTag* tags, hipStream_t s);
// which 0: sigma, 1: eps = C^-1:sigma + eps*, 2: eps* alone; out is float or double.
hipError_t launch_sig_to_out(const double* sig, const int32_t* own, const int2* lnk, const DevDefect* defs, int ndef,
                             int64_t n3, Cubic C, int which, bool fp32, void* out, hipStream_t s);

constexpr int KWIN = 24;  // doubles per window point (21 used: the symmetric 6x6 kernel)

}  // namespace ec
