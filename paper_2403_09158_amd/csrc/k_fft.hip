// k_fft.hip - FFT passes and the Green operator of the periodic eigenstrain solve.
//
// Half-spectrum layout: [kz][ky][kx][6] complex (the six components of a bin
// adjacent), kx in [0, n/2] with row pitch P (spec_pitch).  The solve runs:
//   x-forward (R2C, two real rows per complex transform), y-forward,
//   z-forward + Green operator + z-inverse, y-inverse, x-inverse (C2R) + stress.
// All butterflies, twiddles and the Green operator run in FP64 registers; the
// storage type S (float or double) only sets what is kept in HBM between passes.
#include <algorithm>

#include "ec_internal.h"
#include "fft_core.h"

namespace ec {

namespace {

constexpr int max_nb(int N, int F) {
  Plan2 p = plan_of(N);
  int m = 0;
  for (int s = 0; s < p.nstage; ++s) {
    int b = F * (N / p.r[s]);
    if (b > m) m = b;
  }
  return m;
}
constexpr int pick_T(int nb) { return nb >= 256 ? 256 : ((nb + 63) / 64) * 64; }


// ----------------------------------------------------------------- Green operator
//
// Sec. 3.2: eps_hat = Gamma(xi):(C:eps*_hat) with Gamma built from N = K^-1,
// K_ik = C_ijkl xi_j xi_l; here eps_hat = sym(xi (x) N (tau xi)), tau = C:eps*_hat,
// and the kernel returns sigma_hat = C:eps_hat - tau (the stress spectrum, so the
// inverse transform yields sigma directly).  Gamma is homogeneous of degree 0 in
// xi, so the integer labels stand in for xi = 2 pi k / L.

// tau = C:e for cubic C (components xx yy zz yz xz xy; the shear entries of
// e are tensor components, so they take 2 C44).
__device__ __forceinline__ void cubic_stress(const double2* e, const Cubic& C, double2* tau) {
  const double d = C.C11 - C.C12, c44x2 = 2.0 * C.C44;
  const double trx = e[0].x + e[1].x + e[2].x, try_ = e[0].y + e[1].y + e[2].y;
  const double ctx = C.C12 * trx, cty = C.C12 * try_;
#pragma unroll
  for (int c = 0; c < 3; ++c) tau[c] = make_double2(fma(d, e[c].x, ctx), fma(d, e[c].y, cty));
#pragma unroll
  for (int c = 3; c < 6; ++c) tau[c] = make_double2(c44x2 * e[c].x, c44x2 * e[c].y);
}

// w = wgt N(xi) (tau xi), N = K^-1 by the adjugate, K_ik = C_ijkl xi_j xi_l.
__device__ __forceinline__ void green_w(double ax, double ay, double az, const Cubic& C, const double2* tau,
                                        double wgt, double2* w) {
  const double x2 = ax * ax, y2 = ay * ay, z2 = az * az, r2 = x2 + y2 + z2;
  const double c44r2 = C.C44 * r2, dd = C.C11 - C.C44;
  const double K00 = fma(dd, x2, c44r2), K11 = fma(dd, y2, c44r2), K22 = fma(dd, z2, c44r2);
  const double cc = C.C12 + C.C44;
  const double ccx = cc * ax;
  const double K01 = ccx * ay, K02 = ccx * az, K12 = cc * ay * az;
  const double A00 = K11 * K22 - K12 * K12;
  const double A11 = K00 * K22 - K02 * K02;
  const double A22 = K00 * K11 - K01 * K01;
  const double A01 = K02 * K12 - K01 * K22;
  const double A02 = K01 * K12 - K02 * K11;
  const double A12 = K01 * K02 - K00 * K12;
  const double inv = wgt / (K00 * A00 + K01 * A01 + K02 * A02);
  // v = tau . xi (tau symmetric: xx yy zz yz xz xy)
  double2 v0, v1, v2;
  v0.x = tau[0].x * ax + tau[5].x * ay + tau[4].x * az;
  v0.y = tau[0].y * ax + tau[5].y * ay + tau[4].y * az;
  v1.x = tau[5].x * ax + tau[1].x * ay + tau[3].x * az;
  v1.y = tau[5].y * ax + tau[1].y * ay + tau[3].y * az;
  v2.x = tau[4].x * ax + tau[3].x * ay + tau[2].x * az;
  v2.y = tau[4].y * ax + tau[3].y * ay + tau[2].y * az;
  w[0].x = (A00 * v0.x + A01 * v1.x + A02 * v2.x) * inv;
  w[0].y = (A00 * v0.y + A01 * v1.y + A02 * v2.y) * inv;
  w[1].x = (A01 * v0.x + A11 * v1.x + A12 * v2.x) * inv;
  w[1].y = (A01 * v0.y + A11 * v1.y + A12 * v2.y) * inv;
  w[2].x = (A02 * v0.x + A12 * v1.x + A22 * v2.x) * inv;
  w[2].y = (A02 * v0.y + A12 * v1.y + A22 * v2.y) * inv;
}

// s = C:sym(xi (x) w) - tau (FIRST) or s += C:sym(xi (x) w), cubic C: normal
// entries C12 (xi . w) + (C11 - C12) xi_i w_i, shear entries
// C44 (xi_i w_j + xi_j w_i).
template <bool FIRST>
__device__ __forceinline__ void add_cubic_sym(double ax, double ay, double az, const Cubic& C, const double2* w,
                                              const double2* tau, double2* s) {
  const double d = C.C11 - C.C12;
  const double a[3] = {ax, ay, az};
  const double dx = ax * w[0].x + ay * w[1].x + az * w[2].x;
  const double dy = ax * w[0].y + ay * w[1].y + az * w[2].y;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double bx = FIRST ? fma(C.C12, dx, -tau[c].x) : fma(C.C12, dx, s[c].x);
    const double by = FIRST ? fma(C.C12, dy, -tau[c].y) : fma(C.C12, dy, s[c].y);
    s[c] = make_double2(fma(d, a[c] * w[c].x, bx), fma(d, a[c] * w[c].y, by));
  }
  // shear (yz, xz, xy) = pairs (1, 2), (0, 2), (0, 1)
  constexpr int P[3][2] = {{1, 2}, {0, 2}, {0, 1}};
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int i = P[q][0], j = P[q][1];
    const double mx = fma(a[i], w[j].x, a[j] * w[i].x), my = fma(a[i], w[j].y, a[j] * w[i].y);
    const double bx = FIRST ? -tau[3 + q].x : s[3 + q].x, by = FIRST ? -tau[3 + q].y : s[3 + q].y;
    s[3 + q] = make_double2(fma(C.C44, mx, bx), fma(C.C44, my, by));
  }
}

// Centred integer label of DFT bin k in [0, n) (Sec. 3.4): k up to (n - 1) / 2,
// k - n above.  Only an even n has a Nyquist bin (k = n / 2), whose label the
// callers choose.
__device__ __forceinline__ int centred(int k, int n) { return k <= (n - 1) / 2 ? k : k - n; }
__device__ __forceinline__ bool nyquist(int k, int n) { return (n & 1) == 0 && k == n / 2; }

// sigma_hat at bin (kx in [0, n/2], ky, kz in [0, n)) from eps*_hat (in place).
// Even-n Nyquist rule: a bin with any index at n/2 gets the mean of the
// operators at the all -n/2 and all +n/2 labels (real part of the centred
// full-complex solution).  xi = 0: zero (the mean is added in FP64 later).
__device__ __forceinline__ void green_bin(double2* e, int kx, int ky, int kz, int n, const Cubic& C) {
  if (kx == 0 && ky == 0 && kz == 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) e[c] = make_double2(0.0, 0.0);
    return;
  }
  double2 tau[6], w[3];
  cubic_stress(e, C, tau);
  const int h = n / 2;
  const bool nx = nyquist(kx, n), ny = nyquist(ky, n), nz = nyquist(kz, n), nq = nx || ny || nz;
  const double lx = nx ? -h : kx, ly = ny ? -h : centred(ky, n), lz = nz ? -h : centred(kz, n);
  // every bin takes its (first) label; a Nyquist bin weighs it 1/2 and adds
  // the all +n/2 label, so the lanes of a wavefront part for one label only
  green_w(lx, ly, lz, C, tau, nq ? 0.5 : 1.0, w);
  add_cubic_sym<true>(lx, ly, lz, C, w, tau, e);
  if (nq) {
    const double px = nx ? h : lx, py = ny ? h : ly, pz = nz ? h : lz;
    green_w(px, py, pz, C, tau, 0.5, w);
    add_cubic_sym<false>(px, py, pz, C, w, tau, e);
  }
}

// Rotated crystal (C.frm set): the cubic operator applied in the cube frame,
// eps*_hat and the frequency labels rotated in and sigma_hat rotated back, so
// that the cell-frame operator is built from C' = A^T-rotated C without
// forming its 21 constants.
// The cubic operator on a bin whose eps*_hat is already in the cube frame, with
// the frequency label rotated there; sigma_hat stays in the cube frame.
__device__ __forceinline__ void green_core_rot(double2* ec, int kx, int ky, int kz, int n, const Cubic& C) {
  if (kx == 0 && ky == 0 && kz == 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) ec[c] = make_double2(0.0, 0.0);
    return;
  }
  const double* A = C.frm + 72;
  double2 tau[6], w[3];
  cubic_stress(ec, C, tau);
  const int h = n / 2;
  const bool nx = nyquist(kx, n), ny = nyquist(ky, n), nz = nyquist(kz, n), nq = nx || ny || nz;
  const double lx = nx ? -h : kx, ly = ny ? -h : centred(ky, n), lz = nz ? -h : centred(kz, n);
  auto label = [&](double x, double y, double z, double* r) {
    r[0] = A[0] * x + A[3] * y + A[6] * z;
    r[1] = A[1] * x + A[4] * y + A[7] * z;
    r[2] = A[2] * x + A[5] * y + A[8] * z;
  };
  double r[3];
  label(lx, ly, lz, r);
  green_w(r[0], r[1], r[2], C, tau, nq ? 0.5 : 1.0, w);
  add_cubic_sym<true>(r[0], r[1], r[2], C, w, tau, ec);
  if (nq) {
    label(nx ? h : lx, ny ? h : ly, nz ? h : lz, r);
    green_w(r[0], r[1], r[2], C, tau, 0.5, w);
    add_cubic_sym<false>(r[0], r[1], r[2], C, w, tau, ec);
  }
}

__device__ __forceinline__ void green_bin_rot(double2* e, int kx, int ky, int kz, int n, const Cubic& C) {
  double2 ec[6];
  rot6(C.frm, e, ec);
  green_core_rot(ec, kx, ky, kz, n, C);
  rot6(C.frm + 36, ec, e);
}

// Tile order of a persistent pass.  The tiles are split into eight
// contiguous ranges, one per XCD (dispatch puts workgroup b on XCD b % 8), so
// that neighbouring tiles share an L2.  With a counter per XCD (zero at
// launch) the workgroups of an XCD claim its tiles one at a time, so that one
// starting late behind other work on its CU takes fewer tiles instead of
// holding up the pass; without counters each takes every (grid / 8)-th tile
// of the range.  The tile after the current one is known an iteration ahead
// (for the prefetch): next() at the top of an iteration gives it, the claim
// for the one after it is issued then and stored before the iteration's last
// barrier.
struct TileWalk {
  int lo, hi, g8, xcd;
  uint32_t* ctr;  // nullptr: static order
  int* slot;      // two LDS entries
  __device__ TileWalk(int ntiles, uint32_t* c, int* sl) : ctr(c), slot(sl) {
    g8 = (int)gridDim.x / 8;
    const int per = (ntiles + 7) / 8;
    xcd = (int)(blockIdx.x % 8);
    lo = xcd * per;
    hi = min(ntiles, lo + per);
  }
  // the first two tiles (a barrier must follow before first())
  __device__ void claim_first() {
    if (ctr && threadIdx.x == 0) {
      slot[0] = lo + (int)atomicAdd(&ctr[xcd], 1u);
      slot[1] = lo + (int)atomicAdd(&ctr[xcd], 1u);
    }
  }
  __device__ int first() const { return ctr ? slot[0] : lo + (int)(blockIdx.x / 8); }
  __device__ int next(int t, int it) const { return ctr ? slot[(it + 1) & 1] : t + g8; }
  __device__ uint32_t claim_issue() { return (ctr && threadIdx.x == 0) ? atomicAdd(&ctr[xcd], 1u) : 0u; }
  __device__ void claim_store(int it, uint32_t v) {
    if (ctr && threadIdx.x == 0) slot[it & 1] = lo + (int)v;
  }
};

// ----------------------------------------------------------------- x forward (R2C)

// x forward pass with a two-stage plan of equal radices: each thread reads
// the twiddles of its second-stage butterfly from the global table into
// registers, and the block keeps no LDS copy of the table (more resident
// blocks for these short-lived ones; the inverse pass, which holds more
// registers, keeps the table).
template <int N>
constexpr bool x_twreg() {
  constexpr Plan2 P = plan_of(N);
  return P.nstage == 2 && P.r[0] == P.r[1];
}

template <int N, int NF, int T>
__device__ __forceinline__ auto x_twiddles(const double2* tw_lds, const double2* twg) {
  if constexpr (x_twreg<N>()) {
    constexpr int R = plan_of(N).r[1];
    return make_twreg<N, R, R, Map::Row, NF, T>(twg, threadIdx.x);
  } else {
    return tw_lds;
  }
}

// Persistent: each workgroup walks row groups (ROWS rows of one z plane) in a
// fixed order within its XCD's contiguous range, and loads the next group's
// owner links into registers while it decodes and transforms the current one,
// so the HBM latency of the owner map overlaps the work of the group before.
// The eigenstrains of the next group's single-owner voxels are loaded after
// the current group's transform and before its spectrum stores: vector memory
// operations complete in issue order as far as a wave's wait counter is
// concerned, so a load issued after the stores would wait for them to drain,
// and loads issued one voxel at a time would each wait for the one before.
// Voxels of several owners (a few per cent of the row groups) are decoded in
// place.
// DM: the input, 0 = owner lists, 1 = a dense field [6][n^3], 2 = a dense
// voxel-major field [n^3][6] (the resident stress).
template <int N, typename S, int DM>
__global__ __launch_bounds__(pick_T(max_nb(N, 3 * x_rows(N)))) void k_x_forward(
    const int32_t* __restrict__ own, const int2* __restrict__ lnk, const DevDefect* __restrict__ defs,
    const double* __restrict__ dense, typename Cplx<S>::T* __restrict__ spec, int P, const double2* __restrict__ twg,
    uint32_t* __restrict__ zero_ctr, int max_links) {
  constexpr int ROWS = x_rows(N);
  constexpr int NF = 3 * ROWS;  // (xx,yy), (zz,yz), (xz,xy) per row
  constexpr int T = pick_T(max_nb(N, NF));
  constexpr int LDN = N + N / 16 + 1;
  constexpr int NH = N / 2 + 1;
  constexpr int bpp = N / ROWS;
  constexpr int NG = N * bpp;  // row groups
  __shared__ double2 buf[NF * LDN];
  __shared__ double2 tw[x_twreg<N>() ? 1 : N];
  __shared__ int tslot[2];
  if constexpr (!x_twreg<N>())
    for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  if (zero_ctr && blockIdx.x == 0 && threadIdx.x < NTILECTR) zero_ctr[threadIdx.x] = 0u;
  const size_t n3 = (size_t)N * N * N;
  auto lds = [&](int f, int i) -> double2* { return &buf[f * LDN + i + (i >> 4)]; };
  constexpr int KV = (ROWS * N + T - 1) / T;
  // a group's voxels: ROWS consecutive rows, so ROWS * N consecutive ids
  // The loads below are issued without branches (a lane past the group reads
  // its last voxel and is skipped by the gather, one without an owner reads
  // the twiddle table and is masked), so that the compiler can count them and
  // wait for exactly the ones a use needs.
  auto load_links = [&](int grp, int32_t* lk) {
#pragma unroll
    for (int k = 0; k < KV; ++k) {
      const int i = threadIdx.x + k * T;
      if constexpr (DM == 0) {
        lk[k] = own[(size_t)grp * (ROWS * N) + min(i, ROWS * N - 1)];
      } else {
        lk[k] = -1;
      }
    }
  };
  // single-owner eigenstrains of a group's voxels (zero elsewhere)
  double2 ev[KV][3];
  auto load_vals = [&](const int32_t* lk) {
#pragma unroll
    for (int k = 0; k < KV; ++k) {
      if constexpr (DM == 0) {
        const double2* f = lk[k] >= 0 ? reinterpret_cast<const double2*>(defs[lk[k]].efd) : twg;
#pragma unroll
        for (int c = 0; c < 3; ++c) ev[k][c] = f[c];
      }
    }
  };
  TileWalk walk(NG, nullptr, tslot);
  int grp = walk.first();
  const int hi = walk.hi;
  int32_t link[KV], nlink[KV];
  if (grp < hi) {
    load_links(grp, link);
    load_vals(link);
  }
  const auto twp = x_twiddles<N, NF, T>(tw, twg);
  // Nothing loaded so far stays pending into the loop: the loop's waits are
  // then counted from its own steady state alone (with loads of the set-up
  // still in flight at entry, each wait would have to cover them, and in
  // every later pass it would also wait for the stores of the group before).
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int it = 0; grp < hi; ++it) {
    const int gn = walk.next(grp, it);
    // past the range the loads repeat the current group, unused (so that no
    // branch makes their count uncertain)
    load_links(gn < hi ? gn : grp, nlink);
    const int z = grp / bpp;
    const int y0 = (grp % bpp) * ROWS;
    // gather the rows' six components into the transform inputs (xx + i yy, ...)
#pragma unroll
    for (int k = 0; k < KV; ++k) {
      const int i = threadIdx.x + k * T;
      if (i < ROWS * N) {
        const int r = i / N, x = i - r * N;
        double e[6];
        if (DM == 1) {
          const size_t v = ((size_t)z * N + y0 + r) * N + x;
#pragma unroll
          for (int c = 0; c < 6; ++c) e[c] = dense[c * n3 + v];
        } else if (DM == 2) {
          const double2* vp = reinterpret_cast<const double2*>(dense + 6 * (((size_t)z * N + y0 + r) * N + x));
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            const double2 t = vp[p];
            e[2 * p] = t.x;
            e[2 * p + 1] = t.y;
          }
        } else {  // one owner (loaded with the group before), or none; several: below
          const bool one = link[k] >= 0;
#pragma unroll
          for (int p = 0; p < 3; ++p) {
            e[2 * p] = one ? ev[k][p].x : 0.0;
            e[2 * p + 1] = one ? ev[k][p].y : 0.0;
          }
        }
#pragma unroll
        for (int p = 0; p < 3; ++p) st2(lds(3 * r + p, x), make_double2(e[2 * p], e[2 * p + 1]));
      }
    }
    if constexpr (DM == 0) {
      // voxels of several owners: the exact fixed-point sum over the chain
#pragma unroll
      for (int k = 0; k < KV; ++k) {
        const int i = threadIdx.x + k * T;
        if (i < ROWS * N && link[k] < -1) {
          const int r = i / N, x = i - r * N;
          double e[6];
          decode_voxel(link[k], lnk, defs, e, max_links);
#pragma unroll
          for (int p = 0; p < 3; ++p) st2(lds(3 * r + p, x), make_double2(e[2 * p], e[2 * p + 1]));
        }
      }
    }
    __syncthreads();
    auto from_lds = [&](int f, int i) { return ld2(lds(f, i)); };
    auto to_lds = [&](int f, int i, double2 v) { st2(lds(f, i), v); };
    transform<N, false, Map::Row, NF, T, true, true>(twp, from_lds, from_lds, to_lds, to_lds);
    __syncthreads();
    load_vals(nlink);
    // Hermitian split of the three pair transforms of a row into the six
    // interleaved half-spectrum components.  FP64 storage: one output value per
    // thread, so consecutive threads write consecutive 16-byte values of the
    // row; FP32 storage: one bin (six values, 48 bytes) per thread, which
    // halves the LDS reads and index work where the narrower writes matter less.
    // The loops run over bins k < n/2; the thread of bin 0 of a row also does
    // its bin n/2 (k = n/2 is its own mirror), so no loop pass is left with two
    // busy threads.
    if constexpr (sizeof(S) == 8) {
      auto value = [&](int r, int k, int c) {
        const int p = c >> 1;
        const double2 zk = ld2(lds(3 * r + p, k));
        const double2 zc = conjd(ld2(lds(3 * r + p, k == 0 ? 0 : N - k)));
        const double2 v = (c & 1) ? make_double2(0.5 * (zk.y - zc.y), -0.5 * (zk.x - zc.x))
                                  : make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y));
        st2(spec + spec_at(z, y0 + r, k, c, N, P), v);
      };
      for (int e = threadIdx.x; e < ROWS * (N / 2) * 6; e += T) {
        const int r = e / ((N / 2) * 6), q = e % ((N / 2) * 6), k = q / 6, c = q % 6;
        value(r, k, c);
        if (k == 0) value(r, N / 2, c);
      }
    } else {
      auto bin = [&](int r, int k) {
        typename Cplx<S>::T* const out = spec + spec_at(z, y0 + r, k, 0, N, P);
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const double2 zk = ld2(lds(3 * r + p, k));
          const double2 zc = conjd(ld2(lds(3 * r + p, k == 0 ? 0 : N - k)));
          st2(out + 2 * p, make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y)));
          st2(out + 2 * p + 1, make_double2(0.5 * (zk.y - zc.y), -0.5 * (zk.x - zc.x)));
        }
      };
      // a compile-time trip count, so that the compiler counts the stores
      // (the next group's gather then waits for its loads and leaves these
      // in flight)
      constexpr int NB = ROWS * (N / 2);
#pragma unroll
      for (int q0 = 0; q0 < (NB + T - 1) / T; ++q0) {
        const int e = threadIdx.x + q0 * T;
        if (NB % T == 0 || e < NB) {
          const int r = e / (N / 2), k = e % (N / 2);
          bin(r, k);
          if (k == 0) bin(r, N / 2);
        }
      }
    }
    __syncthreads();  // the next group rewrites the LDS rows
#pragma unroll
    for (int k = 0; k < KV; ++k) link[k] = nlink[k];
    grp = gn;
  }
}

// Update variant: the rows of the eigenstrain change
// dE = E_new chi_new - E_old chi_old (E: E_old in [0, 6), E_new in [6, 12))
// are built in LDS from the two footprint lists (new ids = old ids shifted by
// (sx, sy, sz) voxels when new_ids == nullptr), for rows y in [y_lo, y_lo+y_len),
// z in [z_lo, z_lo+z_len) (cyclic); other rows are zero and never touched.
// One row block (ROWS rows of one z plane) of one move; buf and tw are the
// caller's LDS (tw filled).
template <int N, typename S>
__device__ __forceinline__ void xfs_block(double2* buf, const double2* tw, const int32_t* __restrict__ old_ids,
                                          int old_cnt, const int32_t* __restrict__ new_ids, int new_cnt, int sx, int sy,
                                          int sz, const double* __restrict__ E, typename Cplx<S>::T* __restrict__ spec,
                                          int P, int y_lo, int y_len, int z_lo, int blk) {
  constexpr int ROWS = x_rows(N);
  constexpr int NF = 3 * ROWS;
  constexpr int T = pick_T(max_nb(N, NF));
  constexpr int LDN = N + N / 16 + 1;
  constexpr int NH = N / 2 + 1;
  if (!new_ids) new_cnt = old_cnt;
  for (int i = threadIdx.x; i < NF * LDN; i += T) buf[i] = make_double2(0.0, 0.0);
  const int rb = (y_len + ROWS - 1) / ROWS;
  const int zi = blk / rb;
  const int y0i = (blk % rb) * ROWS;
  int z = z_lo + zi;
  if (z >= N) z -= N;
  __syncthreads();
  auto lds = [&](int f, int i) -> double2& { return buf[f * LDN + i + (i >> 4)]; };
  // scatter sgn * Ev of the voxels that fall in this block's rows (one row per y)
  auto scatter = [&](int id, double sgn, const double* Ev) {
    const int x = id % N, y = (id / N) % N, zz = id / (N * N);
    if (zz != z) return;
    int yi = y - y_lo;
    if (yi < 0) yi += N;
    yi -= y0i;
    if (yi < 0 || yi >= ROWS || y0i + yi >= y_len) return;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      double2& slot = lds(3 * yi + p, x);
      slot.x += sgn * Ev[2 * p];
      slot.y += sgn * Ev[2 * p + 1];
    }
  };
  // Each voxel is owned by one thread per list pass; a voxel can sit in both
  // lists, so the two passes are separated by a barrier.
  for (int i = threadIdx.x; i < old_cnt; i += T) scatter(old_ids[i], -1.0, E);
  __syncthreads();
  for (int i = threadIdx.x; i < new_cnt; i += T) {
    int id;
    if (new_ids) {
      id = new_ids[i];
    } else {
      const int o = old_ids[i];
      int x = o % N + sx, y = (o / N) % N + sy, zz = o / (N * N) + sz;
      x = (x % N + N) % N;
      y = (y % N + N) % N;
      zz = (zz % N + N) % N;
      id = (zz * N + y) * N + x;
    }
    scatter(id, 1.0, E + 6);
  }
  __syncthreads();
  auto from_lds = [&](int f, int i) { return lds(f, i); };
  auto to_lds = [&](int f, int i, double2 v) { lds(f, i) = v; };
  transform<N, false, Map::Row, NF, T, true, true>(tw, from_lds, from_lds, to_lds, to_lds);
  __syncthreads();
  for (int e = threadIdx.x; e < ROWS * NH * 6; e += T) {
    const int yi = e / (NH * 6), q = e % (NH * 6), k = q / 6, c = q % 6, p = c >> 1;
    if (y0i + yi >= y_len) continue;
    int y = y_lo + y0i + yi;
    if (y >= N) y -= N;
    const double2 zk = lds(3 * yi + p, k);
    const double2 zc = conjd(lds(3 * yi + p, k == 0 ? 0 : N - k));
    const double2 v = (c & 1) ? make_double2(0.5 * (zk.y - zc.y), -0.5 * (zk.x - zc.x))
                              : make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y));
    st2(spec + spec_at(z, y, k, c, N, P), v);
  }
  __syncthreads();  // the caller's next block rewrites LDS
}

template <int N, typename S>
__global__ __launch_bounds__(pick_T(max_nb(N, 3 * x_rows(N)))) void k_x_forward_sparse(
    const int32_t* __restrict__ old_ids, const int32_t* __restrict__ old_cnt_p, const int32_t* __restrict__ new_ids,
    int new_cnt, int sx, int sy, int sz, const double* __restrict__ E, typename Cplx<S>::T* __restrict__ spec, int P,
    int y_lo, int y_len, int z_lo, const double2* __restrict__ twg, uint32_t* __restrict__ zero_ctr) {
  constexpr int NF = 3 * x_rows(N);
  constexpr int T = pick_T(max_nb(N, NF));
  constexpr int LDN = N + N / 16 + 1;
  __shared__ double2 buf[NF * LDN];
  __shared__ double2 tw[N];
  if (zero_ctr && blockIdx.x == 0 && threadIdx.x < NTILECTR) zero_ctr[threadIdx.x] = 0u;
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  xfs_block<N, S>(buf, tw, old_ids, *old_cnt_p, new_ids, new_cnt, sx, sy, sz, E, spec, P, y_lo, y_len, z_lo,
                  blockIdx.x);
}

// Batched hops: the row blocks of every job, job after job, over a fixed grid
// (a block takes every gridDim-th one).
template <int N, typename S>
__global__ __launch_bounds__(pick_T(max_nb(N, 3 * x_rows(N)))) void k_x_forward_sparse_batch(
    const HopJob* __restrict__ jobs, int njob, int P, const double2* __restrict__ twg, uint32_t* __restrict__ zero_ctr) {
  constexpr int NF = 3 * x_rows(N);
  constexpr int T = pick_T(max_nb(N, NF));
  constexpr int LDN = N + N / 16 + 1;
  __shared__ double2 buf[NF * LDN];
  __shared__ double2 tw[N];
  if (zero_ctr && blockIdx.x == 0 && threadIdx.x < NTILECTR) zero_ctr[threadIdx.x] = 0u;
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  int total = 0;
  for (int j = 0; j < njob; ++j) total += jobs[j].xitems;
  for (int item = blockIdx.x; item < total; item += gridDim.x) {
    int j = 0, first = 0;
    while (item >= first + jobs[j].xitems) first += jobs[j++].xitems;
    const HopJob& J = jobs[j];
    xfs_block<N, S>(buf, tw, J.ids + J.slot, J.cnt[J.idx], nullptr, 0, J.sx, J.sy, J.sz, J.E12,
                    (typename Cplx<S>::T*)J.spec, P, J.ylo, J.ylen, J.zlo, item - first);
  }
}

// --------------------------------------------------------------- y / z pencils
//
// A tile is WX consecutive kx columns x all six components (6 WX transforms)
// of one z plane (y pass) or one y row (z pass), transformed along y or z.  In
// the component-interleaved layout every row of the tile is one contiguous
// run of 6 WX values; thread lane f = 6 w + c keeps its (column, component)
// across butterflies (the workgroup size is a multiple of 6 WX).  The last kx
// tile holds the n/2 column and idle lanes.

// largest radix of the pencil factorisation
template <int N>
constexpr int pencil_rmax() {
  constexpr Plan2 P = plan_of(N);
  return P.r[0] > P.r[1] ? (P.r[0] > P.r[2] ? P.r[0] : P.r[2]) : (P.r[1] > P.r[2] ? P.r[1] : P.r[2]);
}

// kx columns per tile: LDS for 6 WX transforms of N points stays at 48 KB
template <int N, typename LT>
constexpr int pencil_wx() {
  constexpr int w = sizeof(LT) == 8 ? 4 : 2;
  return N >= 512 ? w / 2 : w;
}

// Threads of a tile pass over NF transforms: one butterfly per thread in the
// widest-radix stage.  With a direct radix that stage has few butterflies, so
// the size is set by the other stages instead: the least multiple of NF that
// fills whole wavefronts.
template <int N>
constexpr int tile_threads(int NF, int rmax) {
  if (!has_direct(plan_of(N)) && !has_direct(plan_fused(N))) return NF * (N / rmax);
  int t = NF;
  while (t % 64) t += NF;
  return t;
}

template <int N, typename LT>
constexpr int pencil_threads() {
  return tile_threads<N>(6 * pencil_wx<N, LT>(), pencil_rmax<N>());
}

// the pencil pass prefetches the next tile's operands (FP32 storage, plans
// without a direct radix)
template <int N, typename S>
constexpr bool pencil_pipe() {
  return sizeof(S) == 4 && !has_direct(plan_of(N));
}

// Tiles of a batch of hops: job j holds cnt(j) consecutive tiles; (job, local
// tile) of tile t by a walk over the (at most MAXBATCH) jobs.
template <class Count>
__device__ __forceinline__ int job_of_tile(int t, int njob, Count&& cnt, int& local) {
  int j = 0, first = 0;
  while (j + 1 < njob && t >= first + cnt(j)) first += cnt(j++);
  local = t - first;
  return j;
}

// BATCH: the tiles of njob hops of a batch (jobs), job after job: a job's
// spectrum and (y pass, PRUNE) its planes and input rows come from its record;
// spec, pr and ntiles are then unused.
template <int N, typename S, bool INV, typename LT, bool PRUNE, int AXIS, bool BATCH = false>
__global__ __launch_bounds__((pencil_threads<N, LT>())) void k_pencil(typename Cplx<S>::T* __restrict__ spec,
                                                                     Prune pr, const double2* __restrict__ twg,
                                                                     int ntiles, uint32_t* __restrict__ ctr,
                                                                     const HopJob* __restrict__ jobs = nullptr,
                                                                     int njob = 0) {
  constexpr int WX = pencil_wx<N, LT>();
  constexpr int NF = 6 * WX;
  constexpr int T = pencil_threads<N, LT>();
  constexpr int NH = N / 2 + 1;
  constexpr int KB = (NH + WX - 1) / WX;
  constexpr Plan2 PL = plan_of(N);
  constexpr int R0 = PL.r[0];
  constexpr int NOP = ((NF * (N / R0) + T - 1) / T) * R0;  // first-stage operands per thread
  static_assert(T % NF == 0, "a thread must keep its column across butterflies");
  constexpr int P = spec_pitch(N, sizeof(S) == 8);
  // element stride along the transform axis; all offsets fit 32 bits
  constexpr int SI = AXIS == 1 ? 6 * P : 6 * N * P;
  static_assert(6LL * N * N * P < (1LL << 31), "32-bit element offsets");
  using C2 = typename Cplx<S>::T;
  __shared__ LT buf[N * NF];
  __shared__ double2 tw[N];
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  // tiles per job in a batch: the planes of its pruned range (y pass, PRUNE)
  // or all of them
  auto job_tiles = [&](int j) { return (PRUNE && AXIS == 1 ? jobs[j].zlen : N) * KB; };
  if constexpr (BATCH) {
    ntiles = 0;
    for (int j = 0; j < njob; ++j) ntiles += job_tiles(j);
  }
  // the spectrum, pruning and local tile index of tile t
  auto tile_of = [&](int t, C2*& base, Prune& p) -> int {
    if constexpr (BATCH) {
      int lt;
      const int j = job_of_tile(t, njob, job_tiles, lt);
      base = (C2*)jobs[j].spec;
      p = Prune{jobs[j].ylo, jobs[j].ylen, jobs[j].zlo, jobs[j].zlen};
      return lt;
    } else {
      base = spec;
      p = pr;
      return t;
    }
  };
  auto in_range_of = [&](const Prune& p, int i) {
    if (!PRUNE) return true;
    int d = i - p.in_lo;
    if (d < 0) d += N;
    return d < p.in_len;
  };
  // lane f's column in tile t (the base of the spectrum if the lane is idle)
  auto column = [&](int t, int f, bool& valid, Prune& p) -> C2* {
    C2* base;
    const int lt = tile_of(t, base, p);
    const int o = lt / KB, kx = (lt % KB) * WX + f / 6;
    valid = kx < NH;
    if (!valid) return base;
    if (AXIS == 1) {
      int z = p.z_lo + o;
      if (z >= N) z -= N;
      return base + (z * N * P + kx) * 6 + f % 6;
    }
    return base + (o * P + kx) * 6 + f % 6;
  };
  // FP32 storage: raw first-stage operands of the next tile are loaded while
  // the current one is transformed (rows outside the input range read row
  // in_lo, a cache hit, and are zeroed when consumed).  FP64 storage would
  // need twice the registers for them and loads each tile's operands in turn,
  // and so does a plan with a direct radix.
  constexpr bool PIPE = pencil_pipe<N, S>();
  C2 nxt[NOP];
  auto fetch = [&](int t, int tid) {
    if constexpr (!PIPE) return;
    bool v;
    Prune p;
    const C2* colp = column(t, tid % NF, v, p);
    for_operands<N, R0, Map::Pencil, NF, T>(
        [&](int, int i, int slot) { nxt[slot] = colp[(in_range_of(p, i) ? i : p.in_lo) * SI]; }, tid);
  };
  auto from_lds = [&](int f, int i) { return ld2(&buf[i * NF + f]); };
  auto to_lds = [&](int f, int i, double2 v) { st2(&buf[i * NF + f], v); };
  __shared__ int tslot[2];
  TileWalk walk(ntiles, PIPE ? ctr : nullptr, tslot);
  walk.claim_first();
  __syncthreads();
  int t = walk.first();
  const int hi = walk.hi;
  if (t < hi) fetch(t, threadIdx.x);
  __syncthreads();
  // two equal radices: the second stage gives a thread the same butterfly in
  // every tile, so its twiddles stay in registers (FP32 storage; with FP64
  // storage the extra registers would cost occupancy)
  constexpr bool TWREG = PL.nstage == 2 && PL.r[0] == PL.r[1] && NF * (N / R0) == T && sizeof(S) == 4;
  const auto twp = [&] {
    if constexpr (TWREG)
      return make_twreg<N, R0, R0, Map::Pencil, NF, T>(tw, threadIdx.x);
    else
      return (const double2*)tw;
  }();
  for (int it = 0; t < hi; ++it) {
    const int tn = walk.next(t, it);
    const uint32_t claim = walk.claim_issue();
    // laundered thread index: index arithmetic is redone per tile instead of
    // being held in registers across the loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    bool valid;
    Prune pt;
    C2* const colp = column(t, tid % NF, valid, pt);
    // a lane past the last column transforms whatever its loads returned
    // (finite spectrum values) and stores nothing
    // without the prefetch every operand is loaded (a row outside the input
    // range reads row in_lo, a cache hit) and zeroed afterwards, so that the
    // loads are issued together rather than one branch at a time
    auto load0 = [&](int, int i, int slot) -> double2 {
      const bool in = !PRUNE || (valid && in_range_of(pt, i));
      if constexpr (PIPE) return in ? ld2(&nxt[slot]) : make_double2(0.0, 0.0);
      const double2 v = ld2(colp + (in ? i : pt.in_lo) * SI);
      return in ? v : make_double2(0.0, 0.0);
    };
    auto store_last = [&](int, int i, double2 v) {
      if (valid) st2(colp + i * SI, v);
    };
    const bool more = tn < hi;
    if constexpr (PL.nstage == 1) {
      stage<N, R0, 1, INV, Map::Pencil, NF, T>(tw, load0, store_last, false, tid);
      if (more) fetch(tn, tid);
    } else {
      stage<N, R0, 1, INV, Map::Pencil, NF, T>(tw, load0, to_lds, false, tid);
      if (more) fetch(tn, tid);
      __syncthreads();
      if constexpr (PL.nstage == 2) {
        stage<N, PL.r[1], R0, INV, Map::Pencil, NF, T>(twp, from_lds, store_last, false, tid);
      } else {
        stage<N, PL.r[1], R0, INV, Map::Pencil, NF, T>(tw, from_lds, to_lds, true, tid);
        __syncthreads();
        stage<N, PL.r[2], R0 * PL.r[1], INV, Map::Pencil, NF, T>(tw, from_lds, store_last, false, tid);
      }
    }
    walk.claim_store(it, claim);
    __syncthreads();  // the next tile's first stage rewrites LDS
    t = tn;
  }
}

// ------------------------------------------- z-forward + Green + z-inverse (fused)
//
// One workgroup owns W kx columns of one ky row for all six components (6 W
// transforms of length N along z, each row of the tile one contiguous run of
// the interleaved spectrum) in one LDS tile: forward transforms, the Green
// step per bin in place, inverse transforms.  The spectrum is read and written
// once per solve instead of three times, and every stage has all six
// components' butterflies to spread over the workgroup.

template <int N>
struct FusedPlan {
  static constexpr Plan2 P = plan_fused(N);
  static constexpr int NSTG = P.nstage;
  static constexpr int R0 = P.r[0], R1 = P.r[1], R2 = P.r[2];
  static constexpr int RL = NSTG == 1 ? R0 : (NSTG == 2 ? R1 : R2);
  static constexpr int I0 = RL;
  static constexpr int I1 = NSTG == 1 ? 1 : (NSTG == 2 ? R0 : R1);
  static constexpr int I2 = NSTG == 3 ? R0 : 1;
};

// Two-column tiles without the operand prefetch and register twiddles (which
// would take their registers) for the even lengths 64 .. 256: three or more
// resident workgroups per CU hide more latency than one four-column one with
// the prefetch (FP32 pass at 256^3 0.33 -> 0.27 ms, 240^3 0.33 -> 0.27, 160^3
// 0.098 -> 0.077, 128^3 0.070 -> 0.042, 64^3 0.030 -> 0.013).  At 512 the
// two-column tile keeps the prefetch (without it 3.6 -> 4.2 ms), and the odd
// 129 keeps four columns (two: 0.83 -> 1.03 ms per solve).
template <int N>
constexpr bool zg_narrow() {
  return N >= 64 && N <= 256 && !has_direct(plan_fused(N));
}

// columns per tile: four, or two for the lengths above, at N = 512 (where a
// four-column tile would not fit) and with FP64 storage from N = 256 on
template <int N, typename S>
constexpr int zg_width() {
  return (N >= 512 || zg_narrow<N>() || (sizeof(S) == 8 && N >= 256)) ? 2 : 4;
}

// one butterfly per thread in the widest-radix stage; a multiple of the 6 W
// transforms, so every lane keeps its transform
template <int N, typename S>
constexpr int zg_fft_threads() {
  using FP = FusedPlan<N>;
  constexpr int rmax = FP::R0 > FP::R1 ? (FP::R0 > FP::R2 ? FP::R0 : FP::R2) : (FP::R1 > FP::R2 ? FP::R1 : FP::R2);
  return tile_threads<N>(6 * zg_width<N, S>(), rmax);
}

// Workgroup size: the butterfly threads, or for the two-column tile at 256
// four whole wavefronts (the fourth idle in the transform stages, every one
// busy in the Green step): three resident workgroups then put three
// wavefronts on every SIMD, where three-wavefront groups would put three on
// one SIMD and two on the others, and every workgroup has a wavefront on the
// busiest one.
template <int N, typename S>
constexpr int zg_threads() {
  constexpr int t = zg_fft_threads<N, S>();
  return (N == 256 && zg_narrow<N>() && zg_width<N, S>() == 2) ? ((t + 255) / 256) * 256 : t;
}

template <int N, typename S>
constexpr bool zg_pipe() {
  return sizeof(S) == 4 && !zg_narrow<N>() && !has_direct(plan_fused(N));
}

// Wavefronts per SIMD the compiler must leave registers for: three for the
// two-column tiles of 64 .. 256 (three resident workgroups; at 256 twelve
// wavefronts per CU), else one (no bound beyond the workgroup size).
template <int N, typename S>
constexpr int zg_waves_per_eu() {
  return zg_narrow<N>() ? 3 : 1;
}

// LDS row swizzle: the low three bits of the z index are XORed with the next
// three, so stride-R stores of the first stages spread over all banks.
__device__ __forceinline__ int zg_swz(int i) { return (i & ~7) | ((i ^ (i >> 3)) & 7); }

// BATCH: the tiles of njob hops of a batch, job after job (NT each), a job's
// spectrum and input planes from its record (spec and pr unused).
template <int N, typename S, bool PRUNE, bool ROT, bool BATCH = false>
__global__ __launch_bounds__((zg_threads<N, S>())) __attribute__((amdgpu_waves_per_eu(zg_waves_per_eu<N, S>())))
void k_zgreen(typename Cplx<S>::T* __restrict__ spec, Cubic C,
                                                                Prune pr, const double2* __restrict__ twg,
                                                                uint32_t* __restrict__ ctr,
                                                                const HopJob* __restrict__ jobs = nullptr,
                                                                int njob = 0) {
  using FP = FusedPlan<N>;
  constexpr int W = zg_width<N, S>();
  constexpr int T = zg_threads<N, S>();
  constexpr int NH = N / 2 + 1;
  constexpr int KB = (NH + W - 1) / W;
  constexpr int NT = N * KB;  // tiles
  constexpr int NF = 6 * W;   // transforms per tile
  constexpr int R0 = FP::R0, R1 = FP::R1, R2 = FP::R2;
  constexpr int NOP = ((NF * (N / R0) + T - 1) / T) * R0;  // first-stage operands per thread
  static_assert(FP::NSTG >= 2, "the first stage must not be the last");
  using C2 = typename Cplx<S>::T;
  // FP64 tile in both storage precisions: rounding the whole spectrum to FP32
  // next to the Green step and between stages roughly doubles the FP32-storage
  // energy error, while the extra LDS costs little here
  __shared__ double2 buf[6 * N * W];
  __shared__ double2 tw[N];
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  constexpr int P = spec_pitch(N, sizeof(S) == 8);
  constexpr int SI = 6 * N * P;  // kz stride; all offsets fit 32 bits
  static_assert(6LL * N * N * P < (1LL << 31), "32-bit element offsets");
  // the row swizzle permutes whole groups of eight rows; it pays for
  // four-column tiles, while with two columns its index arithmetic costs more
  // than the bank conflicts it removes (0.27 against 0.28 ms at 256^3)
  constexpr bool SWZ = N % 8 == 0 && W == 4;
  auto lds = [&](int f, int i) -> double2* { return &buf[__umul24(SWZ ? zg_swz(i) : i, NF) + f]; };
  auto from_lds = [&](int f, int i) { return ld2(lds(f, i)); };
  auto to_lds = [&](int f, int i, double2 v) { st2(lds(f, i), v); };
  // the spectrum and input planes of tile t, and its index within its job
  auto tile_of = [&](int t, C2*& base, Prune& p) -> int {
    if constexpr (BATCH) {
      const int j = t / NT;
      base = (C2*)jobs[j].spec;
      p = Prune{jobs[j].zlo, jobs[j].zlen, 0, N};
      return t - j * NT;
    } else {
      base = spec;
      p = pr;
      return t;
    }
  };
  auto in_z_of = [&](const Prune& p, int i) {
    if (!PRUNE) return true;
    int d = i - p.in_lo;
    if (d < 0) d += N;
    return d < p.in_len;
  };
  // FP32 storage: raw first-stage operands of the next tile, loaded while the
  // current one is transformed (rows outside the input range read row in_lo
  // instead, a cache hit, and are zeroed when consumed).  FP64 storage, and
  // a plan with a direct radix (whose operands already fill the registers),
  // load each tile's operands in turn.
  constexpr bool PIPE = zg_pipe<N, S>();
  C2 nxt[NOP];
  auto fetch = [&](int t, int tid) {
    if constexpr (!PIPE) return;
    C2* base;
    Prune p;
    const int lt = tile_of(t, base, p);
    const int f0 = tid % NF, kx = (lt % KB) * W + f0 / 6;
    const C2* col0 = base + (kx < NH ? ((lt / KB) * P + kx) * 6 + f0 % 6 : 0);
    for_operands<N, R0, Map::Pencil, NF, T>(
        [&](int, int i, int slot) { nxt[slot] = col0[(in_z_of(p, i) ? i : p.in_lo) * SI]; }, tid);
  };
  __shared__ int tslot[2];
  TileWalk walk(BATCH ? NT * njob : NT, PIPE ? ctr : nullptr, tslot);
  walk.claim_first();
  __syncthreads();
  int t = walk.first();
  const int hi = walk.hi;
  if (t < hi) fetch(t, threadIdx.x);
  __syncthreads();
  // two equal radices: the twiddled stage of either direction gives a thread
  // the same butterfly in every tile, so its twiddles stay in registers (with
  // the prefetch, FP32 storage; otherwise the extra registers would cost
  // occupancy)
  constexpr bool TWREG = FP::NSTG == 2 && R0 == R1 && PIPE;
  const auto twz = [&] {
    if constexpr (TWREG)
      return make_twreg<N, R1, R0, Map::Pencil, NF, T>(tw, threadIdx.x);
    else
      return (const double2*)tw;
  }();
  for (int it = 0; t < hi; ++it) {
    const int tn = walk.next(t, it);
    const uint32_t claim = walk.claim_issue();
    // the thread index is laundered per tile so that the many index
    // expressions derived from it are recomputed, not held in registers
    // across the loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    C2* tbase;
    Prune pt;
    const int lt = tile_of(t, tbase, pt);
    const int ky = lt / KB;
    const int f0 = tid % NF, w = f0 / 6;  // lane f = 6 w + c keeps its column
    const int kx = (lt % KB) * W + w;
    const bool valid = kx < NH;
    C2* const col0 = tbase + (valid ? (ky * P + kx) * 6 + f0 % 6 : 0);
    // a lane past the last column transforms whatever its loads returned
    // (finite spectrum values), takes no part in the Green step and stores
    // nothing
    // without the prefetch every operand is loaded (a plane outside the input
    // range reads plane in_lo, a cache hit) and zeroed afterwards, so that the
    // loads are issued together rather than one branch at a time
    auto load0 = [&](int, int i, int slot) -> double2 {
      const bool in = !PRUNE || (valid && in_z_of(pt, i));
      if constexpr (PIPE) return in ? ld2(&nxt[slot]) : make_double2(0.0, 0.0);
      const double2 v = ld2(col0 + (in ? i : pt.in_lo) * SI);
      return in ? v : make_double2(0.0, 0.0);
    };
    stage<N, R0, 1, false, Map::Pencil, NF, T>(tw, load0, to_lds, false, tid);
    if (tn < hi) fetch(tn, tid);
    __syncthreads();
    if constexpr (R2 == 1) {
      stage<N, R1, R0, false, Map::Pencil, NF, T>(twz, from_lds, to_lds, true, tid);
    } else {
      stage<N, R1, R0, false, Map::Pencil, NF, T>(tw, from_lds, to_lds, true, tid);
      __syncthreads();
      stage<N, R2, R0 * R1, false, Map::Pencil, NF, T>(tw, from_lds, to_lds, true, tid);
    }
    __syncthreads();
    // Green step: one bin (all six components) per iteration, in place.  For
    // a rotated crystal eps*_hat arrives in the cube frame (the rasterised
    // eigenstrain is kept there), the cubic operator takes rotated labels, and
    // a second loop over the same bins of each thread turns sigma_hat back to
    // the cell frame (one loop for both pushed the FP32 tile past 256 VGPRs).
#pragma unroll 1
    for (int b = tid; b < N * W; b += T) {
      const int bw = b % W, kz = b / W, bkx = kx - w + bw;
      if (bkx >= NH) continue;
      double2 e[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = from_lds(bw * 6 + c, kz);
      if constexpr (ROT)
        green_core_rot(e, bkx, ky, kz, N, C);
      else
        green_bin(e, bkx, ky, kz, N, C);
#pragma unroll
      for (int c = 0; c < 6; ++c) to_lds(bw * 6 + c, kz, e[c]);
    }
    if constexpr (ROT) {
#pragma unroll 1
      for (int b = tid; b < N * W; b += T) {
        const int bw = b % W, kz = b / W;
        if (kx - w + bw >= NH) continue;
        double2 e[6], r[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) e[c] = from_lds(bw * 6 + c, kz);
        rot6(C.frm + 36, e, r);
#pragma unroll
        for (int c = 0; c < 6; ++c) to_lds(bw * 6 + c, kz, r[c]);
      }
    }
    __syncthreads();
    auto store_last = [&](int, int i, double2 v) {
      if (valid) st2(col0 + i * SI, v);
    };
    transform_plan<N, FP::I0, FP::I1, FP::I2, true, Map::Pencil, NF, T, NF, true, false>(twz, from_lds, from_lds,
                                                                                    to_lds, store_last, tid);
    walk.claim_store(it, claim);
    __syncthreads();  // the next tile's first stage rewrites the tile
    t = tn;
  }
}

// Pointwise Green step over the half spectrum (one thread per bin).
template <typename S>
__global__ __launch_bounds__(256) void k_green(typename Cplx<S>::T* __restrict__ spec, int n, int P, Cubic C) {
  const int NH = n / 2 + 1;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)n * n * NH) return;
  const int kx = (int)(t % NH);
  const size_t r = t / NH;
  const int ky = (int)(r % n), kz = (int)(r / n);
  typename Cplx<S>::T* const bin = spec + spec_at(kz, ky, kx, 0, n, P);
  double2 e[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = ld2(bin + c);
  if (C.frm)
    green_bin_rot(e, kx, ky, kz, n, C);
  else
    green_bin(e, kx, ky, kz, n, C);
#pragma unroll
  for (int c = 0; c < 6; ++c) st2(bin + c, e[c]);
}

// --------------------------------------------------------- x inverse (C2R) + stress

// ACC: the result is added to a field of the stress's layout: add3 (a stress
// held beside the solve, such as that of dislocation loops), or sig itself when
// add3 is null.
// BG: the stress planes of dislocation lines along the axes in bg_mask
// ([3][n^2][6], FP64) are added as well.
// BATCH: njob hops of a batch, N N / ROWS blocks each, a job's spectrum and
// stress from its record (spec and sig unused).
// MASK: the stress is stored only at voxels some defect covers (own[v] & keep
// != -1), the voxels an energy reduction reads; the others keep what they
// held.  keep = 0 stores every voxel: the pass that forms the whole field runs
// this same code, so a covered voxel gets the same bits either way (separate
// code for the two could fuse multiplies and adds differently).
template <int N, typename S, bool ACC, bool BG, bool BATCH = false, bool MASK = false>
__global__ __launch_bounds__(pick_T(max_nb(N, 3 * x_rows(N)))) void k_x_inverse(
    const typename Cplx<S>::T* __restrict__ spec, double* __restrict__ sig, const double* __restrict__ mean6,
    const double2* __restrict__ twg, const double* __restrict__ bg, int bg_mask,
    const HopJob* __restrict__ jobs = nullptr, const double* add3 = nullptr,
    const int32_t* __restrict__ own = nullptr, int32_t keep = -1) {
  constexpr int ROWS = x_rows(N);
  constexpr int NF = 3 * ROWS;
  constexpr int T = pick_T(max_nb(N, NF));
  constexpr int LDN = N + N / 16 + 1;
  constexpr int P = spec_pitch(N, sizeof(S) == 8);
  constexpr int N3 = N * N * N;
  static_assert(6LL * N * N * P < (1LL << 31) && 6LL * N3 < (1LL << 31), "32-bit element offsets");
  __shared__ double2 buf[NF * LDN];
  __shared__ double2 tw[N];
  __shared__ double mean_s[6];
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  if (threadIdx.x < 6) mean_s[threadIdx.x] = mean6[threadIdx.x];
  const int bpp = N / ROWS;
  int blk = blockIdx.x;
  if constexpr (BATCH) {
    const int j = blk / (N * bpp);
    blk -= j * (N * bpp);
    spec = (const typename Cplx<S>::T*)jobs[j].spec;
    sig = jobs[j].sig;
  }
  const int z = blk / bpp;
  const int y0 = (blk % bpp) * ROWS;
  const double scale = 1.0 / (double)N3;
  __syncthreads();
  auto load0 = [&](int f, int k) -> double2 {
    const int p = f % 3, y = y0 + f / 3;
    // components 2p and 2p+1 of bin k (or of its mirror n - k) are adjacent
    const typename Cplx<S>::T* a = spec + ((z * N + y) * P + (k <= N / 2 ? k : N - k)) * 6 + 2 * p;
    double2 A = ld2(a), B = ld2(a + 1);
    if (k > N / 2) {
      A = conjd(A);
      B = conjd(B);
    } else if (k == 0 || (N % 2 == 0 && k == N / 2)) {  // bins that are their own mirror
      A.y = 0.0;
      B.y = 0.0;
    }
    return make_double2(A.x - B.y, A.y + B.x);
  };
  auto from_lds = [&](int f, int i) { return buf[f * LDN + i + (i >> 4)]; };
  auto to_lds = [&](int f, int i, double2 v) { buf[f * LDN + i + (i >> 4)] = v; };
  // sigma is voxel-major, [n^3][6]: components 2p and 2p+1 of a voxel are one
  // aligned 16-byte pair, and the lanes of a store cover whole voxel records
  auto sig_at = [&](int f, int x) -> double2* {
    const int p = f % 3, y = y0 + f / 3;
    return reinterpret_cast<double2*>(sig + (6 * ((z * N + y) * N + x) + 2 * p));
  };
  auto add_at = [&](int f, int x) -> double2 {
    const int p = f % 3, y = y0 + f / 3;
    return *reinterpret_cast<const double2*>((add3 ? add3 : sig) + (6 * ((z * N + y) * N + x) + 2 * p));
  };
  // accumulate: the thread's old values of the last stage's outputs are read
  // before the transform, so their latency overlaps it
  constexpr Plan2 PLX = plan_of(N);
  constexpr int RL = PLX.r[PLX.nstage - 1];
  constexpr int NSL = PLX.nstage == 1 ? 1 : (PLX.nstage == 2 ? PLX.r[0] : PLX.r[0] * PLX.r[1]);
  constexpr int NOUT = ((NF * (N / RL) + T - 1) / T) * RL;
  double2 old[ACC ? NOUT : 1];
  int32_t ow[MASK ? NOUT : 1];
  if constexpr (MASK) {
    bool any = false;
    for_outputs<N, RL, NSL, Map::Row, NF, T>([&](int f, int x, int slot) {
      // keep = 0 (every voxel): the loads all read the map's first entry, one
      // cached line, instead of the whole map
      ow[slot] = own[((z * N + y0 + f / 3) * N + x) & keep] & keep;
      any |= ow[slot] != -1;
    });
    // rows that no defect covers store nothing: their transform is skipped
    if (!__syncthreads_or(any)) return;
  }
  if constexpr (ACC)
    for_outputs<N, RL, NSL, Map::Row, NF, T>([&](int f, int x, int slot) {
      if (!MASK || ow[slot] != -1)
        old[slot] = add_at(f, x);
      else
        old[slot] = make_double2(0.0, 0.0);
    });
  auto store_last = [&](int f, int x, double2 v, int slot) {
    if constexpr (MASK)
      if (ow[slot] == -1) return;
    const int p = f % 3, y = y0 + f / 3;
    double2* s01 = sig_at(f, x);
    double2 r = make_double2(v.x * scale + mean_s[2 * p], v.y * scale + mean_s[2 * p + 1]);
    if constexpr (ACC) {
      const double2 o = old[slot];
      r.x += o.x;
      r.y += o.y;
    }
    if constexpr (BG) {
      const int v[3] = {x, y, z};
      for (int a = 0; a < 3; ++a) {
        if (!(bg_mask & (1 << a))) continue;
        const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
        const double2 o = *reinterpret_cast<const double2*>(bg + ((a * N + v[a2]) * N + v[a1]) * 6 + 2 * p);
        r.x += o.x;
        r.y += o.y;
      }
    }
    *s01 = r;
  };
  transform<N, true, Map::Row, NF, T>(tw, load0, from_lds, to_lds, store_last);
}

// ------------------------------------------------------------------ launchers

// Grid of a tile-loop kernel, a multiple of eight.  Kernels that prefetch the
// next tile (FP32 storage) get as many workgroups as stay resident; the others
// get one tile per workgroup, so tiles overlap through the hardware scheduler.
template <class K>
int tile_grid(K kernel, int threads, int ntiles, bool prefetch) {
  if (!prefetch) return ((ntiles + 7) / 8) * 8;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess)
    return -1;
  const int g = std::min(ncu * std::max(per_cu, 1), ntiles);
  return std::max(8, (g / 8) * 8);
}

template <int N, typename S>
hipError_t go_xf(const int32_t* own, const int2* lnk, const DevDefect* defs, int ndef, const double* dense,
                 void* spec, SpecGeom g, const double2* tw, uint32_t* zero_ctr, hipStream_t s) {
  constexpr int T = pick_T(max_nb(N, 3 * x_rows(N)));
  static_assert(T >= NTILECTR, "the first block zeroes the tile counters");
  const int ngroups = N * (N / x_rows(N));
  using C2 = typename Cplx<S>::T;
  // as many workgroups as stay resident (a multiple of eight), at most one
  // per row group
  const int grid = tile_grid(k_x_forward<N, S, 0>, T, ngroups, true);
  if (grid < 0) return hipErrorInvalidValue;
  if (dense)
    hipLaunchKernelGGL((k_x_forward<N, S, 1>), dim3(grid), dim3(T), 0, s, own, lnk, defs, dense, (C2*)spec, g.P, tw,
                       zero_ctr, ndef);
  else
    hipLaunchKernelGGL((k_x_forward<N, S, 0>), dim3(grid), dim3(T), 0, s, own, lnk, defs, dense, (C2*)spec, g.P,
                       tw, zero_ctr, ndef);
  return hipGetLastError();
}

template <int N, typename S>
hipError_t go_xf_vm(const double* vm, void* spec, SpecGeom g, const double2* tw, hipStream_t s) {
  constexpr int T = pick_T(max_nb(N, 3 * x_rows(N)));
  const int grid = tile_grid(k_x_forward<N, S, 2>, T, N * (N / x_rows(N)), true);
  if (grid < 0 || g.P != spec_pitch(N, sizeof(S) == 8)) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_x_forward<N, S, 2>), dim3(grid), dim3(T), 0, s, (const int32_t*)nullptr,
                     (const int2*)nullptr, (const DevDefect*)nullptr, vm, (typename Cplx<S>::T*)spec, g.P, tw,
                     (uint32_t*)nullptr, 0);
  return hipGetLastError();
}

template <int N, typename S>
hipError_t go_xfs(const int32_t* oi, const int32_t* oc, const int32_t* ni, int nc, int sx, int sy, int sz, const double* E,
                  void* spec, SpecGeom g, int ylo, int ylen, int zlo, int zlen, const double2* tw, uint32_t* zero_ctr,
                  hipStream_t s) {
  constexpr int T = pick_T(max_nb(N, 3 * x_rows(N)));
  static_assert(T >= NTILECTR, "the first block zeroes the tile counters");
  const int grid = zlen * ((ylen + x_rows(N) - 1) / x_rows(N));
  if (grid == 0) return zero_ctr ? launch_fill_i32((int32_t*)zero_ctr, NTILECTR, 0, s) : hipSuccess;
  hipLaunchKernelGGL((k_x_forward_sparse<N, S>), dim3(grid), dim3(T), 0, s, oi, oc, ni, nc, sx, sy, sz, E,
                     (typename Cplx<S>::T*)spec, g.P, ylo, ylen, zlo, tw, zero_ctr);
  return hipGetLastError();
}

// FP32 storage stages the inter-stage exchange in FP32 (half the LDS, so
// twice the columns per tile); FP64 storage keeps FP64 staging.
template <int N, typename S>
hipError_t go_pencil(bool inv, int axis, void* spec, SpecGeom g, Prune pr, const double2* tw, uint32_t* ctr,
                     hipStream_t s) {
  using LT = typename Cplx<S>::T;
  constexpr int T = pencil_threads<N, LT>();
  constexpr int KB = (N / 2 + 1 + pencil_wx<N, LT>() - 1) / pencil_wx<N, LT>();
  const int nouter = axis == 1 ? pr.z_len : N;
  const int ntiles = nouter * KB;
  using C2 = typename Cplx<S>::T;
  const bool prune = pr.in_len < N;
  if (g.P != spec_pitch(N, sizeof(S) == 8) || (axis != 1 && axis != 2)) return hipErrorInvalidValue;
  if (axis == 2 && prune) return hipErrorInvalidValue;  // z pruning runs in the fused z pass
  auto* k = axis == 1 ? (inv ? (prune ? k_pencil<N, S, true, LT, true, 1> : k_pencil<N, S, true, LT, false, 1>)
                             : (prune ? k_pencil<N, S, false, LT, true, 1> : k_pencil<N, S, false, LT, false, 1>))
                      : (inv ? k_pencil<N, S, true, LT, false, 2> : k_pencil<N, S, false, LT, false, 2>);
  const int grid = tile_grid(k, T, ntiles, pencil_pipe<N, S>());
  if (grid < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(grid), dim3(T), 0, s, (C2*)spec, pr, tw, ntiles, ctr, (const HopJob*)nullptr, 0);
  return hipGetLastError();
}

template <int N, typename S, bool ACC, bool BG>
void go_xi_k(const void* spec, double* sig, const double* mean6, const double2* tw, const double* bg, int bg_mask,
             const double* add3, const int32_t* own, bool all, hipStream_t s) {
  constexpr int T = pick_T(max_nb(N, 3 * x_rows(N)));
  const int grid = N * (N / x_rows(N));
  using C2 = typename Cplx<S>::T;
  // with an owner map: the covered voxels, or all of them (all) by the same code
  if (own)
    hipLaunchKernelGGL((k_x_inverse<N, S, ACC, BG, false, true>), dim3(grid), dim3(T), 0, s, (const C2*)spec, sig,
                       mean6, tw, bg, BG ? bg_mask : 0, (const HopJob*)nullptr, add3, own, all ? 0 : -1);
  else
    hipLaunchKernelGGL((k_x_inverse<N, S, ACC, BG>), dim3(grid), dim3(T), 0, s, (const C2*)spec, sig, mean6, tw, bg,
                       BG ? bg_mask : 0, (const HopJob*)nullptr, add3);
}

template <int N, typename S>
hipError_t go_xi(bool acc, const void* spec, double* sig, SpecGeom g, const double* mean6, const double2* tw,
                 const double* bg, int bg_mask, const double* add3, const int32_t* own, bool all, hipStream_t s) {
  if (g.P != spec_pitch(N, sizeof(S) == 8) || (acc && add3) || (acc && own)) return hipErrorInvalidValue;
  if (add3 && bg && bg_mask)
    go_xi_k<N, S, true, true>(spec, sig, mean6, tw, bg, bg_mask, add3, own, all, s);
  else if (acc || add3)
    go_xi_k<N, S, true, false>(spec, sig, mean6, tw, bg, 0, add3, own, all, s);
  else if (bg && bg_mask)
    go_xi_k<N, S, false, true>(spec, sig, mean6, tw, bg, bg_mask, nullptr, own, all, s);
  else
    go_xi_k<N, S, false, false>(spec, sig, mean6, tw, bg, 0, nullptr, own, all, s);
  return hipGetLastError();
}

template <int N, typename S>
hipError_t go_hop_batch(const HopJob* jobs, int njob, SpecGeom g, Cubic C, const double2* tw, uint32_t* ctr,
                        const double* zero6, hipStream_t s) {
  using C2 = typename Cplx<S>::T;
  using LT = typename Cplx<S>::T;
  if (g.P != spec_pitch(N, sizeof(S) == 8) || njob < 1 || njob > MAXBATCH) return hipErrorInvalidValue;
  constexpr bool pipe = pencil_pipe<N, S>(), zpipe = zg_pipe<N, S>();
  constexpr int TX = pick_T(max_nb(N, 3 * x_rows(N)));
  // sparse x forward: a fixed grid walks the row blocks of every job
  hipLaunchKernelGGL((k_x_forward_sparse_batch<N, S>), dim3(256), dim3(TX), 0, s, jobs, njob, g.P, tw, ctr);
  // y forward (pruned planes and rows), fused z pass, y inverse: persistent
  // grids over the jobs' tiles
  constexpr int TP = pencil_threads<N, LT>();
  constexpr int KB = (N / 2 + 1 + pencil_wx<N, LT>() - 1) / pencil_wx<N, LT>();
  const Prune none{0, N, 0, N};
  {
    auto* k = k_pencil<N, S, false, LT, true, 1, true>;
    const int grid = pipe ? tile_grid(k, TP, njob * N * KB, true) : ((njob * N * KB + 7) / 8) * 8;
    if (grid < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(TP), 0, s, (C2*)nullptr, none, tw, 0, ctr, jobs, njob);
  }
  {
    constexpr int W = zg_width<N, S>();
    constexpr int T = zg_threads<N, S>();
    constexpr int NT = N * ((N / 2 + 1 + W - 1) / W);
    auto* k = C.frm ? k_zgreen<N, S, true, true, true> : k_zgreen<N, S, true, false, true>;
    const int grid = tile_grid(k, T, njob * NT, zpipe);
    if (grid < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(T), 0, s, (C2*)nullptr, C, none, tw, ctr + 8, jobs, njob);
  }
  {
    auto* k = k_pencil<N, S, true, LT, false, 1, true>;
    const int grid = tile_grid(k, TP, njob * N * KB, pipe);
    if (grid < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(TP), 0, s, (C2*)nullptr, none, tw, 0, ctr + 16, jobs, njob);
  }
  // accumulating x inverse (a hop's mean-stress change is zero)
  hipLaunchKernelGGL((k_x_inverse<N, S, true, false, true>), dim3(njob * N * (N / x_rows(N))), dim3(TX), 0, s,
                     (const C2*)nullptr, (double*)nullptr, zero6, tw, (const double*)nullptr, 0, jobs);
  return hipGetLastError();
}

}  // namespace

#define EC_FOR_SIZES(X) X(8) X(16) X(24) X(32) X(45) X(48) X(64) X(96) X(128) X(129) X(160) X(240) X(256) X(512)

bool fft_supported(int n) {
  switch (n) {
#define EC_CASE(NN) case NN:
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
    return true;
    default:
      return false;
  }
}

int pencil_width(int n, bool) { return n >= 512 ? 8 : 16; }

hipError_t launch_x_forward(bool fp64, const int32_t* own, const int2* lnk, const DevDefect* defs, int ndef,
                            const double* dense, void* spec, SpecGeom g, const double2* tw, uint32_t* zero_ctr,
                            hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN)                                                                     \
  case NN:                                                                              \
    return fp64 ? go_xf<NN, double>(own, lnk, defs, ndef, dense, spec, g, tw, zero_ctr, s) \
                : go_xf<NN, float>(own, lnk, defs, ndef, dense, spec, g, tw, zero_ctr, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_x_forward_vm(bool fp64, const double* vm, void* spec, SpecGeom g, const double2* tw, hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN) \
  case NN:          \
    return fp64 ? go_xf_vm<NN, double>(vm, spec, g, tw, s) : go_xf_vm<NN, float>(vm, spec, g, tw, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_x_forward_sparse(bool fp64, const int32_t* old_ids, const int32_t* old_cnt, const int32_t* new_ids,
                                   int new_cnt, int sx, int sy, int sz, const double* E, void* spec, SpecGeom g,
                                   int y_lo, int y_len, int z_lo, int z_len, const double2* tw, uint32_t* zero_ctr,
                                   hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN)                                                                                          \
  case NN:                                                                                                   \
    return fp64 ? go_xfs<NN, double>(old_ids, old_cnt, new_ids, new_cnt, sx, sy, sz, E, spec, g, y_lo, y_len, \
                                     z_lo, z_len, tw, zero_ctr, s)                                            \
                : go_xfs<NN, float>(old_ids, old_cnt, new_ids, new_cnt, sx, sy, sz, E, spec, g, y_lo, y_len,  \
                                    z_lo, z_len, tw, zero_ctr, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pencil(bool fp64, bool inv, int axis, void* spec, SpecGeom g, Prune pr, const double2* tw,
                         uint32_t* ctr, hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN)                                                        \
  case NN:                                                                 \
    return fp64 ? go_pencil<NN, double>(inv, axis, spec, g, pr, tw, ctr, s) \
                : go_pencil<NN, float>(inv, axis, spec, g, pr, tw, ctr, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_green(bool fp64, void* spec, SpecGeom g, Cubic C, hipStream_t s) {
  const size_t bins = (size_t)g.n * g.n * (g.n / 2 + 1);
  const int grid = (int)((bins + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(k_green<double>, dim3(grid), dim3(256), 0, s, (double2*)spec, g.n, g.P, C);
  else
    hipLaunchKernelGGL(k_green<float>, dim3(grid), dim3(256), 0, s, (float2*)spec, g.n, g.P, C);
  return hipGetLastError();
}

template <int N, typename S>
hipError_t go_zgreen(void* spec, SpecGeom g, Cubic C, Prune pr, const double2* tw, uint32_t* ctr, hipStream_t s) {
  constexpr int W = zg_width<N, S>();
  constexpr int T = zg_threads<N, S>();
  constexpr int NT = N * ((N / 2 + 1 + W - 1) / W);
  using C2 = typename Cplx<S>::T;
  const bool prune = pr.in_len < N;
  if (g.P != spec_pitch(N, sizeof(S) == 8)) return hipErrorInvalidValue;
  auto* k = C.frm ? (prune ? k_zgreen<N, S, true, true> : k_zgreen<N, S, false, true>)
                  : (prune ? k_zgreen<N, S, true, false> : k_zgreen<N, S, false, false>);
  const int grid = tile_grid(k, T, NT, zg_pipe<N, S>());
  if (grid < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(grid), dim3(T), 0, s, (C2*)spec, C, pr, tw, ctr, (const HopJob*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_z_green(bool fp64, void* spec, SpecGeom g, Cubic C, Prune pr, const double2* tw, uint32_t* ctr,
                          hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN)                                                      \
  case NN:                                                               \
    return fp64 ? go_zgreen<NN, double>(spec, g, C, pr, tw, ctr, s)      \
                : go_zgreen<NN, float>(spec, g, C, pr, tw, ctr, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_hop_batch_fft(bool fp64, const HopJob* jobs, int njob, SpecGeom g, Cubic C, const double2* tw,
                                uint32_t* ctr, const double* zero6, hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN)                                                                  \
  case NN:                                                                           \
    return fp64 ? go_hop_batch<NN, double>(jobs, njob, g, C, tw, ctr, zero6, s)     \
                : go_hop_batch<NN, float>(jobs, njob, g, C, tw, ctr, zero6, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_x_inverse(bool fp64, bool accum, const void* spec, double* sig, SpecGeom g, const double* mean6,
                            const double2* tw, hipStream_t s, const double* bg, int bg_mask, const double* add3,
                            const int32_t* own, bool all) {
  switch (g.n) {
#define EC_CASE(NN)                                                                              \
  case NN:                                                                                       \
    return fp64 ? go_xi<NN, double>(accum, spec, sig, g, mean6, tw, bg, bg_mask, add3, own, all, s) \
                : go_xi<NN, float>(accum, spec, sig, g, mean6, tw, bg, bg_mask, add3, own, all, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

// ------------------------------------------------------ dislocation lines (Sec. 3.1)
//
// A straight line along cell axis a is uniform along a, so its Nye tensor,
// plastic distortion and stress live on the plane k_a = 0 of the spectrum.
// Per bin (k1, k2) over the other two axes (a1 < a2): rho_hat of each spread
// line (bilinear weights over the four grid points around it, density 1/h^2),
// the distortion U_hat_ij = -i xi_k / xi^2 e_jkl b_i t_l rho_hat (Nyquist bins:
// the mean over the all -n/2 and all +n/2 representatives, the real part of the
// centred solution), eps*_hat = sym(U_hat) summed over the lines, then the Green
// step of the bin (the operator is even in xi, so a bin past n/2 along x uses its
// mirror in the half-spectrum indexing of green_bin).
__global__ __launch_bounds__(256) void k_disl_spectrum(const DevLine* __restrict__ lines, int nl, int axis, int n,
                                                       double L, Cubic C, double2* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nn = n * n;
  if (t >= nn) return;
  const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
  const int k1 = t % n, k2 = t / n;
  int kb[3];
  kb[axis] = 0;
  kb[a1] = k1;
  kb[a2] = k2;
  const int hn = n / 2;
  const double s2pi = 2.0 * M_PI / L;
  double2 e[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = make_double2(0.0, 0.0);
  if (k1 != 0 || k2 != 0) {
    // the representatives of the bin: one, or two for a Nyquist bin
    double lab[2][3];
    bool nyq = false;
    for (int d = 0; d < 3; ++d) {
      const int k = kb[d];
      const bool ny = nyquist(k, n);
      nyq |= ny;
      lab[0][d] = ny ? -hn : centred(k, n);
      lab[1][d] = ny ? hn : lab[0][d];
    }
    const int nrep = nyq ? 2 : 1;
    const double h = L / n;
    for (int li = 0; li < nl; ++li) {
      const DevLine ln = lines[li];
      // rho_hat = sum_c w_c exp(-2 pi i (k1 i1 + k2 i2) / n) / h^2
      const double f1 = floor(ln.u1), f2 = floor(ln.u2);
      double2 rho = make_double2(0.0, 0.0);
      for (int c1 = 0; c1 < 2; ++c1)
        for (int c2 = 0; c2 < 2; ++c2) {
          const double w = (1.0 - fabs(ln.u1 - (f1 + c1))) * (1.0 - fabs(ln.u2 - (f2 + c2)));
          if (w == 0.0) continue;
          const int64_t i1 = (((int64_t)f1 + c1) % n + n) % n, i2 = (((int64_t)f2 + c2) % n + n) % n;
          const int64_t m = ((int64_t)k1 * i1 + (int64_t)k2 * i2) % n;
          double sn, cs;
          sincospi(-2.0 * (double)m / n, &sn, &cs);
          rho.x += w * cs;
          rho.y += w * sn;
        }
      rho.x /= h * h;
      rho.y /= h * h;
      // F = mean over the representatives of (xi x t) / xi^2
      double F[3] = {0.0, 0.0, 0.0};
      for (int r = 0; r < nrep; ++r) {
        const double x0 = s2pi * lab[r][0], x1 = s2pi * lab[r][1], x2 = s2pi * lab[r][2];
        const double q = 1.0 / ((x0 * x0 + x1 * x1 + x2 * x2) * nrep);
        F[0] += (x1 * ln.t[2] - x2 * ln.t[1]) * q;
        F[1] += (x2 * ln.t[0] - x0 * ln.t[2]) * q;
        F[2] += (x0 * ln.t[1] - x1 * ln.t[0]) * q;
      }
      // w = -i F rho
      double2 w[3];
      for (int j = 0; j < 3; ++j) w[j] = make_double2(F[j] * rho.y, -F[j] * rho.x);
      const double* b = ln.b;
      e[0].x += b[0] * w[0].x;
      e[0].y += b[0] * w[0].y;
      e[1].x += b[1] * w[1].x;
      e[1].y += b[1] * w[1].y;
      e[2].x += b[2] * w[2].x;
      e[2].y += b[2] * w[2].y;
      e[3].x += 0.5 * (b[1] * w[2].x + b[2] * w[1].x);
      e[3].y += 0.5 * (b[1] * w[2].y + b[2] * w[1].y);
      e[4].x += 0.5 * (b[0] * w[2].x + b[2] * w[0].x);
      e[4].y += 0.5 * (b[0] * w[2].y + b[2] * w[0].y);
      e[5].x += 0.5 * (b[0] * w[1].x + b[1] * w[0].x);
      e[5].y += 0.5 * (b[0] * w[1].y + b[1] * w[0].y);
    }
    int gx = kb[0], gy = kb[1], gz = kb[2];
    if (gx > hn) {
      gx = n - gx;
      gy = (n - gy) % n;
      gz = (n - gz) % n;
    }
    if (C.frm)
      green_bin_rot(e, gx, gy, gz, n, C);
    else
      green_bin(e, gx, gy, gz, n, C);
  }
#pragma unroll
  for (int c = 0; c < 6; ++c) out[(size_t)c * nn + t] = e[c];
}

// One direction of the inverse 2-D transform by direct sums (exact phase
// reduction, m = k i mod n): DIM 0 over k1 (in [c][k2][k1] -> out [c][k2][i1]),
// DIM 1 over k2 with the 1/n^2 scale and the real part into plane [i2 * n + i1][c].
template <int DIM>
__global__ __launch_bounds__(256) void k_disl_idft(const double2* __restrict__ in, int n, double2* __restrict__ out,
                                                   double* __restrict__ plane) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int nn = n * n;
  if (t >= 6 * nn) return;
  const int c = t / nn, r = t % nn;
  const int i = r % n, o = r / n;  // output index along the transformed axis, the other axis
  double2 acc = make_double2(0.0, 0.0);
  for (int k = 0; k < n; ++k) {
    const double2 v = DIM == 0 ? in[(size_t)c * nn + (size_t)o * n + k] : in[(size_t)c * nn + (size_t)k * n + o];
    const int64_t m = ((int64_t)k * i) % n;
    double sn, cs;
    sincospi(2.0 * (double)m / n, &sn, &cs);
    acc.x += v.x * cs - v.y * sn;
    acc.y += v.x * sn + v.y * cs;
  }
  if (DIM == 0)
    out[(size_t)c * nn + (size_t)o * n + i] = acc;
  else
    plane[((size_t)i * n + o) * 6 + c] = acc.x / ((double)n * n);
}

__global__ __launch_bounds__(256) void k_bg_add(double* __restrict__ sig, const double* __restrict__ planes, int mask,
                                                int n, double sgn) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (v >= nn * n) return;
  const int x[3] = {(int)(v % n), (int)((v / n) % n), (int)(v / nn)};
  double add[6] = {0, 0, 0, 0, 0, 0};
  for (int a = 0; a < 3; ++a) {
    if (!(mask & (1 << a))) continue;
    const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
    const double* p = planes + ((size_t)a * nn + (size_t)x[a2] * n + x[a1]) * 6;
    for (int c = 0; c < 6; ++c) add[c] += p[c];
  }
  double* q = sig + 6 * v;
  for (int c = 0; c < 6; ++c) q[c] += sgn * add[c];
}

// Dislocation paths in any direction (Sec. 3.1): per bin of the half spectrum
// the Nye tensor alpha_hat_il = sum over pieces of M_il rho_hat, with the
// trilinear spread of a piece separable per axis,
//   rho_hat = prod_a e^{-2 pi i k_a f_a / n} ((1 - fr_a) + fr_a e^{-2 pi i k_a / n}),
// the exponents reduced exactly (k_a f_a mod n) and read from the twiddle
// table; then U_hat_ij = -i e_jkl xi_k alpha_hat_il / |xi|^2 (at an even n's
// Nyquist bins the mean over the all -n/2 and all +n/2 representatives),
// eps*_hat = sym(U_hat) and the Green step.  Pieces are staged in LDS in
// chunks; one thread per bin.
constexpr int PATH_CHUNK = 128;

template <typename S>
__global__ __launch_bounds__(256) void k_path_spectrum(const DevPiece* __restrict__ pieces, int np, int n, int P,
                                                       double L, Cubic C, const double2* __restrict__ tw,
                                                       typename Cplx<S>::T* __restrict__ spec) {
  __shared__ DevPiece sp[PATH_CHUNK];
  const int NH = n / 2 + 1;
  const int64_t bins = (int64_t)n * n * NH;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = b < bins;
  const int kx = live ? (int)(b % NH) : 0;
  const int64_t r = live ? b / NH : 0;
  const int ky = (int)(r % n), kz = (int)(r / n);
  const int k[3] = {kx, ky, kz};
  double2 e1[3];  // e^{-2 pi i k_a / n}
#pragma unroll
  for (int a = 0; a < 3; ++a) e1[a] = tw[k[a]];
  double2 al[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) al[c] = make_double2(0.0, 0.0);
  for (int p0 = 0; p0 < np; p0 += PATH_CHUNK) {
    const int m = min(PATH_CHUNK, np - p0);
    __syncthreads();
    for (int i = threadIdx.x; i < m; i += blockDim.x) sp[i] = pieces[p0 + i];
    __syncthreads();
    if (!live) continue;
    for (int i = 0; i < m; ++i) {
      const DevPiece& q = sp[i];
      double2 rho = make_double2(1.0, 0.0);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double2 ph = tw[(k[a] * q.f[a]) % n];
        const double w = q.fr[a];
        const double2 f = make_double2((1.0 - w) + w * e1[a].x, w * e1[a].y);
        const double2 t = make_double2(ph.x * f.x - ph.y * f.y, ph.x * f.y + ph.y * f.x);
        rho = make_double2(rho.x * t.x - rho.y * t.y, rho.x * t.y + rho.y * t.x);
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        al[c].x += q.M[c] * rho.x;
        al[c].y += q.M[c] * rho.y;
      }
    }
  }
  if (!live) return;
  double2 e[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = make_double2(0.0, 0.0);
  if (kx != 0 || ky != 0 || kz != 0) {
    const bool nyq = nyquist(kx, n) || nyquist(ky, n) || nyquist(kz, n);
    const int nrep = nyq ? 2 : 1;
    const double s2pi = 2.0 * M_PI / L;
    double2 U[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) U[i][j] = make_double2(0.0, 0.0);
    for (int rep = 0; rep < nrep; ++rep) {
      double x[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int h = n / 2;
        x[a] = s2pi * (nyquist(k[a], n) ? (rep == 0 ? -h : h) : centred(k[a], n));
      }
      const double q = 1.0 / ((x[0] * x[0] + x[1] * x[1] + x[2] * x[2]) * nrep);
      // U_ij += -i (xi x alpha_i.)_j / |xi|^2, alpha_i. the row i of alpha_hat
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double2 a0 = al[3 * i], a1 = al[3 * i + 1], a2 = al[3 * i + 2];
        const double2 c0 = make_double2(x[1] * a2.x - x[2] * a1.x, x[1] * a2.y - x[2] * a1.y);
        const double2 c1 = make_double2(x[2] * a0.x - x[0] * a2.x, x[2] * a0.y - x[0] * a2.y);
        const double2 c2 = make_double2(x[0] * a1.x - x[1] * a0.x, x[0] * a1.y - x[1] * a0.y);
        // -i c = (c.y, -c.x)
        U[i][0].x += q * c0.y;
        U[i][0].y -= q * c0.x;
        U[i][1].x += q * c1.y;
        U[i][1].y -= q * c1.x;
        U[i][2].x += q * c2.y;
        U[i][2].y -= q * c2.x;
      }
    }
    e[0] = U[0][0];
    e[1] = U[1][1];
    e[2] = U[2][2];
    e[3] = make_double2(0.5 * (U[1][2].x + U[2][1].x), 0.5 * (U[1][2].y + U[2][1].y));
    e[4] = make_double2(0.5 * (U[0][2].x + U[2][0].x), 0.5 * (U[0][2].y + U[2][0].y));
    e[5] = make_double2(0.5 * (U[0][1].x + U[1][0].x), 0.5 * (U[0][1].y + U[1][0].y));
    if (C.frm)
      green_bin_rot(e, kx, ky, kz, n, C);
    else
      green_bin(e, kx, ky, kz, n, C);
  }
  typename Cplx<S>::T* const out = spec + spec_at(kz, ky, kx, 0, n, P);
#pragma unroll
  for (int c = 0; c < 6; ++c) st2(out + c, e[c]);
}

__global__ __launch_bounds__(256) void k_bg3_add(double* __restrict__ sig, const double* __restrict__ bg3,
                                                 int64_t count, double sgn) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) sig[i] += sgn * bg3[i];
}

hipError_t launch_path_spectrum(bool fp64, const DevPiece* pieces, int np, SpecGeom g, double L, Cubic C,
                                const double2* tw, void* spec, hipStream_t s) {
  const int64_t bins = (int64_t)g.n * g.n * (g.n / 2 + 1);
  const int grid = (int)((bins + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(k_path_spectrum<double>, dim3(grid), dim3(256), 0, s, pieces, np, g.n, g.P, L, C, tw,
                       (double2*)spec);
  else
    hipLaunchKernelGGL(k_path_spectrum<float>, dim3(grid), dim3(256), 0, s, pieces, np, g.n, g.P, L, C, tw,
                       (float2*)spec);
  return hipGetLastError();
}

hipError_t launch_bg3_add(double* sig, const double* bg3, int64_t n3, double sgn, hipStream_t s) {
  const int64_t count = 6 * n3;
  hipLaunchKernelGGL(k_bg3_add, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, sig, bg3, count, sgn);
  return hipGetLastError();
}

hipError_t launch_disl_plane(const DevLine* lines, int nl, int axis, int n, double L, Cubic C, double2* spec,
                             double2* tmp, double* plane, hipStream_t s) {
  const int nn = n * n;
  hipLaunchKernelGGL(k_disl_spectrum, dim3((nn + 255) / 256), dim3(256), 0, s, lines, nl, axis, n, L, C, spec);
  hipLaunchKernelGGL(k_disl_idft<0>, dim3((6 * nn + 255) / 256), dim3(256), 0, s, (const double2*)spec, n, tmp,
                     (double*)nullptr);
  hipLaunchKernelGGL(k_disl_idft<1>, dim3((6 * nn + 255) / 256), dim3(256), 0, s, (const double2*)tmp, n,
                     (double2*)nullptr, plane);
  return hipGetLastError();
}

hipError_t launch_bg_add(double* sig, const double* planes, int mask, int n, double sgn, hipStream_t s) {
  const int64_t n3 = (int64_t)n * n * n;
  hipLaunchKernelGGL(k_bg_add, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, sig, planes, mask, n, sgn);
  return hipGetLastError();
}

}  // namespace ec
