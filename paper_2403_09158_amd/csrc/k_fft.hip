// k_fft.hip - FFT passes and the Green operator of the periodic eigenstrain solve.
//
// Half-spectrum layout: [6][kz][ky][kx] complex, kx in [0, n/2] with row pitch P
// (padded so every row starts on a 128-byte boundary).  The solve runs:
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
constexpr int pencil_W_of(int N) { return N >= 512 ? 8 : 16; }
constexpr int x_rows(int N) {
  int best = 1;
  for (int r = 1; r <= N; ++r)
    if (N % r == 0 && 3 * r * N <= 1536) best = r;
  return best;
}

// ----------------------------------------------------------------- Green operator
//
// Sec. 3.2: eps_hat = Gamma(xi):(C:eps*_hat) with Gamma built from N = K^-1,
// K_ik = C_ijkl xi_j xi_l; here eps_hat = sym(xi (x) N (tau xi)), tau = C:eps*_hat,
// and the kernel returns sigma_hat = C:eps_hat - tau (the stress spectrum, so the
// inverse transform yields sigma directly).  Gamma is homogeneous of degree 0 in
// xi, so the integer labels stand in for xi = 2 pi k / L.

__device__ __forceinline__ void acc_eps(double ax, double ay, double az, const Cubic& C, const double2* tau,
                                        double2* eps, double wgt) {
  const double x2 = ax * ax, y2 = ay * ay, z2 = az * az, r2 = x2 + y2 + z2;
  const double K00 = C.C11 * x2 + C.C44 * (r2 - x2);
  const double K11 = C.C11 * y2 + C.C44 * (r2 - y2);
  const double K22 = C.C11 * z2 + C.C44 * (r2 - z2);
  const double cc = C.C12 + C.C44;
  const double K01 = cc * ax * ay, K02 = cc * ax * az, K12 = cc * ay * az;
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
  double2 w0, w1, w2;  // w = N v (scaled by wgt)
  w0.x = (A00 * v0.x + A01 * v1.x + A02 * v2.x) * inv;
  w0.y = (A00 * v0.y + A01 * v1.y + A02 * v2.y) * inv;
  w1.x = (A01 * v0.x + A11 * v1.x + A12 * v2.x) * inv;
  w1.y = (A01 * v0.y + A11 * v1.y + A12 * v2.y) * inv;
  w2.x = (A02 * v0.x + A12 * v1.x + A22 * v2.x) * inv;
  w2.y = (A02 * v0.y + A12 * v1.y + A22 * v2.y) * inv;
  eps[0].x += ax * w0.x;
  eps[0].y += ax * w0.y;
  eps[1].x += ay * w1.x;
  eps[1].y += ay * w1.y;
  eps[2].x += az * w2.x;
  eps[2].y += az * w2.y;
  eps[3].x += 0.5 * (ay * w2.x + az * w1.x);
  eps[3].y += 0.5 * (ay * w2.y + az * w1.y);
  eps[4].x += 0.5 * (ax * w2.x + az * w0.x);
  eps[4].y += 0.5 * (ax * w2.y + az * w0.y);
  eps[5].x += 0.5 * (ax * w1.x + ay * w0.x);
  eps[5].y += 0.5 * (ax * w1.y + ay * w0.y);
}

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
  double2 tau[6];
  const double c44x2 = 2.0 * C.C44;
  tau[0].x = C.C11 * e[0].x + C.C12 * (e[1].x + e[2].x);
  tau[0].y = C.C11 * e[0].y + C.C12 * (e[1].y + e[2].y);
  tau[1].x = C.C11 * e[1].x + C.C12 * (e[0].x + e[2].x);
  tau[1].y = C.C11 * e[1].y + C.C12 * (e[0].y + e[2].y);
  tau[2].x = C.C11 * e[2].x + C.C12 * (e[0].x + e[1].x);
  tau[2].y = C.C11 * e[2].y + C.C12 * (e[0].y + e[1].y);
#pragma unroll
  for (int c = 3; c < 6; ++c) tau[c] = make_double2(c44x2 * e[c].x, c44x2 * e[c].y);
  double2 eps[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) eps[c] = make_double2(0.0, 0.0);
  const int h = n / 2;
  const bool nx = kx == h, ny = ky == h, nz = kz == h;
  const double lx = kx, ly = ky < h ? ky : ky - n, lz = kz < h ? kz : kz - n;
  if (!(nx || ny || nz)) {
    acc_eps(lx, ly, lz, C, tau, eps, 1.0);
  } else {
    acc_eps(nx ? -h : lx, ny ? -h : ly, nz ? -h : lz, C, tau, eps, 0.5);
    acc_eps(nx ? h : lx, ny ? h : ly, nz ? h : lz, C, tau, eps, 0.5);
  }
  e[0].x = C.C11 * eps[0].x + C.C12 * (eps[1].x + eps[2].x) - tau[0].x;
  e[0].y = C.C11 * eps[0].y + C.C12 * (eps[1].y + eps[2].y) - tau[0].y;
  e[1].x = C.C11 * eps[1].x + C.C12 * (eps[0].x + eps[2].x) - tau[1].x;
  e[1].y = C.C11 * eps[1].y + C.C12 * (eps[0].y + eps[2].y) - tau[1].y;
  e[2].x = C.C11 * eps[2].x + C.C12 * (eps[0].x + eps[1].x) - tau[2].x;
  e[2].y = C.C11 * eps[2].y + C.C12 * (eps[0].y + eps[1].y) - tau[2].y;
#pragma unroll
  for (int c = 3; c < 6; ++c) e[c] = make_double2(c44x2 * eps[c].x - tau[c].x, c44x2 * eps[c].y - tau[c].y);
}

// ----------------------------------------------------------------- x forward (R2C)

// LDS staging type of the x-forward transforms
template <typename S>
struct XfStage {
  using T = double2;
};

template <int N, typename S, bool DENSE>
__global__ __launch_bounds__(pick_T(max_nb(N, 3 * x_rows(N)))) void k_x_forward(
    const int32_t* __restrict__ own, const int2* __restrict__ lnk, const DevDefect* __restrict__ defs,
    const double* __restrict__ dense, typename Cplx<S>::T* __restrict__ spec, int P, const double2* __restrict__ twg) {
  constexpr int ROWS = x_rows(N);
  constexpr int NF = 3 * ROWS;  // (xx,yy), (zz,yz), (xz,xy) per row
  constexpr int T = pick_T(max_nb(N, NF));
  constexpr int LDN = N + N / 16 + 1;
  constexpr int NH = N / 2 + 1;
  using LT = typename XfStage<S>::T;
  __shared__ LT buf[NF * LDN];
  __shared__ double2 tw[N];
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  const int bpp = N / ROWS;
  const int z = blockIdx.x / bpp;
  const int y0 = (blockIdx.x % bpp) * ROWS;
  const size_t n3 = (size_t)N * N * N;
  const size_t cs = (size_t)N * N * P;
  auto lds = [&](int f, int i) -> LT* { return &buf[f * LDN + i + (i >> 4)]; };
  // gather the rows' six components into the transform inputs (xx + i yy, ...);
  // all of a thread's voxel links are loaded first, then the owners' records
  constexpr int KV = (ROWS * N + T - 1) / T;
  int32_t link[KV];
#pragma unroll
  for (int k = 0; k < KV; ++k) {
    const int i = threadIdx.x + k * T;
    link[k] = -1;
    if (!DENSE && i < ROWS * N) {
      const int r = i / N, x = i - r * N;
      link[k] = own[((size_t)z * N + y0 + r) * N + x];
    }
  }
#pragma unroll
  for (int k = 0; k < KV; ++k) {
    const int i = threadIdx.x + k * T;
    if (i < ROWS * N) {
      const int r = i / N, x = i - r * N;
      double e[6];
      if (DENSE) {
        const size_t v = ((size_t)z * N + y0 + r) * N + x;
#pragma unroll
        for (int c = 0; c < 6; ++c) e[c] = dense[c * n3 + v];
      } else {
        int64_t acc[6] = {0, 0, 0, 0, 0, 0};
        decode_voxel(link[k], lnk, defs, acc);
#pragma unroll
        for (int c = 0; c < 6; ++c) e[c] = (double)acc[c] * FIX_INV;
      }
#pragma unroll
      for (int p = 0; p < 3; ++p) st2(lds(3 * r + p, x), make_double2(e[2 * p], e[2 * p + 1]));
    }
  }
  __syncthreads();
  auto from_lds = [&](int f, int i) { return ld2(lds(f, i)); };
  auto to_lds = [&](int f, int i, double2 v) { st2(lds(f, i), v); };
  transform<N, false, Map::Row, NF, T, true, true>(tw, from_lds, from_lds, to_lds, to_lds);
  __syncthreads();
  for (int e = threadIdx.x; e < NF * NH; e += T) {
    const int f = e / NH, k = e % NH;
    const double2 zk = ld2(lds(f, k));
    const double2 zc = conjd(ld2(lds(f, k == 0 ? 0 : N - k)));
    const double2 A = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y));
    const double2 B = make_double2(0.5 * (zk.y - zc.y), -0.5 * (zk.x - zc.x));
    const int p = f % 3, y = y0 + f / 3;
    const size_t row = ((size_t)z * N + y) * P + k;
    st2(&spec[(size_t)(2 * p) * cs + row], A);
    st2(&spec[(size_t)(2 * p + 1) * cs + row], B);
  }
}

// Update variant: the rows of the eigenstrain change dE = E (chi_new - chi_old)
// are built in LDS from the two footprint lists (new ids = old ids shifted by
// (sx, sy, sz) voxels when new_ids == nullptr), for rows y in [y_lo, y_lo+y_len),
// z in [z_lo, z_lo+z_len) (cyclic); other rows are zero and never touched.
template <int N, typename S>
__global__ __launch_bounds__(pick_T(max_nb(N, 3 * x_rows(N)))) void k_x_forward_sparse(
    const int32_t* __restrict__ old_ids, const int32_t* __restrict__ old_cnt_p, const int32_t* __restrict__ new_ids,
    int new_cnt, int sx, int sy, int sz, const double* __restrict__ E, typename Cplx<S>::T* __restrict__ spec, int P,
    int y_lo, int y_len, int z_lo, const double2* __restrict__ twg) {
  const int old_cnt = *old_cnt_p;
  if (!new_ids) new_cnt = old_cnt;
  constexpr int ROWS = x_rows(N);
  constexpr int NF = 3 * ROWS;
  constexpr int T = pick_T(max_nb(N, NF));
  constexpr int LDN = N + N / 16 + 1;
  constexpr int NH = N / 2 + 1;
  __shared__ double2 buf[NF * LDN];
  __shared__ double2 tw[N];
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  for (int i = threadIdx.x; i < NF * LDN; i += T) buf[i] = make_double2(0.0, 0.0);
  const int rb = (y_len + ROWS - 1) / ROWS;
  const int zi = blockIdx.x / rb;
  const int y0i = (blockIdx.x % rb) * ROWS;
  int z = z_lo + zi;
  if (z >= N) z -= N;
  const size_t cs = (size_t)N * N * P;
  __syncthreads();
  auto lds = [&](int f, int i) -> double2& { return buf[f * LDN + i + (i >> 4)]; };
  // scatter +-E of the voxels that fall in this block's rows (one row per y)
  auto scatter = [&](int id, double sgn) {
    const int x = id % N, y = (id / N) % N, zz = id / (N * N);
    if (zz != z) return;
    int yi = y - y_lo;
    if (yi < 0) yi += N;
    yi -= y0i;
    if (yi < 0 || yi >= ROWS || y0i + yi >= y_len) return;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      double2& slot = lds(3 * yi + p, x);
      slot.x += sgn * E[2 * p];
      slot.y += sgn * E[2 * p + 1];
    }
  };
  // Each voxel is owned by one thread per list pass; a voxel can sit in both
  // lists, so the two passes are separated by a barrier.
  for (int i = threadIdx.x; i < old_cnt; i += T) scatter(old_ids[i], -1.0);
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
    scatter(id, 1.0);
  }
  __syncthreads();
  auto from_lds = [&](int f, int i) { return lds(f, i); };
  auto to_lds = [&](int f, int i, double2 v) { lds(f, i) = v; };
  transform<N, false, Map::Row, NF, T, true, true>(tw, from_lds, from_lds, to_lds, to_lds);
  __syncthreads();
  for (int e = threadIdx.x; e < NF * NH; e += T) {
    const int f = e / NH, k = e % NH;
    const int yi = f / 3, p = f % 3;
    if (y0i + yi >= y_len) continue;
    int y = y_lo + y0i + yi;
    if (y >= N) y -= N;
    const double2 zk = lds(f, k);
    const double2 zc = conjd(lds(f, k == 0 ? 0 : N - k));
    const double2 A = make_double2(0.5 * (zk.x + zc.x), 0.5 * (zk.y + zc.y));
    const double2 B = make_double2(0.5 * (zk.y - zc.y), -0.5 * (zk.x - zc.x));
    const size_t row = ((size_t)z * N + y) * P + k;
    st2(&spec[(size_t)(2 * p) * cs + row], A);
    st2(&spec[(size_t)(2 * p + 1) * cs + row], B);
  }
}

// --------------------------------------------------------------- y / z pencils
//
// A tile is W consecutive kx columns of one (component, z) plane (y pass) or one
// (component, y) row (z pass), transformed along y or z; the kx = n/2 column is
// tiled separately, W planes (y pass) or rows (z pass) at a time.

template <int N, int W>
struct PencilTile {
  static constexpr int KXB = (N / 2 + W - 1) / W;
  int c, outer, kx0, nouter, z_lo;
  bool nyq;
  __device__ PencilTile(int bid, int nouter_, int z_lo_) : nouter(nouter_), z_lo(z_lo_) {
    const int nreg = 6 * nouter * KXB;
    nyq = bid >= nreg;
    if (!nyq) {
      kx0 = (bid % KXB) * W;
      const int rest = bid / KXB;
      outer = rest % nouter;
      c = rest / nouter;
    } else {
      bid -= nreg;
      const int nb = (nouter + W - 1) / W;
      outer = (bid % nb) * W;
      c = bid / nb;
      kx0 = N / 2;
    }
  }
  // column w -> (outer index, kx); false if outside the tile
  __device__ __forceinline__ bool col(int w, int& o, int& kx) const {
    if (!nyq) {
      kx = kx0 + w;
      o = outer;
      return kx < N / 2;
    }
    kx = N / 2;
    o = outer + w;
    return o < nouter;
  }
  // element offset for axis 1 (y pass: transform index i = y) or axis 2 (z pass: i = z)
  __device__ __forceinline__ size_t off(int axis, int o, int kx, int i, int P) const {
    if (axis == 1) {
      int z = z_lo + o;
      if (z >= N) z -= N;
      return (((size_t)c * N + z) * N + i) * P + kx;
    }
    return (((size_t)c * N + i) * N + o) * P + kx;
  }
};

// W columns per tile, LT = LDS staging type (double2, or float2 for FP32 storage),
// TMAX = largest workgroup, PRUNE = input confined to a cyclic range (updates).
constexpr int pick_T2(int nb, int tmax) { return nb >= tmax ? tmax : ((nb + 63) / 64) * 64; }

template <int N, typename S, bool INV, int W, typename LT, int TMAX, bool PRUNE>
__global__ __launch_bounds__(pick_T2(max_nb(N, W), TMAX)) void k_pencil(typename Cplx<S>::T* __restrict__ spec, int P,
                                                                      int axis, Prune pr,
                                                                      const double2* __restrict__ twg, int ntiles) {
  constexpr int T = pick_T2(max_nb(N, W), TMAX);
  static_assert(T % W == 0, "a thread must keep its column across butterflies");
  constexpr Plan2 PL = plan_of(N);
  constexpr int R0 = PL.r[0];
  constexpr int NOP = ((W * (N / R0) + T - 1) / T) * R0;  // first-stage operands per thread
  using C2 = typename Cplx<S>::T;
  __shared__ LT buf[N * W];
  __shared__ double2 tw[N];
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  const int nouter = axis == 1 ? pr.z_len : N;
  const int si = axis == 1 ? P : N * P;  // element stride along the transform axis
  auto in_range = [&](int i) {
    if (!PRUNE) return true;
    int d = i - pr.in_lo;
    if (d < 0) d += N;
    return d < pr.in_len;
  };
  // column of thread lane w in tile t (the base of the spectrum if the lane
  // has no column in this tile)
  auto column = [&](int t, int w, bool& valid) -> C2* {
    const PencilTile<N, W> tile(t, nouter, pr.z_lo);
    int o, kx;
    valid = tile.col(w, o, kx);
    return spec + (valid ? tile.off(axis, o, kx, 0, P) : 0);
  };
  // FP32 storage: raw first-stage operands of the next tile are loaded while
  // the current one is transformed (rows outside the input range read row
  // in_lo, a cache hit, and are zeroed when consumed).  FP64 storage would
  // need twice the registers for them and loads each tile's operands in turn.
  constexpr bool PIPE = sizeof(S) == 4;
  C2 nxt[NOP];
  auto fetch = [&](int t, int tid) {
    if constexpr (!PIPE) return;
    bool v;
    const C2* colp = column(t, tid % W, v);
    for_operands<N, R0, Map::Pencil, W, T>(
        [&](int, int i, int slot) { nxt[slot] = colp[(size_t)(in_range(i) ? i : pr.in_lo) * si]; }, tid);
  };
  auto from_lds = [&](int w, int i) { return ld2(&buf[i * W + w]); };
  auto to_lds = [&](int w, int i, double2 v) { st2(&buf[i * W + w], v); };
  // contiguous tile ranges per XCD (workgroup b runs on XCD b % 8)
  const int g8 = gridDim.x / 8;
  const int per = (ntiles + 7) / 8;
  const int lo = (int)(blockIdx.x % 8) * per;
  const int hi = min(ntiles, lo + per);
  int t = lo + (int)(blockIdx.x / 8);
  if (t < hi) fetch(t, threadIdx.x);
  __syncthreads();
  for (; t < hi; t += g8) {
    // laundered thread index: index arithmetic is redone per tile instead of
    // being held in registers across the loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    bool valid;
    C2* const colp = column(t, tid % W, valid);
    auto load0 = [&](int, int i, int slot) -> double2 {
      if (!(valid && in_range(i))) return make_double2(0.0, 0.0);
      return PIPE ? ld2(&nxt[slot]) : ld2(colp + (size_t)i * si);
    };
    auto store_last = [&](int, int i, double2 v) {
      if (valid) st2(colp + (size_t)i * si, v);
    };
    const bool more = t + g8 < hi;
    if constexpr (PL.nstage == 1) {
      stage<N, R0, 1, INV, Map::Pencil, W, T>(tw, load0, store_last, false, tid);
      if (more) fetch(t + g8, tid);
    } else {
      stage<N, R0, 1, INV, Map::Pencil, W, T>(tw, load0, to_lds, false, tid);
      if (more) fetch(t + g8, tid);
      __syncthreads();
      if constexpr (PL.nstage == 2) {
        stage<N, PL.r[1], R0, INV, Map::Pencil, W, T>(tw, from_lds, store_last, false, tid);
      } else {
        stage<N, PL.r[1], R0, INV, Map::Pencil, W, T>(tw, from_lds, to_lds, true, tid);
        __syncthreads();
        stage<N, PL.r[2], R0 * PL.r[1], INV, Map::Pencil, W, T>(tw, from_lds, store_last, false, tid);
      }
    }
    __syncthreads();  // the next tile's first stage rewrites LDS
  }
}

// ------------------------------------------- z-forward + Green + z-inverse (fused)
//
// One workgroup owns W kx columns of one ky row for all six components (6 W
// transforms of length N along z) in one LDS tile: forward transforms, the
// Green step per bin in place, inverse transforms.  The spectrum is read and
// written once per solve instead of three times, and every stage has all six
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

// columns per tile (two at N = 512, where a four-column tile would not fit)
template <int N, typename S>
constexpr int zg_width() {
  return N >= 512 ? 2 : 4;
}

// one butterfly per thread in the widest-radix stage (at most 1024 threads)
template <int N, typename S>
constexpr int zg_threads() {
  using FP = FusedPlan<N>;
  constexpr int rmin = FP::R0 < FP::R1 ? FP::R0 : FP::R1;
  constexpr int rl = FP::R2 > 1 && FP::R2 < rmin ? FP::R2 : rmin;  // smallest radix
  constexpr int rmax = FP::R0 > FP::R1 ? (FP::R0 > FP::R2 ? FP::R0 : FP::R2) : (FP::R1 > FP::R2 ? FP::R1 : FP::R2);
  constexpr int nb = 6 * zg_width<N, S>() * (N / rmax);
  constexpr int t = ((nb + 63) / 64) * 64;
  static_assert(rl >= 1, "");
  return t > 1024 ? 1024 : t;
}

// LDS row swizzle: the low three bits of the z index are XORed with the next
// three, so stride-R stores of the first stages spread over all banks.
__device__ __forceinline__ int zg_swz(int i) { return (i & ~7) | ((i ^ (i >> 3)) & 7); }

// hardware dispatch places consecutive workgroups on consecutive XCDs; give
// each XCD a contiguous run of tiles so neighbouring kx tiles share its L2
__device__ __forceinline__ int xcd_tile(int bid, int nblk) {
  const int per = nblk / 8;
  return bid < per * 8 ? (bid % 8) * per + bid / 8 : bid;
}

template <int N, typename S, bool PRUNE>
__global__ __launch_bounds__((zg_threads<N, S>())) void k_zgreen(typename Cplx<S>::T* __restrict__ spec, int P,
                                                                Cubic C, Prune pr, const double2* __restrict__ twg) {
  using FP = FusedPlan<N>;
  constexpr int W = zg_width<N, S>();
  constexpr int T = zg_threads<N, S>();
  constexpr int NH = N / 2 + 1;
  constexpr int KB = (NH + W - 1) / W;
  constexpr int NT = N * KB;  // tiles
  constexpr int NF = 6 * W;   // transforms per tile
  constexpr int R0 = FP::R0, R1 = FP::R1, R2 = FP::R2;
  constexpr int NOP = ((NF * (N / R0) + T - 1) / T) * R0;  // first-stage operands per thread
  static_assert(N % 8 == 0, "row swizzle needs whole groups of eight");
  static_assert(FP::NSTG >= 2, "the first stage must not be the last");
  using C2 = typename Cplx<S>::T;
  // FP64 tile in both storage precisions: rounding the whole spectrum to FP32
  // next to the Green step and between stages roughly doubles the FP32-storage
  // energy error, while the extra LDS costs little here
  __shared__ double2 buf[6 * N * W];
  __shared__ double2 tw[N];
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  const int si = N * P;
  const size_t cs = (size_t)N * N * P;
  auto lds = [&](int f, int i) -> double2* { return &buf[((f / W) * N + zg_swz(i)) * W + f % W]; };
  auto from_lds = [&](int f, int i) { return ld2(lds(f, i)); };
  auto to_lds = [&](int f, int i, double2 v) { st2(lds(f, i), v); };
  auto in_z = [&](int i) {
    if (!PRUNE) return true;
    int d = i - pr.in_lo;
    if (d < 0) d += N;
    return d < pr.in_len;
  };
  // FP32 storage: raw first-stage operands of the next tile, loaded while the
  // current one is transformed (rows outside the input range read row in_lo
  // instead, a cache hit, and are zeroed when consumed).  FP64 storage loads
  // each tile's operands in turn.
  constexpr bool PIPE = sizeof(S) == 4;
  C2 nxt[NOP];
  auto fetch = [&](int t, int tid) {
    if constexpr (!PIPE) return;
    const int kx = (t % KB) * W + tid % W;
    const C2* col0 = spec + (kx < NH ? (size_t)(t / KB) * P + kx : 0);
    for_operands<N, R0, Map::Group, NF, T, W>(
        [&](int f, int i, int slot) { nxt[slot] = col0[(f / W) * cs + (size_t)(in_z(i) ? i : pr.in_lo) * si]; }, tid);
  };
  // tiles split into eight contiguous ranges, one per XCD (dispatch order puts
  // workgroup b on XCD b % 8), so neighbouring kx tiles share an L2
  const int g8 = gridDim.x / 8;
  const int per = (NT + 7) / 8;
  const int lo = (int)(blockIdx.x % 8) * per;
  const int hi = min(NT, lo + per);
  int t = lo + (int)(blockIdx.x / 8);
  if (t < hi) fetch(t, threadIdx.x);
  __syncthreads();
  for (; t < hi; t += g8) {
    // the thread index is laundered per tile so that the many index
    // expressions derived from it are recomputed, not held in registers
    // across the loop
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int ky = t / KB;
    const int w = tid % W;  // T and every group size are multiples of W
    const int kx = (t % KB) * W + w;
    const bool valid = kx < NH;
    C2* const col0 = spec + (valid ? (size_t)ky * P + kx : 0);
    auto load0 = [&](int f, int i, int slot) -> double2 {
      if (!(valid && in_z(i))) return make_double2(0.0, 0.0);
      return PIPE ? ld2(&nxt[slot]) : ld2(col0 + (f / W) * cs + (size_t)i * si);
    };
    stage<N, R0, 1, false, Map::Group, NF, T, W>(tw, load0, to_lds, false, tid);
    if (t + g8 < hi) fetch(t + g8, tid);
    __syncthreads();
    if constexpr (R2 == 1) {
      stage<N, R1, R0, false, Map::Group, NF, T, W>(tw, from_lds, to_lds, true, tid);
    } else {
      stage<N, R1, R0, false, Map::Group, NF, T, W>(tw, from_lds, to_lds, true, tid);
      __syncthreads();
      stage<N, R2, R0 * R1, false, Map::Group, NF, T, W>(tw, from_lds, to_lds, true, tid);
    }
    __syncthreads();
    // Green step: one bin (all six components) per iteration, in place
#pragma unroll 1
    for (int b = tid; b < N * W; b += T) {
      const int bw = b % W, kz = b / W, bkx = kx - w + bw;
      if (bkx >= NH) continue;
      double2 e[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] = from_lds(c * W + bw, kz);
      green_bin(e, bkx, ky, kz, N, C);
#pragma unroll
      for (int c = 0; c < 6; ++c) to_lds(c * W + bw, kz, e[c]);
    }
    __syncthreads();
    auto store_last = [&](int f, int i, double2 v) {
      if (valid) st2(col0 + (f / W) * cs + (size_t)i * si, v);
    };
    transform_plan<N, FP::I0, FP::I1, FP::I2, true, Map::Group, NF, T, W, true, false>(tw, from_lds, from_lds, to_lds,
                                                                                    store_last, tid);
    __syncthreads();  // the next tile's first stage rewrites the tile
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
  const size_t cs = (size_t)n * n * P;
  const size_t o = ((size_t)kz * n + ky) * P + kx;
  double2 e[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) e[c] = ld2(&spec[c * cs + o]);
  green_bin(e, kx, ky, kz, n, C);
#pragma unroll
  for (int c = 0; c < 6; ++c) st2(&spec[c * cs + o], e[c]);
}

// --------------------------------------------------------- x inverse (C2R) + stress

template <int N, typename S, bool ACC>
__global__ __launch_bounds__(pick_T(max_nb(N, 3 * x_rows(N)))) void k_x_inverse(
    const typename Cplx<S>::T* __restrict__ spec, double* __restrict__ sig, int P, const double* __restrict__ mean6,
    const double2* __restrict__ twg) {
  constexpr int ROWS = x_rows(N);
  constexpr int NF = 3 * ROWS;
  constexpr int T = pick_T(max_nb(N, NF));
  constexpr int LDN = N + N / 16 + 1;
  __shared__ double2 buf[NF * LDN];
  __shared__ double2 tw[N];
  __shared__ double mean_s[6];
  for (int i = threadIdx.x; i < N; i += T) tw[i] = twg[i];
  if (threadIdx.x < 6) mean_s[threadIdx.x] = mean6[threadIdx.x];
  const int bpp = N / ROWS;
  const int z = blockIdx.x / bpp;
  const int y0 = (blockIdx.x % bpp) * ROWS;
  const size_t n3 = (size_t)N * N * N;
  const size_t cs = (size_t)N * N * P;
  const double scale = 1.0 / (double)n3;
  __syncthreads();
  auto load0 = [&](int f, int k) -> double2 {
    const int p = f % 3, y = y0 + f / 3;
    const size_t row = ((size_t)z * N + y) * P;
    const typename Cplx<S>::T* a = spec + (size_t)(2 * p) * cs + row;
    const typename Cplx<S>::T* b = spec + (size_t)(2 * p + 1) * cs + row;
    double2 A, B;
    if (k <= N / 2) {
      A = ld2(a + k);
      B = ld2(b + k);
      if (k == 0 || k == N / 2) {
        A.y = 0.0;
        B.y = 0.0;
      }
    } else {
      A = conjd(ld2(a + (N - k)));
      B = conjd(ld2(b + (N - k)));
    }
    return make_double2(A.x - B.y, A.y + B.x);
  };
  auto from_lds = [&](int f, int i) { return buf[f * LDN + i + (i >> 4)]; };
  auto to_lds = [&](int f, int i, double2 v) { buf[f * LDN + i + (i >> 4)] = v; };
  auto store_last = [&](int f, int x, double2 v) {
    const int p = f % 3, y = y0 + f / 3;
    const size_t o = ((size_t)z * N + y) * N + x;
    double* s0 = sig + (size_t)(2 * p) * n3 + o;
    double* s1 = sig + (size_t)(2 * p + 1) * n3 + o;
    const double a = v.x * scale + mean_s[2 * p], b = v.y * scale + mean_s[2 * p + 1];
    if (ACC) {
      *s0 += a;
      *s1 += b;
    } else {
      *s0 = a;
      *s1 = b;
    }
  };
  transform<N, true, Map::Row, NF, T>(tw, load0, from_lds, to_lds, store_last);
}

// ------------------------------------------------------------------ launchers

template <int N, typename S>
hipError_t go_xf(const int32_t* own, const int2* lnk, const DevDefect* defs, const double* dense, void* spec,
                 SpecGeom g, const double2* tw, hipStream_t s) {
  constexpr int T = pick_T(max_nb(N, 3 * x_rows(N)));
  const int grid = N * (N / x_rows(N));
  using C2 = typename Cplx<S>::T;
  if (dense)
    hipLaunchKernelGGL((k_x_forward<N, S, true>), dim3(grid), dim3(T), 0, s, own, lnk, defs, dense, (C2*)spec, g.P, tw);
  else
    hipLaunchKernelGGL((k_x_forward<N, S, false>), dim3(grid), dim3(T), 0, s, own, lnk, defs, dense, (C2*)spec, g.P,
                       tw);
  return hipGetLastError();
}

template <int N, typename S>
hipError_t go_xfs(const int32_t* oi, const int32_t* oc, const int32_t* ni, int nc, int sx, int sy, int sz, const double* E,
                  void* spec, SpecGeom g, int ylo, int ylen, int zlo, int zlen, const double2* tw, hipStream_t s) {
  constexpr int T = pick_T(max_nb(N, 3 * x_rows(N)));
  const int grid = zlen * ((ylen + x_rows(N) - 1) / x_rows(N));
  if (grid == 0) return hipSuccess;
  hipLaunchKernelGGL((k_x_forward_sparse<N, S>), dim3(grid), dim3(T), 0, s, oi, oc, ni, nc, sx, sy, sz, E,
                     (typename Cplx<S>::T*)spec, g.P, ylo, ylen, zlo, tw);
  return hipGetLastError();
}

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

template <int N, typename S, int W, typename LT, int TMAX>
hipError_t go_pencil_v(bool inv, int axis, void* spec, SpecGeom g, Prune pr, const double2* tw, hipStream_t s) {
  constexpr int T = pick_T2(max_nb(N, W), TMAX);
  const int nouter = axis == 1 ? pr.z_len : N;
  const int ntiles = 6 * nouter * PencilTile<N, W>::KXB + 6 * ((nouter + W - 1) / W);
  using C2 = typename Cplx<S>::T;
  const bool prune = pr.in_len < N;
  auto* k = inv ? (prune ? k_pencil<N, S, true, W, LT, TMAX, true> : k_pencil<N, S, true, W, LT, TMAX, false>)
                : (prune ? k_pencil<N, S, false, W, LT, TMAX, true> : k_pencil<N, S, false, W, LT, TMAX, false>);
  const int grid = tile_grid(k, T, ntiles, sizeof(S) == 4);
  if (grid < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(grid), dim3(T), 0, s, (C2*)spec, g.P, axis, pr, tw, ntiles);
  return hipGetLastError();
}

// FP32 storage stages the inter-stage exchange in FP32 too (half the LDS, twice
// the resident workgroups); FP64 storage keeps FP64 staging.
template <int N, typename S>
hipError_t go_pencil(bool inv, int axis, void* spec, SpecGeom g, Prune pr, const double2* tw, hipStream_t s) {
  using LT = typename Cplx<S>::T;
  return go_pencil_v<N, S, pencil_W_of(N), LT, 256>(inv, axis, spec, g, pr, tw, s);
}

template <int N, typename S>
hipError_t go_xi(bool acc, const void* spec, double* sig, SpecGeom g, const double* mean6, const double2* tw,
                 hipStream_t s) {
  constexpr int T = pick_T(max_nb(N, 3 * x_rows(N)));
  const int grid = N * (N / x_rows(N));
  using C2 = typename Cplx<S>::T;
  if (acc)
    hipLaunchKernelGGL((k_x_inverse<N, S, true>), dim3(grid), dim3(T), 0, s, (const C2*)spec, sig, g.P, mean6, tw);
  else
    hipLaunchKernelGGL((k_x_inverse<N, S, false>), dim3(grid), dim3(T), 0, s, (const C2*)spec, sig, g.P, mean6, tw);
  return hipGetLastError();
}

}  // namespace

#define EC_FOR_SIZES(X) X(8) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(160) X(240) X(256) X(512)

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

hipError_t launch_x_forward(bool fp64, const int32_t* own, const int2* lnk, const DevDefect* defs, const double* dense,
                            void* spec, SpecGeom g, const double2* tw, hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN)                                                           \
  case NN:                                                                    \
    return fp64 ? go_xf<NN, double>(own, lnk, defs, dense, spec, g, tw, s) \
                : go_xf<NN, float>(own, lnk, defs, dense, spec, g, tw, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_x_forward_sparse(bool fp64, const int32_t* old_ids, const int32_t* old_cnt, const int32_t* new_ids,
                                   int new_cnt, int sx, int sy, int sz, const double* E, void* spec, SpecGeom g,
                                   int y_lo, int y_len, int z_lo, int z_len, const double2* tw, hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN)                                                                                          \
  case NN:                                                                                                   \
    return fp64 ? go_xfs<NN, double>(old_ids, old_cnt, new_ids, new_cnt, sx, sy, sz, E, spec, g, y_lo, y_len, \
                                     z_lo, z_len, tw, s)                                                      \
                : go_xfs<NN, float>(old_ids, old_cnt, new_ids, new_cnt, sx, sy, sz, E, spec, g, y_lo, y_len,  \
                                    z_lo, z_len, tw, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_pencil(bool fp64, bool inv, int axis, void* spec, SpecGeom g, Prune pr, const double2* tw,
                         hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN)                                                   \
  case NN:                                                            \
    return fp64 ? go_pencil<NN, double>(inv, axis, spec, g, pr, tw, s) \
                : go_pencil<NN, float>(inv, axis, spec, g, pr, tw, s);
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
hipError_t go_zgreen(void* spec, SpecGeom g, Cubic C, Prune pr, const double2* tw, hipStream_t s) {
  constexpr int W = zg_width<N, S>();
  constexpr int T = zg_threads<N, S>();
  constexpr int NT = N * ((N / 2 + 1 + W - 1) / W);
  using C2 = typename Cplx<S>::T;
  const bool prune = pr.in_len < N;
  auto* k = prune ? k_zgreen<N, S, true> : k_zgreen<N, S, false>;
  const int grid = tile_grid(k, T, NT, sizeof(S) == 4);
  if (grid < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3(grid), dim3(T), 0, s, (C2*)spec, g.P, C, pr, tw);
  return hipGetLastError();
}

hipError_t launch_z_green(bool fp64, void* spec, SpecGeom g, Cubic C, Prune pr, const double2* tw, hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN) \
  case NN:          \
    return fp64 ? go_zgreen<NN, double>(spec, g, C, pr, tw, s) : go_zgreen<NN, float>(spec, g, C, pr, tw, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

hipError_t launch_x_inverse(bool fp64, bool accum, const void* spec, double* sig, SpecGeom g, const double* mean6,
                            const double2* tw, hipStream_t s) {
  switch (g.n) {
#define EC_CASE(NN)                                                          \
  case NN:                                                                   \
    return fp64 ? go_xi<NN, double>(accum, spec, sig, g, mean6, tw, s) \
                : go_xi<NN, float>(accum, spec, sig, g, mean6, tw, s);
    EC_FOR_SIZES(EC_CASE)
#undef EC_CASE
  }
  return hipErrorInvalidValue;
}

}  // namespace ec
