// k_energy.hip - per-defect interaction energies and the discrete self term.
//
// Sec. 2 (Betti form) with the eigenstrain: E_ij = -h^3 c sum_x eps*_i : sigma_j.
// Summing over j != i with superposition (the total field is the sum of the
// defects' fields) gives E_i = -h^3 c E_i:S_i - B_i, where S_i is the sum of the
// resident FP64 stress over the footprint of i and B_i = -h^3 c sum over pairs
// (x, y) of the footprint of E_i:G(x - y):E_i is the defect's own contribution,
// G being the discrete periodic kernel sigma = G * eps* (a window of it around
// r = 0 is enough because footprints are compact).
#include <algorithm>

#include "ec_internal.h"

namespace ec {

namespace {

// Index of the symmetric pair (a <= b) in the 21-entry window record.
__host__ __device__ constexpr int tri(int a, int b) { return a * 6 - (a * (a - 1)) / 2 + (b - a); }

__device__ __forceinline__ void neumaier(double& s, double& c, double v) {
  const double t = s + v;
  c += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
  s = t;
}

constexpr int RDT = 256;  // threads per defect

// The six stress components of voxel id (sigma is voxel-major, [n^3][6]):
// three aligned 16-byte loads.
__device__ __forceinline__ void ld_voxel(const double* __restrict__ sig, int64_t id, double* v) {
  const double2* q = reinterpret_cast<const double2*>(sig + 6 * id);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double2 w = q[j];
    v[2 * j] = w.x;
    v[2 * j + 1] = w.y;
  }
}

// (s, c) += (s2, c2) for Neumaier pairs
__device__ __forceinline__ void neumaier_merge(double& s, double& c, double s2, double c2) {
  neumaier(s, c, s2);
  c += c2;
}

// One wavefront per defect: S_i = sum of sigma over the footprint (six FP64
// Neumaier sums per lane, four members in flight per lane), combined in a
// fixed tree of lane shuffles, then E_i = -h^3 c E_i:S_i - B_i.  A footprint
// averages a few hundred members, so a wavefront keeps its lanes busy where a
// workgroup per defect would leave most of them idle and add a cross-wavefront
// combine.
constexpr int RDW = 4;  // defects (wavefronts) per workgroup

__device__ __forceinline__ void reduce_defect(const DevDefect* __restrict__ defs, const int32_t* __restrict__ cnt,
                                              const int32_t* __restrict__ ids, const double* __restrict__ sig,
                                              const double* __restrict__ B, double h3c, double* __restrict__ S6,
                                              double* __restrict__ E, double* __restrict__ E2, int i, int lane) {
  const int64_t o = defs[i].slot;
  const int m = cnt[i];
  double s[6], c[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) s[a] = c[a] = 0.0;
  int k = lane;
  for (; k + 3 * 64 < m; k += 4 * 64) {
    int id[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) id[j] = ids[o + k + j * 64];
    double v[4][6];
#pragma unroll
    for (int j = 0; j < 4; ++j) ld_voxel(sig, id[j], v[j]);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int a = 0; a < 6; ++a) neumaier(s[a], c[a], v[j][a]);
  }
  for (; k < m; k += 64) {
    double v[6];
    ld_voxel(sig, ids[o + k], v);
#pragma unroll
    for (int a = 0; a < 6; ++a) neumaier(s[a], c[a], v[a]);
  }
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const double s2 = __shfl_down(s[a], off), c2 = __shfl_down(c[a], off);
      neumaier_merge(s[a], c[a], s2, c2);
    }
  if (lane == 0) {
    double dot = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const double S = s[a] + c[a];
      dot += ddot_w(a) * defs[i].E[a] * S;
      if (S6) S6[6 * i + a] = S;
    }
    const double e = -h3c * dot - B[i];
    E[i] = e;
    if (E2) E2[i] = e;
  }
}

__global__ __launch_bounds__(64 * RDW) void k_reduce(const DevDefect* __restrict__ defs, const int32_t* __restrict__ cnt,
                                                     const int32_t* __restrict__ ids, const double* __restrict__ sig,
                                                     const double* __restrict__ B, double h3c,
                                                     double* __restrict__ S6, double* __restrict__ E, int ndef) {
  const int i = blockIdx.x * RDW + (int)(threadIdx.x >> 6);
  if (i < ndef) reduce_defect(defs, cnt, ids, sig, B, h3c, S6, E, nullptr, i, (int)(threadIdx.x & 63));
}

// Batched hops: the energies of every defect of every job (a fixed grid of
// wavefronts walks them, job after job), also into the job's output buffer
// when it has one.
__global__ __launch_bounds__(64 * RDW) void k_reduce_batch(const HopJob* __restrict__ jobs, int njob) {
  int total = 0;
  for (int j = 0; j < njob; ++j) total += jobs[j].ndef;
  for (int item = blockIdx.x * RDW + (int)(threadIdx.x >> 6); item < total; item += gridDim.x * RDW) {
    int j = 0, first = 0;
    while (item >= first + jobs[j].ndef) first += jobs[j++].ndef;
    const HopJob& J = jobs[j];
    reduce_defect(J.tab, J.cnt, J.ids, J.sig, J.B, J.h3c, J.S6, J.E, J.Eout, item - first, (int)(threadIdx.x & 63));
  }
}

// Window of the kernel from one impulse solve: sigma_a(r) is the response to a
// unit eigenstrain component b at voxel 0; store K_ab(r) = w_a sigma_a(r)
// (w = 1, 1, 1, 2, 2, 2) for a <= b, r in [-D, D]^3.
__global__ void k_window_crop(const double* __restrict__ sig, int n, int D, int b, double* __restrict__ K) {
  const int W = 2 * D + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)W * W * W) return;
  const int rx = (int)(t % W) - D, ry = (int)((t / W) % W) - D, rz = (int)(t / ((int64_t)W * W)) - D;
  const int x = (rx % n + n) % n, y = (ry % n + n) % n, z = (rz % n + n) % n;
  const int64_t id = ((int64_t)z * n + y) * n + x;
  for (int a = 0; a <= b; ++a) K[t * KWIN + tri(a, b)] = ddot_w(a) * sig[6 * id + a];
}

// Scalar window per eigenstrain direction class: g_c(r) = e_c : K(r) : e_c.
__global__ void k_class_windows(const double* __restrict__ K, int64_t W3, const double* __restrict__ dirs, int ncls,
                                double* __restrict__ g) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W3 * ncls) return;
  const int c = (int)(t / W3);
  const int64_t r = t % W3;
  const double* e = dirs + 6 * c;
  const double* k = K + r * KWIN;
  double s = 0.0;
  for (int a = 0; a < 6; ++a) {
    s += e[a] * e[a] * k[tri(a, a)];
    for (int b = a + 1; b < 6; ++b) s += 2.0 * e[a] * e[b] * k[tri(a, b)];
  }
  g[t] = s;
}

constexpr int ST = 256;
constexpr int SMAX = 8192;  // footprint voxels staged in LDS

__device__ __forceinline__ int32_t pack_xyz(int id, int n) {
  return (id % n) | (((id / n) % n) << 10) | ((id / (n * n)) << 20);
}

constexpr double SELF_TARGET = 32768.0;  // pairs per work item
constexpr int SELF_KMAX = 64;            // work items per defect at most

// Work items per defect: ceil(m (m + 1) / 2 / target), between 1 and SELF_KMAX.
__device__ __forceinline__ int self_items_of(int m) {
  const double md = m;
  const int k = (int)ceil(md * (md + 1.0) * 0.5 / SELF_TARGET);
  return k < 1 ? 1 : (k > SELF_KMAX ? SELF_KMAX : k);
}

constexpr int PT = 1024;  // threads of the planning workgroup

// The work list in one workgroup: item counts per defect, their exclusive
// scan into wbeg[0..ndef] (wbeg[ndef] = list length), and the items, rows
// [p0, p1) of a defect's pair triangle with about equal pair counts (rows
// [0, p) hold p m - p (p - 1) / 2 pairs).  Each thread takes a contiguous run
// of defects.
// Self terms by runs: a footprint is a union of runs along its run direction
// t (maximal segments of voxels p, p + t, p + 2t, ...; a convex footprint meets
// each lattice line along t in one run).  For runs A = {P_A + a t, a < L_A} and
// B = {P_B + b t, b < L_B} the pair sum of the class window g is
//   sum_{a, b} g(d + (a - b) t),  d = P_A - P_B,
// and with F, FF the single and double prefix sums of g along the lines of the
// window in direction t (zero before a line enters the window),
//   = FF(d + (L_A - 1) t) - FF(d - t) - FF(d + (L_A - 1 - L_B) t) + FF(d - (L_B + 1) t),
// four lookups per run pair instead of L_A L_B.  g is even, so the ordered
// pairs (A, B) and (B, A) give the same sum.  A defect takes this path when it
// has a run class with a table (the host gives one only when at most
// SELF_RUN_MAX runs can occur, so they fit LDS) and its box fits the tables'
// window (every pair offset within +-rt.D); the host applies the same test to
// size the pair path's work list.
__device__ __forceinline__ bool self_by_runs(const DevDefect& d, int, const RunTables& rt) {
  return d.rcls >= 0 && d.rcls < rt.nrun && d.w[0] <= rt.D + 1 && d.w[1] <= rt.D + 1 && d.w[2] <= rt.D + 1;
}

__global__ __launch_bounds__(PT) void k_self_plan(const int32_t* __restrict__ cnt, const DevDefect* __restrict__ defs,
                                                  int ndef, RunTables rt, int64_t* __restrict__ wbeg,
                                                  SelfWork* __restrict__ work, int64_t cap) {
  auto items = [&](int i) { return self_by_runs(defs[i], cnt[i], rt) ? 0 : self_items_of(cnt[i]); };
  __shared__ int64_t part[2 * (PT / 64)];
  const int per = (ndef + PT - 1) / PT;
  const int b = threadIdx.x * per, e = min(ndef, b + per);
  int64_t s = 0;
  for (int i = b; i < e; ++i) s += items(i);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) part[wv] = x;
  __syncthreads();
  if (wv == 0) {
    int64_t w = lane < PT / 64 ? part[lane] : 0;
    for (int o = 1; o < PT / 64; o <<= 1) {
      const int64_t y = __shfl_up(w, o);
      if (lane >= o) w += y;
    }
    if (lane < PT / 64) part[PT / 64 + lane] = w;
  }
  __syncthreads();
  int64_t at = x - s + (wv > 0 ? part[PT / 64 + wv - 1] : 0);
  if (threadIdx.x == PT - 1) wbeg[ndef] = part[2 * (PT / 64) - 1];
  for (int i = b; i < e; ++i) {
    const int m = cnt[i];
    const int k = items(i);
    const double tot = (double)m * (m + 1.0) * 0.5, a = m + 0.5;
    wbeg[i] = at;
    int p0 = 0;
    for (int j = 1; j <= k; ++j) {
      int p1 = m;
      if (j < k) {
        const double T = j * tot / k;
        p1 = (int)ceil(a - sqrt(fmax(0.0, a * a - 2.0 * T)));
        p1 = p1 < p0 ? p0 : (p1 > m ? m : p1);
      }
      if (at + j - 1 < cap) work[at + j - 1] = SelfWork{i, p0, p1, 0};
      p0 = p1;
    }
    at += k;
  }
}

// Each work item = rows [p0, p1) of a defect's pair triangle q >= p.  Each
// wavefront takes one row p and its lanes walk q = p + lane, p + lane + 64, ...:
// consecutive footprint voxels are x-neighbours, so the lanes read nearly
// consecutive window entries.  Off-diagonal pairs count twice (G(r) = G(-r)).
// A fixed grid walks the item list, whose length is read on the device.
__global__ __launch_bounds__(ST) void k_self(const DevDefect* __restrict__ defs, const int32_t* __restrict__ cnt,
                                             const int32_t* __restrict__ ids, int n, const double* __restrict__ K,
                                             const double* __restrict__ gcls, int D,
                                             const SelfWork* __restrict__ work, const int64_t* __restrict__ nwork_p,
                                             int64_t cap, double* __restrict__ partial) {
  __shared__ int32_t pk[SMAX];
  __shared__ double wsum[ST / 64];
  const int64_t nwork = *nwork_p < cap ? *nwork_p : cap;
  const int W = 2 * D + 1;
  const int h = n / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const SelfWork wk = work[wi];
    const int i = wk.def;
    const int m = cnt[i];
    const int64_t o = defs[i].slot;
    const int cls = defs[i].cls;
    const bool staged = m <= SMAX;
    // Footprints whose bounding box fits the window (every box offset within
    // +-D, the usual case) use box-relative coordinates: the window index of a
    // pair is then a difference of per-voxel linear indices, with no minimum
    // image.  Larger boxes (extent above half the cell) keep the
    // minimum-image path on packed coordinates.
    const int lx = defs[i].lo[0], ly = defs[i].lo[1], lz = defs[i].lo[2];
    const bool lin = defs[i].w[0] <= D + 1 && defs[i].w[1] <= D + 1 && defs[i].w[2] <= D + 1;
    auto linear = [&](int id) -> int32_t {
      int x = id % n - lx, y = (id / n) % n - ly, z = id / (n * n) - lz;
      x += x < 0 ? n : 0;
      y += y < 0 ? n : 0;
      z += z < 0 ? n : 0;
      return (z * W + y) * W + x;
    };
    auto enc = [&](int id) -> int32_t { return lin ? linear(id) : pack_xyz(id, n); };
    if (staged)
      for (int k = threadIdx.x; k < m; k += ST) pk[k] = enc(ids[o + k]);
    __syncthreads();
    auto coord = [&](int k) -> int32_t { return staged ? pk[k] : enc(ids[o + k]); };
    const int C0 = (D * W + D) * W + D;  // window index of offset 0
    auto widx = [&](int32_t P, int32_t Q) -> int {
      if (lin) return P - Q + C0;
      int rx = (P & 1023) - (Q & 1023), ry = ((P >> 10) & 1023) - ((Q >> 10) & 1023), rz = (P >> 20) - (Q >> 20);
      rx += rx < -h ? n : (rx >= n - h ? -n : 0);
      ry += ry < -h ? n : (ry >= n - h ? -n : 0);
      rz += rz < -h ? n : (rz >= n - h ? -n : 0);
      return ((rz + D) * W + (ry + D)) * W + (rx + D);
    };
    double acc = 0.0;
    if (cls >= 0 && staged && lin) {
      // the usual case, kept free of the per-pair choices of the general
      // loop below so that four window loads stay in flight per lane
      const double* g = gcls + (size_t)cls * W * W * W;
      for (int p = wk.p0 + wave; p < wk.p1; p += ST / 64)
        if (lane == 0) acc += g[C0];
      // the item's rows walk the columns q > p in chunks of 256 footprint
      // voxels, all rows of a chunk before the next: the window entries a
      // chunk reaches from neighbouring rows overlap, so they are served
      // from the L1 cache (rows walked whole would cycle through the entire
      // footprint image per row)
      // one row against the chunk [qc, qe), columns q >= q0; q past the
      // chunk reads the chunk's last voxel entry (a valid address) and
      // contributes zero, so the four loads go together
      auto row = [&](int pr, int q0, int qe) {
        const double* gp = g + (pk[pr] + C0);
        double v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int qq = q0 + lane + 64 * k;
          const double x = gp[-pk[qq < qe ? qq : qe - 1]];
          v[k] = qq < qe ? x : 0.0;
        }
        acc += 2.0 * ((v[0] + v[1]) + (v[2] + v[3]));
      };
      for (int qc = wk.p0 + 1; qc < m; qc += 256) {
        const int qe = qc + 256 < m ? qc + 256 : m;
        // rows in pairs (p, p + 1); when p + 1 is p's x-neighbour its window
        // entry for any q is the next one in memory, so one 16-byte load
        // serves both rows (the pair q = p + 1 counts for row p only)
        for (int p = wk.p0 + 2 * wave; p < wk.p1 && p + 1 < qe; p += 2 * (ST / 64)) {
          const int P = pk[p];
          const int q0 = p + 1 > qc ? p + 1 : qc;
          if (p + 1 < wk.p1 && pk[p + 1] == P + 1) {
            const double* gp = g + (P + C0);
            double v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int qq = q0 + lane + 64 * k;
              double2 w;
              __builtin_memcpy(&w, gp - pk[qq < qe ? qq : qe - 1], sizeof w);
              v[k] = qq < qe ? w.x + (qq > p + 1 ? w.y : 0.0) : 0.0;
            }
            acc += 2.0 * ((v[0] + v[1]) + (v[2] + v[3]));
          } else {
            row(p, q0, qe);
            if (p + 1 < wk.p1 && p + 2 < qe) row(p + 1, p + 2 > qc ? p + 2 : qc, qe);
          }
        }
      }
    } else if (cls >= 0) {
      const double* g = gcls + (size_t)cls * W * W * W;
      for (int p = wk.p0 + wave; p < wk.p1; p += ST / 64) {
        const int32_t P = coord(p);
        // the diagonal term once, every other pair twice (q > p)
        if (lane == 0) acc += g[C0];
        int q = p + 1 + lane;
        if (lin) {
          const double* gp = g + (P + C0);
          // four window loads in flight per lane before they are summed
          for (; q + 192 < m; q += 256) {
            const double v0 = gp[-coord(q)], v1 = gp[-coord(q + 64)];
            const double v2 = gp[-coord(q + 128)], v3 = gp[-coord(q + 192)];
            acc += 2.0 * ((v0 + v1) + (v2 + v3));
          }
          for (; q < m; q += 64) acc += 2.0 * gp[-coord(q)];
        } else {
          for (; q < m; q += 64) acc += 2.0 * g[widx(P, coord(q))];
        }
      }
    } else {
      double E[6];
      for (int a = 0; a < 6; ++a) E[a] = defs[i].E[a];
      for (int p = wk.p0 + wave; p < wk.p1; p += ST / 64) {
        const int32_t P = coord(p);
        for (int q = p + lane; q < m; q += 64) {
          const double* k = K + (size_t)widx(P, coord(q)) * KWIN;
          double v = 0.0;
          for (int a = 0; a < 6; ++a) {
            v += E[a] * E[a] * k[tri(a, a)];
            for (int b = a + 1; b < 6; ++b) v += 2.0 * E[a] * E[b] * k[tri(a, b)];
          }
          acc += (q == p) ? v : 2.0 * v;
        }
      }
    }
    for (int s = 32; s > 0; s >>= 1) acc += __shfl_down(acc, s);
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < ST / 64; ++w) t += wsum[w];
      partial[wi] = t;
    }
    __syncthreads();  // pk and wsum are rewritten by the next item
  }
}

// One workgroup per defect on the run path: the runs of the footprint (a run
// starts at a member p whose p - t is not a member; exact integer membership),
// compacted in footprint order into dynamic LDS (rcap runs), then the run
// pairs A <= B over the threads, summed with Neumaier compensation and
// combined in a fixed tree, so the result does not depend on timing.  Defects
// off the run path return at once.
//
// A run's length comes from walking p + k t until the first non-member, with
// the membership quantities updated by additions: for the offset d_k = d + k T
// (T = 1024 t, q units) |d_k|^2 and m.d_k grow by 2 d_k.T + |T|^2 and m.T.  A
// footprint spans less than half the cell, so its runs never reach the
// minimum-image wrap; past it the unwrapped offset is far outside, as the
// wrapped one would be.
__device__ __forceinline__ int wrap_n(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__global__ __launch_bounds__(ST) void k_self_runs(const DevDefect* __restrict__ defs, const int32_t* __restrict__ cnt,
                                                  const int32_t* __restrict__ ids, int n, RunTables rtab, int rcap,
                                                  double* __restrict__ runsum) {
  extern __shared__ int32_t rstart[];  // rcap entries: box-relative x | y << 10 | z << 20 of each run's first voxel
  int16_t* rlen = reinterpret_cast<int16_t*>(rstart + rcap);
  __shared__ int wcnt[ST / 64];
  __shared__ double wsum[ST / 64], wcmp[ST / 64];
  const int i = blockIdx.x;
  const DevDefect d = defs[i];
  const int m = cnt[i];
  if (!self_by_runs(d, m, rtab)) return;
  const int D = rtab.D;
  const int tx = d.rt[0], ty = d.rt[1], tz = d.rt[2];
  const int lx = d.lo[0], ly = d.lo[1], lz = d.lo[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int32_t Lq = QSUB * n, hq = Lq / 2;
  const int64_t T0 = (int64_t)QSUB * tx, T1 = (int64_t)QSUB * ty, T2 = (int64_t)QSUB * tz;
  const int64_t TT = T0 * T0 + T1 * T1 + T2 * T2;
  const int64_t mT = (int64_t)d.m[0] * T0 + (int64_t)d.m[1] * T1 + (int64_t)d.m[2] * T2;
  const int64_t lim = (int64_t)d.eq * d.eq * d.mm, rr = (int64_t)d.mm * d.R2q;
  int nrun = 0;
  for (int k0 = 0; k0 < m; k0 += ST) {
    const int k = k0 + threadIdx.x;
    bool start = false;
    int32_t pk = 0;
    int len = 0;
    if (k < m) {
      const int id = ids[d.slot + k];
      const int x = id % n, y = (id / n) % n, z = id / (n * n);
      start = !member(d, n, wrap_n(x - tx, n), wrap_n(y - ty, n), wrap_n(z - tz, n));
      if (start) {
        const int v[3] = {x, y, z};
        int64_t dd[3];
        for (int a = 0; a < 3; ++a) {
          int32_t q = QSUB * v[a] + QSUB / 2 - d.cq[a];
          q += (q < -hq) ? Lq : 0;
          q -= (q >= hq) ? Lq : 0;
          dd[a] = q;
        }
        int64_t d2 = dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2];
        int64_t dT = dd[0] * T0 + dd[1] * T1 + dd[2] * T2;
        int64_t tm = (int64_t)d.m[0] * dd[0] + (int64_t)d.m[1] * dd[1] + (int64_t)d.m[2] * dd[2];
        len = 1;
        for (; len < n; ++len) {  // offset of p + len t from that of p + (len - 1) t
          d2 += 2 * dT + TT;
          dT += TT;
          tm += mT;
          bool in;
          if (d.kind == 1) {
            in = d2 <= d.R2q;
          } else {
            const bool slab = (tm >= 0) ? (4 * tm * tm < lim) : (4 * tm * tm <= lim);
            in = slab && ((int64_t)d.mm * d2 - tm * tm <= rr);
          }
          if (!in) break;
        }
        const int bx = wrap_n(x - lx, n), by = wrap_n(y - ly, n), bz = wrap_n(z - lz, n);
        pk = bx | (by << 10) | (bz << 20);
      }
    }
    const uint64_t bal = __ballot(start);
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    int before = __popcll(bal & ((1ull << lane) - 1)), tot = 0;
    for (int w = 0; w < ST / 64; ++w) {
      if (w < wave) before += wcnt[w];
      tot += wcnt[w];
    }
    if (start && nrun + before < rcap) {  // always true under the host's run bound
      rstart[nrun + before] = pk;
      rlen[nrun + before] = (int16_t)len;
    }
    nrun += tot;
    __syncthreads();  // wcnt is rewritten by the next chunk; the runs are read below
  }
  nrun = nrun < rcap ? nrun : rcap;
  const int W = 2 * D + 1;
  const double* ff = rtab.ff + (size_t)d.rcls * W * W * W;
  double s = 0.0, c = 0.0;
  const int64_t npair = (int64_t)nrun * (nrun + 1) / 2;
  for (int64_t u = threadIdx.x; u < npair; u += ST) {
    // (A, B), A <= B, from the triangular index u = B (B + 1) / 2 + A
    int Bi = (int)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
    while ((int64_t)Bi * (Bi + 1) / 2 > u) --Bi;
    while ((int64_t)(Bi + 1) * (Bi + 2) / 2 <= u) ++Bi;
    const int Ai = (int)(u - (int64_t)Bi * (Bi + 1) / 2);
    const int32_t PA = rstart[Ai], PB = rstart[Bi];
    const int La = rlen[Ai], Lb = rlen[Bi];
    const int dx = (PA & 1023) - (PB & 1023), dy = ((PA >> 10) & 1023) - ((PB >> 10) & 1023),
              dz = (PA >> 20) - (PB >> 20);
    auto ffat = [&](int kk) -> double {
      const int px = dx + kk * tx, py = dy + kk * ty, pz = dz + kk * tz;
      if (px < -D || px > D || py < -D || py > D || pz < -D || pz > D) return 0.0;  // before the line enters
      return ff[((pz + D) * W + (py + D)) * W + (px + D)];
    };
    const double v = (ffat(La - 1) - ffat(-1)) - (ffat(La - 1 - Lb) - ffat(-Lb - 1));
    neumaier(s, c, Ai == Bi ? v : 2.0 * v);
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double s2 = __shfl_down(s, off), c2 = __shfl_down(c, off);
    neumaier_merge(s, c, s2, c2);
  }
  if (lane == 0) {
    wsum[wave] = s;
    wcmp[wave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ss = wsum[0], cc = wcmp[0];
    for (int w = 1; w < ST / 64; ++w) neumaier_merge(ss, cc, wsum[w], wcmp[w]);
    runsum[i] = ss + cc;
  }
}

// Double prefix sums of the class windows along each run class's direction:
// one thread per (run class, window point); a point whose predecessor along t
// lies outside the window starts a line, and its thread walks the line,
// storing FF = sum of F, F = sum of g (both compensated) at every point.
__global__ void k_run_tables(const double* __restrict__ g, int Dg, int D, const int4* __restrict__ info, int nrun,
                             double* __restrict__ ff) {
  const int W = 2 * D + 1, Wg = 2 * Dg + 1;
  const int64_t W3 = (int64_t)W * W * W, Wg3 = (int64_t)Wg * Wg * Wg;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= W3 * nrun) return;
  const int r = (int)(t / W3);
  const int64_t p = t % W3;
  const int4 q = info[r];
  int x = (int)(p % W) - D, y = (int)((p / W) % W) - D, z = (int)(p / ((int64_t)W * W)) - D;
  auto inside = [&](int a, int b, int c) { return a >= -D && a <= D && b >= -D && b <= D && c >= -D && c <= D; };
  if (inside(x - q.y, y - q.z, z - q.w)) return;  // not the first point of its line
  const double* gc = g + (size_t)q.x * Wg3;
  double* out = ff + (size_t)r * W3;
  double fs = 0.0, fc = 0.0, Fs = 0.0, Fc = 0.0;
  while (inside(x, y, z)) {
    const int64_t idx = ((int64_t)(z + D) * W + (y + D)) * W + (x + D);
    neumaier(fs, fc, gc[((int64_t)(z + Dg) * Wg + (y + Dg)) * Wg + (x + Dg)]);
    neumaier(Fs, Fc, fs + fc);
    out[idx] = Fs + Fc;
    x += q.y;
    y += q.z;
    z += q.w;
  }
}

// B_i = -h^3 c s_i^2 sum(partials) (class windows hold the unit direction) or
// -h^3 c sum(partials) (full-tensor path); partials added in a fixed order.
__global__ void k_self_finish(const int64_t* __restrict__ wbeg, int64_t cap, const double* __restrict__ partial,
                              const double* __restrict__ runsum, const int32_t* __restrict__ cnt, RunTables rt,
                              const DevDefect* __restrict__ defs, int ndef, double h3c, double* __restrict__ B) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndef) return;
  double s = 0.0, c = 0.0;
  if (self_by_runs(defs[i], cnt[i], rt)) s = runsum[i];
  if (cap > 0) {  // no plan ran without pair-path items
    const int64_t we = wbeg[i + 1] < cap ? wbeg[i + 1] : cap;  // the plan stores items below cap only
    for (int64_t w = wbeg[i]; w < we; ++w) neumaier(s, c, partial[w]);
  }
  const double scale = defs[i].cls >= 0 ? defs[i].s * defs[i].s : 1.0;
  B[i] = -h3c * scale * (s + c);
}

// ---- jump probes (the OkMC loop of App. B, biased jumps of Sec. 5) -----------
//
// Defect i translated by a whole-voxel jump lambda, everything else fixed:
//   E_i(X + lambda) = -h^3 c E_i : sum_{x in Omega_i + lambda} (sigma - sigma_i)(x),
//   sigma_i(x) = sum_{y in Omega_i} G(x - y) : E_i,
// so with S(lambda) the sum of the resident stress over the translated
// footprint and X(lambda) = sum over x in Omega_i + lambda, y in Omega_i of
// E_i:G(x - y):E_i (all ordered pairs; X(0) gives the self term, B_i = -h^3 c X(0)),
//   dE = -h^3 c E_i:(S(lambda) - S(0)) + h^3 c X(lambda) + B_i.

__device__ __forceinline__ int wrap_axis(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// One workgroup per (defect, jump): S(lambda) with the footprint ids shifted,
// t1 = -h^3 c E:(S(lambda) - S(0)); S(0) from the energies reduction.  With xc
// (the stored cross part of each jump, h^3 c X(lambda) + B_i, unchanged while
// the footprints only translate) also dE = t1 + xc.
__global__ __launch_bounds__(RDT) void k_jump_sums(const DevDefect* __restrict__ defs, const int32_t* __restrict__ cnt,
                                                   const int32_t* __restrict__ ids, const double* __restrict__ sig,
                                                   int n, const int32_t* __restrict__ jumps, int nj,
                                                   const double* __restrict__ S0, double h3c, double* __restrict__ t1,
                                                   const double* __restrict__ xc, double* __restrict__ dE) {
  const int i = blockIdx.x / nj;
  const int u = blockIdx.x;
  const int lx = jumps[3 * u], ly = jumps[3 * u + 1], lz = jumps[3 * u + 2];
  const int64_t o = defs[i].slot;
  const int m = cnt[i];
  double s[6], c[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) s[a] = c[a] = 0.0;
  for (int k = threadIdx.x; k < m; k += RDT) {
    const int id = ids[o + k];
    const int x = wrap_axis(id % n + lx, n), y = wrap_axis((id / n) % n + ly, n), z = wrap_axis(id / (n * n) + lz, n);
    double v[6];
    ld_voxel(sig, ((int64_t)z * n + y) * n + x, v);
#pragma unroll
    for (int a = 0; a < 6; ++a) neumaier(s[a], c[a], v[a]);
  }
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      const double s2 = __shfl_down(s[a], off), c2 = __shfl_down(c[a], off);
      neumaier_merge(s[a], c[a], s2, c2);
    }
  __shared__ double ws[RDT / 64][6], wc[RDT / 64][6];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      ws[wave][a] = s[a];
      wc[wave][a] = c[a];
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    const DevDefect d = defs[i];
    double dot = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      double ss = ws[0][a], cc = wc[0][a];
      for (int w = 1; w < RDT / 64; ++w) neumaier_merge(ss, cc, ws[w][a], wc[w][a]);
      dot += ddot_w(a) * d.E[a] * ((ss + cc) - S0[6 * i + a]);
    }
    const double v = -h3c * dot;
    t1[u] = v;
    if (xc) dE[u] = v + xc[u];
  }
}

// X(-lambda) = X(lambda) (G(r) = G(-r): swap the two voxels of every pair),
// so a jump whose opposite comes earlier in the defect's list reuses that
// jump's sum, and the zero jump needs none (X(0) is the self-term sum).
// Returns the jump whose cross sum serves jump j of defect i, or -1 for zero.
__device__ __forceinline__ int cross_source(const int32_t* __restrict__ jumps, int i, int j, int nj) {
  const int32_t* l = jumps + 3 * (i * nj + j);
  if (l[0] == 0 && l[1] == 0 && l[2] == 0) return -1;
  for (int k = 0; k < j; ++k) {
    const int32_t* q = jumps + 3 * (i * nj + k);
    if (q[0] == -l[0] && q[1] == -l[1] && q[2] == -l[2]) return k;
  }
  return j;
}

// Work items of the cross sums: per (defect, jump) ceil(m^2 / target) items
// (at most SELF_KMAX), each a range of rows p with all m columns q.
__device__ __forceinline__ int cross_items_of(int m) {
  const double md = m;
  const int k = (int)ceil(md * md / SELF_TARGET);
  return k < 1 ? 1 : (k > SELF_KMAX ? SELF_KMAX : k);
}

__global__ __launch_bounds__(PT) void k_cross_plan(const int32_t* __restrict__ cnt, int ndef, int nj,
                                                   const int32_t* __restrict__ jumps, int64_t* __restrict__ wbeg,
                                                   SelfWork* __restrict__ work, int64_t cap) {
  __shared__ int64_t part[2 * (PT / 64)];
  const int nu = ndef * nj;
  const int per = (nu + PT - 1) / PT;
  const int b = threadIdx.x * per, e = min(nu, b + per);
  int64_t s = 0;
  auto items = [&](int u) { return cross_source(jumps, u / nj, u % nj, nj) == u % nj ? cross_items_of(cnt[u / nj]) : 0; };
  for (int u = b; u < e; ++u) s += items(u);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) part[wv] = x;
  __syncthreads();
  if (wv == 0) {
    int64_t w = lane < PT / 64 ? part[lane] : 0;
    for (int o = 1; o < PT / 64; o <<= 1) {
      const int64_t y = __shfl_up(w, o);
      if (lane >= o) w += y;
    }
    if (lane < PT / 64) part[PT / 64 + lane] = w;
  }
  __syncthreads();
  int64_t at = x - s + (wv > 0 ? part[PT / 64 + wv - 1] : 0);
  if (threadIdx.x == PT - 1) wbeg[nu] = part[2 * (PT / 64) - 1];
  for (int u = b; u < e; ++u) {
    const int m = cnt[u / nj];
    const int k = items(u);
    wbeg[u] = at;
    for (int j = 0; j < k; ++j) {
      const int p0 = (int)((int64_t)m * j / k), p1 = (int)((int64_t)m * (j + 1) / k);
      if (at + j < cap) work[at + j] = SelfWork{u / nj, p0, p1, u % nj};
    }
    at += k;
  }
}

// Each item: rows [p0, p1) of defect def against all of its m footprint voxels,
// for jump `pad` of that defect.  Box-relative linear coordinates when every
// pair offset plus the jump stays within the window, packed coordinates with
// the minimum image otherwise; the class window, or the full tensor window
// for a defect without a class.
__global__ __launch_bounds__(ST) void k_cross(const DevDefect* __restrict__ defs, const int32_t* __restrict__ cnt,
                                              const int32_t* __restrict__ ids, int n, const double* __restrict__ K,
                                              const double* __restrict__ gcls, int D,
                                              const int32_t* __restrict__ jumps, int nj,
                                              const SelfWork* __restrict__ work, const int64_t* __restrict__ nwork_p,
                                              int64_t cap, double* __restrict__ partial) {
  __shared__ int32_t pk[SMAX];
  __shared__ double wsum[ST / 64];
  const int64_t nwork = *nwork_p < cap ? *nwork_p : cap;
  const int W = 2 * D + 1;
  const int h = n / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
    const SelfWork wk = work[wi];
    const int i = wk.def;
    const int m = cnt[i];
    const int64_t o = defs[i].slot;
    const int cls = defs[i].cls;
    const int* lam = jumps + 3 * (i * nj + wk.pad);
    const int lx = lam[0], ly = lam[1], lz = lam[2];
    const bool staged = m <= SMAX;
    const int bx = defs[i].lo[0], by = defs[i].lo[1], bz = defs[i].lo[2];
    const bool lin = defs[i].w[0] + abs(lx) <= D + 1 && defs[i].w[1] + abs(ly) <= D + 1 &&
                     defs[i].w[2] + abs(lz) <= D + 1;
    auto linear = [&](int id) -> int32_t {
      int x = id % n - bx, y = (id / n) % n - by, z = id / (n * n) - bz;
      x += x < 0 ? n : 0;
      y += y < 0 ? n : 0;
      z += z < 0 ? n : 0;
      return (z * W + y) * W + x;
    };
    auto enc = [&](int id) -> int32_t { return lin ? linear(id) : pack_xyz(id, n); };
    if (staged)
      for (int k = threadIdx.x; k < m; k += ST) pk[k] = enc(ids[o + k]);
    __syncthreads();
    auto coord = [&](int k) -> int32_t { return staged ? pk[k] : enc(ids[o + k]); };
    const int C0 = (D * W + D) * W + D;
    const int L0 = (lz * W + ly) * W + lx;  // the jump in window-linear units
    auto widx = [&](int32_t P, int32_t Q) -> int {
      if (lin) return P - Q + L0 + C0;
      int rx = (P & 1023) - (Q & 1023) + lx, ry = ((P >> 10) & 1023) - ((Q >> 10) & 1023) + ly,
          rz = (P >> 20) - (Q >> 20) + lz;
      rx += rx < -h ? n : (rx >= n - h ? -n : 0);
      ry += ry < -h ? n : (ry >= n - h ? -n : 0);
      rz += rz < -h ? n : (rz >= n - h ? -n : 0);
      return ((rz + D) * W + (ry + D)) * W + (rx + D);
    };
    double acc = 0.0;
    if (cls >= 0 && staged && lin) {
      const double* g = gcls + (size_t)cls * W * W * W;
      for (int p = wk.p0 + wave; p < wk.p1; p += ST / 64) {
        const double* gp = g + (pk[p] + L0 + C0);
        for (int q = lane; q < m; q += 256) {
          double v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int qq = q + 64 * k;
            const double x = gp[-pk[qq < m ? qq : m - 1]];
            v[k] = qq < m ? x : 0.0;
          }
          acc += (v[0] + v[1]) + (v[2] + v[3]);
        }
      }
    } else if (cls >= 0) {
      const double* g = gcls + (size_t)cls * W * W * W;
      for (int p = wk.p0 + wave; p < wk.p1; p += ST / 64) {
        const int32_t P = coord(p);
        for (int q = lane; q < m; q += 64) acc += g[widx(P, coord(q))];
      }
    } else {
      double E[6];
      for (int a = 0; a < 6; ++a) E[a] = defs[i].E[a];
      for (int p = wk.p0 + wave; p < wk.p1; p += ST / 64) {
        const int32_t P = coord(p);
        for (int q = lane; q < m; q += 64) {
          const double* k = K + (size_t)widx(P, coord(q)) * KWIN;
          double v = 0.0;
          for (int a = 0; a < 6; ++a) {
            v += E[a] * E[a] * k[tri(a, a)];
            for (int b = a + 1; b < 6; ++b) v += 2.0 * E[a] * E[b] * k[tri(a, b)];
          }
          acc += v;
        }
      }
    }
    for (int sh = 32; sh > 0; sh >>= 1) acc += __shfl_down(acc, sh);
    if (lane == 0) wsum[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < ST / 64; ++w) t += wsum[w];
      partial[wi] = t;
    }
    __syncthreads();  // pk and wsum are rewritten by the next item
  }
}

// dE per (defect, jump): X = the item partials (of the jump itself or of its
// opposite) added in a fixed order; the zero jump keeps only the S term.  The
// cross part xc = h^3 c X + B_i is stored, so that dE = t1 + xc comes out the
// same whether xc is fresh or reused.
__global__ void k_cross_finish(const int64_t* __restrict__ wbeg, const double* __restrict__ partial,
                               const DevDefect* __restrict__ defs, int ndef, int nj, const int32_t* __restrict__ jumps,
                               const double* __restrict__ t1, const double* __restrict__ B, double h3c,
                               double* __restrict__ xc, double* __restrict__ dE) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= ndef * nj) return;
  const int i = u / nj;
  const int src = cross_source(jumps, i, u % nj, nj);
  double x = 0.0;
  if (src >= 0) {
    const int us = i * nj + src;
    double s = 0.0, c = 0.0;
    for (int64_t w = wbeg[us]; w < wbeg[us + 1]; ++w) neumaier(s, c, partial[w]);
    const double scale = defs[i].cls >= 0 ? defs[i].s * defs[i].s : 1.0;
    x = h3c * scale * (s + c) + B[i];
  }
  xc[u] = x;
  dE[u] = t1[u] + x;
}

// Biased frequencies nu = 1/2 nu0 exp(-(Em + dE / 2) / kT) of every jump of a
// defect, and the jump whose frequency-line interval holds xi: the first j
// with xi <= R_j / R_tot (R the running sum in jump order).
__global__ void k_jump_select(const double* __restrict__ dE, int ndef, int nj, const double* __restrict__ Em,
                              double nu0, double kT, const double* __restrict__ xi, const double* __restrict__ u,
                              double dt, double* __restrict__ nu, int32_t* __restrict__ choice) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndef) return;
  double tot = 0.0;
  for (int j = 0; j < nj; ++j) {
    const double v = 0.5 * nu0 * exp(-(Em[i] + 0.5 * dE[i * nj + j]) / kT);
    if (nu) nu[i * nj + j] = v;
    tot += v;
  }
  if (!choice) return;
  // Poisson gate of the time step: no event when u <= P(N = 0) = exp(-nu_i dt),
  // nu_i the defect's nominal frequency
  if (u && u[i] <= exp(-nu0 * exp(-Em[i] / kT) * dt)) {
    choice[i] = -1;
    return;
  }
  double R = 0.0;
  int pick = nj - 1;
  for (int j = 0; j < nj; ++j) {
    R += 0.5 * nu0 * exp(-(Em[i] + 0.5 * dE[i * nj + j]) / kT);
    if (xi[i] <= R / tot) {
      pick = j;
      break;
    }
  }
  choice[i] = pick;
}

// ---- dipole-tensor energies (Sec. 2.1) ------------------------------------------
//
// E_i^dip = -h^3 c m_i E_i : (sigma(x_c) - sigma_i(x_c)), x_c the voxel holding
// the defect centre and sigma_i(x_c) = sum_{y in Omega_i} G(x_c - y) : E_i (the
// window); one workgroup per defect.
__global__ __launch_bounds__(RDT) void k_dipole(const DevDefect* __restrict__ defs, const int32_t* __restrict__ cnt,
                                                const int32_t* __restrict__ ids, const double* __restrict__ sig,
                                                int n, const double* __restrict__ K,
                                                const double* __restrict__ gcls, int D, double h3c,
                                                double* __restrict__ Edip) {
  const int i = blockIdx.x;
  const DevDefect d = defs[i];
  const int64_t o = d.slot;
  const int m = cnt[i];
  const int W = 2 * D + 1;
  const int hn = n / 2;
  int c[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) c[k] = (d.cq[k] / QSUB) % n;
  double acc = 0.0;
  for (int k = threadIdx.x; k < m; k += RDT) {
    const int id = ids[o + k];
    int r[3] = {c[0] - id % n, c[1] - (id / n) % n, c[2] - id / (n * n)};
#pragma unroll
    // minimum image: [-n/2, n/2) for even n, [-(n-1)/2, (n-1)/2] for odd n
    for (int a = 0; a < 3; ++a) r[a] += r[a] < -hn ? n : (r[a] >= n - hn ? -n : 0);
    const int w = ((r[2] + D) * W + (r[1] + D)) * W + (r[0] + D);
    if (d.cls >= 0) {
      acc += gcls[(size_t)d.cls * W * W * W + w];
    } else {
      const double* kk = K + (size_t)w * KWIN;
      double v = 0.0;
      for (int a = 0; a < 6; ++a) {
        v += d.E[a] * d.E[a] * kk[tri(a, a)];
        for (int b = a + 1; b < 6; ++b) v += 2.0 * d.E[a] * d.E[b] * kk[tri(a, b)];
      }
      acc += v;
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
  __shared__ double ws[RDT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) ws[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double own = 0.0;
    for (int w = 0; w < RDT / 64; ++w) own += ws[w];
    if (d.cls >= 0) own *= d.s * d.s;
    double s6[6];
    ld_voxel(sig, ((int64_t)c[2] * n + c[1]) * n + c[0], s6);
    double dot = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) dot += ddot_w(a) * d.E[a] * s6[a];
    Edip[i] = -h3c * m * (dot - own);
  }
}

// Dense component-major outputs [6][n^3] from the voxel-major sigma: which
// 0 -> sigma, 1 -> eps = C^-1:sigma + eps* (cubic compliance, in the cube
// frame for a rotated crystal), 2 -> eps*
// (owner-list gather).
template <typename OT>
__global__ void k_sig_to_out(const double* __restrict__ sig, const int32_t* __restrict__ own,
                             const int2* __restrict__ lnk, const DevDefect* __restrict__ defs, int max_links,
                             int64_t n3, Cubic C, int which, OT* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n3) return;
  double es[6] = {0, 0, 0, 0, 0, 0};
  if (which > 0) {
    decode_voxel(own[t], lnk, defs, es, max_links);
  }
  if (which == 2) {
    double el[6];
    if (C.frm)
      rot6(C.frm + 36, es, el);  // the rasterised eigenstrain is kept in the cube frame
    else
      for (int a = 0; a < 6; ++a) el[a] = es[a];
    for (int a = 0; a < 6; ++a) out[a * n3 + t] = (OT)el[a];
    return;
  }
  double s[6];
  ld_voxel(sig, t, s);
  if (which == 0) {
#pragma unroll
    for (int a = 0; a < 6; ++a) out[a * n3 + t] = (OT)s[a];
    return;
  }
  const double den = (C.C11 - C.C12) * (C.C11 + 2.0 * C.C12);
  const double S11 = (C.C11 + C.C12) / den, S12 = -C.C12 / den, S44h = 0.5 / C.C44;
  double sc[6], ec[6], e[6];
  if (C.frm)
    rot6(C.frm, s, sc);  // the compliance applied in the cube frame
  else
    for (int a = 0; a < 6; ++a) sc[a] = s[a];
  ec[0] = S11 * sc[0] + S12 * (sc[1] + sc[2]);
  ec[1] = S11 * sc[1] + S12 * (sc[0] + sc[2]);
  ec[2] = S11 * sc[2] + S12 * (sc[0] + sc[1]);
  for (int a = 3; a < 6; ++a) ec[a] = S44h * sc[a];
  if (C.frm) {
    // eps = C^-1:sigma + eps*, both in the cube frame, then back to the cell
    for (int a = 0; a < 6; ++a) ec[a] += es[a];
    rot6(C.frm + 36, ec, e);
  } else {
    for (int a = 0; a < 6; ++a) e[a] = ec[a] + es[a];
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) out[a * n3 + t] = (OT)e[a];
}

__global__ __launch_bounds__(256) void k_set_class(DevDefect* __restrict__ defs, int ndef,
                                                   const ClassTag* __restrict__ tags) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < ndef) {
    defs[i].cls = tags[i].cls;
    defs[i].s = tags[i].s;
    defs[i].rcls = tags[i].rcls;
  }
}

}  // namespace

hipError_t launch_set_class(DevDefect* d, int ndef, const ClassTag* tags, hipStream_t s) {
  if (ndef <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_class, dim3((ndef + 255) / 256), dim3(256), 0, s, d, ndef, tags);
  return hipGetLastError();
}

hipError_t launch_reduce(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids, const double* sig,
                         const double* B, double h3c, double* S6, double* E, hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce, dim3((ndef + RDW - 1) / RDW), dim3(64 * RDW), 0, s, d, counts, ids, sig, B, h3c, S6, E,
                     ndef);
  return hipGetLastError();
}

hipError_t launch_hop_batch_energies(const HopJob* jobs, int njob, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_batch, dim3(1024), dim3(64 * RDW), 0, s, jobs, njob);
  return hipGetLastError();
}

hipError_t launch_window_crop(const double* sig, int n, int D, int b, double* K, hipStream_t s) {
  const int W = 2 * D + 1;
  const int64_t W3 = (int64_t)W * W * W;
  hipLaunchKernelGGL(k_window_crop, dim3((unsigned)((W3 + 255) / 256)), dim3(256), 0, s, sig, n, D, b, K);
  return hipGetLastError();
}

hipError_t launch_class_windows(const double* K, int D, const double* dirs, int ncls, double* g, hipStream_t s) {
  if (ncls == 0) return hipSuccess;
  const int W = 2 * D + 1;
  const int64_t W3 = (int64_t)W * W * W;
  hipLaunchKernelGGL(k_class_windows, dim3((unsigned)((W3 * ncls + 255) / 256)), dim3(256), 0, s, K, W3, dirs, ncls,
                     g);
  return hipGetLastError();
}

hipError_t launch_self_terms(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids, int n,
                             const double* K, const double* gcls, int D, RunTables rt, SelfWork* work,
                             int64_t work_cap, int64_t* wbeg, double* partial, double* runsum, double h3c, double* B,
                             hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  const int g1 = (ndef + 255) / 256;
  if (rt.nrun > 0) {
    const int rcap = std::max(1, std::min(rt.max_runs, SELF_RUN_MAX));
    const size_t lds = (size_t)rcap * (sizeof(int32_t) + sizeof(int16_t));
    hipLaunchKernelGGL(k_self_runs, dim3(ndef), dim3(ST), lds, s, d, counts, ids, n, rt, rcap, runsum);
  }
  // the pair path only for the defects off the run path (work_cap bounds their
  // items; none: neither the plan nor the pair kernel runs)
  if (work_cap > 0) {
    hipLaunchKernelGGL(k_self_plan, dim3(1), dim3(PT), 0, s, counts, d, ndef, rt, wbeg, work, work_cap);
    const int grid = (int)std::min<int64_t>(work_cap, 4096);
    hipLaunchKernelGGL(k_self, dim3(grid), dim3(ST), 0, s, d, counts, ids, n, K, gcls, D, work, wbeg + ndef,
                       work_cap, partial);
  }
  hipLaunchKernelGGL(k_self_finish, dim3(g1), dim3(256), 0, s, wbeg, work_cap, partial, runsum, counts, rt, d, ndef,
                     h3c, B);
  return hipGetLastError();
}

hipError_t launch_run_tables(const double* g, int Dg, int Drun, const int4* info, int nrun, double* ff,
                             hipStream_t s) {
  if (nrun == 0) return hipSuccess;
  if (Drun > Dg) return hipErrorInvalidValue;
  const int W = 2 * Drun + 1;
  const int64_t tot = (int64_t)W * W * W * nrun;
  hipLaunchKernelGGL(k_run_tables, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, g, Dg, Drun, info, nrun,
                     ff);
  return hipGetLastError();
}

hipError_t launch_jump_energies(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids,
                                const double* sig, int n, const int32_t* jumps, int nj, const double* S0,
                                const double* K, const double* gcls, int D, SelfWork* work, int64_t work_cap,
                                int64_t* wbeg, double* partial, double* t1, const double* B, double h3c, double* xc,
                                bool xc_valid, double* dE, hipStream_t s) {
  if (ndef == 0 || nj == 0) return hipSuccess;
  const int nu = ndef * nj;
  if (xc_valid) {
    hipLaunchKernelGGL(k_jump_sums, dim3(nu), dim3(RDT), 0, s, d, counts, ids, sig, n, jumps, nj, S0, h3c, t1,
                       (const double*)xc, dE);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_jump_sums, dim3(nu), dim3(RDT), 0, s, d, counts, ids, sig, n, jumps, nj, S0, h3c, t1,
                     (const double*)nullptr, (double*)nullptr);
  hipLaunchKernelGGL(k_cross_plan, dim3(1), dim3(PT), 0, s, counts, ndef, nj, jumps, wbeg, work, work_cap);
  const int grid = (int)std::min<int64_t>(work_cap, 4096);
  hipLaunchKernelGGL(k_cross, dim3(grid), dim3(ST), 0, s, d, counts, ids, n, K, gcls, D, jumps, nj, work, wbeg + nu,
                     work_cap, partial);
  hipLaunchKernelGGL(k_cross_finish, dim3((nu + 255) / 256), dim3(256), 0, s, wbeg, partial, d, ndef, nj, jumps, t1, B,
                     h3c, xc, dE);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_apply_jumps(const DevDefect* __restrict__ src, DevDefect* __restrict__ dst,
                                                     int ndef, const int32_t* __restrict__ choice,
                                                     const int32_t* __restrict__ jumps, int nj, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ndef) return;
  DevDefect d = src[i];
  const int c = choice[i];
  if (c >= 0) {
    const int32_t* l = jumps + ((size_t)i * nj + c) * 3;
    const int64_t Lq = (int64_t)QSUB * n;
    for (int k = 0; k < 3; ++k) {
      d.cq[k] = (int32_t)((((int64_t)d.cq[k] + (int64_t)l[k] * QSUB) % Lq + Lq) % Lq);
      d.lo[k] = ((d.lo[k] + l[k]) % n + n) % n;
    }
  }
  dst[i] = d;
}

hipError_t launch_apply_jumps(const DevDefect* src, DevDefect* dst, int ndef, const int32_t* choice,
                              const int32_t* jumps, int nj, int n, hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_apply_jumps, dim3((ndef + 255) / 256), dim3(256), 0, s, src, dst, ndef, choice, jumps, nj, n);
  return hipGetLastError();
}

hipError_t launch_jump_select(const double* dE, int ndef, int nj, const double* Em, double nu0, double kT,
                              const double* xi, const double* u, double dt, double* nu, int32_t* choice,
                              hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_jump_select, dim3((ndef + 255) / 256), dim3(256), 0, s, dE, ndef, nj, Em, nu0, kT, xi, u, dt,
                     nu, choice);
  return hipGetLastError();
}

hipError_t launch_dipole(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids, const double* sig,
                         int n, const double* K, const double* gcls, int D, double h3c, double* Edip, hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dipole, dim3(ndef), dim3(RDT), 0, s, d, counts, ids, sig, n, K, gcls, D, h3c, Edip);
  return hipGetLastError();
}

hipError_t launch_sig_to_out(const double* sig, const int32_t* own, const int2* lnk, const DevDefect* defs, int ndef,
                             int64_t n3, Cubic C, int which, bool fp32, void* out, hipStream_t s) {
  const unsigned grid = (unsigned)((n3 + 255) / 256);
  if (fp32)
    hipLaunchKernelGGL(k_sig_to_out<float>, dim3(grid), dim3(256), 0, s, sig, own, lnk, defs, ndef, n3, C, which,
                       (float*)out);
  else
    hipLaunchKernelGGL(k_sig_to_out<double>, dim3(grid), dim3(256), 0, s, sig, own, lnk, defs, ndef, n3, C, which,
                       (double*)out);
  return hipGetLastError();
}

}  // namespace ec
