// k_raster.hip - defects to the eigenstrain field and footprint lists.
//
// Sec. 3.1: loop eigenstrain sym(b x n)/e over a slab of thickness e around the
// loop disk; point-defect clusters as dilatational spheres.  Sec. 3.4: fields
// live at voxel centres h (m + 1/2).  One workgroup per defect walks the
// defect's bounding box row by row in ascending voxel-id order, tests
// membership in exact integer arithmetic, compacts the members with a
// workgroup prefix sum (so the footprint list is sorted) and pushes every
// membership onto its voxel's list with one 32-bit atomic exchange.
#include "ec_internal.h"

namespace ec {

namespace {

constexpr int RT = 256;  // threads per rasteriser workgroup

// Exclusive scan of counts into offsets[0..ndef] (offsets[ndef] = total); one workgroup.
__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ counts, int ndef,
                                               int64_t* __restrict__ offsets) {
  constexpr int T = 1024;
  __shared__ int64_t part[2 * (T / 64)];
  const int per = (ndef + T - 1) / T;
  const int b = threadIdx.x * per, e = min(ndef, b + per);
  int64_t s = 0;
  for (int i = b; i < e; ++i) s += counts[i];
  // exclusive scan of the per-thread sums: within each wavefront by lane
  // shuffles, then over the sixteen wavefront totals
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int64_t x = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) part[wv] = x;
  __syncthreads();
  if (wv == 0) {
    int64_t w = lane < T / 64 ? part[lane] : 0;
    for (int o = 1; o < T / 64; o <<= 1) {
      const int64_t y = __shfl_up(w, o);
      if (lane >= o) w += y;
    }
    if (lane < T / 64) part[T / 64 + lane] = w;  // inclusive wavefront totals
  }
  __syncthreads();
  int64_t acc = x - s + (wv > 0 ? part[T / 64 + wv - 1] : 0);
  if (threadIdx.x == T - 1) offsets[ndef] = part[T / 64 + T / 64 - 1];
  for (int i = b; i < e; ++i) {
    offsets[i] = acc;
    acc += counts[i];
  }
}

// One workgroup per defect.  The bounding box is taken in chunks of RCH rows
// (y, z) in ascending order; each row's candidate x range comes from the
// geometry, a scan flattens the chunk's candidates in ascending voxel id, and
// each thread tests one candidate at a time.  A ballot scan gives every member
// its place, so the footprint list comes out sorted with no per-row serial
// work, and the atomics of a pass are independent of each other.
constexpr int RCH = 1024;

__device__ __forceinline__ void row_yz(const DevDefect& d, int n, int r, int& y, int& z) {
  const int iz = r / d.w[1], iy = r - iz * d.w[1];
  y = box_axis(d.lo[1], d.w[1], n, iy);
  z = box_axis(d.lo[2], d.w[2], n, iz);
}

__global__ __launch_bounds__(RT) void k_raster_fill(const DevDefect* __restrict__ defs, int n,
                                                    int32_t* __restrict__ ids, int2* __restrict__ lnk,
                                                    int32_t* __restrict__ counts, int32_t* __restrict__ own) {
  const DevDefect d = defs[blockIdx.x];
  const int nrows = d.w[1] * d.w[2];
  __shared__ int roff[RCH + 1];  // candidates before each row of the chunk
  __shared__ int rxa[RCH];       // first candidate x of each row, unwrapped (may be >= n)
  __shared__ int wsum[RT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int PER = RCH / RT;
  int run = 0;  // members placed so far (same value in every thread)
  for (int r0 = 0; r0 < nrows; r0 += RCH) {
    const int nr = min(RCH, nrows - r0);
    // candidate counts of this thread's PER consecutive rows, then a scan
    int c[PER], s = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int j = threadIdx.x * PER + k;
      c[k] = 0;
      if (j < nr) {
        int y, z, u0, u1;
        row_yz(d, n, r0 + j, y, z);
        if (row_range(d, n, y, z, u0, u1)) {
          c[k] = u1 - u0 + 1;
          rxa[j] = d.lo[0] + u0;
        }
      }
      s += c[k];
    }
    int incl = s;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int acc = incl - s, ctot = 0;
    for (int w = 0; w < RT / 64; ++w) {
      if (w < wave) acc += wsum[w];
      ctot += wsum[w];
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int j = threadIdx.x * PER + k;
      if (j < nr) roff[j] = acc;
      acc += c[k];
    }
    if (threadIdx.x == 0) roff[nr] = ctot;
    __syncthreads();
    for (int k0 = 0; k0 < ctot; k0 += RT) {
      const int k = k0 + threadIdx.x;
      bool is = false;
      int id = 0;
      if (k < ctot) {
        int lo = 0, hi = nr - 1;  // the row holding candidate k
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (roff[mid] <= k) lo = mid;
          else hi = mid - 1;
        }
        const int ci = k - roff[lo];
        const int xa = rxa[lo], xb = xa + (roff[lo + 1] - roff[lo]) - 1;
        int x;
        if (xa < n && xb >= n) {  // wrapped row: [0, xb - n] comes before [xa, n - 1]
          const int nlow = xb - n + 1;
          x = ci < nlow ? ci : xa + (ci - nlow);
        } else {
          x = (xa >= n ? xa - n : xa) + ci;
        }
        int y, z;
        row_yz(d, n, r0 + lo, y, z);
        is = member(d, n, x, y, z);
        id = (z * n + y) * n + x;
      }
      const uint64_t m = __ballot(is);
      if (lane == 0) wsum[wave] = __popcll(m);
      __syncthreads();
      int before = __popcll(m & ((1ull << lane) - 1)), tot = 0;
      for (int w = 0; w < RT / 64; ++w) {
        if (w < wave) before += wsum[w];
        tot += wsum[w];
      }
      if (is) {
        const int64_t e = d.slot + run + before;
        ids[e] = id;
        int32_t next = -1;
        if (atomicCAS(&own[id], -1, (int32_t)blockIdx.x) != -1) next = atomicExch(&own[id], entry_link(e));
        lnk[e] = make_int2((int)blockIdx.x, next);
      }
      run += tot;
      __syncthreads();  // wsum is rewritten by the next pass
    }
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = run;
}

// Empty the lists of all voxels of all listed footprints (plain stores).
__global__ __launch_bounds__(RT) void k_unraster(const DevDefect* __restrict__ defs,
                                                 const int32_t* __restrict__ counts, const int32_t* __restrict__ ids,
                                                 int32_t* __restrict__ own) {
  const int64_t o = defs[blockIdx.x].slot;
  const int cnt = counts[blockIdx.x];
  for (int i = threadIdx.x; i < cnt; i += RT) own[ids[o + i]] = -1;
}

__device__ __forceinline__ int shift_id(int id, int sx, int sy, int sz, int n) {
  int x = id % n + sx, y = (id / n) % n + sy, z = id / (n * n) + sz;
  x += (x < 0) ? n : ((x >= n) ? -n : 0);
  y += (y < 0) ? n : ((y >= n) ? -n : 0);
  z += (z < 0) ? n : ((z >= n) ? -n : 0);
  return (z * n + y) * n + x;
}

// Remove defect `def` from the chains of its old voxels.  Each voxel of one
// footprint is visited by exactly one thread, and no other chain changes
// meanwhile.  The defect sits on the chain either as a terminal id or as an
// entry; either way the link that points to it is redirected past it.
__global__ __launch_bounds__(RT) void k_unlink(int def, int max_links, const int32_t* __restrict__ cnt_p,
                                               int64_t slot, const int32_t* __restrict__ ids, int2* __restrict__ lnk,
                                               int32_t* __restrict__ own) {
  const int cnt = *cnt_p;
  for (int k = blockIdx.x * RT + threadIdx.x; k < cnt; k += gridDim.x * RT) {
    int32_t* p = &own[ids[slot + k]];
    for (int guard = 0; guard < max_links; ++guard) {  // a chain holds each defect once
      const int32_t link = *p;
      if (link == -1) break;  // not found (cannot happen for a consistent chain)
      if (link >= 0) {
        if (link == def) *p = -1;
        break;
      }
      int2* L = &lnk[-2 - link];
      if (L->x == def) {
        *p = L->y;
        break;
      }
      p = &L->y;
    }
  }
}

// Link the moved defect's new entries (ids shifted in place, or copied from new_ids).
__global__ __launch_bounds__(RT) void k_link(int def, const int32_t* __restrict__ cnt_p, int64_t old_slot,
                                             const int32_t* __restrict__ new_ids, int cnt_new, int64_t new_slot,
                                             int sx, int sy, int sz, int n, int32_t* __restrict__ ids,
                                             int2* __restrict__ lnk, int32_t* __restrict__ own) {
  const int cnt = new_ids ? cnt_new : *cnt_p;
  for (int k = blockIdx.x * RT + threadIdx.x; k < cnt; k += gridDim.x * RT) {
    const int64_t e = new_slot + k;
    const int id = new_ids ? new_ids[k] : shift_id(ids[old_slot + k], sx, sy, sz, n);
    ids[e] = id;
    int32_t next = -1;
    if (atomicCAS(&own[id], -1, def) != -1) next = atomicExch(&own[id], entry_link(e));
    lnk[e] = make_int2(def, next);
  }
}

// Batched hops: unlink every job's moved defect from its old voxels, then (a
// second launch) link it at its voxels shifted by the hop, then copy every
// job's moved record into its table.  Sixteen blocks per job.
__global__ __launch_bounds__(RT) void k_unlink_batch(const HopJob* __restrict__ jobs) {
  const HopJob& J = jobs[blockIdx.x / 16];
  const int lb = blockIdx.x % 16;
  const int cnt = J.cnt[J.idx];
  for (int k = lb * RT + threadIdx.x; k < cnt; k += 16 * RT) {
    int32_t* p = &J.own[J.ids[J.slot + k]];
    for (int guard = 0; guard < J.ndef; ++guard) {  // a chain holds each defect once
      const int32_t link = *p;
      if (link == -1) break;
      if (link >= 0) {
        if (link == J.idx) *p = -1;
        break;
      }
      int2* L = &J.lnk[-2 - link];
      if (L->x == J.idx) {
        *p = L->y;
        break;
      }
      p = &L->y;
    }
  }
}

__global__ __launch_bounds__(RT) void k_link_batch(const HopJob* __restrict__ jobs, int n) {
  const HopJob& J = jobs[blockIdx.x / 16];
  const int lb = blockIdx.x % 16;
  const int cnt = J.cnt[J.idx];
  for (int k = lb * RT + threadIdx.x; k < cnt; k += 16 * RT) {
    const int64_t e = J.slot + k;
    const int id = shift_id(J.ids[e], J.sx, J.sy, J.sz, n);
    J.ids[e] = id;
    int32_t next = -1;
    if (atomicCAS(&J.own[id], -1, J.idx) != -1) next = atomicExch(&J.own[id], entry_link(e));
    J.lnk[e] = make_int2(J.idx, next);
  }
}

__global__ __launch_bounds__(64) void k_set_records(const HopJob* __restrict__ jobs) {
  const HopJob& J = jobs[blockIdx.x];
  const int32_t* src = reinterpret_cast<const int32_t*>(&J.rec);
  int32_t* dst = reinterpret_cast<int32_t*>(J.tab + J.idx);
  for (int w = threadIdx.x; w < (int)(sizeof(DevDefect) / 4); w += 64) dst[w] = src[w];
}

// Additive constant of the stress for the xi = 0 condition.  Mean strain zero:
// sigma gets -C:<eps*>, <eps*> = (1/n^3) sum_i |Omega_i| E_i, compensated FP64
// sums over a fixed partition of the defects (deterministic).  Mean stress
// zero: nothing to add (the host does not launch this kernel).
constexpr int MT = 256;
__global__ __launch_bounds__(MT) void k_mean_stress(const DevDefect* __restrict__ defs,
                                                    const int32_t* __restrict__ counts, int ndef, double inv_n3,
                                                    Cubic C, double* __restrict__ add6) {
  __shared__ double ps[6][MT], pc[6][MT];
  double s[6], c[6];
  for (int a = 0; a < 6; ++a) s[a] = c[a] = 0.0;
  for (int i = threadIdx.x; i < ndef; i += MT) {
    const double k = (double)counts[i];
    for (int a = 0; a < 6; ++a) {
      const double v = k * defs[i].E[a];
      const double t = s[a] + v;
      c[a] += (fabs(s[a]) >= fabs(v)) ? ((s[a] - t) + v) : ((v - t) + s[a]);
      s[a] = t;
    }
  }
  for (int a = 0; a < 6; ++a) {
    ps[a][threadIdx.x] = s[a];
    pc[a][threadIdx.x] = c[a];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double m[6];
  for (int a = 0; a < 6; ++a) {
    double ss = 0.0, cc = 0.0;
    for (int t = 0; t < MT; ++t) {
      const double v = ps[a][t];
      const double u = ss + v;
      cc += (fabs(ss) >= fabs(v)) ? ((ss - u) + v) : ((v - u) + ss);
      ss = u;
      cc += pc[a][t];
    }
    m[a] = (ss + cc) * inv_n3;
  }
  double mc[6], t[6];
  if (C.frm)
    rot6(C.frm, m, mc);  // the mean eigenstrain in the cube frame
  else
    for (int a = 0; a < 6; ++a) mc[a] = m[a];
  t[0] = -(C.C11 * mc[0] + C.C12 * (mc[1] + mc[2]));
  t[1] = -(C.C11 * mc[1] + C.C12 * (mc[0] + mc[2]));
  t[2] = -(C.C11 * mc[2] + C.C12 * (mc[0] + mc[1]));
  for (int a = 3; a < 6; ++a) t[a] = -2.0 * C.C44 * mc[a];
  if (C.frm)
    rot6(C.frm + 36, t, add6);
  else
    for (int a = 0; a < 6; ++a) add6[a] = t[a];
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

}  // namespace

hipError_t launch_scan(const int32_t* counts, int ndef, int64_t* offsets, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, ndef, offsets);
  return hipGetLastError();
}

hipError_t launch_raster_fill(const DevDefect* d, int ndef, int n, int32_t* ids, int2* lnk, int32_t* counts,
                              int32_t* own, hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_fill, dim3(ndef), dim3(RT), 0, s, d, n, ids, lnk, counts, own);
  return hipGetLastError();
}

hipError_t launch_unraster(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids, int32_t* own,
                           hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unraster, dim3(ndef), dim3(RT), 0, s, d, counts, ids, own);
  return hipGetLastError();
}

hipError_t launch_move_lists(int def, int ndef, const int32_t* cnt_old, int64_t old_slot, const int32_t* new_ids,
                             int cnt_new, int64_t new_slot, int sx, int sy, int sz, int n, int32_t* ids, int2* lnk,
                             int32_t* own, hipStream_t s) {
  hipLaunchKernelGGL(k_unlink, dim3(16), dim3(RT), 0, s, def, ndef, cnt_old, old_slot, ids, lnk, own);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_link, dim3(16), dim3(RT), 0, s, def, cnt_old, old_slot, new_ids, cnt_new, new_slot, sx, sy, sz,
                     n, ids, lnk, own);
  return hipGetLastError();
}

hipError_t launch_hop_batch_lists(const HopJob* jobs, int njob, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_unlink_batch, dim3(16 * njob), dim3(RT), 0, s, jobs);
  hipLaunchKernelGGL(k_link_batch, dim3(16 * njob), dim3(RT), 0, s, jobs, n);
  hipLaunchKernelGGL(k_set_records, dim3(njob), dim3(64), 0, s, jobs);
  return hipGetLastError();
}

hipError_t launch_mean_stress(const DevDefect* d, const int32_t* counts, int ndef, int64_t n3, Cubic C, int bc,
                              double* add6, hipStream_t s) {
  if (bc == 0) return hipSuccess;  // mean stress zero: the additive term stays 0
  hipLaunchKernelGGL(k_mean_stress, dim3(1), dim3(MT), 0, s, d, counts, ndef, 1.0 / (double)n3, C, add6);
  return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, int64_t count, int64_t v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

}  // namespace ec

namespace ec {
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}
}  // namespace ec
