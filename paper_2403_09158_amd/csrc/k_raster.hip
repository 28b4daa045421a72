// k_raster.hip - defects to the eigenstrain field and footprint lists.
//
// Sec. 3.1: loop eigenstrain sym(b x n)/e over a slab of thickness e around the
// loop disk; point-defect clusters as dilatational spheres.  Sec. 3.4: fields
// live at voxel centres h (m + 1/2).  One workgroup per defect enumerates the
// defect's bounding box in ascending voxel-id order, tests membership in exact
// integer arithmetic, compacts the members with a workgroup prefix sum (so the
// footprint list is sorted) and adds the fixed-point eigenstrain with integer
// atomics (exact and order independent, so overlaps are deterministic).
#include "ec_internal.h"

namespace ec {

namespace {

constexpr int RT = 256;  // threads per rasteriser workgroup

// Exclusive scan of counts into offsets[0..ndef] (offsets[ndef] = total); one workgroup.
__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ counts, int ndef,
                                               int64_t* __restrict__ offsets) {
  __shared__ int64_t part[1024];
  const int T = 1024;
  const int per = (ndef + T - 1) / T;
  const int b = threadIdx.x * per, e = min(ndef, b + per);
  int64_t s = 0;
  for (int i = b; i < e; ++i) s += counts[i];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int t = 0; t < T; ++t) {
      const int64_t v = part[t];
      part[t] = acc;
      acc += v;
    }
    offsets[ndef] = acc;
  }
  __syncthreads();
  int64_t acc = part[threadIdx.x];
  for (int i = b; i < e; ++i) {
    offsets[i] = acc;
    acc += counts[i];
  }
}

__device__ __forceinline__ void add_fix(int64_t* es, size_t n3, int id, const int64_t* efix, int64_t sgn) {
#pragma unroll
  for (int c = 0; c < 6; ++c)
    if (efix[c] != 0) atomicAdd((unsigned long long*)&es[c * n3 + id], (unsigned long long)(sgn * efix[c]));
}

// One workgroup per defect, one thread per bounding-box row (y, z) in ascending
// order: the row's candidate x range comes from the geometry, each candidate is
// tested exactly, a workgroup scan orders the rows, and every row writes its
// members in ascending x.  The footprint list of the defect is therefore sorted.
__global__ __launch_bounds__(RT) void k_raster_fill(const DevDefect* __restrict__ defs, int n,
                                                    int32_t* __restrict__ ids, int32_t* __restrict__ counts,
                                                    int64_t* __restrict__ es) {
  const DevDefect d = defs[blockIdx.x];
  const int nrows = d.w[1] * d.w[2];
  const size_t n3 = (size_t)n * n * n;
  __shared__ int wsum[RT / 64];
  __shared__ int run;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) run = 0;
  __syncthreads();
  for (int r0 = 0; r0 < nrows; r0 += RT) {
    const int r = r0 + threadIdx.x;
    int y = 0, z = 0, u0 = 0, u1 = -1, cnt = 0;
    if (r < nrows) {
      const int iz = r / d.w[1], iy = r - iz * d.w[1];
      y = box_axis(d.lo[1], d.w[1], n, iy);
      z = box_axis(d.lo[2], d.w[2], n, iz);
      if (row_range(d, n, y, z, u0, u1))
        for (int u = u0; u <= u1; ++u) {
          int x = d.lo[0] + u;
          x -= x >= n ? n : 0;
          cnt += member(d, n, x, y, z) ? 1 : 0;
        }
    }
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o);
      if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = incl - cnt, tot = 0;
    for (int w = 0; w < RT / 64; ++w) {
      if (w < wave) before += wsum[w];
      tot += wsum[w];
    }
    if (cnt > 0) {
      int64_t pos = d.slot + run + before;
      // candidates in ascending x: a range that wraps past n - 1 is emitted low part first
      const int xa = d.lo[0] + u0, xb = d.lo[0] + u1;
      const int segs = (xa < n && xb >= n) ? 2 : 1;
      for (int sgi = 0; sgi < segs; ++sgi) {
        int lo, hi;
        if (segs == 2) {
          lo = sgi == 0 ? 0 : xa;
          hi = sgi == 0 ? xb - n : n - 1;
        } else {
          lo = xa >= n ? xa - n : xa;
          hi = xb >= n ? xb - n : xb;
        }
        for (int x = lo; x <= hi; ++x)
          if (member(d, n, x, y, z)) {
            const int id = (z * n + y) * n + x;
            ids[pos++] = id;
            add_fix(es, n3, id, d.efix, 1);
          }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) run += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = run;
}

// Remove the defects' contributions (exact inverse of the fill).
__global__ __launch_bounds__(RT) void k_unraster(const DevDefect* __restrict__ defs,
                                                 const int32_t* __restrict__ counts, const int32_t* __restrict__ ids,
                                                 int64_t n3, int64_t* __restrict__ es) {
  const int64_t o = defs[blockIdx.x].slot;
  const int cnt = counts[blockIdx.x];
  int64_t efix[6];
  for (int c = 0; c < 6; ++c) efix[c] = defs[blockIdx.x].efix[c];
  for (int i = threadIdx.x; i < cnt; i += RT) add_fix(es, n3, ids[o + i], efix, -1);
}

__device__ __forceinline__ int shift_id(int id, int sx, int sy, int sz, int n) {
  int x = id % n + sx, y = (id / n) % n + sy, z = id / (n * n) + sz;
  x += (x < 0) ? n : ((x >= n) ? -n : 0);
  y += (y < 0) ? n : ((y >= n) ? -n : 0);
  z += (z < 0) ? n : ((z >= n) ? -n : 0);
  return (z * n + y) * n + x;
}

// Move one defect in the fixed-point field: subtract on the old footprint, add
// on the new one (new = old shifted by whole voxels when new_ids == nullptr).
// Grid-stride over 2 * cap threads; the old count is read on the device.
__global__ __launch_bounds__(RT) void k_update_es(const int64_t* __restrict__ efix, const int32_t* __restrict__ old_ids,
                                                  const int32_t* __restrict__ cnt_old_p,
                                                  const int32_t* __restrict__ new_ids, int cnt_new, int sx, int sy,
                                                  int sz, int n, int64_t* __restrict__ es) {
  const size_t n3 = (size_t)n * n * n;
  const int cnt_old = *cnt_old_p;
  const int nn = new_ids ? cnt_new : cnt_old;
  int64_t f[6];
  for (int c = 0; c < 6; ++c) f[c] = efix[c];
  for (int t = blockIdx.x * RT + threadIdx.x; t < cnt_old + nn; t += gridDim.x * RT) {
    if (t < cnt_old) {
      add_fix(es, n3, old_ids[t], f, -1);
    } else {
      const int i = t - cnt_old;
      add_fix(es, n3, new_ids ? new_ids[i] : shift_id(old_ids[i], sx, sy, sz, n), f, 1);
    }
  }
}

__global__ __launch_bounds__(RT) void k_translate_ids(int32_t* __restrict__ ids, const int32_t* __restrict__ cnt_p,
                                                      int sx, int sy, int sz, int n) {
  const int cnt = *cnt_p;
  for (int t = blockIdx.x * RT + threadIdx.x; t < cnt; t += gridDim.x * RT) ids[t] = shift_id(ids[t], sx, sy, sz, n);
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
  add6[0] = -(C.C11 * m[0] + C.C12 * (m[1] + m[2]));
  add6[1] = -(C.C11 * m[1] + C.C12 * (m[0] + m[2]));
  add6[2] = -(C.C11 * m[2] + C.C12 * (m[0] + m[1]));
  for (int a = 3; a < 6; ++a) add6[a] = -2.0 * C.C44 * m[a];
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

}  // namespace

hipError_t launch_scan(const int32_t* counts, int ndef, int64_t* offsets, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, ndef, offsets);
  return hipGetLastError();
}

hipError_t launch_raster_fill(const DevDefect* d, int ndef, int n, int32_t* ids, int32_t* counts, int64_t* es,
                              hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_fill, dim3(ndef), dim3(RT), 0, s, d, n, ids, counts, es);
  return hipGetLastError();
}

hipError_t launch_unraster(const DevDefect* d, int ndef, const int32_t* counts, const int32_t* ids, int64_t n3,
                           int64_t* es, hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unraster, dim3(ndef), dim3(RT), 0, s, d, counts, ids, n3, es);
  return hipGetLastError();
}

hipError_t launch_update_es(const int64_t* efix, const int32_t* old_ids, const int32_t* cnt_old,
                            const int32_t* new_ids, int cnt_new, int sx, int sy, int sz, int n, int64_t* es,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_update_es, dim3(64), dim3(RT), 0, s, efix, old_ids, cnt_old, new_ids, cnt_new, sx, sy, sz, n,
                     es);
  return hipGetLastError();
}

hipError_t launch_translate_ids(int32_t* ids, const int32_t* cnt, int sx, int sy, int sz, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_translate_ids, dim3(16), dim3(RT), 0, s, ids, cnt, sx, sy, sz, n);
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
