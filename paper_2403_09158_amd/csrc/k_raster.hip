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

__device__ __forceinline__ void box_cell(const DevDefect& d, int n, long e, int& x, int& y, int& z) {
  const long wxy = (long)d.w[0] * d.w[1];
  const int iz = (int)(e / wxy);
  const long r = e - (long)iz * wxy;
  const int iy = (int)(r / d.w[0]);
  const int ix = (int)(r - (long)iy * d.w[0]);
  x = box_axis(d.lo[0], d.w[0], n, ix);
  y = box_axis(d.lo[1], d.w[1], n, iy);
  z = box_axis(d.lo[2], d.w[2], n, iz);
}

__global__ __launch_bounds__(RT) void k_raster_count(const DevDefect* __restrict__ defs, int n,
                                                     int32_t* __restrict__ counts) {
  const DevDefect d = defs[blockIdx.x];
  const long total = (long)d.w[0] * d.w[1] * d.w[2];
  int c = 0;
  for (long e = threadIdx.x; e < total; e += RT) {
    int x, y, z;
    box_cell(d, n, e, x, y, z);
    c += member(d, n, x, y, z) ? 1 : 0;
  }
  __shared__ int red[RT];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int s = RT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

// Exclusive scan of the counts into offsets[0..ndef]; one workgroup.
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

__global__ __launch_bounds__(RT) void k_raster_fill(const DevDefect* __restrict__ defs, int n,
                                                    const int64_t* __restrict__ offsets, int32_t* __restrict__ ids,
                                                    int64_t* __restrict__ es) {
  const DevDefect d = defs[blockIdx.x];
  const long total = (long)d.w[0] * d.w[1] * d.w[2];
  const int64_t base0 = offsets[blockIdx.x];
  const size_t n3 = (size_t)n * n * n;
  __shared__ int wsum[RT / 64];
  __shared__ int64_t base_s;
  if (threadIdx.x == 0) base_s = base0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  for (long r0 = 0; r0 < total; r0 += RT) {
    const long e = r0 + threadIdx.x;
    int x = 0, y = 0, z = 0;
    bool in = false;
    if (e < total) {
      box_cell(d, n, e, x, y, z);
      in = member(d, n, x, y, z);
    }
    const unsigned long long mask = __ballot(in);
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(mask);
    __syncthreads();
    int64_t pos = base_s + before;
    int tot = 0;
    for (int w = 0; w < RT / 64; ++w) {
      if (w < wave) pos += wsum[w];
      tot += wsum[w];
    }
    if (in) {
      const int id = (z * n + y) * n + x;
      ids[pos] = id;
#pragma unroll
      for (int c = 0; c < 6; ++c)
        if (d.efix[c] != 0) atomicAdd((unsigned long long*)&es[c * n3 + id], (unsigned long long)d.efix[c]);
    }
    __syncthreads();
    if (threadIdx.x == 0) base_s += tot;
    __syncthreads();
  }
}

// Remove the defects' contributions (exact inverse of the fill).
__global__ __launch_bounds__(RT) void k_unraster(const DevDefect* __restrict__ defs,
                                                 const int64_t* __restrict__ offsets,
                                                 const int32_t* __restrict__ counts, const int32_t* __restrict__ ids,
                                                 int64_t n3, int64_t* __restrict__ es) {
  const DevDefect d = defs[blockIdx.x];
  const int64_t o = offsets[blockIdx.x];
  const int cnt = counts[blockIdx.x];
  for (int i = threadIdx.x; i < cnt; i += RT) {
    const int id = ids[o + i];
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (d.efix[c] != 0) atomicAdd((unsigned long long*)&es[c * n3 + id], (unsigned long long)(-d.efix[c]));
  }
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
__global__ __launch_bounds__(RT) void k_update_es(const int64_t* __restrict__ efix, const int32_t* __restrict__ old_ids,
                                                  int cnt_old, const int32_t* __restrict__ new_ids, int cnt_new,
                                                  int sx, int sy, int sz, int n, int64_t* __restrict__ es) {
  const size_t n3 = (size_t)n * n * n;
  const int t = blockIdx.x * RT + threadIdx.x;
  if (t < cnt_old) {
    const int id = old_ids[t];
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (efix[c] != 0) atomicAdd((unsigned long long*)&es[c * n3 + id], (unsigned long long)(-efix[c]));
  } else if (t < cnt_old + cnt_new) {
    const int i = t - cnt_old;
    const int id = new_ids ? new_ids[i] : shift_id(old_ids[i], sx, sy, sz, n);
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (efix[c] != 0) atomicAdd((unsigned long long*)&es[c * n3 + id], (unsigned long long)efix[c]);
  }
}

__global__ __launch_bounds__(RT) void k_translate_ids(int32_t* __restrict__ ids, int cnt, int sx, int sy, int sz,
                                                      int n) {
  const int t = blockIdx.x * RT + threadIdx.x;
  if (t < cnt) ids[t] = shift_id(ids[t], sx, sy, sz, n);
}

// Additive constant of the stress for the xi = 0 condition.  Mean strain zero:
// sigma gets -C:<eps*>, <eps*> = (1/n^3) sum_i |Omega_i| E_i (compensated FP64).
// Mean stress zero: nothing to add.
__global__ void k_mean_stress(const DevDefect* __restrict__ defs, const int32_t* __restrict__ counts, int ndef,
                              double inv_n3, Cubic C, int bc, double* __restrict__ add6) {
  if (threadIdx.x != 0) return;
  double m[6];
  for (int c = 0; c < 6; ++c) {
    double s = 0.0, comp = 0.0;
    for (int i = 0; i < ndef; ++i) {
      const double v = (double)counts[i] * defs[i].E[c];
      const double t = s + v;
      comp += (fabs(s) >= fabs(v)) ? ((s - t) + v) : ((v - t) + s);
      s = t;
    }
    m[c] = (s + comp) * inv_n3;
  }
  if (bc == 0) {
    for (int c = 0; c < 6; ++c) add6[c] = 0.0;
    return;
  }
  add6[0] = -(C.C11 * m[0] + C.C12 * (m[1] + m[2]));
  add6[1] = -(C.C11 * m[1] + C.C12 * (m[0] + m[2]));
  add6[2] = -(C.C11 * m[2] + C.C12 * (m[0] + m[1]));
  for (int c = 3; c < 6; ++c) add6[c] = -2.0 * C.C44 * m[c];
}

__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}

}  // namespace

hipError_t launch_raster_count(const DevDefect* d, int ndef, int n, int32_t* counts, hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_count, dim3(ndef), dim3(RT), 0, s, d, n, counts);
  return hipGetLastError();
}

hipError_t launch_scan(const int32_t* counts, int ndef, int64_t* offsets, hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, counts, ndef, offsets);
  return hipGetLastError();
}

hipError_t launch_raster_fill(const DevDefect* d, int ndef, int n, const int64_t* offsets, int32_t* ids,
                              int64_t* es, hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_raster_fill, dim3(ndef), dim3(RT), 0, s, d, n, offsets, ids, es);
  return hipGetLastError();
}

hipError_t launch_unraster(const DevDefect* d, int ndef, const int64_t* offsets, const int32_t* counts,
                           const int32_t* ids, int64_t n3, int64_t* es, hipStream_t s) {
  if (ndef == 0) return hipSuccess;
  hipLaunchKernelGGL(k_unraster, dim3(ndef), dim3(RT), 0, s, d, offsets, counts, ids, n3, es);
  return hipGetLastError();
}

hipError_t launch_update_es(const int64_t* efix, const int32_t* old_ids, int cnt_old, const int32_t* new_ids,
                            int cnt_new, int sx, int sy, int sz, int n, int64_t* es, hipStream_t s) {
  const int tot = cnt_old + cnt_new;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_update_es, dim3((tot + RT - 1) / RT), dim3(RT), 0, s, efix, old_ids, cnt_old, new_ids, cnt_new,
                     sx, sy, sz, n, es);
  return hipGetLastError();
}

hipError_t launch_translate_ids(int32_t* ids, int cnt, int sx, int sy, int sz, int n, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(k_translate_ids, dim3((cnt + RT - 1) / RT), dim3(RT), 0, s, ids, cnt, sx, sy, sz, n);
  return hipGetLastError();
}

hipError_t launch_mean_stress(const DevDefect* d, const int32_t* counts, int ndef, int64_t n3, Cubic C, int bc,
                              double* add6, hipStream_t s) {
  hipLaunchKernelGGL(k_mean_stress, dim3(1), dim3(64), 0, s, d, counts, ndef, 1.0 / (double)n3, C, bc, add6);
  return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, int64_t count, int64_t v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
  return hipGetLastError();
}

}  // namespace ec
