// k_shift.hip - energies of a stored defect type translated by the shift
// theorem (Sec. 3.3, eq. shift).
//
// A defect type's eigenstrain spectrum eps*_hat_0 (and stress spectrum
// sigma_hat_0) is stored once for its reference centre X0.  The type translated
// by d = X - X0 has the spectrum phi_d(xi) eps*_hat_0(xi), and its energy with a
// stress field sigma follows from Parseval's identity on the half spectrum:
//   sum_x eps*_d(x) : sigma(x) = (1/N) sum_k w(k_x) Re[phi_d(k) eps*_hat_0(k) : conj(sigma_hat(k))],
// w = 1 on the planes k_x = 0 and (even n) k_x = n/2, which hold their own
// Hermitian partners, and 2 elsewhere; the contraction weighs the shear
// components twice.  phi_d is exp(-i xi . d) with the centred labels of
// Sec. 3.4; at a bin with even-n Nyquist components it is the mean of the
// factors of the -n/2 and +n/2 representatives, which is the transform of the
// real part of the translated field.  With an excluded mover at offset d'
// (its own stress, translated, taken out of sigma) the contraction is with
// conj(sigma_hat - phi_d' sigma_hat_0).
//
// One pass over the three spectra serves up to TYPE_NP positions; each block
// leaves one FP64 partial sum per position and the partials are added in a
// fixed order, so results do not depend on scheduling.
#include "ec_internal.h"

namespace ec {

namespace {

constexpr int TT = 256;

__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// The phase of entry p at bin (kx, ky, kz): tab[(p * 3 + a) * n + k] is the
// factor of axis a at bin k (the -n/2 label at a Nyquist bin), nyq[p * 3 + a]
// the factor of the +n/2 representative.
__device__ __forceinline__ double2 phase(const double2* __restrict__ tab, const double2* __restrict__ nyq, int p,
                                         int n, int kx, int ky, int kz, bool nx, bool ny, bool nz) {
  const double2* t = tab + (size_t)p * 3 * n;
  const double2 a = t[kx], b = t[n + ky], c = t[2 * n + kz];
  double2 m = cmul2(cmul2(a, b), c);
  if (nx || ny || nz) {
    // values loaded first and then chosen, so that no local needs an address
    const double2 na = nyq[3 * p], nb = nyq[3 * p + 1], nc = nyq[3 * p + 2];
    const double2 ap = nx ? na : a, bp = ny ? nb : b, cp = nz ? nc : c;
    const double2 mp = cmul2(cmul2(ap, bp), cp);
    m = make_double2(0.5 * (m.x + mp.x), 0.5 * (m.y + mp.y));
  }
  return m;
}

template <typename S>
__global__ __launch_bounds__(TT) void k_type_energy(const typename Cplx<S>::T* __restrict__ sig,
                                                    const typename Cplx<S>::T* __restrict__ te,
                                                    const typename Cplx<S>::T* __restrict__ ts, int n, int P,
                                                    const double2* __restrict__ tab, const double2* __restrict__ nyq,
                                                    int np, int excl, double* __restrict__ partial) {
  __shared__ double red[TT];
  const int NH = n / 2 + 1;
  const bool even = (n & 1) == 0;
  const int64_t bins = (int64_t)n * n * NH;
  double acc[TYPE_NP];
#pragma unroll
  for (int p = 0; p < TYPE_NP; ++p) acc[p] = 0.0;
  for (int64_t b = (int64_t)blockIdx.x * TT + threadIdx.x; b < bins; b += (int64_t)gridDim.x * TT) {
    const int kx = (int)(b % NH);
    const int64_t r = b / NH;
    const int ky = (int)(r % n), kz = (int)(r / n);
    const size_t o = spec_at(kz, ky, kx, 0, n, P);
    // A = eps*_hat_0 : conj(sigma_hat), B = eps*_hat_0 : conj(sigma_hat_0)
    double2 A = make_double2(0.0, 0.0), B = make_double2(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double w = c < 3 ? 1.0 : 2.0;
      const double2 e = ld2(te + o + c), s = ld2(sig + o + c);
      A.x += w * (e.x * s.x + e.y * s.y);
      A.y += w * (e.y * s.x - e.x * s.y);
      if (excl) {
        const double2 q = ld2(ts + o + c);
        B.x += w * (e.x * q.x + e.y * q.y);
        B.y += w * (e.y * q.x - e.x * q.y);
      }
    }
    const bool nx = even && kx == n / 2, ny = even && ky == n / 2, nz = even && kz == n / 2;
    if (excl) {  // D = A - B conj(phi_d')
      const double2 f = phase(tab, nyq, np, n, kx, ky, kz, nx, ny, nz);
      A.x -= B.x * f.x + B.y * f.y;
      A.y -= B.y * f.x - B.x * f.y;
    }
    const double wx = (kx == 0 || nx) ? 1.0 : 2.0;
#pragma unroll
    for (int p = 0; p < TYPE_NP; ++p) {
      if (p < np) {
        const double2 f = phase(tab, nyq, p, n, kx, ky, kz, nx, ny, nz);
        acc[p] += wx * (f.x * A.x - f.y * A.y);
      }
    }
  }
  // block sums by a fixed tree (np is the same for every thread)
#pragma unroll
  for (int p = 0; p < TYPE_NP; ++p) {
    if (p >= np) break;
    red[threadIdx.x] = acc[p];
    __syncthreads();
    for (int w = TT / 2; w > 0; w >>= 1) {
      if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(size_t)p * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// E_p = scale * sum of the grid partials of position p: one workgroup per
// position, strided Neumaier sums per thread, then a fixed tree.
__global__ __launch_bounds__(256) void k_type_finish(const double* __restrict__ partial, int grid, double scale,
                                                     double* __restrict__ E) {
  __shared__ double rs[256], rc[256];
  const int p = blockIdx.x;
  double s = 0.0, c = 0.0;
  for (int b = threadIdx.x; b < grid; b += 256) {
    const double v = partial[(size_t)p * grid + b], t = s + v;
    c += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
    s = t;
  }
  rs[threadIdx.x] = s;
  rc[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double a = rs[threadIdx.x], v = rs[threadIdx.x + w], t = a + v;
      rc[threadIdx.x] += rc[threadIdx.x + w] + (fabs(a) >= fabs(v) ? (a - t) + v : (v - t) + a);
      rs[threadIdx.x] = t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) E[p] = scale * (rs[0] + rc[0]);
}

}  // namespace

int type_energy_grid(int n) {
  const int64_t bins = (int64_t)n * n * (n / 2 + 1);
  return (int)std::min<int64_t>(1024, (bins + TT - 1) / TT);
}

hipError_t launch_type_energies(bool fp64, const void* sig, const void* te, const void* ts, SpecGeom g,
                                const double2* tab, const double2* nyq, int np, bool excl, double* partial,
                                double scale, double* E, hipStream_t s) {
  if (np < 1 || np > TYPE_NP) return hipErrorInvalidValue;
  const int grid = type_energy_grid(g.n);
  if (fp64)
    hipLaunchKernelGGL(k_type_energy<double>, dim3(grid), dim3(TT), 0, s, (const double2*)sig, (const double2*)te,
                       (const double2*)ts, g.n, g.P, tab, nyq, np, excl ? 1 : 0, partial);
  else
    hipLaunchKernelGGL(k_type_energy<float>, dim3(grid), dim3(TT), 0, s, (const float2*)sig, (const float2*)te,
                       (const float2*)ts, g.n, g.P, tab, nyq, np, excl ? 1 : 0, partial);
  hipLaunchKernelGGL(k_type_finish, dim3(np), dim3(256), 0, s, partial, grid, scale, E);
  return hipGetLastError();
}

}  // namespace ec
