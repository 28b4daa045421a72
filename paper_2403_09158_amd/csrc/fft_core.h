// fft_core.h - mixed-radix (2/3/4/5/8/16, and the prime 43) Stockham FFT building blocks for gfx950.
//
// Every transform here is a 1-D DFT of compile-time length N computed by a
// workgroup in FP64 registers.  The first stage reads its operands straight from
// HBM (or from an input rule), intermediate stages exchange through LDS, and the
// last stage hands its outputs to a store rule, so a two-stage length makes one
// LDS round trip.  Stockham indexing (self-sorting, no bit reversal):
//   stage with radix R after a product Ns of earlier radices, butterfly j in [0, N/R):
//     k = j mod Ns, inputs x[j + r N/R], twiddles W_N^{k r N/(Ns R)},
//     outputs y[(j/Ns) Ns R + k + r Ns].
// Twiddles W_N^e = exp(-2 pi i e / N) come from a table computed on the host in
// extended precision and staged in LDS; the inverse transform uses conjugates.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace ec {

struct Plan2 {
  int nstage;
  int r[3];
};

// Radix sequence per supported length (first stage first).
__host__ __device__ constexpr Plan2 plan_of(int N) {
  return N == 8     ? Plan2{1, {8, 1, 1}}
         : N == 16  ? Plan2{1, {16, 1, 1}}
         : N == 24  ? Plan2{2, {8, 3, 1}}
         : N == 32  ? Plan2{2, {8, 4, 1}}
         : N == 48  ? Plan2{2, {16, 3, 1}}
         : N == 64  ? Plan2{2, {8, 8, 1}}
         : N == 96  ? Plan2{2, {16, 6, 1}}
         : N == 128 ? Plan2{2, {16, 8, 1}}
         : N == 160 ? Plan2{2, {16, 10, 1}}
         : N == 240 ? Plan2{2, {16, 15, 1}}
         : N == 256 ? Plan2{2, {16, 16, 1}}
         : N == 512 ? Plan2{3, {8, 8, 8}}
         : N == 45  ? Plan2{2, {15, 3, 1}}
         : N == 129 ? Plan2{2, {43, 3, 1}}
                    : Plan2{0, {1, 1, 1}};
}

// Radices whose butterfly is evaluated output by output (dft_direct) rather
// than all at once in registers: the large prime of an odd length.  A plan
// puts it first, where it needs no twiddles.
__host__ __device__ constexpr bool direct_radix(int R) { return R == 43; }
__host__ __device__ constexpr bool has_direct(Plan2 p) {
  return direct_radix(p.r[0]) || direct_radix(p.r[1]) || direct_radix(p.r[2]);
}

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 conjd(double2 a) { return make_double2(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ double2 rot90(double2 a) {
  return INV ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// exp(-+ 2 pi i e / R) for the small in-register composites (R = 8, 16).
template <int R, bool INV>
__device__ __forceinline__ double2 wsmall(int e) {
  // cos(2 pi k / 16), k = 0..15
  constexpr double c16[16] = {1.0,
                              0.92387953251128675613,
                              0.70710678118654752440,
                              0.38268343236508977173,
                              0.0,
                              -0.38268343236508977173,
                              -0.70710678118654752440,
                              -0.92387953251128675613,
                              -1.0,
                              -0.92387953251128675613,
                              -0.70710678118654752440,
                              -0.38268343236508977173,
                              0.0,
                              0.38268343236508977173,
                              0.70710678118654752440,
                              0.92387953251128675613};
  const int k = (e * (16 / R)) & 15;
  const double c = c16[k];
  const double s = c16[(k + 12) & 15];  // sin(2 pi k/16) = cos(2 pi (k - 4)/16)
  return INV ? make_double2(c, s) : make_double2(c, -s);
}

template <int R, bool INV>
__device__ __forceinline__ double2 twid_small(double2 a, int e) {
  const int q = (e * (16 / R)) & 15;
  if (q == 0) return a;
  if (q == 8) return make_double2(-a.x, -a.y);
  if (q == 4) return rot90<INV>(a);
  if (q == 12) return rot90<!INV>(a);
  return cmul(a, wsmall<R, INV>(e));
}

template <int R, bool INV>
struct Dft;

template <bool INV>
struct Dft<1, INV> {
  __device__ __forceinline__ static void run(double2*) {}
};

template <bool INV>
struct Dft<2, INV> {
  __device__ __forceinline__ static void run(double2* v) {
    double2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <bool INV>
struct Dft<3, INV> {
  __device__ __forceinline__ static void run(double2* v) {
    constexpr double h = 0.86602540378443864676;  // sin(2 pi / 3)
    double2 a = v[0], s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    double2 t = make_double2(a.x - 0.5 * s.x, a.y - 0.5 * s.y);
    double2 u = rot90<INV>(cscale(d, h));
    v[0] = cadd(a, s);
    v[1] = cadd(t, u);
    v[2] = csub(t, u);
  }
};

template <bool INV>
struct Dft<4, INV> {
  __device__ __forceinline__ static void run(double2* v) {
    double2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    double2 t2 = cadd(v[1], v[3]), t3 = rot90<INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <bool INV>
struct Dft<5, INV> {
  __device__ __forceinline__ static void run(double2* v) {
    constexpr double c1 = 0.30901699437494742410;   // cos(2 pi/5)
    constexpr double c2 = -0.80901699437494742410;  // cos(4 pi/5)
    constexpr double s1 = 0.95105651629515357212;   // sin(2 pi/5)
    constexpr double s2 = 0.58778525229247312917;   // sin(4 pi/5)
    double2 a = v[0];
    double2 p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
    double2 p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
    double2 r1 = make_double2(a.x + c1 * p1.x + c2 * p2.x, a.y + c1 * p1.y + c2 * p2.y);
    double2 r2 = make_double2(a.x + c2 * p1.x + c1 * p2.x, a.y + c2 * p1.y + c1 * p2.y);
    double2 q1 = rot90<INV>(make_double2(s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y));
    double2 q2 = rot90<INV>(make_double2(s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y));
    v[0] = cadd(a, cadd(p1, p2));
    v[1] = cadd(r1, q1);
    v[4] = csub(r1, q1);
    v[2] = cadd(r2, q2);
    v[3] = csub(r2, q2);
  }
};

// Composite R = R1*R2 in registers: inputs x[n1 + R1 n2], outputs X[k2 + R2 k1].
template <int R1, int R2, bool INV>
__device__ __forceinline__ void dft_composite(double2* v) {
  constexpr int R = R1 * R2;
  double2 y[R];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    double2 t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = v[n1 + R1 * n2];
    Dft<R2, INV>::run(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[n1 * R2 + k2] = twid_small<R, INV>(t[k2], n1 * k2);
  }
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    double2 t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = y[n1 * R2 + k2];
    Dft<R1, INV>::run(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) v[k2 + R2 * k1] = t[k1];
  }
}

template <bool INV>
struct Dft<8, INV> {
  __device__ __forceinline__ static void run(double2* v) { dft_composite<2, 4, INV>(v); }
};

template <bool INV>
struct Dft<16, INV> {
  __device__ __forceinline__ static void run(double2* v) { dft_composite<4, 4, INV>(v); }
};

// R = R1 x R2 with R1, R2 coprime, by the prime-factor (Good-Thomas) mapping,
// no inner twiddles: input n = (R2 n1 + R1 n2) mod R, output k = (E1 k1 + E2 k2)
// mod R with E1 = 1 mod R1, 0 mod R2 and E2 = 0 mod R1, 1 mod R2, so the
// exponent n k reduces to R2 n1 k1 + R1 n2 k2 mod R: an R1 x R2 two-dimensional
// DFT.
template <int R1, int R2, int E1, int E2, bool INV>
__device__ __forceinline__ void dft_pfa(double2* v) {
  constexpr int R = R1 * R2;
  static_assert(E1 % R1 == 1 && E1 % R2 == 0 && E2 % R1 == 0 && E2 % R2 == 1, "CRT output map");
  double2 y[R];
#pragma unroll
  for (int n1 = 0; n1 < R1; ++n1) {
    double2 t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = v[(R2 * n1 + R1 * n2) % R];
    Dft<R2, INV>::run(t);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) y[n1 * R2 + k2] = t[k2];
  }
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    double2 t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = y[n1 * R2 + k2];
    Dft<R1, INV>::run(t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) v[(E1 * k1 + E2 * k2) % R] = t[k1];
  }
}

template <bool INV>
struct Dft<6, INV> {
  __device__ __forceinline__ static void run(double2* v) { dft_pfa<2, 3, 3, 4, INV>(v); }
};

template <bool INV>
struct Dft<10, INV> {
  __device__ __forceinline__ static void run(double2* v) { dft_pfa<2, 5, 5, 6, INV>(v); }
};

template <bool INV>
struct Dft<15, INV> {
  __device__ __forceinline__ static void run(double2* v) { dft_pfa<3, 5, 10, 6, INV>(v); }
};

// Length-R DFT of v[0..R) for an odd prime R, each output handed to put(r,
// X_r) as soon as it is formed, so the butterfly never holds R outputs beside
// its R inputs.  The inputs are first folded into symmetric pairs,
// a_j = x_j + x_{R-j} and b_j = x_j - x_{R-j} (j = 1 .. (R-1)/2), in place; then
//   X_0 = x_0 + sum a_j,  X_k, X_{R-k} = C_k -+ i S_k  (forward; +- inverse),
//   C_k = x_0 + sum_j a_j cos(2 pi j k / R),  S_k = sum_j b_j sin(2 pi j k / R),
// with the cosines and sines read from the length-N twiddle table
// (W_N^{m N / R} = cos - i sin of 2 pi m / R).
template <int N, int R, bool INV, class Put>
__device__ __forceinline__ void dft_direct(double2* v, const double2* tw, Put&& put) {
  static_assert(R % 2 == 1 && N % R == 0, "odd radix dividing N");
  constexpr int H = (R - 1) / 2;
  double2 x0 = v[0], sum = v[0];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    const double2 a = cadd(v[j], v[R - j]), b = csub(v[j], v[R - j]);
    v[j] = a;
    v[R - j] = b;
    sum = cadd(sum, a);
  }
  put(0, sum);
#pragma unroll 1
  for (int k = 1; k <= H; ++k) {
    double2 C = x0, S = make_double2(0.0, 0.0);
    int m = 0;
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      m += k;
      if (m >= R) m -= R;
      const double2 w = tw[m * (N / R)];  // (cos, -sin) of 2 pi m / R
      C.x += v[j].x * w.x;
      C.y += v[j].y * w.x;
      S.x -= v[R - j].x * w.y;
      S.y -= v[R - j].y * w.y;
    }
    // forward: X_k = C - i S, X_{R-k} = C + i S; the inverse swaps them
    const double2 mi = make_double2(C.x + S.y, C.y - S.x), pi = make_double2(C.x - S.y, C.y + S.x);
    put(k, INV ? pi : mi);
    put(R - k, INV ? mi : pi);
  }
}

// Twiddle from the LDS table (forward W_N^e; conjugated for the inverse).
template <bool INV>
__device__ __forceinline__ double2 tw_at(const double2* tw, int e) {
  double2 t = tw[e];
  return INV ? make_double2(t.x, -t.y) : t;
}

// The R twiddles of one butterfly in registers (forward sign), w[r] for its
// r-th operand: for kernels whose threads keep the same butterfly of a stage
// from tile to tile, so the table is read once per kernel instead of once per
// tile.  A stage given a TwReg uses it in place of the table.
template <int R>
struct TwReg {
  double2 w[R];
};

template <class TW>
struct is_twreg : std::false_type {};
template <int R>
struct is_twreg<TwReg<R>> : std::true_type {};

template <bool INV>
__device__ __forceinline__ double2 twiddle(const double2* tw, int, int e) {
  return tw_at<INV>(tw, e);
}
template <bool INV, int R>
__device__ __forceinline__ double2 twiddle(const TwReg<R>& t, int r, int) {
  return INV ? conjd(t.w[r]) : t.w[r];
}

// One Stockham stage over `nfft` transforms of length N with radix R after
// Ns = product of earlier radices.  Butterfly b -> (transform f, index j) by
// MAP (pencil: f fastest across lanes, so columns stay contiguous; row: j
// fastest, so positions along a contiguous row stay contiguous).  Operands are
// all read (LOAD) before the barrier and written (STORE) after it, so the
// stage may run in place on LDS.  BPT = butterflies per thread.
// Butterfly b of a stage -> (transform f, butterfly j within it).  Pencil:
// transforms interleaved (f = b % NFFT); Row: one transform after another;
// Group: transforms in groups of GW, one group after another, interleaved
// inside a group, so a thread keeps its lane of the group in every group.
enum class Map { Pencil, Row, Group };

template <Map M, int N, int R, int NFFT, int GW>
__device__ __forceinline__ void bfly_index(int b, int& f, int& j) {
  if constexpr (M == Map::Pencil) {
    f = b % NFFT;
    j = b / NFFT;
  } else if constexpr (M == Map::Row) {
    f = b / (N / R);
    j = b % (N / R);
  } else {
    constexpr int PER = GW * (N / R);
    const int rem = b % PER;
    f = (b / PER) * GW + rem % GW;
    j = rem / GW;
  }
}

template <int N, int R, int NS, bool INV, Map M, int NFFT, int T, int GW = NFFT, class TW, class Load, class Store>
__device__ __forceinline__ void stage(const TW& tw, Load&& load, Store&& store, bool sync_between,
                                      int tid = threadIdx.x) {
  constexpr int NB = NFFT * (N / R);
  constexpr int BPT = (NB + T - 1) / T;
  static_assert(!is_twreg<TW>::value || NB <= T, "register twiddles need at most one butterfly per thread");
  double2 v[BPT][R];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = tid + q * T;
    if (NB % T == 0 || b < NB) {
      int f, j;
      bfly_index<M, N, R, NFFT, GW>(b, f, j);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // a 3-argument rule also receives the operand's slot q R + r (see
        // for_operands), a compile-time index into register-held operands
        if constexpr (std::is_invocable_v<Load, int, int, int>)
          v[q][r] = load(f, j + r * (N / R), q * R + r);
        else
          v[q][r] = load(f, j + r * (N / R));
      }
    }
  }
  if (sync_between) __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = tid + q * T;
    if (NB % T == 0 || b < NB) {
      int f, j;
      bfly_index<M, N, R, NFFT, GW>(b, f, j);
      const int k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], twiddle<INV>(tw, r, k * r * (N / (NS * R))));
      }
      const int base = (j / NS) * NS * R + k;
      if constexpr (direct_radix(R)) {
        // outputs leave one by one in a loop, so a store rule that needs a
        // compile-time slot cannot follow a direct radix
        static_assert(!is_twreg<TW>::value, "a direct radix reads the twiddle table");
        static_assert(!std::is_invocable_v<Store, int, int, double2, int>, "no slot-indexed store after a direct radix");
        dft_direct<N, R, INV>(v[q], tw, [&](int r, double2 x) { store(f, base + r * NS, x); });
      } else {
        Dft<R, INV>::run(v[q]);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // a 4-argument rule also receives the output's slot q R + r (see
          // for_outputs), a compile-time index into register-held values
          if constexpr (std::is_invocable_v<Store, int, int, double2, int>)
            store(f, base + r * NS, v[q][r], q * R + r);
          else
            store(f, base + r * NS, v[q][r]);
        }
      }
    }
  }
}

// Visit the operands a thread reads in a radix-R stage, in the order stage()
// reads them: fn(f, i, slot) with slot = q R + r for its q-th butterfly.
template <int N, int R, Map M, int NFFT, int T, int GW = NFFT, class F>
__device__ __forceinline__ void for_operands(F&& fn, int tid = threadIdx.x) {
  constexpr int NB = NFFT * (N / R);
  constexpr int BPT = (NB + T - 1) / T;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = tid + q * T;
    if (NB % T == 0 || b < NB) {
      int f, j;
      bfly_index<M, N, R, NFFT, GW>(b, f, j);
#pragma unroll
      for (int r = 0; r < R; ++r) fn(f, j + r * (N / R), q * R + r);
    }
  }
}

// Visit the outputs a thread writes in a radix-R stage after NS, in the order
// stage() writes them: fn(f, i, slot) with slot = q R + r for its q-th
// butterfly.
template <int N, int R, int NS, Map M, int NFFT, int T, int GW = NFFT, class F>
__device__ __forceinline__ void for_outputs(F&& fn, int tid = threadIdx.x) {
  constexpr int NB = NFFT * (N / R);
  constexpr int BPT = (NB + T - 1) / T;
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = tid + q * T;
    if (NB % T == 0 || b < NB) {
      int f, j;
      bfly_index<M, N, R, NFFT, GW>(b, f, j);
      const int k = j % NS;
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) fn(f, base + r * NS, q * R + r);
    }
  }
}

// Register twiddles of the radix-R stage after NS for the thread whose
// butterfly in that stage is b = tid (one butterfly per thread).
template <int N, int R, int NS, Map M, int NFFT, int T, int GW = NFFT>
__device__ __forceinline__ TwReg<R> make_twreg(const double2* tw, int tid) {
  // a thread without a butterfly (b >= NFFT N / R) reads in-range entries it
  // never uses
  static_assert(NFFT * (N / R) <= T, "at most one butterfly per thread");
  int f, j;
  bfly_index<M, N, R, NFFT, GW>(tid, f, j);
  const int k = j % NS;
  TwReg<R> t;
#pragma unroll
  for (int r = 0; r < R; ++r) t.w[r] = tw[k * r * (N / (NS * R))];
  return t;
}

// Full transform: first stage LOAD0 -> LDS (or -> STORE_LAST for one stage),
// middle stages in place on LDS, last stage LDS -> STORE_LAST.  LDS is reached
// through `lds_ld(f, i)` / `lds_st(f, i, v)` (element i of transform f), so the
// staging precision is the caller's choice.  LAST_LDS: the last stage's store
// writes LDS too (operands are then all read before the barrier), LOAD0_LDS:
// the first stage reads LDS in place.
template <int N, bool INV, Map M, int NFFT, int T, bool LOAD0_LDS = false, bool LAST_LDS = false, class TW,
          class Load0, class LdsLd, class LdsSt, class StoreLast>
__device__ __forceinline__ void transform(const TW& tw, Load0&& load0, LdsLd&& from_lds, LdsSt&& to_lds,
                                          StoreLast&& store_last) {
  constexpr Plan2 P = plan_of(N);
  static_assert(P.nstage >= 1, "unsupported FFT length");
  static_assert(!is_twreg<TW>::value || P.nstage == 2, "register twiddles need a two-stage plan");
  if constexpr (P.nstage == 1) {
    stage<N, P.r[0], 1, INV, M, NFFT, T>(tw, load0, store_last, LOAD0_LDS && LAST_LDS);
  } else if constexpr (P.nstage == 2) {
    stage<N, P.r[0], 1, INV, M, NFFT, T>(tw, load0, to_lds, LOAD0_LDS);
    __syncthreads();
    stage<N, P.r[1], P.r[0], INV, M, NFFT, T>(tw, from_lds, store_last, LAST_LDS);
  } else {
    stage<N, P.r[0], 1, INV, M, NFFT, T>(tw, load0, to_lds, LOAD0_LDS);
    __syncthreads();
    stage<N, P.r[1], P.r[0], INV, M, NFFT, T>(tw, from_lds, to_lds, true);
    __syncthreads();
    stage<N, P.r[2], P.r[0] * P.r[1], INV, M, NFFT, T>(tw, from_lds, store_last, LAST_LDS);
  }
}

// Transform with an explicit radix sequence (R1 = 1: one stage, R2 = 1: two
// stages); LOAD0_LDS / LAST_LDS as for transform().
template <int N, int R0, int R1, int R2, bool INV, Map M, int NFFT, int T, int GW, bool LOAD0_LDS, bool LAST_LDS,
          class TW, class Load0, class LdsLd, class LdsSt, class StoreLast>
__device__ __forceinline__ void transform_plan(const TW& tw, Load0&& load0, LdsLd&& from_lds, LdsSt&& to_lds,
                                               StoreLast&& store_last, int tid = threadIdx.x) {
  static_assert(R0 * R1 * R2 == N, "radices must multiply to N");
  // register twiddles serve one twiddled stage only
  static_assert(!is_twreg<TW>::value || R2 == 1, "register twiddles need a two-stage plan");
  if constexpr (R1 == 1) {
    stage<N, R0, 1, INV, M, NFFT, T, GW>(tw, load0, store_last, LOAD0_LDS && LAST_LDS, tid);
  } else if constexpr (R2 == 1) {
    stage<N, R0, 1, INV, M, NFFT, T, GW>(tw, load0, to_lds, LOAD0_LDS, tid);
    __syncthreads();
    stage<N, R1, R0, INV, M, NFFT, T, GW>(tw, from_lds, store_last, LAST_LDS, tid);
  } else {
    stage<N, R0, 1, INV, M, NFFT, T, GW>(tw, load0, to_lds, LOAD0_LDS, tid);
    __syncthreads();
    stage<N, R1, R0, INV, M, NFFT, T, GW>(tw, from_lds, to_lds, true, tid);
    __syncthreads();
    stage<N, R2, R0 * R1, INV, M, NFFT, T, GW>(tw, from_lds, store_last, LAST_LDS, tid);
  }
}

// Factorisation for the fused z pass: radices whose butterfly counts divide
// evenly over the workgroup when six components are transformed together.
__host__ __device__ constexpr Plan2 plan_fused(int N) {
  return N == 8     ? Plan2{2, {4, 2, 1}}
         : N == 16  ? Plan2{2, {4, 4, 1}}
         : N == 24  ? Plan2{2, {8, 3, 1}}
         : N == 32  ? Plan2{2, {8, 4, 1}}
         : N == 48  ? Plan2{2, {16, 3, 1}}
         : N == 64  ? Plan2{3, {8, 2, 4}}
         : N == 96  ? Plan2{2, {16, 6, 1}}
         : N == 128 ? Plan2{3, {8, 4, 4}}
         : N == 160 ? Plan2{2, {16, 10, 1}}
         : N == 240 ? Plan2{2, {16, 15, 1}}
         : N == 256 ? Plan2{2, {16, 16, 1}}
         : N == 512 ? Plan2{3, {8, 16, 4}}
         : N == 45  ? Plan2{2, {15, 3, 1}}
         : N == 129 ? Plan2{2, {43, 3, 1}}
                    : Plan2{0, {1, 1, 1}};
}

}  // namespace ec
