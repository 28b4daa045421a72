// Host-side checks of the defect quantisation, validation and footprint
// enumeration of the C-ABI library, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side (the library source is
// included whole so that its internal functions are reachable; no HIP call
// is made).  Exit status 0 when every check holds.
#include "../../paper_2403_09158_amd/csrc/ec_api.hip"

#include <cstdio>
#include <random>
#include <set>

namespace {

int failures = 0;
#define CHECK(c, ...)                          \
  do {                                         \
    if (!(c)) {                                \
      ++failures;                              \
      std::fprintf(stderr, "FAIL: " __VA_ARGS__); \
      std::fprintf(stderr, "\n");              \
    }                                          \
  } while (0)

ec_problem cell(int n, double L) {
  ec_problem P{};
  P.n = n;
  P.L = L;
  P.C11 = 243.0;
  P.C12 = 145.0;
  P.C44 = 116.0;
  return P;
}

ec_defect loop(const double c[3], double R, const double b[3], const double nrm[3], double e = 0.0) {
  ec_defect d{};
  d.kind = EC_LOOP;
  for (int k = 0; k < 3; ++k) {
    d.c[k] = c[k];
    d.b[k] = b[k];
    d.normal[k] = nrm[k];
  }
  d.radius = R;
  d.thickness = e;
  return d;
}

// Every member voxel of the grid (brute force over all n^3) is in the
// footprint enumeration and nothing else is.
void footprint_complete(const ec_problem& P, const ec_defect& rec, const char* what) {
  DevDefect d;
  std::string err;
  if (!quantise(P, rec, d, err)) {
    CHECK(false, "%s: valid defect rejected (%s)", what, err.c_str());
    return;
  }
  std::vector<int32_t> ids;
  footprint_ids(d, P.n, ids);
  for (size_t i = 1; i < ids.size(); ++i) CHECK(ids[i - 1] < ids[i], "%s: footprint not ascending", what);
  std::set<int32_t> got(ids.begin(), ids.end()), want;
  for (int z = 0; z < P.n; ++z)
    for (int y = 0; y < P.n; ++y)
      for (int x = 0; x < P.n; ++x)
        if (member(d, P.n, x, y, z)) want.insert((z * P.n + y) * P.n + x);
  CHECK(got == want, "%s: footprint %zu voxels, brute force %zu", what, got.size(), want.size());
}

void rejects(const ec_problem& P, const ec_defect& rec, const char* what) {
  DevDefect d;
  std::string err;
  CHECK(!quantise(P, rec, d, err) && !err.empty(), "%s: invalid defect accepted", what);
}

}  // namespace

int main() {
  std::mt19937_64 rng(240309158);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const double a = 0.2866;
  const int normals[][3] = {{1, 1, 1}, {1, -1, 1}, {1, 0, 0}, {0, 1, 0}, {1, 1, 0}, {2, 1, 0}, {3, -1, 2}};
  for (int n : {16, 21, 24}) {
    const double L = n * 0.3125;
    const ec_problem P = cell(n, L);
    for (int t = 0; t < 60; ++t) {
      const double c[3] = {U(rng) * L * 3.0 - L, U(rng) * L, U(rng) * L};  // also outside the cell
      const int* m = normals[t % 7];
      const double nrm[3] = {(double)m[0], (double)m[1], (double)m[2]};
      const double s = 0.5 * a / std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
      const double b[3] = {s * nrm[0], s * nrm[1], s * nrm[2]};
      const double R = 0.2 + U(rng) * 0.35 * L;
      const double e = (t % 3 == 0) ? 0.0 : 0.3125 * (0.5 + 2.0 * U(rng));
      footprint_complete(P, loop(c, R, b, nrm, e), "loop");
      ec_defect sp{};
      sp.kind = EC_SPHERE;
      for (int k = 0; k < 3; ++k) sp.c[k] = c[k];
      sp.radius = 0.1 + U(rng) * 0.45 * L;
      sp.eig_v = 0.01;
      footprint_complete(P, sp, "sphere");
    }
    // invalid records are refused with a message
    const double c[3] = {1.0, 1.0, 1.0}, b[3] = {0.1, 0.1, 0.1}, nrm[3] = {1, 1, 1};
    rejects(P, loop(c, -1.0, b, nrm), "negative radius");
    rejects(P, loop(c, std::nan(""), b, nrm), "NaN radius");
    rejects(P, loop(c, 0.5 * L, b, nrm), "loop reaching half the cell");
    const double zero[3] = {0, 0, 0}, odd[3] = {1.0, 0.37, 0.0}, nanc[3] = {std::nan(""), 0, 0},
                 huge[3] = {1e300, 0, 0};
    rejects(P, loop(c, 1.0, zero, nrm), "zero Burgers vector");
    rejects(P, loop(c, 1.0, b, odd), "irrational habit normal");
    rejects(P, loop(c, 1.0, b, zero), "zero habit normal");
    rejects(P, loop(nanc, 1.0, b, nrm), "NaN centre");
    rejects(P, loop(huge, 1.0, b, nrm), "centre out of range");
    rejects(P, loop(c, 1.0, b, nrm, -0.1), "negative thickness");
    rejects(P, loop(c, 1.0, b, nrm, 1e-9), "thickness below the quantisation step");
    const double big_b[3] = {100.0, 0, 0};
    rejects(P, loop(c, 1.0, big_b, nrm, 0.5), "eigenstrain too large");
    ec_defect bad{};
    bad.kind = 7;
    bad.radius = 1.0;
    rejects(P, bad, "unknown kind");
  }
  std::printf("%s: %d failure(s)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
