// Host-side driver for a sanitizer build (AddressSanitizer + UndefinedBehavior-
// Sanitizer) of the library's CPU code: element derivation, mesh preprocessing
// (DOF numbering, patches, gather words, shared-DOF lists), scheduling checks,
// point location, the Gershgorin bound and the boundary mass, on jittered
// structured meshes of every supported element, plus the rejection of bad meshes.
// Built and run by tests/test_host_sanitize.py with g++ (no GPU code involved).
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "element.hpp"
#include "mesh.hpp"

namespace {

uint64_t g_state = 0x2545F4914F6CDD1Dull;
double uniform() {  // xorshift64*, a fixed test sequence
  g_state ^= g_state >> 12;
  g_state ^= g_state << 25;
  g_state ^= g_state >> 27;
  return (double)((g_state * 2685821657736338717ull) >> 11) * 0x1.0p-53;
}

// n x n squares split into two triangles, interior vertices jittered
void square_mesh(int n, std::vector<double>& xy, std::vector<int32_t>& cells) {
  const double h = 1.0 / n;
  for (int j = 0; j <= n; ++j)
    for (int i = 0; i <= n; ++i) {
      double x = i * h, z = j * h;
      if (i > 0 && i < n && j > 0 && j < n) {
        x += 0.2 * h * (uniform() - 0.5);
        z += 0.2 * h * (uniform() - 0.5);
      }
      xy.push_back(x);
      xy.push_back(z);
    }
  auto v = [n](int i, int j) { return (int32_t)(j * (n + 1) + i); };
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      cells.insert(cells.end(), {v(i, j), v(i + 1, j), v(i + 1, j + 1)});
      cells.insert(cells.end(), {v(i, j), v(i + 1, j + 1), v(i, j + 1)});
    }
}

// n^3 cubes split into six Kuhn tetrahedra, interior vertices jittered
void cube_mesh(int n, std::vector<double>& xyz, std::vector<int32_t>& cells) {
  const double h = 1.0 / n;
  for (int k = 0; k <= n; ++k)
    for (int j = 0; j <= n; ++j)
      for (int i = 0; i <= n; ++i) {
        double p[3] = {i * h, j * h, k * h};
        const bool inner = i > 0 && i < n && j > 0 && j < n && k > 0 && k < n;
        for (double& q : p) {
          if (inner) q += 0.15 * h * (uniform() - 0.5);
          xyz.push_back(q);
        }
      }
  auto v = [n](int i, int j, int k) { return (int32_t)((k * (n + 1) + j) * (n + 1) + i); };
  const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        for (const auto& pm : perm) {
          int c[3] = {i, j, k};
          cells.push_back(v(c[0], c[1], c[2]));
          for (int s = 0; s < 3; ++s) {
            c[pm[s]] += 1;
            cells.push_back(v(c[0], c[1], c[2]));
          }
        }
}

int g_fail = 0;
void check(bool ok, const std::string& what) {
  if (!ok) {
    std::printf("FAIL %s\n", what.c_str());
    ++g_fail;
  }
}

void exercise(int dim, int degree, int n, int patch) {
  std::vector<double> x;
  std::vector<int32_t> cells;
  if (dim == 2)
    square_mesh(n, x, cells);
  else
    cube_mesh(n, x, cells);
  const int64_t nv = (int64_t)x.size() / dim, ne = (int64_t)cells.size() / (dim + 1);
  kmv::Mesh* m = kmv::build_mesh(dim, degree, x.data(), nv, cells.data(), ne, patch);
  const std::string tag = std::to_string(dim) + "D k=" + std::to_string(degree) + " patch=" + std::to_string(patch);
  std::string why;
  check(kmv::validate_mesh(*m, why), tag + " validate: " + why);
  double msum = 0;
  for (double v : m->mass) msum += v;
  check(std::fabs(msum - 1.0) < 1e-12, tag + " mass sums to the volume");
  std::vector<double> c(m->n_dofs, 1.5);
  const double rho = kmv::gershgorin_rho(*m, c.data());
  check(rho > 0 && std::isfinite(rho), tag + " gershgorin");
  std::vector<int32_t> bd;
  std::vector<double> bb;
  kmv::boundary_weights(*m, bd, bb);
  double bsum = 0;
  for (double v : bb) bsum += v;
  check(std::fabs(bsum - (dim == 2 ? 4.0 : 6.0)) < 1e-10, tag + " boundary mass sums to the boundary measure");
  for (int t = 0; t < 50; ++t) {
    double p[3] = {uniform(), uniform(), uniform()};
    kmv::PointLoc loc;
    check(m->locate(p, loc), tag + " locate inside");
    double s = 0;
    for (double v : loc.phi) s += v;
    check(std::fabs(s - 1.0) < 1e-10, tag + " partition of unity at a located point");
  }
  double out[3] = {1.5, 0.5, 0.5};
  kmv::PointLoc loc;
  check(!m->locate(out, loc), tag + " locate outside");
  delete m;
}

}  // namespace

int main() {
  for (int k = 1; k <= 5; ++k) {
    exercise(2, k, 6, 0);
    exercise(2, k, 6, 9);
  }
  for (int k = 1; k <= 3; ++k) {
    exercise(3, k, 3, 0);
    exercise(3, k, 3, 7);
  }
  // bad meshes are rejected with an exception, not an out-of-range access
  {
    std::vector<double> x = {0, 0, 1, 0, 0, 1};
    std::vector<int32_t> bad = {0, 1, 7};
    bool thrown = false;
    try {
      delete kmv::build_mesh(2, 2, x.data(), 3, bad.data(), 1, 0);
    } catch (...) {
      thrown = true;
    }
    check(thrown, "vertex index out of range");
    std::vector<double> flat = {0, 0, 1, 0, 2, 0};
    std::vector<int32_t> one = {0, 1, 2};
    thrown = false;
    try {
      delete kmv::build_mesh(2, 2, flat.data(), 3, one.data(), 1, 0);
    } catch (...) {
      thrown = true;
    }
    check(thrown, "zero-area cell");
  }
  std::printf("%s\n", g_fail ? "FAILED" : "OK");
  return g_fail ? 1 : 0;
}
