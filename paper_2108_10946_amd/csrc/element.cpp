// KMV reference elements (host).  Derived at library load from the definitions:
// nodes = orbits of the reference simplex (coordinates printed in figures
// fig:2dels / fig:3dels for KMV2tri, KMV3tri, KMV2tet, KMV3tet; degree-4 and
// degree-5 triangles solved for from the moment equations), weights = the nodal
// quadrature rule exact to degree 2k - 1 (1, 3, 5, 7 on triangles of degree 1..4,
// 1, 3, 5 on tetrahedra; 10 for the degree-5 triangle), basis = Lagrange basis of
// the enriched space at the nodes, all in long double.
#include "element.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <stdexcept>
#include <string>

namespace kmv {
namespace {

using LD = long double;

// ------------------------------------------------------------ dense polynomials
struct Basis {
  int dim, maxdeg;
  std::vector<std::array<int, 3>> exps;
  std::map<std::array<int, 3>, int> index;
  Basis(int d, int m) : dim(d), maxdeg(m) {
    for (int t = 0; t <= m; ++t)
      for (int i = t; i >= 0; --i)
        for (int j = t - i; j >= 0; --j) {
          int k = t - i - j;
          if (dim == 2 && k != 0) continue;
          std::array<int, 3> e{i, j, k};
          index[e] = (int)exps.size();
          exps.push_back(e);
        }
  }
  int size() const { return (int)exps.size(); }
};

using Poly = std::vector<LD>;

Poly mono(const Basis& B, int i, int j, int k) {
  Poly p(B.size(), 0.0L);
  p[B.index.at({i, j, k})] = 1.0L;
  return p;
}

Poly mul(const Basis& B, const Poly& a, const Poly& b) {
  Poly r(B.size(), 0.0L);
  for (int x = 0; x < B.size(); ++x) {
    if (a[x] == 0.0L) continue;
    for (int y = 0; y < B.size(); ++y) {
      if (b[y] == 0.0L) continue;
      std::array<int, 3> e{B.exps[x][0] + B.exps[y][0], B.exps[x][1] + B.exps[y][1],
                           B.exps[x][2] + B.exps[y][2]};
      auto it = B.index.find(e);
      if (it == B.index.end()) throw std::logic_error("polynomial degree overflow");
      r[it->second] += a[x] * b[y];
    }
  }
  return r;
}

Poly add(const Poly& a, const Poly& b, LD sb = 1.0L) {
  Poly r(a);
  for (size_t i = 0; i < r.size(); ++i) r[i] += sb * b[i];
  return r;
}

LD peval(const Basis& B, const Poly& p, const LD* x) {
  LD s = 0.0L;
  for (int m = 0; m < B.size(); ++m) {
    if (p[m] == 0.0L) continue;
    LD t = p[m];
    for (int r = 0; r < B.dim; ++r)
      for (int e = 0; e < B.exps[m][r]; ++e) t *= x[r];
    s += t;
  }
  return s;
}

Poly pderiv(const Basis& B, const Poly& p, int r) {
  Poly d(B.size(), 0.0L);
  for (int m = 0; m < B.size(); ++m) {
    if (p[m] == 0.0L || B.exps[m][r] == 0) continue;
    std::array<int, 3> e = B.exps[m];
    LD c = p[m] * e[r];
    e[r] -= 1;
    d[B.index.at(e)] += c;
  }
  return d;
}

// barycentric lambda_i as polynomials in the reference coordinates
std::vector<Poly> barycentrics(const Basis& B) {
  std::vector<Poly> lam;
  Poly one = mono(B, 0, 0, 0);
  Poly l0 = one;
  for (int r = 0; r < B.dim; ++r) {
    int e[3] = {0, 0, 0};
    e[r] = 1;
    l0 = add(l0, mono(B, e[0], e[1], e[2]), -1.0L);
  }
  lam.push_back(l0);
  for (int r = 0; r < B.dim; ++r) {
    int e[3] = {0, 0, 0};
    e[r] = 1;
    lam.push_back(mono(B, e[0], e[1], e[2]));
  }
  return lam;
}

// Spanning set of the KMV space: P_k plus bubbles.
std::vector<Poly> kmv_space(const Basis& B, int dim, int k) {
  std::vector<Poly> f;
  for (int m = 0; m < B.size(); ++m) {
    const auto& e = B.exps[m];
    if (e[0] + e[1] + e[2] <= k) f.push_back(mono(B, e[0], e[1], e[2]));
  }
  auto lam = barycentrics(B);
  if (dim == 2) {
    Poly b = mul(B, mul(B, lam[0], lam[1]), lam[2]);
    if (k == 2) f.push_back(b);
    if (k == 3) {
      f.push_back(mul(B, b, lam[1]));
      f.push_back(mul(B, b, lam[2]));
    }
    if (k == 4) {
      // b * (degree-2 part not already in P4): x^2, xy, y^2
      f.push_back(mul(B, b, mono(B, 2, 0, 0)));
      f.push_back(mul(B, b, mono(B, 1, 1, 0)));
      f.push_back(mul(B, b, mono(B, 0, 2, 0)));
    }
    if (k == 5) {
      // b * P4 modulo b * P2 (already in P5): homogeneous degrees 3 and 4
      for (int t = 3; t <= 4; ++t)
        for (int i = t; i >= 0; --i) f.push_back(mul(B, b, mono(B, i, t - i, 0)));
    }
  } else {
    Poly bT = mul(B, mul(B, lam[0], lam[1]), mul(B, lam[2], lam[3]));
    if (k >= 2) {
      for (int j = 0; j < 4; ++j) {
        std::vector<int> F;
        for (int i = 0; i < 4; ++i)
          if (i != j) F.push_back(i);
        Poly bF = mul(B, mul(B, lam[F[0]], lam[F[1]]), lam[F[2]]);
        if (k == 2) f.push_back(bF);
        if (k == 3) {
          f.push_back(mul(B, bF, lam[F[1]]));
          f.push_back(mul(B, bF, lam[F[2]]));
        }
      }
      if (k == 2) f.push_back(bT);
      if (k == 3)
        for (int j = 0; j < 4; ++j) f.push_back(mul(B, bT, lam[j]));
    }
  }
  return f;
}

// -------------------------------------------------------------------- orbits
enum Kind { V, M, E, C, S3, S6, FC, F3, I4 };

struct OrbitDef {
  Kind kind;
  std::vector<LD> p0;  // starting / fixed parameters
  bool free;
};

std::vector<std::vector<LD>> orbit_points(int dim, Kind kind, const LD* p) {
  // label pattern and label values
  std::vector<int> pat;
  std::vector<LD> val;
  const LD h = 0.5L, t3 = 1.0L / 3.0L;
  if (dim == 2) {
    switch (kind) {
      case V: pat = {0, 1, 1}; val = {1, 0}; break;
      case M: pat = {0, 0, 1}; val = {h, 0}; break;
      case E: pat = {0, 1, 2}; val = {p[0], 1 - p[0], 0}; break;
      case C: pat = {0, 0, 0}; val = {t3}; break;
      case S3: pat = {0, 0, 1}; val = {p[0], 1 - 2 * p[0]}; break;
      case S6: pat = {0, 1, 2}; val = {p[0], p[1], 1 - p[0] - p[1]}; break;
      default: throw std::logic_error("orbit");
    }
  } else {
    switch (kind) {
      case V: pat = {0, 1, 1, 1}; val = {1, 0}; break;
      case M: pat = {0, 0, 1, 1}; val = {h, 0}; break;
      case E: pat = {0, 1, 2, 2}; val = {p[0], 1 - p[0], 0}; break;
      case FC: pat = {0, 0, 0, 1}; val = {t3, 0}; break;
      case F3: pat = {0, 0, 1, 2}; val = {p[0], 1 - 2 * p[0], 0}; break;
      case C: pat = {0, 0, 0, 0}; val = {0.25L}; break;
      case I4: pat = {0, 0, 0, 1}; val = {p[0], 1 - 3 * p[0]}; break;
      default: throw std::logic_error("orbit");
    }
  }
  std::sort(pat.begin(), pat.end());
  std::vector<std::vector<LD>> pts;
  do {
    std::vector<LD> b;
    for (int l : pat) b.push_back(val[l]);
    pts.push_back(b);
  } while (std::next_permutation(pat.begin(), pat.end()));
  return pts;
}

struct RuleDef {
  std::vector<OrbitDef> orbits;
  int degree;
  std::vector<LD> w0;
};

RuleDef rule_def(int dim, int k) {
  const LD s6 = 1.0L / 6.0L;
  if (dim == 2) {
    switch (k) {
      case 1: return {{{V, {}, false}}, 1, {}};
      case 2: return {{{V, {}, false}, {M, {}, false}, {C, {}, false}}, 3, {}};
      case 3:  // fig:2dels, KMV3tri
        return {{{V, {}, false}, {E, {0.2934695559090401L}, true}, {S3, {0.2073451756635909L}, true}},
                5, {}};
      case 4:  // solved for: vertices, midpoints, an edge pair, two interior 3-orbits
        return {{{V, {}, false}, {M, {}, false}, {E, {0.2L}, true}, {S3, {0.4L}, true},
                 {S3, {0.15L}, true}},
                7,
                {0.003L, 0.013L, 0.011L, 0.08L, 0.05L}};
      case 5:  // solved for: vertices, two edge pairs, three 3-orbits, one 6-orbit
        return {{{V, {}, false},
                 {E, {0.36330L}, true},
                 {E, {0.13226L}, true},
                 {S3, {0.25686L}, true},
                 {S3, {0.45784L}, true},
                 {S3, {0.05753L}, true},
                 {S6, {0.22100L, 0.70081L}, true}},
                10,
                {0.00071L, 0.0062L, 0.0035L, 0.0459L, 0.0345L, 0.0116L, 0.0273L}};
    }
  } else {
    switch (k) {
      case 1: return {{{V, {}, false}}, 1, {}};
      case 2: return {{{V, {}, false}, {M, {}, false}, {FC, {}, false}, {C, {}, false}}, 3, {}};
      case 3:  // fig:3dels, KMV3tet (32 nodes)
        return {{{V, {}, false}, {E, {0.314210342418033L}, true}, {F3, {0.21548220313557542L}, true},
                 {I4, {s6}, false}},
                5, {}};
    }
  }
  throw std::invalid_argument("unsupported KMV element");
}

LD factorial(int n) {
  LD f = 1.0L;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// Moment residuals: sum_i w_i m(x_i) - int_ref m for monomials m of degree <= q,
// plus, for the degree-2 tetrahedron, the interior bubble (its degree-3 system
// leaves one weight free).
std::vector<LD> residual(int dim, int k, const RuleDef& R, const std::vector<LD>& x) {
  Basis B(dim, R.degree);
  size_t npar = 0;
  for (auto& o : R.orbits)
    if (o.free) npar += o.p0.size();
  std::vector<std::vector<std::vector<LD>>> pts;
  size_t pi = 0;
  for (auto& o : R.orbits) {
    const LD* p = o.p0.data();
    if (o.free) {
      p = x.data() + pi;
      pi += o.p0.size();
    }
    pts.push_back(orbit_points(dim, o.kind, p));
  }
  std::vector<LD> res;
  for (int m = 0; m < B.size(); ++m) {
    const auto& e = B.exps[m];
    LD s = 0.0L;
    for (size_t o = 0; o < pts.size(); ++o)
      for (auto& b : pts[o]) {
        LD t = 1.0L;
        for (int r = 0; r < dim; ++r)
          for (int q = 0; q < e[r]; ++q) t *= b[r + 1];
        s += x[npar + o] * t;
      }
    LD exact = factorial(e[0]) * factorial(e[1]) * factorial(e[2]) / factorial(e[0] + e[1] + e[2] + dim);
    res.push_back((s - exact) / exact);  // relative: high-degree moments are small
  }
  if (dim == 3 && k == 2) {
    LD s = 0.0L;
    for (size_t o = 0; o < pts.size(); ++o)
      for (auto& b : pts[o]) s += x[npar + o] * b[0] * b[1] * b[2] * b[3];
    res.push_back(s * factorial(7) - 1.0L);
  }
  return res;
}

std::vector<LD> solve_dense(std::vector<std::vector<LD>> A, std::vector<LD> b) {
  const int n = (int)b.size();
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    std::swap(A[c], A[piv]);
    std::swap(b[c], b[piv]);
    if (A[c][c] == 0.0L) throw std::runtime_error("singular system");
    for (int r = c + 1; r < n; ++r) {
      LD f = A[r][c] / A[c][c];
      for (int j = c; j < n; ++j) A[r][j] -= f * A[c][j];
      b[r] -= f * b[c];
    }
  }
  std::vector<LD> x(n);
  for (int r = n - 1; r >= 0; --r) {
    LD s = b[r];
    for (int j = r + 1; j < n; ++j) s -= A[r][j] * x[j];
    x[r] = s / A[r][r];
  }
  return x;
}

// Gauss-Newton on the (consistent, possibly overdetermined) moment system.
std::vector<LD> solve_rule(int dim, int k, const RuleDef& R) {
  std::vector<LD> x;
  for (auto& o : R.orbits)
    if (o.free) x.insert(x.end(), o.p0.begin(), o.p0.end());
  size_t npar = x.size();
  size_t nw = R.orbits.size();
  for (size_t o = 0; o < nw; ++o) x.push_back(R.w0.empty() ? 0.1L / nw : R.w0[o]);
  const LD h = 1e-9L;
  for (int it = 0; it < 100; ++it) {
    auto r = residual(dim, k, R, x);
    LD nr = 0;
    for (LD v : r) nr = std::max(nr, std::fabs(v));
    if (nr < 1e-18L) break;
    const size_t ne = r.size(), nx = x.size();
    std::vector<std::vector<LD>> J(ne, std::vector<LD>(nx));
    for (size_t j = 0; j < nx; ++j) {
      auto xp = x, xm = x;
      xp[j] += h;
      xm[j] -= h;
      auto rp = residual(dim, k, R, xp), rm = residual(dim, k, R, xm);
      for (size_t i = 0; i < ne; ++i) J[i][j] = (rp[i] - rm[i]) / (2 * h);
    }
    std::vector<std::vector<LD>> A(nx, std::vector<LD>(nx, 0.0L));
    std::vector<LD> g(nx, 0.0L);
    for (size_t a = 0; a < nx; ++a) {
      for (size_t b = 0; b < nx; ++b)
        for (size_t i = 0; i < ne; ++i) A[a][b] += J[i][a] * J[i][b];
      for (size_t i = 0; i < ne; ++i) g[a] -= J[i][a] * r[i];
    }
    auto dx = solve_dense(A, g);
    for (size_t j = 0; j < nx; ++j) x[j] += dx[j];
  }
  auto r = residual(dim, k, R, x);
  LD nr = 0;
  for (LD v : r) nr = std::max(nr, std::fabs(v));
  if (!(nr < 1e-15L)) throw std::runtime_error("KMV rule did not converge");
  (void)npar;
  return x;
}

std::vector<std::vector<LD>> invert(std::vector<std::vector<LD>> A) {
  const int n = (int)A.size();
  std::vector<std::vector<LD>> I(n, std::vector<LD>(n, 0.0L));
  for (int i = 0; i < n; ++i) I[i][i] = 1.0L;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    std::swap(A[c], A[piv]);
    std::swap(I[c], I[piv]);
    LD d = A[c][c];
    if (d == 0.0L) throw std::runtime_error("KMV nodes are not unisolvent");
    for (int j = 0; j < n; ++j) {
      A[c][j] /= d;
      I[c][j] /= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      LD f = A[r][c];
      if (f == 0.0L) continue;
      for (int j = 0; j < n; ++j) {
        A[r][j] -= f * A[c][j];
        I[r][j] -= f * I[c][j];
      }
    }
  }
  return I;
}

Element build(int dim, int k) {
  RuleDef R = rule_def(dim, k);
  auto x = solve_rule(dim, k, R);
  Element el;
  el.dim = dim;
  el.degree = k;
  size_t pi = 0, npar = 0;
  for (auto& o : R.orbits)
    if (o.free) npar += o.p0.size();
  std::vector<std::vector<LD>> bary;
  std::vector<LD> w;
  for (size_t o = 0; o < R.orbits.size(); ++o) {
    const auto& od = R.orbits[o];
    const LD* p = od.p0.data();
    if (od.free) {
      p = x.data() + pi;
      pi += od.p0.size();
    }
    for (auto& b : orbit_points(dim, od.kind, p)) {
      bary.push_back(b);
      w.push_back(x[npar + o]);
    }
  }
  const int n = (int)bary.size();
  el.n = n;
  const int maxdeg = dim == 2 ? 7 : 5;
  Basis B(dim, maxdeg);
  auto f = kmv_space(B, dim, k);
  if ((int)f.size() != n) throw std::logic_error("KMV space dimension != node count");
  std::vector<std::vector<LD>> V(n, std::vector<LD>(n));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) V[i][j] = peval(B, f[j], &bary[i][1]);
  auto Cm = invert(V);
  el.nodes.resize(n * dim);
  el.bary.resize(n * (dim + 1));
  el.weights.resize(n);
  el.grads.resize((size_t)n * n * dim);
  el.entity.resize(n);
  el.entity_id.resize(n);
  for (int i = 0; i < n; ++i) {
    for (int r = 0; r < dim; ++r) el.nodes[i * dim + r] = (double)bary[i][r + 1];
    for (int r = 0; r <= dim; ++r) el.bary[i * (dim + 1) + r] = (double)bary[i][r];
    el.weights[i] = (double)w[i];
  }
  for (int r = 0; r < dim; ++r) {
    std::vector<Poly> df;
    for (auto& p : f) df.push_back(pderiv(B, p, r));
    for (int q = 0; q < n; ++q) {
      std::vector<LD> dv(n);
      for (int j = 0; j < n; ++j) dv[j] = peval(B, df[j], &bary[q][1]);
      for (int a = 0; a < n; ++a) {
        LD s = 0.0L;
        for (int j = 0; j < n; ++j) s += dv[j] * Cm[j][a];
        el.grads[((size_t)q * n + a) * dim + r] = (double)s;
      }
    }
  }
  // entries that vanish by symmetry come out as round-off; make them exact zeros
  double gmax = 0;
  for (double v : el.grads) gmax = std::max(gmax, std::fabs(v));
  for (double& v : el.grads)
    if (std::fabs(v) < 1e-14 * gmax) v = 0.0;
  // entity of each node from its zero barycentric coordinates
  static const int edges2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  static const int edges3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  for (int i = 0; i < n; ++i) {
    std::vector<int> nz;
    for (int r = 0; r <= dim; ++r)
      if (std::fabs(bary[i][r]) > 1e-12L) nz.push_back(r);
    const int nnz = (int)nz.size();
    if (nnz == 1) {
      el.entity[i] = ENT_VERTEX;
      el.entity_id[i] = nz[0];
    } else if (nnz == 2) {
      el.entity[i] = ENT_EDGE;
      int id = -1;
      const int ne = dim == 2 ? 3 : 6;
      for (int e = 0; e < ne; ++e) {
        const int* ed = dim == 2 ? edges2[e] : edges3[e];
        if (ed[0] == nz[0] && ed[1] == nz[1]) id = e;
      }
      el.entity_id[i] = id;
    } else if (nnz == 3 && dim == 3) {
      el.entity[i] = ENT_FACE;
      int zero = 0;
      for (int r = 0; r <= 3; ++r)
        if (std::fabs(bary[i][r]) <= 1e-12L) zero = r;
      el.entity_id[i] = zero;  // face opposite vertex `zero`
    } else {
      el.entity[i] = ENT_CELL;
      el.entity_id[i] = 0;
    }
  }
  for (int i = 0; i < n; ++i) {
    if (el.entity_id[i] != 0) continue;
    if (el.entity[i] == ENT_VERTEX) el.n_vertex++;
    if (el.entity[i] == ENT_EDGE) el.n_edge++;
    if (el.entity[i] == ENT_FACE) el.n_face++;
    if (el.entity[i] == ENT_CELL) el.n_cell++;
  }
  el.span_polys = f;
  el.mono = B.exps;
  el.coef.resize((size_t)n * n);
  for (int j = 0; j < n; ++j)
    for (int a = 0; a < n; ++a) el.coef[(size_t)j * n + a] = Cm[j][a];
  return el;
}

std::mutex g_mu;
std::map<std::pair<int, int>, Element> g_cache;

}  // namespace

bool element_supported(int dim, int degree) {
  return (dim == 2 && degree >= 1 && degree <= 5) || (dim == 3 && degree >= 1 && degree <= 3);
}

const Element& element(int dim, int degree) {
  if (!element_supported(dim, degree)) throw std::invalid_argument("unsupported (dim, degree)");
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_pair(dim, degree);
  auto it = g_cache.find(key);
  if (it == g_cache.end()) it = g_cache.emplace(key, build(dim, degree)).first;
  return it->second;
}

void Element::eval(const double* xi, double* phi) const {
  const size_t nf = span_polys.size();
  std::vector<long double> fv(nf);
  for (size_t j = 0; j < nf; ++j) {
    long double s = 0.0L;
    const auto& p = span_polys[j];
    for (size_t m = 0; m < p.size(); ++m) {
      if (p[m] == 0.0L) continue;
      long double t = p[m];
      for (int r = 0; r < dim; ++r)
        for (int e = 0; e < mono[m][r]; ++e) t *= xi[r];
      s += t;
    }
    fv[j] = s;
  }
  for (int a = 0; a < n; ++a) {
    long double s = 0.0L;
    for (size_t j = 0; j < nf; ++j) s += fv[j] * coef[j * n + a];
    phi[a] = (double)s;
  }
}

}  // namespace kmv
