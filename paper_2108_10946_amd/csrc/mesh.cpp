// Mesh preprocessing (host): topological DOF numbering, geometry, lumped mass,
// recursive-coordinate-bisection patches, in-patch colouring, owned/shared DOF
// split and patch-local maps for the GPU kernels.
#include "mesh.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <stdexcept>
#include <unordered_map>

namespace kmv {
namespace {

const int kEdges2[3][2] = {{0, 1}, {0, 2}, {1, 2}};
const int kEdges3[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

void invert_small(int d, const double* J, double* Ji, double* det) {
  if (d == 2) {
    const double a = J[0], b = J[1], c = J[2], e = J[3];
    const double dt = a * e - b * c;
    *det = dt;
    Ji[0] = e / dt;
    Ji[1] = -b / dt;
    Ji[2] = -c / dt;
    Ji[3] = a / dt;
  } else {
    const double a = J[0], b = J[1], c = J[2], d_ = J[3], e = J[4], f = J[5], g = J[6], h = J[7],
                 i = J[8];
    const double A = e * i - f * h, B = -(d_ * i - f * g), C = d_ * h - e * g;
    const double dt = a * A + b * B + c * C;
    *det = dt;
    Ji[0] = A / dt;
    Ji[1] = -(b * i - c * h) / dt;
    Ji[2] = (b * f - c * e) / dt;
    Ji[3] = B / dt;
    Ji[4] = (a * i - c * g) / dt;
    Ji[5] = -(a * f - c * d_) / dt;
    Ji[6] = C / dt;
    Ji[7] = -(a * h - b * g) / dt;
    Ji[8] = (a * e - b * d_) / dt;
  }
}

// Recursive coordinate bisection of cell centroids into leaves of <= P cells.
void rcb(std::vector<int64_t>& ids, int64_t b, int64_t e, const std::vector<double>& cen, int dim,
         int P, std::vector<int64_t>& leaf_start) {
  const int64_t n = e - b;
  if (n <= P) {
    leaf_start.push_back(b);
    return;
  }
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t i = b; i < e; ++i)
    for (int r = 0; r < dim; ++r) {
      lo[r] = std::min(lo[r], cen[ids[i] * dim + r]);
      hi[r] = std::max(hi[r], cen[ids[i] * dim + r]);
    }
  int ax = 0;
  for (int r = 1; r < dim; ++r)
    if (hi[r] - lo[r] > hi[ax] - lo[ax]) ax = r;
  const int64_t leaves = (n + P - 1) / P;
  const int64_t nl = n * (leaves / 2) / leaves;
  std::nth_element(ids.begin() + b, ids.begin() + b + nl, ids.begin() + e,
                   [&](int64_t x, int64_t y) {
                     const double cx = cen[x * dim + ax], cy = cen[y * dim + ax];
                     return cx < cy || (cx == cy && x < y);
                   });
  rcb(ids, b, b + nl, cen, dim, P, leaf_start);
  rcb(ids, b + nl, e, cen, dim, P, leaf_start);
}

int64_t nearest(const std::vector<std::array<double, 2>>& list, double a, double b) {
  int64_t best = -1;
  double bd = 1e300;
  for (size_t i = 0; i < list.size(); ++i) {
    const double d = std::fabs(list[i][0] - a) + std::fabs(list[i][1] - b);
    if (d < bd) {
      bd = d;
      best = (int64_t)i;
    }
  }
  if (bd > 1e-9) throw MeshError{"node does not match its entity's canonical nodes"};
  return best;
}

}  // namespace

Mesh* build_mesh(int dim, int degree, const double* coords, int64_t nv, const int32_t* cells,
                 int64_t ne, int patch_cells) {
  if (dim != 2 && dim != 3) throw std::invalid_argument("dim must be 2 or 3");
  if (!coords || !cells || nv <= 0 || ne <= 0) throw std::invalid_argument("empty mesh");
  const Element& el = element(dim, degree);
  std::unique_ptr<Mesh> m(new Mesh());
  m->dim = dim;
  m->degree = degree;
  m->el = &el;
  m->nd = el.n;
  m->ng = dim == 2 ? 3 : 6;
  m->n_vertices = nv;
  m->n_cells = ne;
  m->coords.assign(coords, coords + nv * dim);
  m->cells_in.assign(cells, cells + ne * (dim + 1));
  const int nvc = dim + 1, nd = el.n, dd = dim * dim;
  for (int64_t i = 0; i < ne * nvc; ++i)
    if (cells[i] < 0 || cells[i] >= nv) {
      throw MeshError{"cell vertex index out of range"};
    }

  // ---- geometry per input cell
  std::vector<double> J(ne * dd), Ji(ne * dd), det(ne), cen(ne * dim);
  for (int64_t c = 0; c < ne; ++c) {
    const double* p0 = coords + (int64_t)cells[c * nvc] * dim;
    double hmax = 0;
    for (int r = 0; r < dim; ++r) {
      const double* pr = coords + (int64_t)cells[c * nvc + r + 1] * dim;
      double l2 = 0;
      for (int i = 0; i < dim; ++i) {
        J[c * dd + i * dim + r] = pr[i] - p0[i];
        l2 += (pr[i] - p0[i]) * (pr[i] - p0[i]);
      }
      hmax = std::max(hmax, std::sqrt(l2));
    }
    invert_small(dim, &J[c * dd], &Ji[c * dd], &det[c]);
    if (!(std::fabs(det[c]) > 1e-13 * std::pow(hmax, dim))) {
      throw MeshError{"degenerate (zero-measure) cell"};
    }
    for (int i = 0; i < dim; ++i) {
      double s = 0;
      for (int v = 0; v < nvc; ++v) s += coords[(int64_t)cells[c * nvc + v] * dim + i];
      cen[c * dim + i] = s / nvc;
    }
  }

  // ---- topological DOF numbering (initial ids)
  std::vector<int64_t> vdof(nv, -1);
  int64_t nvd = 0;
  for (int64_t i = 0; i < ne * nvc; ++i)
    if (vdof[cells[i]] < 0) vdof[cells[i]] = nvd++;
  const int nedge_loc = dim == 2 ? 3 : 6;
  std::unordered_map<uint64_t, int64_t> edge_id;
  edge_id.reserve(ne * nedge_loc);
  std::vector<int64_t> cell_edge(ne * nedge_loc);
  for (int64_t c = 0; c < ne; ++c)
    for (int e = 0; e < nedge_loc; ++e) {
      const int* ed = dim == 2 ? kEdges2[e] : kEdges3[e];
      uint64_t a = cells[c * nvc + ed[0]], b = cells[c * nvc + ed[1]];
      if (a > b) std::swap(a, b);
      auto it = edge_id.emplace(a * (uint64_t)nv + b, (int64_t)edge_id.size()).first;
      cell_edge[c * nedge_loc + e] = it->second;
    }
  const int64_t n_edges = (int64_t)edge_id.size();
  std::vector<int64_t> cell_face;
  int64_t n_faces = 0;
  if (dim == 3) {
    std::vector<std::array<int64_t, 5>> fk;  // a, b, c, cell, local face
    fk.reserve(ne * 4);
    for (int64_t c = 0; c < ne; ++c)
      for (int j = 0; j < 4; ++j) {
        std::array<int64_t, 3> v;
        int t = 0;
        for (int i = 0; i < 4; ++i)
          if (i != j) v[t++] = cells[c * 4 + i];
        std::sort(v.begin(), v.end());
        fk.push_back({v[0], v[1], v[2], c, j});
      }
    std::sort(fk.begin(), fk.end());
    cell_face.assign(ne * 4, -1);
    for (size_t i = 0; i < fk.size(); ++i) {
      if (i == 0 || fk[i][0] != fk[i - 1][0] || fk[i][1] != fk[i - 1][1] || fk[i][2] != fk[i - 1][2])
        ++n_faces;
      cell_face[fk[i][3] * 4 + fk[i][4]] = n_faces - 1;
    }
  }
  // canonical node lists on one reference edge / face
  std::vector<std::array<double, 2>> edge_can, face_can;
  for (int q = 0; q < nd; ++q) {
    if (el.entity[q] == ENT_EDGE && el.entity_id[q] == 0)  // edge (0,1): coordinate lambda_0
      edge_can.push_back({el.bary[q * (dim + 1) + 0], 0.0});
    if (el.entity[q] == ENT_FACE && el.entity_id[q] == 3)  // face (0,1,2): (lambda_0, lambda_1)
      face_can.push_back({el.bary[q * 4 + 0], el.bary[q * 4 + 1]});
  }
  std::sort(edge_can.begin(), edge_can.end());
  std::sort(face_can.begin(), face_can.end());
  const int64_t edge_base = nvd, face_base = edge_base + n_edges * el.n_edge;
  const int64_t cell_base = face_base + n_faces * el.n_face;
  const int64_t ndof = cell_base + ne * el.n_cell;
  std::vector<int64_t> cdof0(ne * nd);
  for (int64_t c = 0; c < ne; ++c) {
    int icell = 0;
    const int32_t* cv = cells + c * nvc;
    for (int q = 0; q < nd; ++q) {
      const double* bq = &el.bary[q * (dim + 1)];
      const int id = el.entity_id[q];
      int64_t g = -1;
      switch (el.entity[q]) {
        case ENT_VERTEX: g = vdof[cv[id]]; break;
        case ENT_EDGE: {
          const int* ed = dim == 2 ? kEdges2[id] : kEdges3[id];
          const int lo_loc = cv[ed[0]] < cv[ed[1]] ? ed[0] : ed[1];
          g = edge_base + cell_edge[c * nedge_loc + id] * el.n_edge + nearest(edge_can, bq[lo_loc], 0.0);
          break;
        }
        case ENT_FACE: {
          int f[3], t = 0;
          for (int i = 0; i < 4; ++i)
            if (i != id) f[t++] = i;
          std::sort(f, f + 3, [&](int x, int y) { return cv[x] < cv[y]; });
          g = face_base + cell_face[c * 4 + id] * el.n_face + nearest(face_can, bq[f[0]], bq[f[1]]);
          break;
        }
        default: g = cell_base + c * el.n_cell + (icell++);
      }
      cdof0[c * nd + q] = g;
    }
  }

  // ---- patches by recursive coordinate bisection
  if (patch_cells <= 0) {
    double dofs_per_cell = dim == 2 ? 0.5 + 1.5 * el.n_edge + el.n_cell
                                    : 1.0 / 6.0 + 7.0 / 6.0 * el.n_edge + 2.0 * el.n_face + el.n_cell;
    int P = (int)(2048.0 / (dofs_per_cell * 1.25));
    P = (P / 64) * 64;
    patch_cells = std::max(64, std::min(512, P));
  }
  m->patch_cells = patch_cells;
  std::vector<int64_t> order(ne);
  std::iota(order.begin(), order.end(), 0);
  std::vector<int64_t> leaf_start;
  rcb(order, 0, ne, cen, dim, patch_cells, leaf_start);
  leaf_start.push_back(ne);
  const int64_t np = (int64_t)leaf_start.size() - 1;
  m->n_patches = np;

  // ---- colour cells inside each patch (no two same-colour cells share a DOF)
  std::vector<uint64_t> dof_mask(ndof, 0);
  std::vector<int> colour(ne, -1);
  m->patch_ncol.assign(np, 0);
  for (int64_t p = 0; p < np; ++p) {
    int ncol = 0;
    for (int64_t i = leaf_start[p]; i < leaf_start[p + 1]; ++i) {
      const int64_t c = order[i];
      uint64_t forbid = 0;
      for (int q = 0; q < nd; ++q) forbid |= dof_mask[cdof0[c * nd + q]];
      if (forbid == ~0ull) {
          throw MeshError{"more than 64 colours needed inside a patch"};
      }
      int col = __builtin_ctzll(~forbid);
      colour[c] = col;
      ncol = std::max(ncol, col + 1);
      for (int q = 0; q < nd; ++q) dof_mask[cdof0[c * nd + q]] |= 1ull << col;
    }
    for (int64_t i = leaf_start[p]; i < leaf_start[p + 1]; ++i) {
      const int64_t c = order[i];
      for (int q = 0; q < nd; ++q) dof_mask[cdof0[c * nd + q]] = 0;
    }
    std::stable_sort(order.begin() + leaf_start[p], order.begin() + leaf_start[p + 1],
                     [&](int64_t x, int64_t y) { return colour[x] < colour[y]; });
    m->patch_ncol[p] = ncol;
    m->max_colours = std::max(m->max_colours, ncol);
  }
  m->cell_input = order;

  // ---- owned / shared classification
  std::vector<int32_t> last(ndof, -1), npat(ndof, 0), first_patch(ndof, -1);
  for (int64_t p = 0; p < np; ++p)
    for (int64_t i = leaf_start[p]; i < leaf_start[p + 1]; ++i) {
      const int64_t c = order[i];
      for (int q = 0; q < nd; ++q) {
        const int64_t g = cdof0[c * nd + q];
        if (last[g] != p) {
          last[g] = (int32_t)p;
          if (npat[g]++ == 0) first_patch[g] = (int32_t)p;
        }
      }
    }
  std::vector<int64_t> newid(ndof, -1);
  int64_t next = 0;
  m->patch_own_start.assign(np + 1, 0);
  for (int64_t p = 0; p < np; ++p) {
    m->patch_own_start[p] = (int32_t)next;
    for (int64_t i = leaf_start[p]; i < leaf_start[p + 1]; ++i) {
      const int64_t c = order[i];
      for (int q = 0; q < nd; ++q) {
        const int64_t g = cdof0[c * nd + q];
        if (npat[g] == 1 && newid[g] < 0) newid[g] = next++;
      }
    }
  }
  m->patch_own_start[np] = (int32_t)next;
  m->n_own_total = next;
  for (int64_t p = 0; p < np; ++p)
    for (int64_t i = leaf_start[p]; i < leaf_start[p + 1]; ++i) {
      const int64_t c = order[i];
      for (int q = 0; q < nd; ++q) {
        const int64_t g = cdof0[c * nd + q];
        if (newid[g] < 0) newid[g] = next++;
      }
    }
  if (next != ndof) {
    throw MeshError{"DOF numbering incomplete (unused vertices?)"};
  }
  m->n_dofs = ndof;
  m->n_shared = ndof - m->n_own_total;
  {
    std::vector<int32_t> fp(ndof);
    for (int64_t g = 0; g < ndof; ++g) fp[newid[g]] = first_patch[g];
    first_patch.swap(fp);
  }
  if (ndof >= (int64_t)1 << 31) {
    throw std::invalid_argument("more than 2^31 DOFs");
  }

  // ---- final per-cell arrays in internal order
  m->cell_dofs.resize(ne * nd);
  m->x0.resize(ne * dim);
  m->jac.resize(ne * dd);
  m->jinv.resize(ne * dd);
  m->absdet.resize(ne);
  m->geom.resize(ne * m->ng);
  for (int64_t i = 0; i < ne; ++i) {
    const int64_t c = order[i];
    for (int q = 0; q < nd; ++q) m->cell_dofs[i * nd + q] = newid[cdof0[c * nd + q]];
    for (int r = 0; r < dim; ++r) m->x0[i * dim + r] = coords[(int64_t)cells[c * nvc] * dim + r];
    std::memcpy(&m->jac[i * dd], &J[c * dd], dd * sizeof(double));
    std::memcpy(&m->jinv[i * dd], &Ji[c * dd], dd * sizeof(double));
    const double ad = std::fabs(det[c]);
    m->absdet[i] = ad;
    const double* Jv = &Ji[c * dd];
    int t = 0;
    for (int r = 0; r < dim; ++r)
      for (int s = r; s < dim; ++s) {
        double v = 0;
        for (int k = 0; k < dim; ++k) v += Jv[r * dim + k] * Jv[s * dim + k];
        m->geom[i * m->ng + (t++)] = ad * v;
      }
  }
  // lumped mass and DOF coordinates
  m->mass.assign(ndof, 0.0);
  m->dof_coords.assign(ndof * dim, 0.0);
  std::vector<char> seen(ndof, 0);
  for (int64_t i = 0; i < ne; ++i)
    for (int q = 0; q < nd; ++q) {
      const int64_t g = m->cell_dofs[i * nd + q];
      m->mass[g] += el.weights[q] * m->absdet[i];
      if (!seen[g]) {
        seen[g] = 1;
        for (int k = 0; k < dim; ++k) {
          double x = m->x0[i * dim + k];
          for (int r = 0; r < dim; ++r) x += m->jac[i * dd + k * dim + r] * el.nodes[q * dim + r];
          m->dof_coords[g * dim + k] = x;
        }
      }
    }

  // ---- patch-local maps
  m->patch_cell_start.assign(leaf_start.begin(), leaf_start.end());
  m->patch_sh_start.assign(np + 1, 0);
  m->colour_start.assign(np * (kMaxColours + 1), 0);
  m->lmap.assign((size_t)nd * ne, 0);
  m->dof_patch.assign(ndof, -1);
  m->dof_local.assign(ndof, -1);
  std::vector<int32_t> loc(ndof, -1);
  std::vector<int32_t> sh_list;
  for (int64_t p = 0; p < np; ++p) {
    m->patch_sh_start[p] = (int32_t)sh_list.size();
    const int32_t own0 = m->patch_own_start[p];
    const int32_t nown = m->patch_own_start[p + 1] - own0;
    int32_t nsh = 0;
    std::vector<int32_t> touched;
    // colour boundaries
    int32_t* cs = &m->colour_start[p * (kMaxColours + 1)];
    for (int col = 0; col <= kMaxColours; ++col) cs[col] = (int32_t)leaf_start[p + 1];
    for (int64_t i = leaf_start[p + 1] - 1; i >= leaf_start[p]; --i) cs[colour[order[i]]] = (int32_t)i;
    for (int col = m->patch_ncol[p] - 1; col >= 0; --col)
      if (cs[col] > cs[col + 1]) cs[col] = cs[col + 1];
    for (int64_t i = leaf_start[p]; i < leaf_start[p + 1]; ++i)
      for (int q = 0; q < nd; ++q) {
        const int64_t g = m->cell_dofs[i * nd + q];
        if (loc[g] < 0) {
          if (g < m->n_own_total) {
            loc[g] = (int32_t)(g - own0);
          } else {
            loc[g] = nown + nsh++;
            sh_list.push_back((int32_t)g);
          }
          touched.push_back((int32_t)g);
        }
        m->lmap[(size_t)q * ne + i] = (uint16_t)loc[g];
      }
    const int nloc = nown + nsh;
    if (nloc > 65535) {
      throw std::invalid_argument("patch too large for 16-bit local indices");
    }
    m->max_nloc = std::max(m->max_nloc, nloc);
    m->max_patch_cells = std::max(m->max_patch_cells, (int)(leaf_start[p + 1] - leaf_start[p]));
    for (int32_t g : touched) {
      if (first_patch[g] == p) {  // owner patch of an owned DOF, or first of a shared one
        m->dof_patch[g] = (int32_t)p;
        m->dof_local[g] = loc[g];
      }
      loc[g] = -1;
    }
  }
  // gather lists (inverse of lmap per patch), entries in (cell, node) order
  if ((int64_t)m->max_patch_cells * nd > 65535) throw std::invalid_argument("patch too large for 16-bit slots");
  m->gl_ptr_off.assign(np + 1, 0);
  m->gl_ent_off.assign(np + 1, 0);
  auto pad8 = [](int64_t x) { return (x + 7) / 8 * 8; };
  for (int64_t p = 0; p < np; ++p) {
    const int32_t nloc = (m->patch_own_start[p + 1] - m->patch_own_start[p]) +
                         ((p + 1 < np ? m->patch_sh_start[p + 1] : (int32_t)sh_list.size()) - m->patch_sh_start[p]);
    m->gl_ptr_off[p + 1] = (int32_t)(m->gl_ptr_off[p] + pad8(nloc + 1));
    m->gl_ent_off[p + 1] = (int32_t)(m->gl_ent_off[p] + pad8((leaf_start[p + 1] - leaf_start[p]) * nd));
  }
  m->gl_ptr.assign(m->gl_ptr_off[np], 0);
  m->gl_ent.assign(m->gl_ent_off[np], 0);
  for (int64_t p = 0; p < np; ++p) {
    const int32_t c0 = (int32_t)leaf_start[p], c1 = (int32_t)leaf_start[p + 1];
    const int32_t nloc = (m->patch_own_start[p + 1] - m->patch_own_start[p]) +
                         ((p + 1 < np ? m->patch_sh_start[p + 1] : (int32_t)sh_list.size()) - m->patch_sh_start[p]);
    uint16_t* gp = &m->gl_ptr[m->gl_ptr_off[p]];
    uint16_t* ge = &m->gl_ent[m->gl_ent_off[p]];
    std::vector<int32_t> cnt(nloc + 1, 0);
    for (int32_t e = c0; e < c1; ++e)
      for (int a = 0; a < nd; ++a) cnt[m->lmap[(size_t)a * ne + e] + 1]++;
    for (int32_t i = 0; i < nloc; ++i) cnt[i + 1] += cnt[i];
    for (int32_t i = 0; i <= nloc; ++i) gp[i] = (uint16_t)cnt[i];
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t e = c0; e < c1; ++e)
      for (int a = 0; a < nd; ++a) {
        const int li = m->lmap[(size_t)a * ne + e];
        ge[fill[li]++] = (uint16_t)((e - c0) * nd + a);
      }
  }
  // designated patch of a shared DOF: the first patch touching it
  for (int64_t g = 0; g < ndof; ++g)
    if (m->dof_patch[g] < 0) {
      throw std::logic_error("DOF without a designated patch");
    }
  m->patch_sh_start[np] = (int32_t)sh_list.size();
  m->sh_idx = sh_list;
  m->n_shared_refs = (int64_t)sh_list.size();
  m->shp_ptr.assign(m->n_shared + 1, 0);
  for (int32_t g : sh_list) m->shp_ptr[g - m->n_own_total + 1]++;
  for (int64_t s = 0; s < m->n_shared; ++s) m->shp_ptr[s + 1] += m->shp_ptr[s];
  m->shp_slot.assign(sh_list.size(), 0);
  {
    std::vector<int32_t> fill(m->shp_ptr.begin(), m->shp_ptr.end() - 1);
    for (size_t k = 0; k < sh_list.size(); ++k) {
      const int64_t s = sh_list[k] - m->n_own_total;
      m->shp_slot[fill[s]++] = (int32_t)k;  // patches visited in order -> slots increase
    }
  }
  // inline copy of each shared ref's slot list (first entry = designated patch)
  for (int64_t s = 0; s < m->n_shared; ++s)
    m->max_share = std::max(m->max_share, m->shp_ptr[s + 1] - m->shp_ptr[s]);
  // inline pair {first slot, second slot} for DOFs on the interface of two
  // patches; {first slot, -count} otherwise (the kernels then walk the CSR list)
  m->ref_slots.assign(sh_list.size() * kMaxShare, -1);
  for (size_t r = 0; r < sh_list.size(); ++r) {
    const int64_t s = sh_list[r] - m->n_own_total;
    const int32_t k0 = m->shp_ptr[s], k1 = m->shp_ptr[s + 1];
    m->ref_slots[r * kMaxShare + 0] = m->shp_slot[k0];
    m->ref_slots[r * kMaxShare + 1] = k1 - k0 == 2 ? m->shp_slot[k0 + 1] : -(k1 - k0);
  }

  // ---- point location grid (bucket by cell bounding boxes)
  for (int r = 0; r < dim; ++r) {
    m->lo[r] = 1e300;
    m->hi[r] = -1e300;
  }
  for (int64_t v = 0; v < nv; ++v)
    for (int r = 0; r < dim; ++r) {
      m->lo[r] = std::min(m->lo[r], coords[v * dim + r]);
      m->hi[r] = std::max(m->hi[r], coords[v * dim + r]);
    }
  {
    double vol = 1;
    for (int r = 0; r < dim; ++r) vol *= std::max(m->hi[r] - m->lo[r], 1e-300);
    const double cell_size = std::pow(vol / std::max<int64_t>(1, ne / 2), 1.0 / dim);
    int64_t nb = 1;
    for (int r = 0; r < dim; ++r) {
      m->grid_n[r] = (int)std::max(1.0, std::min(4096.0, std::ceil((m->hi[r] - m->lo[r]) / cell_size)));
      nb *= m->grid_n[r];
    }
    auto bucket_range = [&](int64_t i, int* b0, int* b1) {
      for (int r = 0; r < dim; ++r) {
        double mn = 1e300, mx = -1e300;
        for (int v = 0; v < nvc; ++v) {
          const int64_t c = order[i];
          const double x = coords[(int64_t)cells[c * nvc + v] * dim + r];
          mn = std::min(mn, x);
          mx = std::max(mx, x);
        }
        const double w = (m->hi[r] - m->lo[r]) / m->grid_n[r];
        b0[r] = std::max(0, std::min(m->grid_n[r] - 1, (int)std::floor((mn - m->lo[r]) / w - 1e-9)));
        b1[r] = std::max(0, std::min(m->grid_n[r] - 1, (int)std::floor((mx - m->lo[r]) / w + 1e-9)));
      }
      for (int r = dim; r < 3; ++r) b0[r] = b1[r] = 0;
    };
    m->grid_ptr.assign(nb + 1, 0);
    for (int pass = 0; pass < 2; ++pass) {
      std::vector<int64_t> fill;
      if (pass == 1) {
        for (int64_t b = 0; b < nb; ++b) m->grid_ptr[b + 1] += m->grid_ptr[b];
        m->grid_cells.assign(m->grid_ptr[nb], 0);
        fill.assign(m->grid_ptr.begin(), m->grid_ptr.end() - 1);
      }
      for (int64_t i = 0; i < ne; ++i) {
        int b0[3], b1[3];
        bucket_range(i, b0, b1);
        for (int x = b0[0]; x <= b1[0]; ++x)
          for (int y = b0[1]; y <= b1[1]; ++y)
            for (int z = b0[2]; z <= b1[2]; ++z) {
              const int64_t b = ((int64_t)x * m->grid_n[1] + y) * m->grid_n[2] + z;
              if (pass == 0)
                m->grid_ptr[b + 1]++;
              else
                m->grid_cells[fill[b]++] = i;
            }
      }
    }
  }
  return m.release();
}

bool Mesh::locate(const double* x, PointLoc& out) const {
  const double tol = 1e-12;
  int b[3] = {0, 0, 0};
  for (int r = 0; r < dim; ++r) {
    const double w = (hi[r] - lo[r]) / grid_n[r];
    const double f = (x[r] - lo[r]) / w;
    if (f < -1e-9 || f > grid_n[r] + 1e-9) return false;
    b[r] = std::max(0, std::min(grid_n[r] - 1, (int)std::floor(f)));
  }
  const int64_t bi = ((int64_t)b[0] * grid_n[1] + b[1]) * grid_n[2] + b[2];
  int64_t best = -1, best_in = -1;
  double best_xi[3] = {0, 0, 0};
  const int dd = dim * dim;
  for (int64_t k = grid_ptr[bi]; k < grid_ptr[bi + 1]; ++k) {
    const int64_t i = grid_cells[k];
    double xi[3] = {0, 0, 0}, s = 0;
    for (int r = 0; r < dim; ++r) {
      for (int j = 0; j < dim; ++j) xi[r] += jinv[i * dd + r * dim + j] * (x[j] - x0[i * dim + j]);
      s += xi[r];
    }
    bool inside = 1.0 - s >= -tol;
    for (int r = 0; r < dim; ++r) inside = inside && xi[r] >= -tol;
    if (inside && (best < 0 || cell_input[i] < best_in)) {
      best = i;
      best_in = cell_input[i];
      for (int r = 0; r < 3; ++r) best_xi[r] = xi[r];
    }
  }
  if (best < 0) return false;
  out.cell = best;
  out.phi.assign(nd, 0.0);
  el->eval(best_xi, out.phi.data());
  return true;
}

double gershgorin_rho(const Mesh& m, const double* c) {
  const int nd = m.nd, dim = m.dim, ng = m.ng;
  const int64_t ne = m.n_cells, N = m.n_dofs;
  const Element& el = *m.el;
  // DOF -> (cell, local node) incidence
  std::vector<int64_t> ptr(N + 1, 0), inc;
  for (int64_t i = 0; i < ne * nd; ++i) ptr[m.cell_dofs[i] + 1]++;
  for (int64_t g = 0; g < N; ++g) ptr[g + 1] += ptr[g];
  inc.resize(ne * nd);
  {
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < ne * nd; ++i) inc[fill[m.cell_dofs[i]]++] = i;
  }
  std::vector<double> acc(N, 0.0);
  std::vector<int64_t> cols;
  double rho = 0;
  std::vector<double> row(nd);
  for (int64_t g = 0; g < N; ++g) {
    cols.clear();
    for (int64_t k = ptr[g]; k < ptr[g + 1]; ++k) {
      const int64_t e = inc[k] / nd;
      const int a = (int)(inc[k] % nd);
      const double* G = &m.geom[e * ng];
      std::fill(row.begin(), row.end(), 0.0);
      for (int q = 0; q < nd; ++q) {
        const double c2 = c[m.cell_dofs[e * nd + q]] * c[m.cell_dofs[e * nd + q]];
        const double* da = &el.grads[((size_t)q * nd + a) * dim];
        double v[3];
        if (dim == 2) {
          v[0] = G[0] * da[0] + G[1] * da[1];
          v[1] = G[1] * da[0] + G[2] * da[1];
        } else {
          v[0] = G[0] * da[0] + G[1] * da[1] + G[2] * da[2];
          v[1] = G[1] * da[0] + G[3] * da[1] + G[4] * da[2];
          v[2] = G[2] * da[0] + G[4] * da[1] + G[5] * da[2];
        }
        const double s = el.weights[q] * c2;
        for (int b = 0; b < nd; ++b) {
          const double* db = &el.grads[((size_t)q * nd + b) * dim];
          double t = 0;
          for (int r = 0; r < dim; ++r) t += v[r] * db[r];
          row[b] += s * t;
        }
      }
      for (int b = 0; b < nd; ++b) {
        const int64_t h = m.cell_dofs[e * nd + b];
        if (acc[h] == 0.0) cols.push_back(h);
        acc[h] += row[b];
        if (acc[h] == 0.0) acc[h] = 1e-300;  // keep it listed
      }
    }
    double s = 0;
    for (int64_t h : cols) {
      s += std::fabs(acc[h]);
      acc[h] = 0.0;
    }
    rho = std::max(rho, s / m.mass[g]);
  }
  return rho;
}

bool validate_mesh(const Mesh& m, std::string& why) {
  const int nd = m.nd;
  const int64_t ne = m.n_cells, N = m.n_dofs;
  for (int64_t g = 0; g < N; ++g)
    if (!(m.mass[g] > 0)) {
      why = "non-positive lumped mass at DOF " + std::to_string(g);
      return false;
    }
  std::vector<int64_t> stamp(N, -1), lastp(N, -1), npatch(N, 0);
  int64_t st = 0;
  for (int64_t p = 0; p < m.n_patches; ++p) {
    const int32_t c0 = m.patch_cell_start[p], c1 = m.patch_cell_start[p + 1];
    const int32_t own0 = m.patch_own_start[p], nown = m.patch_own_start[p + 1] - own0;
    const int32_t sh0 = m.patch_sh_start[p], nsh = m.patch_sh_start[p + 1] - sh0;
    const int32_t* cs = &m.colour_start[p * (kMaxColours + 1)];
    const int ncol = m.patch_ncol[p];
    if (cs[0] != c0 || cs[ncol] != c1) {
      why = "colour ranges do not cover patch " + std::to_string(p);
      return false;
    }
    for (int c = 0; c < ncol; ++c) {
      if (cs[c] > cs[c + 1]) {
        why = "colour ranges out of order";
        return false;
      }
      ++st;
      for (int32_t e = cs[c]; e < cs[c + 1]; ++e)
        for (int a = 0; a < nd; ++a) {
          const int64_t g = m.cell_dofs[e * nd + a];
          if (stamp[g] == st) {
            why = "two cells of colour " + std::to_string(c) + " in patch " + std::to_string(p) +
                  " share DOF " + std::to_string(g);
            return false;
          }
          stamp[g] = st;
        }
    }
    for (int32_t e = c0; e < c1; ++e)
      for (int a = 0; a < nd; ++a) {
        const int64_t g = m.cell_dofs[e * nd + a];
        const int loc = m.lmap[(size_t)a * ne + e];
        if (loc < nown) {
          if (g != own0 + loc) {
            why = "owned local index does not match the DOF map";
            return false;
          }
        } else if (loc - nown >= nsh || m.sh_idx[sh0 + loc - nown] != g) {
          why = "shared local index does not match the DOF map";
          return false;
        }
        if (lastp[g] != p) {
          lastp[g] = p;
          npatch[g]++;
        }
      }
  }
  for (int64_t g = 0; g < m.n_own_total; ++g)
    if (npatch[g] != 1) {
      why = "owned DOF " + std::to_string(g) + " touched by " + std::to_string(npatch[g]) + " patches";
      return false;
    }
  for (int64_t s = 0; s < m.n_shared; ++s) {
    const int64_t g = m.n_own_total + s;
    const int32_t k0 = m.shp_ptr[s], k1 = m.shp_ptr[s + 1];
    if (npatch[g] < 2 || k1 - k0 != npatch[g]) {
      why = "shared DOF " + std::to_string(g) + " has a wrong partial list";
      return false;
    }
    for (int32_t k = k0; k < k1; ++k) {
      if (m.sh_idx[m.shp_slot[k]] != g || (k > k0 && m.shp_slot[k] <= m.shp_slot[k - 1])) {
        why = "partial slots of shared DOF " + std::to_string(g) + " are wrong or unordered";
        return false;
      }
    }
  }
  // gather lists: per patch a permutation of the cell-node slots, grouped by DOF
  for (int64_t p = 0; p < m.n_patches; ++p) {
    const int32_t c0 = m.patch_cell_start[p], c1 = m.patch_cell_start[p + 1];
    const int32_t nloc = (m.patch_own_start[p + 1] - m.patch_own_start[p]) +
                         (m.patch_sh_start[p + 1] - m.patch_sh_start[p]);
    const uint16_t* gp = &m.gl_ptr[m.gl_ptr_off[p]];
    const uint16_t* ge = &m.gl_ent[m.gl_ent_off[p]];
    const int nslot = (c1 - c0) * nd;
    if (m.gl_ptr_off[p] % 8 || m.gl_ent_off[p] % 8 || m.gl_ptr_off[p + 1] - m.gl_ptr_off[p] < nloc + 1 ||
        m.gl_ent_off[p + 1] - m.gl_ent_off[p] < nslot || gp[0] != 0 || gp[nloc] != nslot) {
      why = "gather list of patch " + std::to_string(p) + " does not cover its cells";
      return false;
    }
    std::vector<char> seen(nslot, 0);
    for (int32_t i = 0; i < nloc; ++i)
      for (int k = gp[i]; k < gp[i + 1]; ++k) {
        const int slot = ge[k];
        const int e = c0 + slot / nd, a = slot % nd;
        if (slot >= nslot || seen[slot] || m.lmap[(size_t)a * ne + e] != i || (k > gp[i] && slot <= ge[k - 1])) {
          why = "gather list of patch " + std::to_string(p) + " is not the inverse of the local map";
          return false;
        }
        seen[slot] = 1;
      }
  }
  // inline slot lists of every shared ref agree with the CSR lists
  for (int64_t r = 0; r < m.n_shared_refs; ++r) {
    const int64_t s = m.sh_idx[r] - m.n_own_total;
    const int32_t k0 = m.shp_ptr[s], k1 = m.shp_ptr[s + 1];
    const int32_t* rs = &m.ref_slots[r * kMaxShare];
    const bool ok = rs[0] == m.shp_slot[k0] && rs[1] == (k1 - k0 == 2 ? m.shp_slot[k0 + 1] : -(k1 - k0));
    if (!ok) {
      why = "inline partial slots of shared ref " + std::to_string(r) + " disagree with the CSR list";
      return false;
    }
  }
  return true;
}

}  // namespace kmv
