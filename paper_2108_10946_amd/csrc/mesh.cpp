// Mesh preprocessing (host): topological DOF numbering, geometry, lumped mass,
// recursive-coordinate-bisection patches, the owned/shared DOF split, the
// interior-DOF layout and the patch-local gather words of the GPU kernels.
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
  // cells, DOFs and shared refs are indexed with 32-bit integers on the device
  if (ne >= (int64_t)1 << 31 || nv >= (int64_t)1 << 31) throw std::invalid_argument("more than 2^31 cells or vertices");
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
    // LDS holds the patch's non-interior DOFs (three float values each in the
    // adjoint, plus shared refs) and its cells' non-interior slots (two each): aim
    // at about 4096 such DOFs and 64 KiB of float LDS, at most 256 cells (4 waves)
    const double nonint_per_cell = dim == 2 ? 0.5 + 1.5 * el.n_edge
                                            : 1.0 / 6.0 + 7.0 / 6.0 * el.n_edge + 2.0 * el.n_face;
    const int nb_cell = el.n - el.n_cell;
    const double lds_per_cell = 4.0 * (3.0 * 1.2 * nonint_per_cell + 2.0 * nb_cell);
    int P = (int)std::min(4096.0 / (std::max(nonint_per_cell, 1.0) * 1.25), 65536.0 / lds_per_cell);
    P = (P / 64) * 64;
    patch_cells = std::max(64, std::min(256, P));
    // measured on the GPU: KMV4 triangles step about 4% faster with 224-cell
    // patches than with 256 (both directions); degrees 2, 3 are flat and 5 is
    // slower there
    if (dim == 2 && degree == 4) patch_cells = std::min(patch_cells, 224);
    // KMV3 tetrahedra: the estimate above gives 128, but with the slot arrays
    // overlaying the staging their float LDS is 49 / 77 KiB (forward / adjoint) at
    // 256 cells, the same waves per CU as at 128, and a quarter fewer shared refs:
    // measured 12% faster per misfit + gradient (the FP64 adjoint needs ~146 KiB)
    if (dim == 3 && degree == 3) patch_cells = 256;
  }
  m->patch_cells = patch_cells;
  std::vector<int64_t> order(ne);
  std::iota(order.begin(), order.end(), 0);
  std::vector<int64_t> leaf_start;
  rcb(order, 0, ne, cen, dim, patch_cells, leaf_start);
  leaf_start.push_back(ne);
  const int64_t np = (int64_t)leaf_start.size() - 1;
  m->n_patches = np;

  m->cell_input = order;
  for (int q = 0; q < nd; ++q) (el.entity[q] == ENT_CELL ? m->int_nodes : m->bnd_nodes).push_back(q);
  const int ni = (int)m->int_nodes.size(), nb = (int)m->bnd_nodes.size();
  m->ni = ni;
  m->nb = nb;

  // ---- owned / shared classification
  std::vector<int32_t> last(ndof, -1), npat(ndof, 0), ncell_of(ndof, 0);
  for (int64_t p = 0; p < np; ++p)
    for (int64_t i = leaf_start[p]; i < leaf_start[p + 1]; ++i) {
      const int64_t c = order[i];
      for (int q = 0; q < nd; ++q) {
        const int64_t g = cdof0[c * nd + q];
        ncell_of[g]++;
        if (last[g] != p) {
          last[g] = (int32_t)p;
          npat[g]++;
        }
      }
    }
  std::vector<int64_t> newid(ndof, -1);
  int64_t next = 0;
  m->patch_own_start.assign(np + 1, 0);
  for (int64_t p = 0; p < np; ++p) {
    m->patch_own_start[p] = (int32_t)next;
    const int64_t c0 = leaf_start[p], nc = leaf_start[p + 1] - c0;
    // interior DOFs: node j of the patch's t-th cell at next + j*nc + t
    for (int64_t t = 0; t < nc; ++t)
      for (int j = 0; j < ni; ++j) newid[cdof0[order[c0 + t] * nd + m->int_nodes[j]]] = next + j * nc + t;
    next += (int64_t)ni * nc;
    // the other owned DOFs: those with one or two cells first, then the rest,
    // each group in first-touch order
    for (int pass = 0; pass < 2; ++pass)
      for (int64_t t = 0; t < nc; ++t)
        for (int b = 0; b < nb; ++b) {
          const int64_t g = cdof0[order[c0 + t] * nd + m->bnd_nodes[b]];
          if (npat[g] == 1 && newid[g] < 0 && (ncell_of[g] > 2) == (pass == 1)) newid[g] = next++;
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

  // ---- patch-local maps of the non-interior DOFs and their gather words
  m->patch_cell_start.assign(leaf_start.begin(), leaf_start.end());
  m->patch_sh_start.assign(np + 1, 0);
  m->lmap.assign((size_t)nb * ne, 0);
  for (int64_t p = 0; p < np; ++p)
    m->max_patch_cells = std::max(m->max_patch_cells, (int)(leaf_start[p + 1] - leaf_start[p]));
  m->slot_stride = m->max_patch_cells;
  if ((int64_t)nb * m->slot_stride + 1 >= (int64_t)kListMark) {
    throw std::invalid_argument("patch too large for 16-bit cell-node slots");
  }
  const uint32_t zslot = (uint32_t)(nb * m->slot_stride);
  m->gword_off.assign(np + 1, 0);
  m->glist_off.assign(np + 1, 0);
  std::vector<int32_t> loc(ndof, -1), pc(ndof, 0);
  std::vector<int32_t> sh_list;
  for (int64_t p = 0; p < np; ++p) {
    m->patch_sh_start[p] = (int32_t)sh_list.size();
    const int32_t c0 = (int32_t)leaf_start[p], nc = (int32_t)(leaf_start[p + 1] - c0);
    const int32_t bo0 = m->patch_own_start[p] + ni * nc;
    const int32_t nbo = m->patch_own_start[p + 1] - bo0;
    // shared refs in first-touch order, those with one or two cells here first
    std::vector<int32_t> refs, touched;
    for (int32_t t = 0; t < nc; ++t)
      for (int b = 0; b < nb; ++b) {
        const int64_t g = m->cell_dofs[(int64_t)(c0 + t) * nd + m->bnd_nodes[b]];
        if (pc[g]++ == 0) {
          touched.push_back((int32_t)g);
          if (g >= m->n_own_total) refs.push_back((int32_t)g);
        }
      }
    std::stable_sort(refs.begin(), refs.end(), [&](int32_t x, int32_t y) { return (pc[x] > 2) < (pc[y] > 2); });
    for (int32_t g : touched) loc[g] = g < m->n_own_total ? g - bo0 : -1;
    for (size_t j = 0; j < refs.size(); ++j) {
      loc[refs[j]] = nbo + (int32_t)j;
      sh_list.push_back(refs[j]);
    }
    const int32_t nbl = nbo + (int32_t)refs.size();
    if (nbl > 65535) {
      throw std::invalid_argument("patch too large for 16-bit local indices");
    }
    m->max_nbl = std::max(m->max_nbl, (int)nbl);
    // slots of every local DOF in (cell, node) order
    std::vector<int32_t> cnt(nbl + 1, 0);
    for (int32_t t = 0; t < nc; ++t)
      for (int b = 0; b < nb; ++b) {
        const int64_t g = m->cell_dofs[(int64_t)(c0 + t) * nd + m->bnd_nodes[b]];
        const int32_t l = loc[g];
        if (l < 0 || l >= nbl) throw std::logic_error("local DOF index out of range");
        m->lmap[(size_t)b * ne + c0 + t] = (uint16_t)l;
        cnt[l + 1]++;
      }
    for (int32_t l = 0; l < nbl; ++l) cnt[l + 1] += cnt[l];
    std::vector<uint16_t> slots(cnt[nbl]);
    {
      std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
      for (int32_t t = 0; t < nc; ++t)
        for (int b = 0; b < nb; ++b) {
          const int32_t l = m->lmap[(size_t)b * ne + c0 + t];
          slots[fill[l]++] = (uint16_t)(b * m->slot_stride + t);
        }
    }
    const size_t list0 = m->glist.size();
    for (int32_t l = 0; l < nbl; ++l) {
      const int32_t k = cnt[l + 1] - cnt[l];
      if (k <= 0) throw std::logic_error("local DOF without a contributing cell");
      if (k <= 2) {
        const uint32_t s1 = k == 2 ? slots[cnt[l] + 1] : zslot;
        m->gword.push_back((uint32_t)slots[cnt[l]] | (s1 << 16));
      } else {
        const size_t off = m->glist.size() - list0;
        if (off > 0xFFFE || k > 0xFFFF) throw std::invalid_argument("patch gather list too long");
        m->gword.push_back((uint32_t)off | (kListMark << 16));
        m->glist.push_back((uint16_t)k);
        for (int32_t q = cnt[l]; q < cnt[l + 1]; ++q) m->glist.push_back(slots[q]);
      }
    }
    while (m->glist.size() % 8) m->glist.push_back(0);
    m->gword_off[p + 1] = (int32_t)m->gword.size();
    m->glist_off[p + 1] = (int32_t)m->glist.size();
    m->max_glist = std::max(m->max_glist, m->glist_off[p + 1] - m->glist_off[p]);
    for (int32_t g : touched) {
      pc[g] = 0;
      loc[g] = -1;
    }
  }
  if (sh_list.size() >= (size_t)1 << 31) {
    throw std::invalid_argument("more than 2^31 shared refs (use larger patches)");
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
  const int nd = m.nd, ni = m.ni, nb = m.nb;
  const int64_t ne = m.n_cells, N = m.n_dofs;
  for (int64_t g = 0; g < N; ++g)
    if (!(m.mass[g] > 0)) {
      why = "non-positive lumped mass at DOF " + std::to_string(g);
      return false;
    }
  if ((int)m.int_nodes.size() != ni || (int)m.bnd_nodes.size() != nb || ni + nb != nd) {
    why = "node classes do not cover the element";
    return false;
  }
  const int64_t cs = m.slot_stride, zslot = (int64_t)nb * cs;
  std::vector<int64_t> lastp(N, -1), npatch(N, 0);
  for (int64_t p = 0; p < m.n_patches; ++p) {
    const int32_t c0 = m.patch_cell_start[p], nc = m.patch_cell_start[p + 1] - c0;
    const int32_t own0 = m.patch_own_start[p], bo0 = own0 + ni * nc;
    const int32_t nbo = m.patch_own_start[p + 1] - bo0;
    const int32_t sh0 = m.patch_sh_start[p], nsh = m.patch_sh_start[p + 1] - sh0;
    const int32_t nbl = nbo + nsh;
    if (nc <= 0 || nc > cs || nbo < 0 || nbl > m.max_nbl || m.gword_off[p + 1] - m.gword_off[p] != nbl) {
      why = "patch " + std::to_string(p) + " has inconsistent ranges";
      return false;
    }
    for (int32_t t = 0; t < nc; ++t) {
      const int64_t e = c0 + t;
      for (int j = 0; j < ni; ++j)
        if (m.cell_dofs[e * nd + m.int_nodes[j]] != own0 + (int64_t)j * nc + t) {
          why = "interior DOF of cell " + std::to_string(e) + " is not at its implicit position";
          return false;
        }
      for (int b = 0; b < nb; ++b) {
        const int64_t g = m.cell_dofs[e * nd + m.bnd_nodes[b]];
        const int l = m.lmap[(size_t)b * ne + e];
        if (l < nbo) {
          if (g != bo0 + l) {
            why = "owned local index does not match the DOF map";
            return false;
          }
        } else if (l >= nbl || m.sh_idx[sh0 + l - nbo] != g) {
          why = "shared local index does not match the DOF map";
          return false;
        }
      }
      for (int a = 0; a < nd; ++a) {
        const int64_t g = m.cell_dofs[e * nd + a];
        if (lastp[g] != p) {
          lastp[g] = p;
          npatch[g]++;
        }
      }
    }
    // gather words: every cell-node slot of the patch exactly once, under its DOF
    std::vector<char> seen((size_t)zslot, 0);
    const uint32_t* gw = &m.gword[m.gword_off[p]];
    const uint16_t* gl = &m.glist[m.glist_off[p]];
    const int32_t gln = m.glist_off[p + 1] - m.glist_off[p];
    if (m.glist_off[p] % 8) {
      why = "gather list of patch " + std::to_string(p) + " is not 16-byte aligned";
      return false;
    }
    for (int32_t l = 0; l < nbl; ++l) {
      std::vector<int64_t> sl;
      const uint32_t lo = gw[l] & 0xFFFFu, hi = gw[l] >> 16;
      if (hi == kListMark) {
        if ((int32_t)lo >= gln || (int32_t)(lo + 1 + gl[lo]) > gln || gl[lo] < 3) {
          why = "gather list entry out of range";
          return false;
        }
        for (int k = 0; k < gl[lo]; ++k) sl.push_back(gl[lo + 1 + k]);
      } else {
        sl.push_back(lo);
        if (hi != zslot) sl.push_back(hi);
      }
      for (int64_t sv : sl) {
        const int64_t b = sv / cs, t = sv % cs;
        if (sv >= zslot || t >= nc || seen[sv] || m.lmap[(size_t)b * ne + c0 + t] != l) {
          why = "gather words of patch " + std::to_string(p) + " are not the inverse of the local map";
          return false;
        }
        seen[sv] = 1;
      }
    }
    for (int32_t t = 0; t < nc; ++t)
      for (int b = 0; b < nb; ++b)
        if (!seen[(size_t)b * cs + t]) {
          why = "a cell-node slot of patch " + std::to_string(p) + " is never gathered";
          return false;
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

namespace {
// n-point Gauss-Legendre rule on [0, 1] (Newton on the three-term recurrence).
void gauss01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double t = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = t;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (t * p1 - p0) / (t * t - 1);
      const double step = p1 / dp;
      t -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[i] = 0.5 * (1 - t);
    w[i] = 1.0 / ((1 - t * t) * dp * dp);  // (2 / ((1-t^2) P_n'^2)) / 2
  }
}
}  // namespace

void boundary_weights(const Mesh& m, std::vector<int32_t>& dofs, std::vector<double>& b) {
  const int dim = m.dim, nv = dim + 1, nd = m.nd, dd = dim * dim;
  // every facet of every cell, as (sorted vertex ids, internal cell, local vertex left out)
  struct F {
    std::array<int32_t, 3> v;
    int64_t cell;
    int skip;
  };
  std::vector<F> fs;
  fs.reserve((size_t)m.n_cells * nv);
  for (int64_t e = 0; e < m.n_cells; ++e) {
    const int32_t* cv = &m.cells_in[(size_t)m.cell_input[e] * nv];
    for (int s = 0; s < nv; ++s) {
      F f{{-1, -1, -1}, e, s};
      int k = 0;
      for (int a = 0; a < nv; ++a)
        if (a != s) f.v[k++] = cv[a];
      std::sort(f.v.begin(), f.v.begin() + dim);
      fs.push_back(f);
    }
  }
  std::sort(fs.begin(), fs.end(), [](const F& a, const F& c) { return a.v < c.v; });
  // facet quadrature: points as barycentric weights of the facet's vertices, weights
  // summing to 1 (times the facet measure below)
  std::vector<double> gx, gw;
  gauss01(8, gx, gw);
  std::vector<std::array<double, 3>> qb;
  std::vector<double> qw;
  if (dim == 2) {
    for (int i = 0; i < 8; ++i) {
      qb.push_back({gx[i], 1 - gx[i], 0});
      qw.push_back(gw[i]);
    }
  } else {  // triangle: t in (0,1) toward vertex 2, the remaining edge (1-t) split by s
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) {
        const double t = gx[i], s = gx[j];
        qb.push_back({(1 - t) * (1 - s), (1 - t) * s, t});
        qw.push_back(2 * gw[i] * gw[j] * (1 - t));
      }
  }
  std::vector<double> acc(m.n_dofs, 0.0), phi(nd);
  for (size_t i = 0; i < fs.size();) {
    size_t j = i + 1;
    while (j < fs.size() && fs[j].v == fs[i].v) ++j;
    if (j - i == 1) {
      const F& f = fs[i];
      const double* X[3];
      for (int a = 0; a < dim; ++a) X[a] = &m.coords[(size_t)f.v[a] * dim];
      double meas;
      if (dim == 2) {
        meas = std::hypot(X[1][0] - X[0][0], X[1][1] - X[0][1]);
      } else {
        double u[3], v[3];
        for (int r = 0; r < 3; ++r) {
          u[r] = X[1][r] - X[0][r];
          v[r] = X[2][r] - X[0][r];
        }
        meas = 0.5 * std::sqrt(std::pow(u[1] * v[2] - u[2] * v[1], 2) + std::pow(u[2] * v[0] - u[0] * v[2], 2) +
                               std::pow(u[0] * v[1] - u[1] * v[0], 2));
      }
      const int64_t e = f.cell;
      for (size_t q = 0; q < qw.size(); ++q) {
        double x[3] = {0, 0, 0}, xi[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a)
          for (int r = 0; r < dim; ++r) x[r] += qb[q][a] * X[a][r];
        for (int r = 0; r < dim; ++r)
          for (int c = 0; c < dim; ++c) xi[r] += m.jinv[e * dd + r * dim + c] * (x[c] - m.x0[e * dim + c]);
        m.el->eval(xi, phi.data());
        for (int a = 0; a < nd; ++a) acc[m.cell_dofs[e * nd + a]] += meas * qw[q] * phi[a];
      }
    }
    i = j;
  }
  // keep the DOFs on the boundary (the traces of the other nodes' basis functions
  // vanish there, up to rounding)
  double bmax = 0;
  for (double v : acc) bmax = std::max(bmax, std::fabs(v));
  dofs.clear();
  b.clear();
  for (int64_t i = 0; i < m.n_dofs; ++i)
    if (std::fabs(acc[i]) > 1e-9 * bmax) {
      dofs.push_back((int32_t)i);
      b.push_back(acc[i]);
    }
}

void boundary_of(const Mesh& m, const std::vector<int32_t>** dofs, const std::vector<double>** b) {
  std::call_once(m.bnd_once, [&m]() { boundary_weights(m, m.bnd_dof, m.bnd_b); });
  *dofs = &m.bnd_dof;
  *b = &m.bnd_b;
}

}  // namespace kmv
