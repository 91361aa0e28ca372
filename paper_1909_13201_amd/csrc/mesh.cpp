// Nested structured hierarchy: element/node/vertex numbering, node types,
// the J2 unknown layout and Dirichlet data (paper Section 3.3: levels are
// midpoint refinements of a conforming coarse mesh with the same
// fluid/solid split; Section 3.1: interface test functions belong to the
// solid-side equations K and S).
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "host.hpp"

namespace fsgmg {

static int64_t lin(const int* ix, const int* n, int D) {
  int64_t out = 0, stride = 1;
  for (int a = 0; a < D; ++a) {
    out += (int64_t)ix[a] * stride;
    stride *= n[a];
  }
  return out;
}

static const int kThree[kMaxDim] = {3, 3, 3};
static const int kTwo[kMaxDim] = {2, 2, 2};

static void unlin(int64_t k, const int* n, int D, int* ix) {
  for (int a = 0; a < D; ++a) {
    ix[a] = (int)(k % n[a]);
    k /= n[a];
  }
}

int64_t Level::node_index(const int* ix) const { return lin(ix, nn, D); }

void Level::node_ijk(int64_t n, int* ix) const { unlin(n, nn, D, ix); }

int64_t Level::vertex_node(int64_t v) const {
  int ix[kMaxDim];
  unlin(v, nv, D, ix);
  for (int a = 0; a < D; ++a) ix[a] *= 2;
  return lin(ix, nn, D);
}

// reference coordinates of the Q2 node lines of level l: the coarse
// breakpoints with midpoints inserted l+1 times
static std::vector<double> node_lines(const double* b, int nc, int l) {
  std::vector<double> cur(b, b + nc + 1);
  for (int t = 0; t < l + 1; ++t) {
    std::vector<double> nxt(2 * cur.size() - 1);
    for (size_t i = 0; i < cur.size(); ++i) nxt[2 * i] = cur[i];
    for (size_t i = 0; i + 1 < cur.size(); ++i) nxt[2 * i + 1] = 0.5 * (cur[i] + cur[i + 1]);
    cur.swap(nxt);
  }
  return cur;
}

static void map_point(const fsgmg_mesh_desc& m, const double* xr, double* x) {
  for (int a = 0; a < m.dim; ++a) x[a] = xr[a];
  if (m.mapping == 0) return;
  if (m.mapping == 1) {
    const double xc = m.map_params[0], R = m.map_params[1];
    const double ya = m.map_params[2], yb = m.map_params[3];
    const double dx = xr[0] - xc;
    const double bump = std::sqrt(std::max(R * R - dx * dx, 0.0));
    double s = (xr[1] - ya) / (yb - ya);
    s = std::min(1.0, std::max(0.0, s));
    x[1] = xr[1] + bump * s;
    return;
  }
  if (m.mapping == 2) {
    // smooth bulge R cos^2(pi dx / (2R)), tangent to the straight wall at
    // |dx| = R (bounded element shear under refinement)
    const double xc = m.map_params[0], R = m.map_params[1];
    const double ya = m.map_params[2], yb = m.map_params[3];
    const double dx = xr[0] - xc;
    const double c = std::cos(M_PI * dx / (2.0 * R));
    const double bump = std::fabs(dx) < R ? R * c * c : 0.0;
    double s = (xr[1] - ya) / (yb - ya);
    s = std::min(1.0, std::max(0.0, s));
    x[1] = xr[1] + bump * s;
    return;
  }
  if (m.mapping == 3) {
    // square cross-section [0,1]^2 onto the disc of centre (cx, cy) and
    // radius R (x' = a sqrt(1 - b^2 / 2), y' = b sqrt(1 - a^2 / 2) with
    // a, b in [-1, 1]: the square's edges land on the circle); z unchanged
    const double cx = m.map_params[0], cy = m.map_params[1], R = m.map_params[2];
    const double a = 2.0 * xr[0] - 1.0, b = 2.0 * xr[1] - 1.0;
    x[0] = cx + R * a * std::sqrt(1.0 - 0.5 * b * b);
    x[1] = cy + R * b * std::sqrt(1.0 - 0.5 * a * a);
    return;
  }
  throw std::invalid_argument("unknown mapping");
}

void build_level(const fsgmg_mesh_desc& m, int l, Level& lv) {
  const int D = m.dim;
  lv.D = D;
  lv.l = l;
  lv.nE = lv.N2 = lv.NV = 1;
  lv.nb = lv.npv = 1;
  for (int a = 0; a < kMaxDim; ++a) {
    lv.ne[a] = lv.nn[a] = lv.nv[a] = 1;
  }
  for (int a = 0; a < D; ++a) {
    lv.ne[a] = m.nc[a] << l;
    lv.nn[a] = 2 * lv.ne[a] + 1;
    lv.nv[a] = lv.ne[a] + 1;
    lv.nE *= lv.ne[a];
    lv.N2 *= lv.nn[a];
    lv.NV *= lv.nv[a];
    lv.nb *= 3;
    lv.npv *= 2;
  }
  const int nb = lv.nb, npv = lv.npv;
  lv.region.resize(lv.nE);
  lv.parent0.resize(lv.nE);
  lv.elem_nodes.resize(lv.nE * nb);
  lv.elem_verts.resize(lv.nE * npv);
  for (int64_t e = 0; e < lv.nE; ++e) {
    int ex[kMaxDim], px[kMaxDim];
    unlin(e, lv.ne, D, ex);
    for (int a = 0; a < D; ++a) px[a] = ex[a] >> l;
    const int64_t p = lin(px, m.nc, D);
    lv.parent0[e] = (int32_t)p;
    lv.region[e] = m.region[p];
    for (int k = 0; k < nb; ++k) {
      int ix[kMaxDim], loc[kMaxDim];
      unlin(k, kThree, D, loc);
      for (int a = 0; a < D; ++a) ix[a] = 2 * ex[a] + loc[a];
      lv.elem_nodes[e * nb + k] = lin(ix, lv.nn, D);
    }
    for (int k = 0; k < npv; ++k) {
      int ix[kMaxDim], loc[kMaxDim];
      unlin(k, kTwo, D, loc);
      for (int a = 0; a < D; ++a) ix[a] = ex[a] + loc[a];
      lv.elem_verts[e * npv + k] = lin(ix, lv.nv, D);
    }
  }

  std::vector<double> lines[kMaxDim];
  for (int a = 0; a < D; ++a) lines[a] = node_lines(m.breaks[a], m.nc[a], l);
  lv.xref.resize(lv.N2 * D);
  lv.X.resize(lv.N2 * D);
  for (int64_t n = 0; n < lv.N2; ++n) {
    int ix[kMaxDim];
    unlin(n, lv.nn, D, ix);
    for (int a = 0; a < D; ++a) lv.xref[n * D + a] = lines[a][ix[a]];
    map_point(m, &lv.xref[n * D], &lv.X[n * D]);
  }

  lv.solid_side.assign(lv.N2, 0);
  lv.fluid_touch.assign(lv.N2, 0);
  lv.vert_solid.assign(lv.NV, 0);
  lv.vert_fluid.assign(lv.NV, 0);
  for (int64_t e = 0; e < lv.nE; ++e) {
    const bool solid = lv.region[e] == 1;
    for (int k = 0; k < nb; ++k) (solid ? lv.solid_side : lv.fluid_touch)[lv.elem_nodes[e * nb + k]] = 1;
    for (int k = 0; k < npv; ++k) (solid ? lv.vert_solid : lv.vert_fluid)[lv.elem_verts[e * npv + k]] = 1;
  }

  lv.Nps = lv.Npf = 0;
  lv.ps_of_vert.assign(lv.NV, -1);
  lv.pf_of_vert.assign(lv.NV, -1);
  lv.off_ps = (int64_t)D * lv.N2;
  for (int64_t v = 0; v < lv.NV; ++v)
    if (lv.vert_solid[v]) lv.ps_of_vert[v] = lv.off_ps + lv.Nps++;
  lv.off_u = lv.off_ps + lv.Nps;
  lv.off_pf = lv.off_u + (int64_t)D * lv.N2;
  for (int64_t v = 0; v < lv.NV; ++v)
    if (lv.vert_fluid[v]) lv.pf_of_vert[v] = lv.off_pf + lv.Npf++;
  lv.N = lv.off_pf + lv.Npf;

  // Dirichlet data: a tag bc[face][region] holds on every node of the face
  // that belongs to an element of that region.
  lv.dir.assign(lv.N, 0);
  lv.dir_val.assign(lv.N, 0.0);
  std::vector<uint8_t> wall(lv.N2, 0), inflow(lv.N2, 0);
  std::vector<double> inflow_val(lv.N2 * D, 0.0);
  for (int f = 0; f < 2 * D; ++f) {
    const int a = f / 2, side = f % 2;
    const int target = side == 0 ? 0 : lv.nn[a] - 1;
    bool any_inflow = false;
    std::vector<int64_t> on_face;
    for (int64_t n = 0; n < lv.N2; ++n) {
      int ix[kMaxDim];
      unlin(n, lv.nn, D, ix);
      if (ix[a] == target) on_face.push_back(n);
    }
    for (int64_t n : on_face) {
      const uint8_t touch[2] = {lv.fluid_touch[n], lv.solid_side[n]};
      bool dmask = false, wmask = false, imask = false;
      for (int r = 0; r < 2; ++r) {
        if (!touch[r]) continue;
        dmask |= m.bc_d[f][r] == 1;
        wmask |= m.bc_u[f][r] == 1;
        imask |= m.bc_u[f][r] == 2;
      }
      if (dmask)
        for (int c = 0; c < D; ++c) lv.dir[D * n + c] = 1;
      if (wmask) wall[n] = 1;
      if (imask) any_inflow = true;
    }
    if (!any_inflow) continue;
    double lo[kMaxDim], hi[kMaxDim];
    for (int b = 0; b < D; ++b) {
      lo[b] = 1e300;
      hi[b] = -1e300;
    }
    for (int64_t n : on_face) {
      if (!lv.fluid_touch[n]) continue;
      for (int b = 0; b < D; ++b) {
        lo[b] = std::min(lo[b], lv.xref[n * D + b]);
        hi[b] = std::max(hi[b], lv.xref[n * D + b]);
      }
    }
    for (int64_t n : on_face) {
      const uint8_t touch[2] = {lv.fluid_touch[n], lv.solid_side[n]};
      bool imask = false;
      for (int r = 0; r < 2; ++r) imask |= touch[r] && m.bc_u[f][r] == 2;
      if (!imask) continue;
      double prof = 1.0;
      for (int b = 0; b < D; ++b) {
        if (b == a) continue;
        const double s = (lv.xref[n * D + b] - lo[b]) / (hi[b] - lo[b]);
        prof *= 4.0 * s * (1.0 - s);
      }
      inflow_val[n * D + a] = (side == 0 ? 1.0 : -1.0) * m.inflow_peak * prof;
      inflow[n] = 1;
    }
  }
  for (int64_t n = 0; n < lv.N2; ++n) {
    if (!(wall[n] || inflow[n])) continue;
    for (int c = 0; c < D; ++c) {
      const int64_t k = lv.off_u + D * n + c;
      lv.dir[k] = 1;
      lv.dir_val[k] = wall[n] ? 0.0 : inflow_val[n * D + c];
    }
  }
}

CsrHost csr_transpose(const CsrHost& A) {
  CsrHost T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.rowptr.assign(T.nrows + 1, 0);
  for (int64_t k = 0; k < A.nnz(); ++k) T.rowptr[A.col[k] + 1]++;
  for (int64_t i = 0; i < T.nrows; ++i) T.rowptr[i + 1] += T.rowptr[i];
  T.col.resize(A.nnz());
  T.val.resize(A.nnz());
  std::vector<int64_t> cur(T.rowptr.begin(), T.rowptr.end() - 1);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
      const int64_t p = cur[A.col[k]]++;
      T.col[p] = (int32_t)i;
      T.val[p] = A.val[k];
    }
  return T;
}

}  // namespace fsgmg
