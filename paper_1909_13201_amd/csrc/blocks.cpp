// Field-split additive Schwarz block index sets (paper Section 3.2).
//
// The level is split into the fields [d, p^s] and [u, p^f] (eq. FS).  Each
// region is tiled by non-overlapping element-aligned cores of core[] elements.
// Vanka rule: a block takes the pressures whose support meets the core (the
// Q1 vertices of the core's elements) and the displacements / velocities
// whose support meets the support of those pressures: the Q2 nodes of the
// core's elements grown by `halo` element layers of the same region.
//   field d, solid core: d of those nodes + p^s      ([S_ds S_ps; V_ds 0])
//   field d, fluid core: d of fluid nodes only        ([A_df], overlapping DD)
//   field u, fluid core: u of fluid nodes + p^f       ([F_uf F_pf; W_uf 0])
//   u^s: Jacobi on the lumped mass (no block).
// Dirichlet unknowns belong to no block.  Order: field d then field u, tiles
// x-fastest, solid before fluid within a tile.  owner(i) = last block that
// contains i (the additive update takes entry i from the last block).
//
// Enlarged interface cores (iface_mult = m > 1, layered walls): per region, a
// tile row whose region elements touch another region across a face normal
// to axis 1 takes over the next m - 1 tile rows on the side away from the
// interface (never a row that touches an interface itself; a row touching
// interfaces on both sides keeps its size).  The enlarged core is emitted in
// the place of the interface tile; the rows taken over emit nothing.
//
// Monolithic comparator (the AS formula of Section 3.2, P^s_1j and P^f_1j):
// no field split; one block per core and region with the displacements,
// velocities and pressures of that region (same selection rule), so u^s and
// the kinematic rows K sit in the solid blocks and only Dirichlet unknowns
// stay outside every block.
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "host.hpp"

namespace fsgmg {

namespace {

// first / last tile row (axis 1) of the core of each tile row, {-1, -1} for
// rows taken over by an enlarged interface core
std::vector<std::pair<int, int>> row_groups(const Level& lv, const int* core, int region,
                                            int mult) {
  const int ny = lv.ne[1];
  const int nt1 = (ny + core[1] - 1) / core[1];
  std::vector<std::pair<int, int>> g(nt1);
  for (int t = 0; t < nt1; ++t) g[t] = {t, t};
  if (mult <= 1) return g;
  // region of each element row (must not vary along x, or z in 3D)
  std::vector<int8_t> rr(ny, -1);
  for (int64_t e = 0; e < lv.nE; ++e) {
    const int y = (int)((e / lv.ne[0]) % ny);
    if (rr[y] < 0)
      rr[y] = lv.region[e];
    else if (rr[y] != lv.region[e])
      throw std::invalid_argument("enlarged interface cores need regions constant along x (and z)");
  }
  struct Flags { bool has, below, above; };
  std::vector<Flags> fl(nt1);
  for (int t = 0; t < nt1; ++t) {
    Flags f{false, false, false};
    for (int y = t * core[1]; y < std::min((t + 1) * core[1], ny); ++y) {
      if (rr[y] != region) continue;
      f.has = true;
      if (y > 0 && rr[y - 1] != region) f.below = true;
      if (y + 1 < ny && rr[y + 1] != region) f.above = true;
    }
    fl[t] = f;
  }
  std::vector<char> taken(nt1, 0);
  for (int t = 0; t < nt1; ++t) {
    if (!fl[t].has || fl[t].below == fl[t].above || taken[t]) continue;
    const int step = fl[t].below ? 1 : -1;
    int lo = t, hi = t;
    for (int k = 1; k < mult; ++k) {
      const int u = t + step * k;
      if (u < 0 || u >= nt1 || taken[u] || !fl[u].has || fl[u].below || fl[u].above) break;
      taken[u] = 1;
      g[u] = {-1, -1};
      lo = std::min(lo, u);
      hi = std::max(hi, u);
    }
    g[t] = {lo, hi};
  }
  return g;
}

}  // namespace

void build_blocks(const Level& lv, const int* core, int halo, int iface_mult, bool monolithic,
                  BlockSet& bs) {
  const int D = lv.D;
  int nt[kMaxDim] = {1, 1, 1};
  int64_t ntiles = 1;
  for (int a = 0; a < D; ++a) {
    if (core[a] < 1) throw std::invalid_argument("core size must be >= 1");
    nt[a] = (lv.ne[a] + core[a] - 1) / core[a];
    ntiles *= nt[a];
  }
  const std::vector<std::pair<int, int>> groups[2] = {row_groups(lv, core, 0, iface_mult),
                                                      row_groups(lv, core, 1, iface_mult)};
  bs.ptr.assign(1, 0);
  bs.dofs.clear();
  bs.colour_ptr.clear();
  std::vector<int32_t> stamp_el(lv.nE, -1), stamp_node(lv.N2, -1), stamp_vert(lv.NV, -1);
  int32_t stamp = 0;
  std::vector<int64_t> core_el, blk_el, dofs;
  // passes: field 0 = [d, p^s] (solid, then fluid cores), field 1 = [u, p^f]
  // (fluid cores); monolithic: field 2 = [d, u, p] (solid, then fluid)
  const int fields[2] = {monolithic ? 2 : 0, 1};
  for (int fi = 0; fi < (monolithic ? 1 : 2); ++fi) {
    const int field = fields[fi];
    for (int64_t t = 0; t < ntiles; ++t) {
      int tx[kMaxDim] = {0, 0, 0};
      int64_t tt = t;
      for (int a = 0; a < D; ++a) {
        tx[a] = (int)(tt % nt[a]);
        tt /= nt[a];
      }
      const int regions[2] = {1, 0};
      for (int ri = (field == 1 ? 1 : 0); ri < 2; ++ri) {
        const int region = regions[ri];
        const std::pair<int, int> g = groups[region][tx[1]];
        if (g.first < 0) continue;
        core_el.clear();
        int lo[kMaxDim] = {0, 0, 0}, hi[kMaxDim] = {1, 1, 1};
        for (int a = 0; a < D; ++a) {
          lo[a] = tx[a] * core[a];
          hi[a] = std::min(lo[a] + core[a], lv.ne[a]);
        }
        lo[1] = g.first * core[1];
        hi[1] = std::min((g.second + 1) * core[1], lv.ne[1]);
        for (int z = lo[2]; z < (D > 2 ? hi[2] : 1); ++z)
          for (int y = lo[1]; y < hi[1]; ++y)
            for (int x = lo[0]; x < hi[0]; ++x) {
              const int64_t e = x + (int64_t)lv.ne[0] * (y + (int64_t)lv.ne[1] * z);
              if (lv.region[e] == region) core_el.push_back(e);
            }
        if (core_el.empty()) continue;
        ++stamp;
        blk_el.clear();
        for (int64_t e : core_el) {
          int ex[kMaxDim] = {0, 0, 0};
          int64_t r = e;
          for (int a = 0; a < D; ++a) {
            ex[a] = (int)(r % lv.ne[a]);
            r /= lv.ne[a];
          }
          const int hz = D > 2 ? halo : 0;
          for (int dz = -hz; dz <= hz; ++dz)
            for (int dy = -halo; dy <= halo; ++dy)
              for (int dx = -halo; dx <= halo; ++dx) {
                const int q[3] = {ex[0] + dx, ex[1] + dy, D > 2 ? ex[2] + dz : 0};
                bool ok = true;
                for (int a = 0; a < D; ++a) ok &= q[a] >= 0 && q[a] < lv.ne[a];
                if (!ok) continue;
                const int64_t n = q[0] + (int64_t)lv.ne[0] * (q[1] + (int64_t)lv.ne[1] * q[2]);
                if (lv.region[n] != region || stamp_el[n] == stamp) continue;
                stamp_el[n] = stamp;
                blk_el.push_back(n);
              }
        }
        dofs.clear();
        for (int64_t e : blk_el)
          for (int k = 0; k < lv.nb; ++k) {
            const int64_t n = lv.elem_nodes[e * lv.nb + k];
            if (stamp_node[n] == stamp) continue;
            stamp_node[n] = stamp;
            const bool ss = lv.solid_side[n];
            if (field == 2) {
              if (region == 1 || !ss)
                for (int c = 0; c < D; ++c) {
                  dofs.push_back((int64_t)D * n + c);
                  dofs.push_back(lv.off_u + (int64_t)D * n + c);
                }
            } else if (field == 0 && region == 1) {
              for (int c = 0; c < D; ++c) dofs.push_back((int64_t)D * n + c);
            } else if (field == 0) {
              if (!ss)
                for (int c = 0; c < D; ++c) dofs.push_back((int64_t)D * n + c);
            } else {
              if (!ss)
                for (int c = 0; c < D; ++c) dofs.push_back(lv.off_u + (int64_t)D * n + c);
            }
          }
        if (!(field == 0 && region == 0))
          for (int64_t e : core_el)
            for (int k = 0; k < lv.npv; ++k) {
              const int64_t v = lv.elem_verts[e * lv.npv + k];
              if (stamp_vert[v] == stamp) continue;
              stamp_vert[v] = stamp;
              dofs.push_back(region == 1 ? lv.ps_of_vert[v] : lv.pf_of_vert[v]);
            }
        std::sort(dofs.begin(), dofs.end());
        size_t before = bs.dofs.size();
        for (int64_t d : dofs)
          if (!lv.dir[d]) bs.dofs.push_back((int32_t)d);
        if (bs.dofs.size() == before) continue;
        bs.ptr.push_back((int64_t)bs.dofs.size());
      }
    }
  }
  bs.owner.assign(lv.N, -1);
  for (int64_t j = 0; j < bs.nblk(); ++j)
    for (int64_t k = bs.ptr[j]; k < bs.ptr[j + 1]; ++k) bs.owner[bs.dofs[k]] = (int32_t)j;
  bs.jac.clear();
  for (int64_t i = 0; i < lv.N; ++i)
    if (bs.owner[i] < 0) bs.jac.push_back((int32_t)i);
}

}  // namespace fsgmg

namespace fsgmg {

void colour_blocks(const CsrHost& A, const std::vector<double>* pieces, int npieces,
                   BlockSet& bs) {
  const int64_t N = A.nrows, nb = bs.nblk();
  // entries that couple (per-piece row-relative threshold)
  std::vector<uint8_t> cpl(A.nnz(), 0);
  for (int64_t i = 0; i < N; ++i)
    for (int q = 0; q < npieces; ++q) {
      const std::vector<double>& P = pieces[q];
      double mx = 0.0;
      for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) mx = std::max(mx, std::fabs(P[k]));
      if (mx == 0.0) continue;
      for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
        if (std::fabs(P[k]) > kCouplingRel * mx) cpl[k] = 1;
    }
  // blocks containing each unknown
  std::vector<int64_t> mptr(N + 1, 0);
  for (int32_t g : bs.dofs) mptr[g + 1]++;
  for (int64_t i = 0; i < N; ++i) mptr[i + 1] += mptr[i];
  std::vector<int32_t> mblk(bs.dofs.size());
  {
    std::vector<int64_t> cur(mptr.begin(), mptr.end() - 1);
    for (int64_t j = 0; j < nb; ++j)
      for (int64_t p = bs.ptr[j]; p < bs.ptr[j + 1]; ++p) mblk[cur[bs.dofs[p]]++] = (int32_t)j;
  }
  // blocks that block j reaches through its rows (shared unknowns included);
  // the conflict graph is this relation made symmetric
  std::vector<std::vector<int32_t>> adj(nb);
  std::vector<int64_t> seen(nb, -1);
  for (int64_t j = 0; j < nb; ++j) {
    auto touch = [&](int64_t g) {
      for (int64_t t = mptr[g]; t < mptr[g + 1]; ++t) {
        const int32_t k = mblk[t];
        if (k == j || seen[k] == j) continue;
        seen[k] = j;
        adj[j].push_back(k);
        adj[k].push_back((int32_t)j);
      }
    };
    for (int64_t p = bs.ptr[j]; p < bs.ptr[j + 1]; ++p) {
      const int32_t a = bs.dofs[p];
      touch(a);
      for (int64_t k = A.rowptr[a]; k < A.rowptr[a + 1]; ++k)
        if (cpl[k]) touch(A.col[k]);
    }
  }
  // first fit in block order
  std::vector<int32_t> colour(nb, -1), mark;
  int32_t ncol = 0;
  for (int64_t j = 0; j < nb; ++j) {
    mark.assign(ncol + 1, 0);
    for (int32_t k : adj[j])
      if (colour[k] >= 0) mark[colour[k]] = 1;
    int32_t c = 0;
    while (mark[c]) ++c;
    colour[j] = c;
    ncol = std::max(ncol, c + 1);
  }
  // regroup colour by colour
  std::vector<int64_t> ord(nb);
  for (int64_t j = 0; j < nb; ++j) ord[j] = j;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int64_t a, int64_t b) { return colour[a] < colour[b]; });
  std::vector<int64_t> ptr(1, 0);
  std::vector<int32_t> dofs;
  dofs.reserve(bs.dofs.size());
  bs.colour_ptr.assign(ncol + 1, 0);
  for (int64_t q = 0; q < nb; ++q) {
    const int64_t j = ord[q];
    dofs.insert(dofs.end(), bs.dofs.begin() + bs.ptr[j], bs.dofs.begin() + bs.ptr[j + 1]);
    ptr.push_back((int64_t)dofs.size());
    bs.colour_ptr[colour[j] + 1] = q + 1;
  }
  for (int32_t c = 0; c < ncol; ++c)
    bs.colour_ptr[c + 1] = std::max(bs.colour_ptr[c + 1], bs.colour_ptr[c]);
  bs.ptr.swap(ptr);
  bs.dofs.swap(dofs);
  for (int64_t j = 0; j < nb; ++j)
    for (int64_t p = bs.ptr[j]; p < bs.ptr[j + 1]; ++p) bs.owner[bs.dofs[p]] = (int32_t)j;
  // the Jacobi unknowns must be mutually uncoupled
  std::vector<uint8_t> isjac(N, 0);
  for (int32_t i : bs.jac) isjac[i] = 1;
  for (int32_t i : bs.jac)
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
      if (cpl[k] && A.col[k] != i && isjac[A.col[k]])
        throw std::invalid_argument(
            "multiplicative Schwarz: two unknowns outside every block are coupled");
}

}  // namespace fsgmg
