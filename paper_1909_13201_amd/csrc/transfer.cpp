// Prolongation (natural injection of the nested Q2/Q1 spaces) and the
// equation-routed restriction R_2 of paper Section 3.3.
//
// The node-level interpolation Pn (fine Q2 node <- coarse Q2 nodes) serves
// every displacement and velocity component; Q1 interpolation inside each
// region serves p^s and p^f.  The restriction walks Pn^T but routes rows by
// equation type: a coarse solid-side node collects fine S rows (d-rows of
// solid-side nodes) and fine F rows (u-rows of fluid nodes) into its S row
// (R_SF = P_{d^f,d^s}^T) and only fine K rows into its K row; a coarse fluid
// node collects fine A rows and fine F rows.  The transpose of P_{u^f,u^s}
// appears nowhere.
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "host.hpp"

namespace fsgmg {

namespace {

struct W1 {
  int idx[3];
  double w[3];
  int n;
};

// 1D weights of the midpoint refinement of a line with nc elements.
std::vector<W1> weights_1d(int nc, bool quadratic) {
  std::vector<W1> out;
  const int nf = quadratic ? 4 * nc + 1 : 2 * nc + 1;
  for (int k = 0; k < nf; ++k) {
    W1 r{};
    if (quadratic) {
      const int c = std::min(k / 4, nc - 1);
      const double x = (k - 4 * c) / 2.0 - 1.0;
      const double L[3] = {0.5 * x * (x - 1.0), 1.0 - x * x, 0.5 * x * (x + 1.0)};
      for (int j = 0; j < 3; ++j)
        if (L[j] != 0.0) {
          r.idx[r.n] = 2 * c + j;
          r.w[r.n++] = L[j];
        }
    } else {
      const int c = std::min(k / 2, nc - 1);
      const double x = (double)(k - 2 * c) - 1.0;
      const double N[2] = {0.5 * (1.0 - x), 0.5 * (1.0 + x)};
      for (int j = 0; j < 2; ++j)
        if (N[j] != 0.0) {
          r.idx[r.n] = c + j;
          r.w[r.n++] = N[j];
        }
    }
    out.push_back(r);
  }
  return out;
}

// Tensor-product interpolation between grids with fine / coarse extents.
CsrHost tensor_interp(int D, const int* nfine, const int* ncoarse, const std::vector<W1>* w1) {
  CsrHost P;
  int64_t nf = 1, nc = 1;
  for (int a = 0; a < D; ++a) {
    nf *= nfine[a];
    nc *= ncoarse[a];
  }
  P.nrows = nf;
  P.ncols = nc;
  P.rowptr.assign(nf + 1, 0);
  for (int64_t i = 0; i < nf; ++i) {
    int ix[kMaxDim] = {0, 0, 0};
    int64_t t = i;
    for (int a = 0; a < D; ++a) {
      ix[a] = (int)(t % nfine[a]);
      t /= nfine[a];
    }
    const W1* r[kMaxDim];
    for (int a = 0; a < D; ++a) r[a] = &w1[a][ix[a]];
    int cnt[kMaxDim] = {1, 1, 1};
    for (int a = 0; a < D; ++a) cnt[a] = r[a]->n;
    for (int k2 = 0; k2 < (D > 2 ? cnt[2] : 1); ++k2)
      for (int k1 = 0; k1 < cnt[1]; ++k1)
        for (int k0 = 0; k0 < cnt[0]; ++k0) {
          const int kk[3] = {k0, k1, k2};
          int64_t c = 0, stride = 1;
          double w = 1.0;
          for (int a = 0; a < D; ++a) {
            c += (int64_t)r[a]->idx[kk[a]] * stride;
            stride *= ncoarse[a];
            w *= r[a]->w[kk[a]];
          }
          P.col.push_back((int32_t)c);
          P.val.push_back(w);
        }
    // columns sorted within a row
    const int64_t b = P.rowptr[i], e = (int64_t)P.col.size();
    std::vector<std::pair<int32_t, double>> tmp;
    for (int64_t k = b; k < e; ++k) tmp.emplace_back(P.col[k], P.val[k]);
    std::sort(tmp.begin(), tmp.end());
    for (int64_t k = b; k < e; ++k) {
      P.col[k] = tmp[k - b].first;
      P.val[k] = tmp[k - b].second;
    }
    P.rowptr[i + 1] = e;
  }
  return P;
}

// Restrict a vertex interpolation to the vertices of one region.
CsrHost region_rows(const CsrHost& Pv, const std::vector<int64_t>& fine_map, int64_t fine_off,
                    int64_t nfine, const std::vector<int64_t>& coarse_map, int64_t coarse_off,
                    int64_t ncoarse) {
  CsrHost P;
  P.nrows = nfine;
  P.ncols = ncoarse;
  P.rowptr.assign(nfine + 1, 0);
  std::vector<int64_t> order(nfine, -1);
  for (int64_t v = 0; v < (int64_t)fine_map.size(); ++v)
    if (fine_map[v] >= 0) order[fine_map[v] - fine_off] = v;
  for (int64_t r = 0; r < nfine; ++r) {
    const int64_t v = order[r];
    for (int64_t k = Pv.rowptr[v]; k < Pv.rowptr[v + 1]; ++k) {
      const int64_t cm = coarse_map[Pv.col[k]];
      if (cm < 0) throw std::runtime_error("pressure interpolation leaves its region");
      P.col.push_back((int32_t)(cm - coarse_off));
      P.val.push_back(Pv.val[k]);
    }
    P.rowptr[r + 1] = (int64_t)P.col.size();
  }
  return P;
}

}  // namespace

void build_transfer(const Level& fine, const Level& coarse, Transfer& t) {
  const int D = fine.D;
  std::vector<W1> q2[kMaxDim], q1[kMaxDim];
  for (int a = 0; a < D; ++a) {
    q2[a] = weights_1d(coarse.ne[a], true);
    q1[a] = weights_1d(coarse.ne[a], false);
  }
  t.Pn = tensor_interp(D, fine.nn, coarse.nn, q2);
  CsrHost Pv = tensor_interp(D, fine.nv, coarse.nv, q1);
  t.Pps = region_rows(Pv, fine.ps_of_vert, fine.off_ps, fine.Nps, coarse.ps_of_vert,
                      coarse.off_ps, coarse.Nps);
  t.Ppf = region_rows(Pv, fine.pf_of_vert, fine.off_pf, fine.Npf, coarse.pf_of_vert,
                      coarse.off_pf, coarse.Npf);
  t.Rn = csr_transpose(t.Pn);
  t.Rps = csr_transpose(t.Pps);
  t.Rpf = csr_transpose(t.Ppf);
}

CsrHost prolongation_full(const Level& fine, const Level& coarse, const Transfer& t) {
  const int D = fine.D;
  std::vector<std::vector<std::pair<int32_t, double>>> rows(fine.N);
  for (int64_t i = 0; i < fine.N2; ++i)
    for (int64_t k = t.Pn.rowptr[i]; k < t.Pn.rowptr[i + 1]; ++k)
      for (int c = 0; c < D; ++c) {
        const int64_t I = t.Pn.col[k];
        rows[D * i + c].emplace_back((int32_t)(D * I + c), t.Pn.val[k]);
        rows[fine.off_u + D * i + c].emplace_back((int32_t)(coarse.off_u + D * I + c), t.Pn.val[k]);
      }
  for (int64_t r = 0; r < fine.Nps; ++r)
    for (int64_t k = t.Pps.rowptr[r]; k < t.Pps.rowptr[r + 1]; ++k)
      rows[fine.off_ps + r].emplace_back((int32_t)(coarse.off_ps + t.Pps.col[k]), t.Pps.val[k]);
  for (int64_t r = 0; r < fine.Npf; ++r)
    for (int64_t k = t.Ppf.rowptr[r]; k < t.Ppf.rowptr[r + 1]; ++k)
      rows[fine.off_pf + r].emplace_back((int32_t)(coarse.off_pf + t.Ppf.col[k]), t.Ppf.val[k]);
  CsrHost P;
  P.nrows = fine.N;
  P.ncols = coarse.N;
  P.rowptr.assign(fine.N + 1, 0);
  for (int64_t i = 0; i < fine.N; ++i) {
    if (!fine.dir[i])
      for (auto& e : rows[i]) {
        P.col.push_back(e.first);
        P.val.push_back(e.second);
      }
    P.rowptr[i + 1] = (int64_t)P.col.size();
  }
  return P;
}

CsrHost restriction_full(const Level& fine, const Level& coarse, const Transfer& t) {
  const int D = fine.D;
  CsrHost R;
  R.nrows = coarse.N;
  R.ncols = fine.N;
  R.rowptr.assign(coarse.N + 1, 0);
  std::vector<std::vector<std::pair<int32_t, double>>> rows(coarse.N);
  for (int64_t I = 0; I < coarse.N2; ++I) {
    const bool ssI = coarse.solid_side[I];
    for (int64_t k = t.Rn.rowptr[I]; k < t.Rn.rowptr[I + 1]; ++k) {
      const int64_t i = t.Rn.col[k];
      const double w = t.Rn.val[k];
      const bool ssi = fine.solid_side[i];
      for (int c = 0; c < D; ++c) {
        if (ssI == ssi) {
          rows[D * I + c].emplace_back((int32_t)(D * i + c), w);
          rows[coarse.off_u + D * I + c].emplace_back((int32_t)(fine.off_u + D * i + c), w);
        } else if (ssI && !ssi) {
          rows[D * I + c].emplace_back((int32_t)(fine.off_u + D * i + c), w);   // R_SF
        }
      }
    }
  }
  for (int64_t r = 0; r < coarse.Nps; ++r)
    for (int64_t k = t.Rps.rowptr[r]; k < t.Rps.rowptr[r + 1]; ++k)
      rows[coarse.off_ps + r].emplace_back((int32_t)(fine.off_ps + t.Rps.col[k]), t.Rps.val[k]);
  for (int64_t r = 0; r < coarse.Npf; ++r)
    for (int64_t k = t.Rpf.rowptr[r]; k < t.Rpf.rowptr[r + 1]; ++k)
      rows[coarse.off_pf + r].emplace_back((int32_t)(fine.off_pf + t.Rpf.col[k]), t.Rpf.val[k]);
  for (int64_t I = 0; I < coarse.N; ++I) {
    if (!coarse.dir[I]) {
      std::sort(rows[I].begin(), rows[I].end());
      for (auto& e : rows[I]) {
        R.col.push_back(e.first);
        R.val.push_back(e.second);
      }
    }
    R.rowptr[I + 1] = (int64_t)R.col.size();
  }
  return R;
}

}  // namespace fsgmg
