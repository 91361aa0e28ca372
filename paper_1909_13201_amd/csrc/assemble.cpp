// Q2/Q1 assembly of the linearized monolithic FSI operator in J2 routing.
//
// Equation groups (paper Section 3.1) and the weak forms of Section 2.2,
// linearized at the stress-free state d = 0 about a frozen advecting
// velocity w:
//   S  solid-side momentum rows: solid elements G(grad d + grad d^T):grad phi
//      - p^s div phi (linearized Mooney-Rivlin, C1 = G/3, C2 = C1/2);
//      fluid elements mu(grad u + grad u^T):grad phi - p^f div phi
//      + rho (w.grad)u.phi (+ SUPG), i.e. the interface rows collect both;
//   A  fluid-node ALE rows: (k (grad d + grad d^T), grad phi), k = 1/V of the
//      coarse element containing the point;
//   K  kinematic rows on u^s: lumped (or consistent) mass; -mass/dt on d^s
//      for a backward-Euler step;
//   F  fluid-node momentum rows (fluid terms above);
//   V  -(div d, q) - (1/lambda_L)(p^s, q);   W  -(div u, q).
// SUPG (eqs. tausupg, lambda_k): tau = 1/max(4 lambda nu, sqrt(lambda)|w|),
// lambda from the element-bubble generalized eigenproblem (dim x dim).
// Operator = base + G*pG + (1/lambda_L)*pC + mu*pMu with tau frozen.
#include <algorithm>
#include <cmath>
#include <memory>
#include <numeric>
#include <exception>
#include <stdexcept>
#include <thread>

#include "host.hpp"

namespace fsgmg {

namespace {

constexpr int kMaxQ = 27, kMaxB = 27, kMaxP = 8;

struct RefElem {
  int D, nq, nb, np, bubble;
  double wq[kMaxQ];
  double phi[kMaxQ][kMaxB];
  double dphi[kMaxQ][kMaxB][3];
  double d2phi[kMaxQ][kMaxB][3][3];
  double psi[kMaxQ][kMaxP];
  double dpsi[kMaxQ][kMaxP][3];

  explicit RefElem(int dim) : D(dim) {
    const double sq = std::sqrt(0.6);
    const double gp[3] = {-sq, 0.0, sq};
    const double gw[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
    auto L = [](int a, double x) {
      return a == 0 ? 0.5 * x * (x - 1.0) : (a == 1 ? 1.0 - x * x : 0.5 * x * (x + 1.0));
    };
    auto dL = [](int a, double x) { return a == 0 ? x - 0.5 : (a == 1 ? -2.0 * x : x + 0.5); };
    auto ddL = [](int a, double) { return a == 1 ? -2.0 : 1.0; };
    auto N = [](int a, double x) { return a == 0 ? 0.5 * (1.0 - x) : 0.5 * (1.0 + x); };
    auto dN = [](int a, double) { return a == 0 ? -0.5 : 0.5; };
    nq = nb = 1;
    np = 1;
    for (int k = 0; k < D; ++k) {
      nq *= 3;
      nb *= 3;
      np *= 2;
    }
    bubble = 0;
    for (int k = 0, s = 1; k < D; ++k, s *= 3) bubble += s;
    for (int q = 0; q < nq; ++q) {
      int qi[3];
      for (int k = 0, t = q; k < D; ++k, t /= 3) qi[k] = t % 3;
      wq[q] = 1.0;
      for (int k = 0; k < D; ++k) wq[q] *= gw[qi[k]];
      for (int a = 0; a < nb; ++a) {
        int ai[3];
        for (int k = 0, t = a; k < D; ++k, t /= 3) ai[k] = t % 3;
        double v = 1.0;
        for (int k = 0; k < D; ++k) v *= L(ai[k], gp[qi[k]]);
        phi[q][a] = v;
        for (int i = 0; i < D; ++i) {
          double g = 1.0;
          for (int k = 0; k < D; ++k) g *= (k == i) ? dL(ai[k], gp[qi[k]]) : L(ai[k], gp[qi[k]]);
          dphi[q][a][i] = g;
          for (int j = 0; j < D; ++j) {
            double h = 1.0;
            for (int k = 0; k < D; ++k) {
              const double x = gp[qi[k]];
              if (k == i && k == j)
                h *= ddL(ai[k], x);
              else if (k == i || k == j)
                h *= dL(ai[k], x);
              else
                h *= L(ai[k], x);
            }
            d2phi[q][a][i][j] = h;
          }
        }
      }
      for (int m = 0; m < np; ++m) {
        int mi[3];
        for (int k = 0, t = m; k < D; ++k, t /= 2) mi[k] = t % 2;
        double v = 1.0;
        for (int k = 0; k < D; ++k) v *= N(mi[k], gp[qi[k]]);
        psi[q][m] = v;
        for (int i = 0; i < D; ++i) {
          double g = 1.0;
          for (int k = 0; k < D; ++k) g *= (k == i) ? dN(mi[k], gp[qi[k]]) : N(mi[k], gp[qi[k]]);
          dpsi[q][m][i] = g;
        }
      }
    }
  }
};

// Geometry of one element at every Gauss point.
struct ElemGeo {
  double dV[kMaxQ];
  double G[kMaxQ][kMaxB][3];
  double H[kMaxQ][kMaxB][3][3];
  double Gp[kMaxQ][kMaxP][3];
};

void invert_small(int D, const double J[3][3], double Ji[3][3], double& det) {
  if (D == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;
    Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det;
    Ji[1][1] = J[0][0] / det;
    return;
  }
  det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
        J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
        J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
}

void element_geometry(const RefElem& R, const Level& lv, int64_t e, ElemGeo& g) {
  const int D = R.D, nb = R.nb;
  double Xe[kMaxB][3];
  for (int b = 0; b < nb; ++b)
    for (int i = 0; i < D; ++i) Xe[b][i] = lv.X[lv.elem_nodes[e * nb + b] * D + i];
  for (int q = 0; q < R.nq; ++q) {
    double J[3][3] = {}, Ji[3][3] = {}, det = 0;
    for (int i = 0; i < D; ++i)
      for (int k = 0; k < D; ++k) {
        double s = 0;
        for (int b = 0; b < nb; ++b) s += Xe[b][i] * R.dphi[q][b][k];
        J[i][k] = s;
      }
    invert_small(D, J, Ji, det);   // Ji[k][i] = d xi_k / d x_i
    if (!(det > 0)) throw std::runtime_error("non-positive Jacobian determinant");
    g.dV[q] = det * R.wq[q];
    for (int a = 0; a < nb; ++a) {
      for (int i = 0; i < D; ++i) {
        double s = 0;
        for (int k = 0; k < D; ++k) s += R.dphi[q][a][k] * Ji[k][i];
        g.G[q][a][i] = s;
      }
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) {
          double s = 0;
          for (int k = 0; k < D; ++k)
            for (int m = 0; m < D; ++m) s += Ji[k][i] * R.d2phi[q][a][k][m] * Ji[m][j];
          g.H[q][a][i][j] = s;
        }
    }
    for (int m = 0; m < R.np; ++m)
      for (int i = 0; i < D; ++i) {
        double s = 0;
        for (int k = 0; k < D; ++k) s += R.dpsi[q][m][k] * Ji[k][i];
        g.Gp[q][m][i] = s;
      }
  }
}

// largest eigenvalue of a symmetric D x D matrix (cyclic Jacobi)
double max_sym_eig(int D, double M[3][3]) {
  if (D == 2) {
    const double a = M[0][0], b = M[0][1], d = M[1][1];
    return 0.5 * (a + d) + std::sqrt(0.25 * (a - d) * (a - d) + b * b);
  }
  double A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = M[i][j];
  for (int sweep = 0; sweep < 50; ++sweep) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    if (off < 1e-300) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        const double th = 0.5 * (A[q][q] - A[p][p]) / A[p][q];
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
      }
  }
  return std::max(A[0][0], std::max(A[1][1], A[2][2]));
}

// Triplets tagged with the affine piece they belong to.
struct Triplets {
  std::vector<int64_t> row;
  std::vector<int32_t> col;
  std::vector<uint8_t> piece;
  std::vector<double> val;
  void add(int64_t r, int64_t c, int p, double v) {
    if (v == 0.0) return;
    add_always(r, c, p, v);
  }
  // append lists in order, releasing them
  void join(std::vector<Triplets>& parts) {
    size_t n = row.size();
    for (const Triplets& p : parts) n += p.row.size();
    row.reserve(n);
    col.reserve(n);
    piece.reserve(n);
    val.reserve(n);
    for (Triplets& p : parts) {
      row.insert(row.end(), p.row.begin(), p.row.end());
      col.insert(col.end(), p.col.begin(), p.col.end());
      piece.insert(piece.end(), p.piece.begin(), p.piece.end());
      val.insert(val.end(), p.val.begin(), p.val.end());
      p = Triplets();
    }
  }
  // terms that depend on the advecting velocity keep their entries when
  // they vanish, so the operator's pattern does not depend on w
  void add_always(int64_t r, int64_t c, int p, double v) {
    if (r < 0) return;
    row.push_back(r);
    col.push_back((int32_t)c);
    piece.push_back((uint8_t)p);
    val.push_back(v);
  }
};

// Run f(i0, i1) over contiguous ranges of [0, n) on up to 16 host threads
// (one when n is small).
template <typename F>
static void parallel_ranges(int64_t n, int64_t min_per_thread, F&& f) {
  const int nthr = (int)std::min<int64_t>(
      std::max(1u, std::min(16u, std::thread::hardware_concurrency())), n / min_per_thread + 1);
  if (nthr <= 1) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::exception_ptr> errs(nthr);
  std::vector<std::thread> pool;
  for (int t = 0; t < nthr; ++t)
    pool.emplace_back([&, t]() {
      try {
        f(n * t / nthr, n * (t + 1) / nthr);
      } catch (...) {
        errs[t] = std::current_exception();
      }
    });
  for (std::thread& th : pool) th.join();
  for (const std::exception_ptr& e : errs)
    if (e) std::rethrow_exception(e);
}

// Combine triplets into a CSR pattern with one value array per piece: the
// triplets of a row are ordered by column (the same sort of the same
// sequence whatever the threading, so the sums are reproducible) and equal
// columns summed per piece.
void to_csr(const Triplets& t, int64_t nrows, int64_t ncols, int npieces, CsrHost& pat,
            std::vector<double>* pieces) {
  const int64_t nt = (int64_t)t.row.size();
  std::vector<int64_t> cnt(nrows + 1, 0);
  for (int64_t k = 0; k < nt; ++k) cnt[t.row[k] + 1]++;
  for (int64_t i = 0; i < nrows; ++i) cnt[i + 1] += cnt[i];
  std::vector<int64_t> order(nt);
  {
    std::vector<int64_t> cur(cnt.begin(), cnt.end() - 1);
    for (int64_t k = 0; k < nt; ++k) order[cur[t.row[k]]++] = k;
  }
  // each row's triplets sorted by column, and its number of distinct columns
  std::vector<int64_t> nu(nrows + 1, 0);
  parallel_ranges(nrows, 4096, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      auto b = order.begin() + cnt[i], e = order.begin() + cnt[i + 1];
      std::sort(b, e, [&](int64_t x, int64_t y) { return t.col[x] < t.col[y]; });
      int64_t u = 0;
      for (auto k = b; k != e; ++k)
        if (k == b || t.col[*k] != t.col[*(k - 1)]) ++u;
      nu[i + 1] = u;
    }
  });
  pat.nrows = nrows;
  pat.ncols = ncols;
  pat.rowptr.assign(nrows + 1, 0);
  for (int64_t i = 0; i < nrows; ++i) pat.rowptr[i + 1] = pat.rowptr[i] + nu[i + 1];
  const int64_t nnz = pat.rowptr[nrows];
  pat.col.assign(nnz, 0);
  for (int p = 0; p < npieces; ++p) pieces[p].assign(nnz, 0.0);
  parallel_ranges(nrows, 4096, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int64_t k = cnt[i], out = pat.rowptr[i];
      while (k < cnt[i + 1]) {
        const int32_t c = t.col[order[k]];
        double acc[4] = {0, 0, 0, 0};
        while (k < cnt[i + 1] && t.col[order[k]] == c) {
          acc[t.piece[order[k]]] += t.val[order[k]];
          ++k;
        }
        pat.col[out] = c;
        for (int p = 0; p < npieces; ++p) pieces[p][out] = acc[p];
        ++out;
      }
    }
  });
}

enum { P_BASE = 0, P_G = 1, P_C = 2, P_MU = 3 };

}  // namespace

std::vector<double> reference_tables(int D) {
  const RefElem R(D);
  constexpr int Q = kMaxQ, B = kMaxB, P = kMaxP;
  // Gauss weights, phi, dphi, d2phi, psi, dpsi at the maximal sizes (zeros
  // beyond the element's own counts)
  std::vector<double> t(Q + Q * B + Q * B * 3 + Q * B * 9 + Q * P + Q * P * 3, 0.0);
  const size_t o_phi = Q, o_dphi = o_phi + Q * B, o_d2 = o_dphi + Q * B * 3,
               o_psi = o_d2 + Q * B * 9, o_dpsi = o_psi + Q * P;
  for (int q = 0; q < R.nq; ++q) {
    t[q] = R.wq[q];
    for (int a = 0; a < R.nb; ++a) {
      t[o_phi + q * B + a] = R.phi[q][a];
      for (int k = 0; k < D; ++k) {
        t[o_dphi + (q * B + a) * 3 + k] = R.dphi[q][a][k];
        for (int m = 0; m < D; ++m) t[o_d2 + ((q * B + a) * 3 + k) * 3 + m] = R.d2phi[q][a][k][m];
      }
    }
    for (int m = 0; m < R.np; ++m) {
      t[o_psi + q * P + m] = R.psi[q][m];
      for (int k = 0; k < D; ++k) t[o_dpsi + (q * P + m) * 3 + k] = R.dpsi[q][m][k];
    }
  }
  return t;
}

void lame(double E, double nu, double& G, double& invlam) {
  G = E / (2.0 * (1.0 + nu));
  invlam = nu >= 0.5 ? 0.0 : (1.0 + nu) * (1.0 - 2.0 * nu) / (E * nu);
}

std::vector<double> element_volumes(const Level& lv) {
  RefElem R(lv.D);
  std::vector<double> vol(lv.nE);
  ElemGeo g;
  for (int64_t e = 0; e < lv.nE; ++e) {
    element_geometry(R, lv, e, g);
    double s = 0;
    for (int q = 0; q < R.nq; ++q) s += g.dV[q];
    vol[e] = s;
  }
  return vol;
}

namespace {

// Unknowns of one element: displacement and velocity components of its
// nodes, the momentum row of each (S on solid-side nodes, F elsewhere) and
// its solid and fluid pressure unknowns (-1 where a vertex has none).
struct ElemDofs {
  int64_t d[kMaxB * 3], u[kMaxB * 3], rowm[kMaxB * 3], ps[kMaxP], pf[kMaxP];
};

void element_dofs(const Level& lv, int64_t e, int nb, int np, ElemDofs& o) {
  const int D = lv.D;
  const int64_t* nodes = &lv.elem_nodes[e * nb];
  const int64_t* verts = &lv.elem_verts[e * np];
  for (int a = 0; a < nb; ++a)
    for (int c = 0; c < D; ++c) {
      o.d[a * D + c] = (int64_t)D * nodes[a] + c;
      o.u[a * D + c] = lv.off_u + (int64_t)D * nodes[a] + c;
      o.rowm[a * D + c] = lv.solid_side[nodes[a]] ? o.d[a * D + c] : o.u[a * D + c];
    }
  for (int m = 0; m < np; ++m) {
    o.ps[m] = lv.ps_of_vert[verts[m]];
    o.pf[m] = lv.pf_of_vert[verts[m]];
  }
}

enum { T_OP = 0, T_TIME = 1, T_LOAD = 2 };

// The terms of fluid element e that depend on the advecting velocity w
// (Section 2.2: the convection rho (w.grad u, phi) and every SUPG term of
// the stabilized momentum balance with tau of eq. tausupg, lambda_k from the
// element bubble), handed in a fixed order to emit(target, row, col, piece,
// value): T_OP the operator, T_TIME the time operator, T_LOAD the load
// operator (the last two on the finest level only).
template <typename Emit>
void advective_terms(const RefElem& R, const Level& lv, const Physics& ph, const ElemGeo& g,
                     int64_t e, const ElemDofs& dof, const std::vector<double>& w, bool finest,
                     Emit&& emit) {
  const int D = R.D, nb = R.nb, np = R.np, nq = R.nq;
  const double rho = ph.rho, inv_dt = ph.inv_dt, theta = ph.theta;
  const bool weighted = inv_dt != 0.0 && theta != 1.0;
  const int64_t* nodes = &lv.elem_nodes[e * nb];
  // a steady term of a momentum row: theta v into the operator and, on the
  // finest level, -(1 - theta) v into the time operator
  auto madd = [&](int64_t r, int64_t c, int p, double v) {
    emit(T_OP, r, c, p, weighted ? theta * v : v);
    if (finest && weighted) emit(T_TIME, r, c, p, -(1.0 - theta) * v);
  };
  double wq[kMaxQ][3], wg[kMaxQ][kMaxB];
  for (int q = 0; q < nq; ++q)
    for (int i = 0; i < D; ++i) {
      double s = 0;
      for (int b = 0; b < nb; ++b) s += w[nodes[b] * D + i] * R.phi[q][b];
      wq[q][i] = s;
    }
  for (int q = 0; q < nq; ++q)
    for (int a = 0; a < nb; ++a) {
      double s = 0;
      for (int i = 0; i < D; ++i) s += wq[q][i] * g.G[q][a][i];
      wg[q][a] = s;
    }
  // convection rho (w.grad u, phi)
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      double s = 0;
      for (int q = 0; q < nq; ++q) s += g.dV[q] * R.phi[q][a] * wg[q][b];
      for (int c = 0; c < D; ++c) madd(dof.rowm[a * D + c], dof.u[b * D + c], P_BASE, rho * s);
    }
  if (!ph.supg) return;
  // lambda_k from the element bubble
  const int bb = R.bubble;
  double Mb[3][3] = {}, Nb = 0;
  for (int q = 0; q < nq; ++q) {
    double lap = 0;
    for (int i = 0; i < D; ++i) lap += g.H[q][bb][i][i];
    double v[3][3];
    for (int a = 0; a < D; ++a)
      for (int i = 0; i < D; ++i) v[a][i] = (i == a ? lap : 0.0) + g.H[q][bb][i][a];
    for (int a = 0; a < D; ++a)
      for (int b = 0; b < D; ++b) {
        double s = 0;
        for (int i = 0; i < D; ++i) s += v[a][i] * v[b][i];
        Mb[a][b] += g.dV[q] * s;
      }
    for (int i = 0; i < D; ++i) Nb += g.dV[q] * g.G[q][bb][i] * g.G[q][bb][i];
  }
  const double lam = max_sym_eig(D, Mb) / Nb;
  const double nu_k = ph.mu / rho;
  double tw[kMaxQ];
  for (int q = 0; q < nq; ++q) {
    double wn = 0;
    for (int i = 0; i < D; ++i) wn += wq[q][i] * wq[q][i];
    wn = std::sqrt(wn);
    const double tau = 1.0 / std::max(4.0 * lam * nu_k, std::sqrt(lam) * wn);
    tw[q] = g.dV[q] * tau * rho;
  }
  for (int a = 0; a < nb; ++a)
    for (int b = 0; b < nb; ++b) {
      // the SUPG inertia: its steady part carries theta, its time part
      // rho/dt phi_b does not
      double s1s = 0, s1t = 0;
      for (int q = 0; q < nq; ++q) {
        s1s += tw[q] * wg[q][a] * rho * wg[q][b];
        s1t += tw[q] * wg[q][a] * rho * inv_dt * R.phi[q][b];
      }
      const double s1 = weighted ? theta * s1s + s1t : s1s + s1t;
      for (int c = 0; c < D; ++c) {
        const int64_t r = dof.rowm[a * D + c], col = dof.u[b * D + c];
        emit(T_OP, r, col, P_BASE, s1);
        if (finest && weighted) emit(T_TIME, r, col, P_BASE, -(1.0 - theta) * s1s);
        if (finest && inv_dt != 0.0) emit(T_TIME, r, col, P_BASE, s1t);
      }
      if (finest) {   // the SUPG load term rho^2 tau (w.grad phi_a, f)
        double sl = 0;
        for (int q = 0; q < nq; ++q) sl += rho * rho * tw[q] * wg[q][a] * R.phi[q][b];
        for (int c = 0; c < D; ++c)
          emit(T_LOAD, dof.rowm[a * D + c], (int64_t)D * nodes[b] + c, P_BASE, sl);
      }
    }
  for (int a = 0; a < nb; ++a)
    for (int c = 0; c < D; ++c)
      for (int b = 0; b < nb; ++b)
        for (int f = 0; f < D; ++f) {
          double s = 0;
          for (int q = 0; q < nq; ++q) {
            double lap = 0;
            if (c == f)
              for (int i = 0; i < D; ++i) lap += g.H[q][b][i][i];
            s += tw[q] * wg[q][a] * (lap + g.H[q][b][c][f]);
          }
          madd(dof.rowm[a * D + c], dof.u[b * D + f], P_MU, -s);
        }
  for (int a = 0; a < nb; ++a)
    for (int c = 0; c < D; ++c)
      for (int m = 0; m < np; ++m) {
        double s = 0;
        for (int q = 0; q < nq; ++q) s += tw[q] * wg[q][a] * g.Gp[q][m][c];
        madd(dof.rowm[a * D + c], dof.pf[m], P_BASE, s);
      }
}

// Position of entry (r, c) in a CSR pattern (columns sorted per row).
int64_t slot_of(const CsrHost& P, int64_t r, int64_t c) {
  const int32_t* b = P.col.data() + P.rowptr[r];
  const int32_t* en = P.col.data() + P.rowptr[r + 1];
  const int32_t* it = std::lower_bound(b, en, (int32_t)c);
  if (it == en || *it != (int32_t)c)
    throw std::logic_error("an advective term falls outside the operator's pattern");
  return it - P.col.data();
}

// Where the advective terms of a level are added.  op: the unreduced
// pattern and pieces on the finest level (nothing skipped), the reduced
// ones elsewhere (entries in a Dirichlet row or column skipped: the reduced
// operator has none); time / load: the finest level's operators with their
// Dirichlet rows removed.
struct AdvTargets {
  const CsrHost* op;
  std::vector<double>* op_piece;
  bool op_reduced;
  const CsrHost* time;
  std::vector<double>* time_piece;
  const CsrHost* load;
  std::vector<double>* load_val;
};

// Add the advective terms of every fluid element of the level.  Elements
// are taken colour by colour (the parity of the element's position along
// each axis: elements of one colour share no node, hence no row) and the
// elements of a colour on host threads, so every entry receives its
// contributions in one order whatever the threading.  Every element emits
// the same number of terms (the branches depend on the physics only), so
// the value slot of each emission can be recorded once (record) and
// replayed (replay) instead of searched for.
void add_advective(const Level& lv, const Physics& ph, const std::vector<double>& w, bool finest,
                   const AdvTargets& t, AdvectionPlan* rec, const std::vector<int32_t>* replay) {
  std::vector<int32_t>* record = rec ? &rec->slots : nullptr;
  const int D = lv.D;
  const RefElem R(D);
  const int ncol = 1 << D;
  std::vector<std::vector<int64_t>> by_colour(ncol);
  for (int64_t e = 0; e < lv.nE; ++e) {
    if (lv.region[e] == 1) continue;
    int ix[kMaxDim] = {0, 0, 0};
    lv.node_ijk(lv.elem_nodes[e * R.nb], ix);   // the element's first corner, 2 x its position
    int colour = 0;
    for (int a = 0; a < D; ++a) colour |= ((ix[a] >> 1) & 1) << a;
    by_colour[colour].push_back(e);
  }
  int64_t nfluid = 0, per = 0;
  for (const std::vector<int64_t>& list : by_colour) nfluid += (int64_t)list.size();
  if (nfluid == 0) return;
  if (record || replay) {   // emissions per element, counted on one element
    const int64_t e = [&] {
      for (const std::vector<int64_t>& list : by_colour)
        if (!list.empty()) return list[0];
      return (int64_t)0;
    }();
    std::unique_ptr<ElemGeo> g(new ElemGeo);
    ElemDofs dof;
    element_geometry(R, lv, e, *g);
    element_dofs(lv, e, R.nb, R.np, dof);
    advective_terms(R, lv, ph, *g, e, dof, w, finest,
                    [&](int, int64_t, int64_t, int, double) { ++per; });
  }
  if (rec) {
    rec->slots.assign(nfluid * per, -1);
    rec->dest.assign(nfluid * per, 0);
    rec->per = (int)per;
    rec->elems.clear();
    for (const std::vector<int64_t>& list : by_colour)
      for (int64_t e : list) rec->elems.push_back((int32_t)e);
  }
  if (replay && (int64_t)replay->size() != nfluid * per)
    throw std::logic_error("re-assembly slots do not match the level");
  int64_t base = 0;
  for (const std::vector<int64_t>& list : by_colour) {
    parallel_ranges((int64_t)list.size(), 32, [&](int64_t i0, int64_t i1) {
      std::unique_ptr<ElemGeo> g(new ElemGeo);
      ElemDofs dof;
      for (int64_t i = i0; i < i1; ++i) {
        const int64_t e = list[i];
        element_geometry(R, lv, e, *g);
        element_dofs(lv, e, R.nb, R.np, dof);
        int64_t k = (base + i) * per;
        if (replay) {
          const int32_t* sl = replay->data() + k;
          advective_terms(R, lv, ph, *g, e, dof, w, finest,
                          [&](int target, int64_t, int64_t, int p, double v) {
                            const int32_t s = *sl++;
                            if (s < 0) return;
                            if (target == T_OP)
                              t.op_piece[p][s] += v;
                            else if (target == T_TIME)
                              t.time_piece[p][s] += v;
                            else
                              (*t.load_val)[s] += v;
                          });
          continue;
        }
        advective_terms(R, lv, ph, *g, e, dof, w, finest,
                        [&](int target, int64_t r, int64_t c, int p, double v) {
                          int64_t s = -1;
                          if (target == T_OP) {
                            if (!(t.op_reduced && (lv.dir[r] || lv.dir[c]))) {
                              s = slot_of(*t.op, r, c);
                              t.op_piece[p][s] += v;
                            }
                          } else if (target == T_TIME) {
                            if (!lv.dir[r]) {
                              s = slot_of(*t.time, r, c);
                              t.time_piece[p][s] += v;
                            }
                          } else if (!lv.dir[r]) {
                            s = slot_of(*t.load, r, c);
                            (*t.load_val)[s] += v;
                          }
                          if (record) {
                            rec->dest[k] = (uint8_t)(4 * target + p);
                            (*record)[k++] = (int32_t)s;
                          }
                        });
      }
    });
    base += (int64_t)list.size();
  }
}

// Copy of a value array on host threads.
void copy_values(const std::vector<double>& from, std::vector<double>& to) {
  to.resize(from.size());
  parallel_ranges((int64_t)from.size(), 1 << 17, [&](int64_t i0, int64_t i1) {
    std::copy(from.begin() + i0, from.begin() + i1, to.begin() + i0);
  });
}

// Reduced operator values (Dirichlet rows and columns removed, unit
// diagonal) from the unreduced pieces on the pattern already in op.A.
void reduce_values(const Level& lv, const CsrHost& full, const std::vector<double>* fp,
                   LevelOperator& op) {
  const CsrHost& A = op.A;
  parallel_ranges(lv.N, 4096, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int64_t o = A.rowptr[i];
      if (lv.dir[i]) {
        op.piece[P_BASE][o] = 1.0;
        for (int p = 1; p < 4; ++p) op.piece[p][o] = 0.0;
        continue;
      }
      for (int64_t k = full.rowptr[i]; k < full.rowptr[i + 1]; ++k) {
        if (lv.dir[full.col[k]]) continue;
        for (int p = 0; p < 4; ++p) op.piece[p][o] = fp[p][k];
        ++o;
      }
    }
  });
}

void combine_values(const std::vector<double>* piece, double G, double invlam, double mu,
                    std::vector<double>& val) {
  const int64_t n = (int64_t)piece[0].size();
  val.resize(n);
  parallel_ranges(n, 1 << 16, [&](int64_t i0, int64_t i1) {
    for (int64_t k = i0; k < i1; ++k)
      val[k] = piece[P_BASE][k] + G * piece[P_G][k] + invlam * piece[P_C][k] + mu * piece[P_MU][k];
  });
}

// Lift pieces: lift = g on Dirichlet rows, -(A_full g) on free rows.
void lift_values(const Level& lv, const CsrHost& full, const std::vector<double>* fp,
                 LevelOperator& op) {
  for (int p = 0; p < 4; ++p) op.lift_piece[p].assign(lv.N, 0.0);
  parallel_ranges(lv.N, 4096, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      if (lv.dir[i]) {
        op.lift_piece[P_BASE][i] = lv.dir_val[i];
        continue;
      }
      for (int64_t k = full.rowptr[i]; k < full.rowptr[i + 1]; ++k) {
        const int32_t j = full.col[k];
        if (!lv.dir[j] || lv.dir_val[j] == 0.0) continue;
        for (int p = 0; p < 4; ++p) op.lift_piece[p][i] -= fp[p][k] * lv.dir_val[j];
      }
    }
  });
}

// Rows of an unreduced CSR with the Dirichlet rows removed (every column
// kept), pattern and npieces value arrays.
void drop_dirichlet_rows(const Level& lv, const CsrHost& M, const std::vector<double>* mp,
                         int npieces, CsrHost& out, std::vector<double>* outp) {
  out.nrows = lv.N;
  out.ncols = M.ncols;
  out.rowptr.assign(lv.N + 1, 0);
  for (int64_t i = 0; i < lv.N; ++i)
    out.rowptr[i + 1] = out.rowptr[i] + (lv.dir[i] ? 0 : M.rowptr[i + 1] - M.rowptr[i]);
  const int64_t nnz = out.rowptr[lv.N];
  out.col.resize(nnz);
  for (int p = 0; p < npieces; ++p) outp[p].resize(nnz);
  parallel_ranges(lv.N, 4096, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      if (lv.dir[i]) continue;
      int64_t o = out.rowptr[i];
      for (int64_t k = M.rowptr[i]; k < M.rowptr[i + 1]; ++k, ++o) {
        out.col[o] = M.col[k];
        for (int p = 0; p < npieces; ++p) outp[p][o] = mp[p][k];
      }
    }
  });
}

// Recorded slots are 32-bit: the patterns they index must be shorter than
// 2^31 entries.
bool slots_fit(const CsrHost& op, const CsrHost* time, const CsrHost* load) {
  const int64_t lim = (int64_t)1 << 31;
  return op.nnz() < lim && (!time || time->nnz() < lim) && (!load || load->nnz() < lim);
}

}  // namespace

void assemble_level(const Level& lv, const Physics& ph, const std::vector<double>& coarse_vol,
                    const std::vector<double>* w_level, bool finest, LevelOperator& op,
                    AdvectionPlan* plan) {
  const int D = lv.D;
  RefElem R(D);
  const int nb = R.nb, np = R.np, nq = R.nq, nbD = nb * D;
  const double rho = ph.rho, inv_dt = ph.inv_dt;
  // weight of the steady terms of the momentum rows (1 = backward Euler,
  // 1/2 = Crank-Nicolson for the momentum balance)
  const double theta = ph.theta;
  const bool weighted = inv_dt != 0.0 && theta != 1.0;
  double Gmod, invlam;
  lame(ph.E, ph.nu, Gmod, invlam);
  op.G = Gmod;
  op.invlam = invlam;
  op.mu = ph.mu;
  const bool have_w = w_level != nullptr;

  // The element loop over [e_begin, e_end) into the given triplet lists
  // (operator pieces, load operator, time operator): every term that does
  // not depend on the advecting velocity, and zero-valued entries where the
  // advective terms land (they are added later, on the fixed pattern).
  auto run_elements = [&](int64_t e_begin, int64_t e_end, Triplets& T, Triplets& TL,
                          Triplets& TT) {
    // a term that carries 1/dt: into the operator and, on the finest level,
    // into the time operator as well
    auto tadd = [&](int64_t r, int64_t c, double v) {
      T.add(r, c, P_BASE, v);
      if (finest) TT.add(r, c, 0, v);
    };
    // a steady term of a momentum row: theta times v into the operator and,
    // on the finest level, -(1 - theta) v into the time operator (the
    // explicit part of the step)
    auto madd = [&](int64_t r, int64_t c, int p, double v) {
      T.add(r, c, p, weighted ? theta * v : v);
      if (finest && weighted) TT.add(r, c, p, -(1.0 - theta) * v);
    };
    ElemGeo g;
    ElemDofs dof;
    static thread_local double Tg[kMaxB][kMaxB][3][3];
    std::vector<double> Ksym(nbD * nbD), Bdiv(np * nbD), M2(nb * nb), M1(np * np);
    for (int64_t e = e_begin; e < e_end; ++e) {
      element_geometry(R, lv, e, g);
      element_dofs(lv, e, nb, np, dof);
      const int64_t* nodes = &lv.elem_nodes[e * nb];
      const int64_t* dofd = dof.d;
      const int64_t* dofu = dof.u;
      const int64_t* rowm = dof.rowm;
      // T[a][b][i][j] = sum_q dV G_ai G_bj
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
          for (int i = 0; i < D; ++i)
            for (int j = 0; j < D; ++j) {
              double s = 0;
              for (int q = 0; q < nq; ++q) s += g.dV[q] * g.G[q][a][i] * g.G[q][b][j];
              Tg[a][b][i][j] = s;
            }
      for (int a = 0; a < nb; ++a)
        for (int c = 0; c < D; ++c)
          for (int b = 0; b < nb; ++b)
            for (int f = 0; f < D; ++f) {
              double v = Tg[a][b][f][c];
              if (c == f)
                for (int i = 0; i < D; ++i) v += Tg[a][b][i][i];
              Ksym[(a * D + c) * nbD + b * D + f] = v;
            }
      for (int m = 0; m < np; ++m)
        for (int b = 0; b < nb; ++b)
          for (int f = 0; f < D; ++f) {
            double s = 0;
            for (int q = 0; q < nq; ++q) s += g.dV[q] * R.psi[q][m] * g.G[q][b][f];
            Bdiv[m * nbD + b * D + f] = s;
          }
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
          double s = 0;
          for (int q = 0; q < nq; ++q) s += g.dV[q] * R.phi[q][a] * R.phi[q][b];
          M2[a * nb + b] = s;
        }
      for (int m = 0; m < np; ++m)
        for (int n = 0; n < np; ++n) {
          double s = 0;
          for (int q = 0; q < nq; ++q) s += g.dV[q] * R.psi[q][m] * R.psi[q][n];
          M1[m * np + n] = s;
        }
      const bool solid = lv.region[e] == 1;

      // load operator: rho (f_h, phi) on momentum rows, columns = nodal force
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
          for (int c = 0; c < D; ++c)
            if (finest) TL.add(rowm[a * D + c], (int64_t)D * nodes[b] + c, 0, rho * M2[a * nb + b]);

      if (solid) {
        const int64_t* dps = dof.ps;
        for (int r = 0; r < nbD; ++r)
          for (int s = 0; s < nbD; ++s) madd(dofd[r], dofd[s], P_G, Ksym[r * nbD + s]);
        for (int m = 0; m < np; ++m)
          for (int r = 0; r < nbD; ++r) {
            madd(dofd[r], dps[m], P_BASE, -Bdiv[m * nbD + r]);
            T.add(dps[m], dofd[r], P_BASE, -Bdiv[m * nbD + r]);
          }
        for (int m = 0; m < np; ++m)
          for (int n = 0; n < np; ++n) T.add(dps[m], dps[n], P_C, -M1[m * np + n]);
        for (int a = 0; a < nb; ++a)
          for (int c = 0; c < D; ++c) {
            const int64_t r = dofu[a * D + c];
            if (ph.k_mass == 0) {
              double lump = 0;
              for (int b = 0; b < nb; ++b) lump += M2[a * nb + b];
              T.add(r, r, P_BASE, lump);
              if (inv_dt != 0.0) tadd(r, dofd[a * D + c], -inv_dt * lump);
            } else {
              for (int b = 0; b < nb; ++b) {
                T.add(r, dofu[b * D + c], P_BASE, M2[a * nb + b]);
                if (inv_dt != 0.0) tadd(r, dofd[b * D + c], -inv_dt * M2[a * nb + b]);
              }
            }
          }
        if (inv_dt != 0.0)
          for (int a = 0; a < nb; ++a)
            for (int b = 0; b < nb; ++b)
              for (int c = 0; c < D; ++c)
                tadd(dofd[a * D + c], dofu[b * D + c], rho * inv_dt * M2[a * nb + b]);
        continue;
      }

      // ---------------- fluid element ----------------
      const int64_t* dpf = dof.pf;
      for (int r = 0; r < nbD; ++r)
        for (int s = 0; s < nbD; ++s) madd(rowm[r], dofu[s], P_MU, Ksym[r * nbD + s]);
      for (int m = 0; m < np; ++m)
        for (int r = 0; r < nbD; ++r) {
          madd(rowm[r], dpf[m], P_BASE, -Bdiv[m * nbD + r]);
          T.add(dpf[m], dofu[r], P_BASE, -Bdiv[m * nbD + r]);
        }
      const double kel = ph.ale_k == 0 ? 1.0 / coarse_vol[lv.parent0[e]] : 1.0;
      for (int a = 0; a < nb; ++a) {
        if (lv.solid_side[nodes[a]]) continue;   // ALE test functions vanish on the interface
        for (int c = 0; c < D; ++c)
          for (int s = 0; s < nbD; ++s)
            T.add(dofd[a * D + c], dofd[s], P_BASE, kel * Ksym[(a * D + c) * nbD + s]);
      }
      if (inv_dt != 0.0)
        for (int a = 0; a < nb; ++a)
          for (int b = 0; b < nb; ++b)
            for (int c = 0; c < D; ++c)
              tadd(rowm[a * D + c], dofu[b * D + c], rho * inv_dt * M2[a * nb + b]);
      if (!have_w) continue;
      // the pattern of the advective terms, whatever their values (an
      // entry stays when w vanishes there)
      advective_terms(R, lv, ph, g, e, dof, *w_level, finest,
                      [&](int target, int64_t r, int64_t c, int p, double) {
                        (target == T_OP ? T : (target == T_TIME ? TT : TL)).add_always(r, c, p, 0.0);
                      });
    }
  };
  // Contiguous element ranges on host threads; their triplets are joined in
  // element order, so the summation order (and every value) is that of one
  // pass over the elements.
  Triplets T, TL, TT;
  const int64_t nE = lv.nE;
  {
    const int nthr = (int)std::min<int64_t>(
        std::max(1u, std::min(16u, std::thread::hardware_concurrency())), nE / 256 + 1);
    std::vector<Triplets> cT(nthr), cL(nthr), cTT(nthr);
    parallel_ranges(nthr, 1, [&](int64_t t0, int64_t t1) {
      for (int64_t t = t0; t < t1; ++t)
        run_elements(nE * t / nthr, nE * (t + 1) / nthr, cT[t], cL[t], cTT[t]);
    });
    T.join(cT);
    TL.join(cL);
    TT.join(cTT);
  }

  // unreduced pattern with pieces
  CsrHost full;
  std::vector<double> fp[4];
  to_csr(T, lv.N, lv.N, 4, full, fp);
  T = Triplets();

  // reduced pattern: Dirichlet rows and columns removed, unit diagonal
  // (rows counted, then filled, on host threads)
  CsrHost& A = op.A;
  A.nrows = A.ncols = lv.N;
  A.rowptr.assign(lv.N + 1, 0);
  parallel_ranges(lv.N, 4096, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int64_t c = 1;
      if (!lv.dir[i]) {
        c = 0;
        for (int64_t k = full.rowptr[i]; k < full.rowptr[i + 1]; ++k) c += !lv.dir[full.col[k]];
      }
      A.rowptr[i + 1] = c;
    }
  });
  for (int64_t i = 0; i < lv.N; ++i) A.rowptr[i + 1] += A.rowptr[i];
  const int64_t annz = A.rowptr[lv.N];
  A.col.assign(annz, 0);
  parallel_ranges(lv.N, 4096, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int64_t o = A.rowptr[i];
      if (lv.dir[i]) {
        A.col[o] = (int32_t)i;
        continue;
      }
      for (int64_t k = full.rowptr[i]; k < full.rowptr[i + 1]; ++k)
        if (!lv.dir[full.col[k]]) A.col[o++] = full.col[k];
    }
  });
  for (int p = 0; p < 4; ++p) op.piece[p].resize(annz);

  if (finest) {
    // load and time operators with their Dirichlet rows removed (the time
    // operator keeps every column: the previous state carries the previous
    // Dirichlet data; its affine pieces are the operator's when theta < 1:
    // the explicit part carries G and mu)
    {
      CsrHost L;
      std::vector<double> lp[4];
      to_csr(TL, lv.N, (int64_t)D * lv.N2, 1, L, lp);
      TL = Triplets();
      drop_dirichlet_rows(lv, L, lp, 1, op.load, &op.load.val);
    }
    {
      CsrHost Tc;
      std::vector<double> tp[4];
      to_csr(TT, lv.N, lv.N, 4, Tc, tp);
      TT = Triplets();
      drop_dirichlet_rows(lv, Tc, tp, 4, op.time, op.time_piece);
    }
    if (have_w) {
      if (plan) {
        for (int p = 0; p < 4; ++p) {
          plan->stat[p] = fp[p];
          plan->tstat[p] = op.time_piece[p];
        }
        plan->lstat = op.load.val;
      }
      add_advective(lv, ph, *w_level, true,
                    AdvTargets{&full, fp, false, &op.time, op.time_piece, &op.load, &op.load.val},
                    plan && slots_fit(full, &op.time, &op.load) ? plan : nullptr, nullptr);
    }
    reduce_values(lv, full, fp, op);
    lift_values(lv, full, fp, op);
    combine_values(op.time_piece, Gmod, invlam, ph.mu, op.time.val);
    op.full = std::move(full);
    for (int p = 0; p < 4; ++p) op.full_piece[p] = std::move(fp[p]);
  } else {
    reduce_values(lv, full, fp, op);
    if (have_w) {
      if (plan)
        for (int p = 0; p < 4; ++p) plan->stat[p] = op.piece[p];
      add_advective(lv, ph, *w_level, false,
                    AdvTargets{&op.A, op.piece, true, nullptr, nullptr, nullptr, nullptr},
                    plan && slots_fit(op.A, nullptr, nullptr) ? plan : nullptr, nullptr);
    }
  }
  combine_values(op.piece, Gmod, invlam, ph.mu, A.val);
  if (plan) plan->ready = have_w;
}

void reassemble_level(const Level& lv, const Physics& ph, const AdvectionPlan& plan,
                      const std::vector<double>& w_level, bool finest, LevelOperator& op) {
  if (!plan.ready) throw std::logic_error("no re-assembly plan for this level");
  const std::vector<int32_t>* replay = plan.slots.empty() ? nullptr : &plan.slots;
  if (finest) {
    for (int p = 0; p < 4; ++p) {
      copy_values(plan.stat[p], op.full_piece[p]);
      copy_values(plan.tstat[p], op.time_piece[p]);
    }
    copy_values(plan.lstat, op.load.val);
    add_advective(lv, ph, w_level, true,
                  AdvTargets{&op.full, op.full_piece, false, &op.time, op.time_piece, &op.load,
                             &op.load.val},
                  nullptr, replay);
    reduce_values(lv, op.full, op.full_piece, op);
    lift_values(lv, op.full, op.full_piece, op);
    combine_values(op.time_piece, op.G, op.invlam, op.mu, op.time.val);
  } else {
    for (int p = 0; p < 4; ++p) copy_values(plan.stat[p], op.piece[p]);
    add_advective(lv, ph, w_level, false,
                  AdvTargets{&op.A, op.piece, true, nullptr, nullptr, nullptr, nullptr}, nullptr,
                  replay);
  }
  combine_values(op.piece, op.G, op.invlam, op.mu, op.A.val);
}

}  // namespace fsgmg
