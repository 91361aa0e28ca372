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

void assemble_level(const Level& lv, const Physics& ph, const std::vector<double>& coarse_vol,
                    const std::vector<double>* w_level, bool finest, LevelOperator& op) {
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
  // (operator pieces, load operator, time operator).
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
    auto madd = [&](int64_t r, int64_t c, int p, double v, bool always) {
      const double tv = weighted ? theta * v : v;
      if (always)
        T.add_always(r, c, p, tv);
      else
        T.add(r, c, p, tv);
      if (finest && weighted) TT.add(r, c, p, -(1.0 - theta) * v);
    };
    ElemGeo g;
    static thread_local double Tg[kMaxB][kMaxB][3][3];
    std::vector<double> Ksym(nbD * nbD), Bdiv(np * nbD), M2(nb * nb), M1(np * np);
    std::vector<int64_t> dofd(nbD), dofu(nbD), rowm(nbD), dps(np), dpf(np);
    for (int64_t e = e_begin; e < e_end; ++e) {
      element_geometry(R, lv, e, g);
      const int64_t* nodes = &lv.elem_nodes[e * nb];
      const int64_t* verts = &lv.elem_verts[e * np];
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
      for (int a = 0; a < nb; ++a)
        for (int c = 0; c < D; ++c) {
          dofd[a * D + c] = (int64_t)D * nodes[a] + c;
          dofu[a * D + c] = lv.off_u + (int64_t)D * nodes[a] + c;
        }
      const bool solid = lv.region[e] == 1;
      // momentum rows: S for solid-side nodes, F for fluid nodes
      for (int a = 0; a < nb; ++a)
        for (int c = 0; c < D; ++c)
          rowm[a * D + c] = lv.solid_side[nodes[a]] ? dofd[a * D + c] : dofu[a * D + c];

      // load operator: rho (f_h, phi) on momentum rows, columns = nodal force
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b)
          for (int c = 0; c < D; ++c)
            if (finest) TL.add(rowm[a * D + c], (int64_t)D * nodes[b] + c, 0, rho * M2[a * nb + b]);

      if (solid) {
        for (int m = 0; m < np; ++m) dps[m] = lv.ps_of_vert[verts[m]];
        for (int r = 0; r < nbD; ++r)
          for (int s = 0; s < nbD; ++s) madd(dofd[r], dofd[s], P_G, Ksym[r * nbD + s], false);
        for (int m = 0; m < np; ++m)
          for (int r = 0; r < nbD; ++r) {
            madd(dofd[r], dps[m], P_BASE, -Bdiv[m * nbD + r], false);
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
      for (int m = 0; m < np; ++m) dpf[m] = lv.pf_of_vert[verts[m]];
      for (int r = 0; r < nbD; ++r)
        for (int s = 0; s < nbD; ++s) madd(rowm[r], dofu[s], P_MU, Ksym[r * nbD + s], false);
      for (int m = 0; m < np; ++m)
        for (int r = 0; r < nbD; ++r) {
          madd(rowm[r], dpf[m], P_BASE, -Bdiv[m * nbD + r], false);
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
      double wq[kMaxQ][3], wg[kMaxQ][kMaxB];
      for (int q = 0; q < nq; ++q)
        for (int i = 0; i < D; ++i) {
          double s = 0;
          for (int b = 0; b < nb; ++b) s += (*w_level)[nodes[b] * D + i] * R.phi[q][b];
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
          for (int c = 0; c < D; ++c) madd(rowm[a * D + c], dofu[b * D + c], P_BASE, rho * s, true);
        }
      if (!ph.supg) continue;
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
          double s1 = 0;
          if (!weighted) {
            for (int q = 0; q < nq; ++q) s1 += tw[q] * wg[q][a] * (rho * wg[q][b] + rho * inv_dt * R.phi[q][b]);
          } else {
            // only the steady part carries theta
            double s1s = 0, s1t = 0;
            for (int q = 0; q < nq; ++q) {
              s1s += tw[q] * wg[q][a] * rho * wg[q][b];
              s1t += tw[q] * wg[q][a] * rho * inv_dt * R.phi[q][b];
            }
            s1 = theta * s1s + s1t;
            if (finest)
              for (int c = 0; c < D; ++c) TT.add(rowm[a * D + c], dofu[b * D + c], 0, -(1.0 - theta) * s1s);
          }
          for (int c = 0; c < D; ++c) T.add_always(rowm[a * D + c], dofu[b * D + c], P_BASE, s1);
          if (finest && inv_dt != 0.0) {   // the SUPG time term of s1, on its own
            double st = 0;
            for (int q = 0; q < nq; ++q) st += tw[q] * wg[q][a] * rho * inv_dt * R.phi[q][b];
            for (int c = 0; c < D; ++c) TT.add(rowm[a * D + c], dofu[b * D + c], 0, st);
          }
          double sl = 0;
          for (int q = 0; q < nq; ++q) sl += rho * rho * tw[q] * wg[q][a] * R.phi[q][b];
          if (finest)
            for (int c = 0; c < D; ++c) TL.add(rowm[a * D + c], (int64_t)D * nodes[b] + c, 0, sl);
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
              madd(rowm[a * D + c], dofu[b * D + f], P_MU, -s, true);
            }
      for (int a = 0; a < nb; ++a)
        for (int c = 0; c < D; ++c)
          for (int m = 0; m < np; ++m) {
            double s = 0;
            for (int q = 0; q < nq; ++q) s += tw[q] * wg[q][a] * g.Gp[q][m][c];
            madd(rowm[a * D + c], dpf[m], P_BASE, s, true);
          }
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

  // reduced operator: Dirichlet rows and columns removed, unit diagonal
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
  for (int p = 0; p < 4; ++p) op.piece[p].assign(annz, 0.0);
  A.val.assign(annz, 0.0);
  parallel_ranges(lv.N, 4096, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int64_t o = A.rowptr[i];
      if (lv.dir[i]) {
        A.col[o] = (int32_t)i;
        op.piece[P_BASE][o] = 1.0;
      } else {
        for (int64_t k = full.rowptr[i]; k < full.rowptr[i + 1]; ++k) {
          if (lv.dir[full.col[k]]) continue;
          A.col[o] = full.col[k];
          for (int p = 0; p < 4; ++p) op.piece[p][o] = fp[p][k];
          ++o;
        }
      }
      for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
        A.val[k] = op.piece[P_BASE][k] + Gmod * op.piece[P_G][k] + invlam * op.piece[P_C][k] +
                   ph.mu * op.piece[P_MU][k];
    }
  });

  if (finest) {
    // lift pieces: lift = g on Dirichlet rows, -(A_full g) on free rows
    for (int p = 0; p < 4; ++p) op.lift_piece[p].assign(lv.N, 0.0);
    for (int64_t i = 0; i < lv.N; ++i) {
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
    // load operator with Dirichlet rows removed
    CsrHost L;
    std::vector<double> lp[4];
    to_csr(TL, lv.N, (int64_t)D * lv.N2, 1, L, lp);
    op.load.nrows = lv.N;
    op.load.ncols = (int64_t)D * lv.N2;
    op.load.rowptr.assign(lv.N + 1, 0);
    op.load.col.clear();
    op.load.val.clear();
    for (int64_t i = 0; i < lv.N; ++i) {
      if (!lv.dir[i])
        for (int64_t k = L.rowptr[i]; k < L.rowptr[i + 1]; ++k) {
          op.load.col.push_back(L.col[k]);
          op.load.val.push_back(lp[0][k]);
        }
      op.load.rowptr[i + 1] = (int64_t)op.load.col.size();
    }
    // time operator with Dirichlet rows removed (every column kept: the
    // previous state carries the previous Dirichlet data)
    // (affine pieces like the operator's when theta < 1: the explicit part
    // carries G and mu)
    CsrHost Tc;
    std::vector<double> tp[4];
    to_csr(TT, lv.N, lv.N, 4, Tc, tp);
    op.time.nrows = op.time.ncols = lv.N;
    op.time.rowptr.assign(lv.N + 1, 0);
    op.time.col.clear();
    op.time.val.clear();
    for (int p = 0; p < 4; ++p) op.time_piece[p].clear();
    for (int64_t i = 0; i < lv.N; ++i) {
      if (!lv.dir[i])
        for (int64_t k = Tc.rowptr[i]; k < Tc.rowptr[i + 1]; ++k) {
          op.time.col.push_back(Tc.col[k]);
          for (int p = 0; p < 4; ++p) op.time_piece[p].push_back(tp[p][k]);
          op.time.val.push_back(tp[P_BASE][k] + Gmod * tp[P_G][k] + invlam * tp[P_C][k] +
                                ph.mu * tp[P_MU][k]);
        }
      op.time.rowptr[i + 1] = (int64_t)op.time.col.size();
    }
    op.full = std::move(full);
    for (int p = 0; p < 4; ++p) op.full_piece[p] = std::move(fp[p]);
  }
}

}  // namespace fsgmg
