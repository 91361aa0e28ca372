// Host-side setup structures of the fsgmg library: nested structured mesh,
// J2 unknown layout, sparse matrices, transfers and Schwarz block index sets.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fsgmg.h"

namespace fsgmg {

constexpr int kMaxDim = 3;

// Compressed sparse rows on the host (64-bit row pointers, 32-bit columns).
struct CsrHost {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
  int64_t nnz() const { return rowptr.empty() ? 0 : rowptr.back(); }
};

CsrHost csr_transpose(const CsrHost& A);

// One level of the nested hierarchy.  Q2 nodes and Q1 vertices are numbered
// x-fastest; the level vector is [d | p^s | u | p^f] (see fsgmg.h).
struct Level {
  int D = 2, l = 0;
  int ne[kMaxDim] = {1, 1, 1};   // elements per axis
  int nn[kMaxDim] = {1, 1, 1};   // Q2 node lines per axis
  int nv[kMaxDim] = {1, 1, 1};   // Q1 vertex lines per axis
  int64_t nE = 0, N2 = 0, NV = 0;
  int nb = 9, npv = 4;           // Q2 / Q1 functions per element
  std::vector<int8_t> region;    // per element
  std::vector<int32_t> parent0;  // level-0 element containing each element
  std::vector<int64_t> elem_nodes;  // nE * nb
  std::vector<int64_t> elem_verts;  // nE * npv
  std::vector<double> xref, X;      // N2 * D reference / physical coordinates
  std::vector<uint8_t> solid_side, fluid_touch;  // per node
  std::vector<uint8_t> vert_solid, vert_fluid;   // per vertex
  int64_t Nps = 0, Npf = 0, off_ps = 0, off_u = 0, off_pf = 0, N = 0;
  std::vector<int64_t> ps_of_vert, pf_of_vert;   // DOF index or -1
  std::vector<uint8_t> dir;      // per DOF
  std::vector<double> dir_val;   // per DOF

  int64_t node_index(const int* ix) const;
  int64_t vertex_node(int64_t v) const;   // Q2 node at a Q1 vertex
  void node_ijk(int64_t n, int* ix) const;
};

// Build level l of the hierarchy described by `mesh`.
void build_level(const fsgmg_mesh_desc& mesh, int l, Level& lv);

// Assembled level operator: reduced matrix A (Dirichlet rows/columns
// eliminated, unit diagonal) and its affine pieces on the same pattern,
// A = base + G*pG + invlam*pC + mu*pMu.  For the finest level also the
// unreduced pieces needed by gradients and the Dirichlet lift pieces.
struct LevelOperator {
  CsrHost A;
  std::vector<double> piece[4];     // reduced pieces (base has the unit diagonal)
  CsrHost full;                     // unreduced pattern (finest only)
  std::vector<double> full_piece[4];
  std::vector<double> lift_piece[4];  // finest: lift = sum coef * lift_piece
  CsrHost load;                     // finest: N x D*N2 load operator
  CsrHost time;                     // finest: the previous state's operator of a time
                                    // step (the terms carrying 1/dt, and -(1 - theta)
                                    // times the steady momentum-row terms), Dirichlet
                                    // rows removed
  std::vector<double> time_piece[4];  // its affine pieces
  double G = 0, invlam = 0, mu = 0;
};

struct Physics {
  double E, nu, mu, rho, inv_dt;
  double theta;      // weight of the steady momentum-row terms (1 = backward Euler)
  int supg, ale_k, k_mass;
  const double* w;   // finest-level nodal advecting velocity or nullptr
  int n_levels;
};

void lame(double E, double nu, double& G, double& invlam);

// The reference element's tables (Gauss weights, Q2 values, first and second
// derivatives, Q1 values and derivatives) at the 27 / 27 / 8 maxima of 3D,
// flattened in that order (the device re-assembly's layout).
std::vector<double> reference_tables(int D);

// What re-assembling a level about a new advecting velocity needs: the sums
// of every term that does not depend on it, on the patterns the advective
// terms (convection and SUPG) are added to.  Those patterns hold every
// entry an advective term can reach, whatever the velocity, so they are
// fixed.  stat: the unreduced pieces on the finest level, the reduced ones
// elsewhere; tstat / lstat: the finest level's time and load operators
// (Dirichlet rows removed); elems: the fluid elements in the order their
// terms are added (colour by colour), each emitting per terms; slots: the
// value slot (-1: none) of every advective term in that order, dest its
// array (4 target + piece; target 0 the operator, 1 the time operator, 2
// the load operator).
struct AdvectionPlan {
  std::vector<double> stat[4];
  std::vector<double> tstat[4];
  std::vector<double> lstat;
  std::vector<int32_t> elems;
  std::vector<int32_t> slots;
  std::vector<uint8_t> dest;
  int per = 0;
  bool ready = false;
};

// Assemble level `lv` (finest = true also keeps unreduced pieces, lift and
// load operator).  coarse_vol: level-0 element volumes (ALE k = 1/V).  The
// advective terms are added after the others, element colour by element
// colour, into the fixed pattern; plan != nullptr keeps what
// reassemble_level needs.
void assemble_level(const Level& lv, const Physics& ph, const std::vector<double>& coarse_vol,
                    const std::vector<double>* w_level, bool finest, LevelOperator& op,
                    AdvectionPlan* plan = nullptr);

// The values of `op` (assembled by assemble_level with this plan, patterns
// kept) about a new advecting velocity w_level: equal, bit for bit, to what
// assemble_level gives about it.
void reassemble_level(const Level& lv, const Physics& ph, const AdvectionPlan& plan,
                      const std::vector<double>& w_level, bool finest, LevelOperator& op);

std::vector<double> element_volumes(const Level& lv);

// Node-level transfer from level l-1 (coarse) to level l (fine).
//  P rows: fine Q2 node -> (coarse node, weight); pressure rows: fine p DOF
//  (local p^s / p^f index) -> (coarse local index, weight).
//  R rows: coarse Q2 node -> (fine node, weight, fine-solid-side flag).
struct Transfer {
  CsrHost Pn;        // N2_fine x N2_coarse
  CsrHost Pps, Ppf;  // Nps_f x Nps_c, Npf_f x Npf_c
  CsrHost Rn;        // N2_coarse x N2_fine (= Pn^T)
  CsrHost Rps, Rpf;  // transposes of Pps, Ppf
};

void build_transfer(const Level& fine, const Level& coarse, Transfer& t);

// Expand to full scalar matrices (Dirichlet-masked), for inspection.
CsrHost prolongation_full(const Level& fine, const Level& coarse, const Transfer& t);
CsrHost restriction_full(const Level& fine, const Level& coarse, const Transfer& t);

// Field-split additive Schwarz block index sets of one level.
struct BlockSet {
  std::vector<int64_t> ptr;     // nblk + 1
  std::vector<int32_t> dofs;    // sorted per block
  std::vector<int32_t> owner;   // N, last block containing the DOF, -1 if none
  std::vector<int32_t> jac;     // DOFs in no block (Jacobi)
  std::vector<int64_t> colour_ptr;  // multiplicative sweep: first block of each colour
  int64_t nblk() const { return ptr.empty() ? 0 : (int64_t)ptr.size() - 1; }
};

void build_blocks(const Level& lv, const int* core, int halo, int iface_mult, bool monolithic,
                  BlockSet& bs);

// Order of the multiplicative sweep (Section 3.2): greedy first-fit colouring
// of the blocks in their current order, then the blocks regrouped colour by
// colour with the order inside a colour kept (owner recomputed, colour_ptr
// filled).  Blocks conflict when they share an unknown or the operator
// couples them in either direction; an entry couples when one of the affine
// pieces holds it above kCouplingRel times that piece's largest magnitude in
// the row (parameter-independent, blind to assembly rounding of entries that
// vanish).  Throws std::invalid_argument when two unknowns outside every
// block are coupled (their Jacobi step would then not be the sequential one).
constexpr double kCouplingRel = 1e-14;
void colour_blocks(const CsrHost& A, const std::vector<double>* pieces, int npieces,
                   BlockSet& bs);

}  // namespace fsgmg
