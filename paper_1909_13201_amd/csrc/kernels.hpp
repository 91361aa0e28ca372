// Device data views and kernel launchers of the fsgmg library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fsgmg {

// Level operator in node-block form.  Node row blocks rb in [0, 2*N2): the
// D scalar rows of one Q2 node's d-equations (rb < N2) or u-equations.
//   NN: D x D blocks against a node's d or u unknowns (column = scalar offset
//       of the block's first column), values row-major per block;
//   NP: D x 1 columns against one pressure unknown.
// Pressure rows p in [0, Nps + Npf):
//   PN: 1 x D rows against a node block; PP: scalar entries.
// Level operator in sliced-ELL node-block form.  Rows are "units": node rows
// (dim outputs: the d or u components of one Q2 node) and pressure rows (one
// output).  Each class is cut into slices of 64 rows (rows sorted by length
// inside windows of 1,024 so a slice holds rows of similar length); slice s
// stores the k-th entry of its row r at entry index off[s] + 64 k + r, so a
// wavefront reads consecutive entries.  Entry kinds: node rows x node columns
// (dim x dim block, row-major), node rows x pressure columns (dim values),
// pressure rows x node columns (dim values), pressure rows x pressure columns
// (one value).  Padding entries have column 0 and value 0.
template <typename T>
struct BOpView {
  int64_t nrb, npr;          // node rows (2 N2), pressure rows (Nps + Npf)
  int64_t nsn, nsp;          // slices of the node / pressure class
  const int32_t* nrow_off;   // node row -> first output unknown
  const int32_t* prow_off;   // pressure row -> output unknown
  // node class: per slice rows[64] (-1 = padding), widths and entry offsets
  const int32_t* n_rows;
  const int32_t* n_wa;
  const int32_t* n_wb;
  const int64_t* n_oa;
  const int64_t* n_ob;
  const int32_t* n_ca;       // per entry: offset of the column node's first unknown
  const int32_t* n_cb;       // per entry: pressure column
  const T* n_va;             // dim*dim per entry
  const T* n_vb;             // dim per entry
  // pressure class
  const int32_t* p_rows;
  const int32_t* p_wa;
  const int32_t* p_wb;
  const int64_t* p_oa;
  const int64_t* p_ob;
  const int32_t* p_ca;
  const int32_t* p_cb;
  const T* p_va;             // dim per entry
  const T* p_vb;             // one per entry
};

// Transfer between level l-1 (coarse) and l (fine), node-level form.
template <typename T>
struct TransferView {
  int64_t N2f, N2c, Npsf, Npff, Npsc, Npfc;
  int64_t offu_f, offps_f, offpf_f, offu_c, offps_c, offpf_c;
  const int32_t* pn_ptr;   // fine node -> coarse nodes
  const int32_t* pn_col;
  const T* pn_val;
  const int32_t* rn_ptr;   // coarse node -> fine nodes (transpose of pn)
  const int32_t* rn_col;
  const T* rn_val;
  const int32_t* pps_ptr;  // fine p^s -> coarse p^s (local indices)
  const int32_t* pps_col;
  const T* pps_val;
  const int32_t* ppf_ptr;
  const int32_t* ppf_col;
  const T* ppf_val;
  const int32_t* rps_ptr;  // coarse p^s -> fine p^s
  const int32_t* rps_col;
  const T* rps_val;
  const int32_t* rpf_ptr;
  const int32_t* rpf_col;
  const T* rpf_val;
  const uint8_t* flags_f;  // per node: 1 solid-side, 2 d Dirichlet, 4 u Dirichlet
  const uint8_t* flags_c;
};

// Schwarz blocks of one level.  W holds, per block, the rows of the block
// inverse that belong to unknowns the block owns, column-major with the
// owned-row count padded to mpad (a multiple of the vector width).
struct BlocksView {
  int64_t nblk, njac;
  const int64_t* dof_ptr;   // nblk + 1
  const int32_t* dofs;
  const int32_t* own_ptr;   // nblk + 1
  const int32_t* own_dof;   // global DOF of each owned row
  const int32_t* own_loc;   // local index (in the block) of each owned row
  const int64_t* w_off;     // element offset of each block in W
  const int32_t* mpad;      // padded owned-row count per block
  const int32_t* jac;       // DOFs in no block
  const void* jac_inv;      // 1 / A_ii in the vector precision
  int max_n, max_mpad;
  // transposed apply: DOF -> positions in the per-block output buffer
  const int32_t* tpos_ptr;  // N + 1
  const int32_t* tpos;
  // launch order of the sweeps: workgroup b works on block order[b]; the
  // blocks are sorted by decreasing inverse size so that the largest start
  // first (longest-processing-time-first over the CUs)
  const int32_t* order;
  // rows of the level operator for the fused residual: block j's rows
  // A[I_j, :] as ELL of width rows_w[j], column-major (entry k of local row i
  // at rows_off[j] + k * n_j + i), padding entries point at the row's own
  // unknown with value 0; the Jacobi unknowns' rows likewise (entry k of
  // Jacobi row q at k * njac + q); values in the vector precision
  const int64_t* rows_off;
  const int32_t* rows_w;
  const int32_t* rows_col;
  const void* rows_val;
  int jrow_w;
  const int32_t* jrow_col;
  const void* jrow_val;
};

enum class WPrec { F64 = 0, F32 = 1, BF16 = 2 };

// ---- level operator ----
// lanes: 1, 2, 4, 8 or 16 lanes per row (the entries of a row are dealt
// round-robin)
template <typename T>
void launch_spmv(const BOpView<T>& A, int D, const T* x, const T* b, T* y, bool residual,
                 hipStream_t s, int lanes = 1);

// scalar CSR (FP64): y = A x (+ beta y)
void launch_csr_spmv(int64_t nrows, const int64_t* rowptr, const int32_t* col, const double* val,
                     const double* x, double* y, double beta, hipStream_t s);

// ---- transfers (mode 0: b_c = D_c R r_f, 1: x_f += D_f P x_c,
//      2: b_c = (D_f P)^T r_f, 3: x_f += (D_c R)^T x_c) ----
template <typename T>
void launch_transfer(const TransferView<T>& t, int D, int mode, const T* in, T* out,
                     hipStream_t s, int lanes = 8);

// ---- smoother: x = (first ? 0 : x) + omega * B r  (transpose: B^T) ----
// threads: workgroup width of the forward sweep (256 / 512 / 1024, 0 = by
// block count); a negative value selects non-temporal loads of the inverses
template <typename TV>
void launch_smooth(const BlocksView& B, WPrec wp, const void* W, const TV* r, TV* x, TV* tbuf,
                   double omega, bool first, bool transpose, int64_t N, hipStream_t s,
                   int threads = 0, int split = 1);

// ---- fused sweep: the residual b - A xin of every block's rows (and of the
// Jacobi rows) is formed inside the launch from B.rows_* (first: xin = 0,
// residual = b), then xout[own] = (first ? 0 : xin[own]) + omega (W_j r)[own],
// xout[jac] likewise.  Additive sweep: xout != xin, every entry of xout is
// written.  Multiplicative colour step (B views one colour, all rows owned,
// no Jacobi rows): xin == xout, omega 1, first 0 (the blocks of a colour
// neither read nor write each other's unknowns) ----
template <typename TV>
void launch_smooth_fused(const BlocksView& B, WPrec wp, const void* W, const TV* b, const TV* xin,
                         TV* xout, double omega, bool first, hipStream_t s, int threads = 0);
// gather B.rows_* / B.jrow_* from the level's FP64 CSR (values cast to TV)
template <typename TV>
void launch_block_rows(const BlocksView& B, const int64_t* rowptr, const int32_t* col,
                       const double* val, hipStream_t s);
// multiplicative sweep end: y[jac] += (b - A y)[jac] / A_jj, then
// x = (first ? 0 : x) + omega (y - (first ? 0 : x))
template <typename TV>
void launch_mult_finish(const BlocksView& B, const TV* b, TV* y, TV* x, int64_t N, double omega,
                        bool first, hipStream_t s);

// ---- several right-hand sides on one operator (K <= 64 columns, entry
// (i, c) at i * K + c): Y = B - A X or A X; restriction (mode 0) /
// prolongation (mode 1, adds) of K columns; X = Ainv B for the dense coarse
// inverse; block apply X[own] = (first ? 0 : X[own]) + omega (W_j R[I_j])[own]
// on the matrix cores (FP64 vectors with FP64 inverses, FP32 vectors with
// FP32 or BF16 inverses), Jacobi unknowns likewise ----
constexpr int kMaxRhs = 64;
constexpr int kMaxRhsBlock = 1024;   // largest block (unknowns) of the K-column block apply
template <typename T>
void launch_spmm(const BOpView<T>& A, int D, const T* X, const T* B, T* Y, int K, bool residual,
                 hipStream_t s);
template <typename T>
void launch_transfer_mc(const TransferView<T>& t, int D, int mode, const T* in, T* out, int K,
                        hipStream_t s);
template <typename TV>
void launch_dense_mc(int64_t n, const double* Ainv, const TV* B, TV* X, int K, hipStream_t s);
template <typename TV>
void launch_smooth_mc(const BlocksView& B, WPrec wp, const void* W, const TV* R, TV* X, int K,
                      double omega, bool first, hipStream_t s);
// transposed K-column sweep: T[I_j] = W_j^T R[own_j] per block (Wt: the
// transposed inverses, column-major over n_j padded to the vector width, at
// wt_off[j]; T: one K-column row per block entry), then X[i] = (first ? 0 :
// X[i]) + omega (fixed-order sum over the blocks containing i), Jacobi
// unknowns likewise
template <typename TV>
void launch_smooth_mc_t(const BlocksView& B, WPrec wp, const void* Wt, const int64_t* wt_off,
                        const TV* R, TV* X, TV* T, int64_t N, int K, double omega, bool first,
                        hipStream_t s);
void launch_transpose_blocks(const BlocksView& B, WPrec wp, const void* W, const int64_t* wt_off,
                             void* Wt, hipStream_t s);

// dst_mapped[i] = src[i], i < n: dst_mapped is the device address of pinned
// host memory (hipHostGetDevicePointer); the host reads it after the stream
// has passed the launch
void launch_store_host(const double* src, double* dst_mapped, int n, hipStream_t s);

// one read pass over `bytes` of zero-filled device memory (cache eviction
// before a timed launch); sink is a separate 4-byte device word
void launch_flush(const void* buf, int64_t bytes, uint32_t* sink, hipStream_t s);

// ---- K-column Krylov (FP64, K <= 64 unknown-major columns; basis vector i
// of a K-column block at V + i * ld; h, out: nv x K, entry (i, c) at i * K + c;
// `part` holds krylov_mc_partials() doubles; fixed-order reductions) ----
int krylov_mc_partials();
void launch_mc_mdot(const double* V, int64_t ld, int nv, const double* w, int64_t N, int K,
                    double* part, double* out, hipStream_t s);
// w -= V h, then out = V^T w (per column)
void launch_mc_maxpy_mdot(const double* V, int64_t ld, int nv, const double* h, double* w,
                          int64_t N, int K, double* part, double* out, hipStream_t s);
// w -= V h, then out[c] = |w[:, c]|
void launch_mc_maxpy_norm(const double* V, int64_t ld, int nv, const double* h, double* w,
                          int64_t N, int K, double* part, double* out, hipStream_t s);
// y[:, c] = scale[c] w[:, c]
void launch_mc_scale(int64_t N, int K, const double* scale, const double* w, double* y,
                     hipStream_t s);
// x[:, c] += sum_{i < nv} y[i, c] Z_i[:, c]
void launch_mc_update(const double* Z, int64_t ld, int nv, const double* y, double* x, int64_t N,
                      int K, hipStream_t s);

// ---- multiplicative sweep, one colour: B views the colour's blocks (all
// rows owned, mutually uncoupled) and no Jacobi unknowns, or no blocks and
// the Jacobi unknowns.  e[I_j] += W_j r[I_j] (transpose: W_j^T r[I_j]);
// Jacobi: e[i] += r[i] / A_ii.  p0..p1: positions of the colour's blocks in
// B.dofs (transposed step, which goes through tbuf) ----
template <typename TV>
void launch_smooth_colour(const BlocksView& B, WPrec wp, const void* W, const TV* r, TV* e,
                          TV* tbuf, int64_t p0, int64_t p1, bool transpose, hipStream_t s,
                          int threads = 0, int split = 1);
// x = (first ? 0 : x) + a e
template <typename TV>
void launch_add_scaled(int64_t n, double a, const TV* e, TV* x, bool first, hipStream_t s);

// ---- block setup ----
// Block setup over a list of block ids (jlist[b], b < nb; launch b of the
// list works on block jlist[b]).  Dense copies of the blocks' principal
// submatrices, row stride np = n rounded up to 16, identity in the padding;
// dense_off[b] = element offset of list entry b.
// The dense copies, the factorization and the extraction run in the factor
// type: FP64 (f32 = false) for FP64 inverses, FP32 (f32 = true) for FP32 and
// BF16 inverses; `dense` holds elements of that type.
void launch_gather_blocks(const int32_t* jlist, int64_t nb, const BlocksView& B,
                          const int64_t* rowptr, const int32_t* col, const double* val,
                          const int64_t* dense_off, void* dense, bool f32, int max_n,
                          hipStream_t s);
// Blocked in-place Gauss-Jordan inversion with partial pivoting of the padded
// dense blocks (16-column panels, MFMA trailing updates in the factor type);
// sigma[sigma_off[b] + q] receives the column permutation that completes the
// inverse; status[j] = 1 on a zero pivot.  max_n bounds the listed blocks'
// sizes (it sizes the LDS); invert_blocks_lds: the LDS bytes one workgroup
// needs for blocks of padded size np_max.
size_t invert_blocks_lds(int np_max, bool f32);
void launch_invert_blocks(const int32_t* jlist, int64_t nb, const int64_t* dof_ptr,
                          const int64_t* dense_off, const int64_t* sigma_off, void* dense,
                          bool f32, int32_t* sigma, int32_t* status, int max_n, hipStream_t s);
void launch_extract_owned(const int32_t* jlist, int64_t nb, const BlocksView& B,
                          const int64_t* dense_off, const int64_t* sigma_off, const void* dense,
                          bool f32, const int32_t* sigma, WPrec wp, void* W, hipStream_t s);

// Dense inverse of the coarse-level matrix (CSR, n rows) by blocked
// Gauss-Jordan with partial pivoting spread over the GPU.  launch_coarse_factor
// gathers the CSR into the work matrix a (np x np, np = n rounded up to 16,
// identity tail) and factors it; piv (np) receives the pivot row of every
// column, status[0] = 1 on a zero pivot (must be 0 on entry).  Where
// coarse_register_path(np) holds and a2 (a second np x np matrix) and src
// (np) are given, 16-column panels held in registers alternate between a
// and a2; otherwise panels of nb (8 or 4, coarse_panel_width) columns in LDS
// are applied to a in place, with ybuf (nb x np) as scratch.  Returns the
// matrix that holds the result.  After piv has been turned into the column
// permutation sigma (inverse[:, q] = result[:, sigma[q]]),
// launch_coarse_finish writes the n x n inverse and its transpose.
// 8 or 4 (LDS panels), or coarse_wide_panel() when np x 5 doubles exceed the
// LDS: then np must be a multiple of coarse_wide_panel() and the scratch
// after the work matrix must hold (3 W + 1) np + 2 W doubles (W the width)
int coarse_panel_width(int64_t np, int max_lds);
int coarse_wide_panel();
bool coarse_register_path(int64_t np);
// sigma from the pivot list on the device (one workgroup, coarse_sigma_lds(np)
// bytes of LDS); the identity when status[0] reports a zero pivot
size_t coarse_sigma_lds(int64_t np);
void launch_coarse_sigma(const int32_t* piv, int64_t np, const int32_t* status, int32_t* sig,
                         hipStream_t s);
const double* launch_coarse_factor(int64_t n, int64_t np, const int64_t* rp, const int32_t* col,
                                   const double* val, double* a, double* ybuf, double* a2,
                                   int32_t* src, int32_t* piv, int32_t* status, int nb,
                                   hipStream_t s);
void launch_coarse_finish(const double* a, int64_t np, int64_t n, const int32_t* sigma, double* inv,
                          double* invT, hipStream_t s);

// ---- coarse solve: y = Ainv * x (transpose: Ainv^T x), FP64 matrix ----
template <typename TV>
void launch_dense_gemv(int64_t n, const double* Ainv, bool transpose, const TV* x, TV* y,
                       hipStream_t s);

// ---- Krylov (FP64): partial sums per workgroup, then a fixed-order
// reduction kernel that writes out[0..k) (deterministic) ----
int krylov_partials();
void launch_mdot(const double* V, int64_t ld, int k, const double* w, int64_t N, double* part,
                 double* out, hipStream_t s);
void launch_maxpy_mdot(const double* V, int64_t ld, int k, const double* h, double* w, int64_t N,
                       double* part, double* out, hipStream_t s);
// w -= V h; out[0] = ||w||
void launch_maxpy_norm(const double* V, int64_t ld, int k, const double* h, double* w,
                       int64_t N, double* part, double* out, hipStream_t s);
// out[0] = ||w||
void launch_norm2(const double* w, int64_t N, double* part, double* out, hipStream_t s);
void launch_scale_copy(const double* w, const double* beta, double* v, int64_t N, hipStream_t s);
void launch_gemv_update(const double* Z, int64_t ld, int k, const double* y, double* x,
                        int64_t N, hipStream_t s);

// ---- elementwise ----
template <typename TA, typename TB>
void launch_cast(const TA* a, TB* b, int64_t n, hipStream_t s);
void launch_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s);
void launch_load_rhs(int64_t n, const int64_t* rowptr, const int32_t* col, const double* val,
                     const double* f, const double* lift, double* b, hipStream_t s);
// b = L f + g lift + T x_prev (load operator L and time operator T in CSR)
void launch_time_rhs(int64_t n, const int64_t* lrp, const int32_t* lcol, const double* lval,
                     const double* f, const double* lift, double g, const int64_t* trp,
                     const int32_t* tcol, const double* tval, const double* x_prev, double* b,
                     hipStream_t s);
// out[0] = sum over unmasked i of a_i b_i
void launch_masked_dot(const double* a, const uint8_t* mask, const double* b, int64_t n,
                       double* part, double* out, hipStream_t s);
template <typename T>
void launch_fill(T* p, T v, int64_t n, hipStream_t s);
// out[map[k]] = v[k] (either output may be null)
void launch_scatter(int64_t n, const double* v, const int64_t* map, double* out64, float* out32,
                    hipStream_t s);
void launch_recombine(int64_t n, const double* p0, const double* p1, const double* p2,
                      const double* p3, double c1, double c2, double c3, double* out64,
                      float* out32, hipStream_t s);

// ---- re-assembly of the advective terms on the device (2D) ----
// Reference element tables, RefElem's layout (Gauss weights, phi, dphi,
// d2phi, psi, dpsi at the 27-point / 27-function / 8-function maxima).
constexpr int kAdvQ = 27, kAdvB = 27, kAdvP = 8;
constexpr int kRefWq = 0, kRefPhi = kRefWq + kAdvQ, kRefDphi = kRefPhi + kAdvQ * kAdvB,
              kRefD2phi = kRefDphi + kAdvQ * kAdvB * 3, kRefPsi = kRefD2phi + kAdvQ * kAdvB * 9,
              kRefDpsi = kRefPsi + kAdvQ * kAdvP, kRefSize = kRefDpsi + kAdvQ * kAdvP * 3;
struct AdvElemView {
  int64_t nfluid = 0;             // fluid elements, in the order their terms are added
  int per = 0;                    // terms each element emits
  const int32_t* elems = nullptr;
  const int64_t* elem_nodes = nullptr;   // nE x 9
  const double* X = nullptr;             // N2 x 2 node coordinates
  const int32_t* node_fine = nullptr;    // the finest-level node of each level node
  const double* x = nullptr;             // finest-level vector; velocity at off_u
  int64_t off_u = 0;
  const double* ref = nullptr;           // reference tables (kRefSize doubles)
  double rho = 1, mu = 1, inv_dt = 0, theta = 1;
  int supg = 1, finest = 0;
  double* emit = nullptr;                // nfluid x per values
  int32_t* flag = nullptr;               // bit 1: an element emitted another number of terms
};
// Every fluid element's advective terms (the host assembly's order and
// arithmetic) into v.emit; one thread per element.
void launch_adv_elements(const AdvElemView& v, hipStream_t s);
// dst[arr[i]][slot[i]] = stat[i] + sum of emit[em[k]], k in [ptr[i], ptr[i+1]);
// where red[i] >= 0 (the finest level's operator arrays) also
// dst_red[arr[i]][red[i]] = the same value.
struct AdvGatherView {
  int64_t n = 0;
  const uint8_t* arr = nullptr;
  const int64_t* slot = nullptr;
  const double* stat = nullptr;
  const int64_t* ptr = nullptr;
  const int64_t* em = nullptr;
  const int64_t* red = nullptr;
  const double* emit = nullptr;
  double* dst[12] = {};
  double* dst_red[4] = {};
};
void launch_adv_gather(const AdvGatherView& g, hipStream_t s);
// lift pieces of the listed rows: lift[p][row[i]] = - sum over k of
// full[p][kk[k]] g[k], k in [ptr[i], ptr[i+1]), in that order
void launch_adv_lift(int64_t n, const int64_t* row, const int64_t* ptr, const int64_t* kk,
                     const double* g, const double* f0, const double* f1, const double* f2,
                     const double* f3, double* l0, double* l1, double* l2, double* l3,
                     hipStream_t s);
// out[j] = in[perm[j]]
void launch_permute_values(int64_t n, const int64_t* perm, const double* in, double* out,
                           hipStream_t s);
// flag[0] |= 1 when any of x[0 .. n) is NaN or infinite
void launch_nonfinite_flag(int64_t n, const double* x, int32_t* flag, hipStream_t s);

// ---- allocation-free scratch ----
// A file-scope device array of kNoAllocScratchBytes bytes (one copy per GPU,
// held until the process ends) for entry points that must not allocate.
// noalloc_scratch(device) returns its device address on `device` (looked up
// once per device with that device current, then cached), or nullptr and a
// message when the lookup fails.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
void* noalloc_scratch(int device, const char** err);

}  // namespace fsgmg
