// fsgmg C ABI: hierarchy setup, field-split additive Schwarz blocks, the
// multigrid V-cycle (and its transpose), right-preconditioned FGMRES with
// classical Gram-Schmidt twice, the adjoint solve and parameter gradients.
//
// Method (paper Sections 3.2-3.3): GMRES preconditioned by one GMG V-cycle;
// damped Richardson with the additive field-split smoother on levels >= 1,
// direct solve on level 0; natural-injection prolongation and the
// equation-routed restriction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "fsgmg.h"
#include "host.hpp"
#include "kernels.hpp"

using namespace fsgmg;

namespace {

struct Fail {
  fsgmg_status st;
  std::string msg;
};

#define HIPCHECK(expr)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) throw Fail{FSGMG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// ---------------------------------------------------------------------------
// node-block operator in sliced-ELL form (see BOpView), and a map from the
// scalar CSR entries to the concatenated value array [n_va | n_vb | p_va | p_vb]
// ---------------------------------------------------------------------------
struct SellClass {
  int64_t nslices = 0, ea = 0, eb = 0;   // slices, entries of kind a / b (padding included)
  std::vector<int32_t> rows, wa, wb, ca, cb;
  std::vector<int64_t> oa, ob;
};

struct BOpHost {
  int64_t nrb = 0, npr = 0;
  std::vector<int32_t> nrow_off, prow_off;
  SellClass node, pres;
  int64_t n_na = 0, n_nb = 0, n_pa = 0, n_pb = 0;   // value counts per region
  std::vector<int64_t> map;
  int64_t nvals() const { return n_na + n_nb + n_pa + n_pb; }
};

namespace {

// Rows' entry lists (CSR of entries, column per entry) -> slices of 64 rows,
// rows sorted by (a-length, b-length) descending inside windows of 1,024.
// pos_a[i] / pos_b[i]: the sliced entry index of CSR entry i.
void make_slices(int64_t nrows, const std::vector<int64_t>& pa, const std::vector<int32_t>& ca,
                 const std::vector<int64_t>& pb, const std::vector<int32_t>& cb, SellClass& S,
                 std::vector<int64_t>& pos_a, std::vector<int64_t>& pos_b) {
  constexpr int64_t C = 64, kWindow = 1024;
  std::vector<int32_t> order(nrows);
  for (int64_t r = 0; r < nrows; ++r) order[r] = (int32_t)r;
  for (int64_t w0 = 0; w0 < nrows; w0 += kWindow) {
    const int64_t w1 = std::min(nrows, w0 + kWindow);
    std::stable_sort(order.begin() + w0, order.begin() + w1, [&](int32_t x, int32_t y) {
      const int64_t ax = pa[x + 1] - pa[x], ay = pa[y + 1] - pa[y];
      if (ax != ay) return ax > ay;
      return pb[x + 1] - pb[x] > pb[y + 1] - pb[y];
    });
  }
  S.nslices = (nrows + C - 1) / C;
  S.rows.assign(S.nslices * C, -1);
  S.wa.assign(S.nslices, 0);
  S.wb.assign(S.nslices, 0);
  S.oa.assign(S.nslices, 0);
  S.ob.assign(S.nslices, 0);
  pos_a.assign(ca.size(), -1);
  pos_b.assign(cb.size(), -1);
  int64_t ea = 0, eb = 0;
  for (int64_t sl = 0; sl < S.nslices; ++sl) {
    int64_t wa = 0, wb = 0;
    for (int64_t r = 0; r < C && sl * C + r < nrows; ++r) {
      const int32_t row = order[sl * C + r];
      S.rows[sl * C + r] = row;
      wa = std::max(wa, pa[row + 1] - pa[row]);
      wb = std::max(wb, pb[row + 1] - pb[row]);
    }
    S.wa[sl] = (int32_t)wa;
    S.wb[sl] = (int32_t)wb;
    S.oa[sl] = ea;
    S.ob[sl] = eb;
    ea += wa * C;
    eb += wb * C;
  }
  S.ea = ea;
  S.eb = eb;
  S.ca.assign(ea, 0);
  S.cb.assign(eb, 0);
  for (int64_t sl = 0; sl < S.nslices; ++sl)
    for (int64_t r = 0; r < C; ++r) {
      const int32_t row = S.rows[sl * C + r];
      if (row < 0) continue;
      for (int64_t k = 0; k < pa[row + 1] - pa[row]; ++k) {
        const int64_t e = S.oa[sl] + k * C + r;
        S.ca[e] = ca[pa[row] + k];
        pos_a[pa[row] + k] = e;
      }
      for (int64_t k = 0; k < pb[row + 1] - pb[row]; ++k) {
        const int64_t e = S.ob[sl] + k * C + r;
        S.cb[e] = cb[pb[row] + k];
        pos_b[pb[row] + k] = e;
      }
    }
}

}  // namespace

BOpHost build_bop(const Level& lv, const CsrHost& A) {
  const int D = lv.D;
  BOpHost b;
  b.nrb = 2 * lv.N2;
  b.npr = lv.Nps + lv.Npf;
  b.map.assign(A.nnz(), -1);
  auto node_col = [&](int64_t c) { return c < lv.off_ps || (c >= lv.off_u && c < lv.off_pf); };
  auto block_off = [&](int64_t c) -> int64_t {
    return c < lv.off_ps ? D * (c / D) : lv.off_u + D * ((c - lv.off_u) / D);
  };
  struct E {
    int64_t key;
    int r, q;
    int64_t k;
  };
  // per class: CSR of entries (kind a: node columns, kind b: pressure columns)
  // and, per scalar entry, (CSR entry, position inside the entry's values)
  std::vector<int64_t> pa[2], pb[2];
  std::vector<int32_t> ca[2], cb[2];
  std::vector<std::pair<int64_t, int>> sa[2], sb[2];   // indexed by scalar entry k
  for (int c = 0; c < 2; ++c) {
    pa[c].assign(1, 0);
    pb[c].assign(1, 0);
  }
  std::vector<int64_t> ka, kb;   // scalar entry of each recorded (CSR entry, offset)
  std::vector<E> ne, pe;
  std::vector<int64_t> ent_a[2], ent_b[2];   // scalar k list per class (parallel to sa/sb)
  auto add_row = [&](int cls, const std::vector<int64_t>& rows_scalar, int nout) {
    ne.clear();
    pe.clear();
    for (int r = 0; r < nout; ++r) {
      const int64_t row = rows_scalar[r];
      for (int64_t k = A.rowptr[row]; k < A.rowptr[row + 1]; ++k) {
        const int64_t c = A.col[k];
        if (node_col(c)) {
          const int64_t bo = block_off(c);
          ne.push_back({bo, r, (int)(c - bo), k});
        } else {
          pe.push_back({c, r, 0, k});
        }
      }
    }
    std::sort(ne.begin(), ne.end(), [](const E& x, const E& y) { return x.key < y.key; });
    std::sort(pe.begin(), pe.end(), [](const E& x, const E& y) { return x.key < y.key; });
    const int wva = cls == 0 ? D * D : D;   // values per entry of kind a
    for (size_t i = 0; i < ne.size(); ++i) {
      if (i == 0 || ne[i].key != ne[i - 1].key) ca[cls].push_back((int32_t)ne[i].key);
      const int off = cls == 0 ? ne[i].r * D + ne[i].q : ne[i].q;
      (void)wva;
      sa[cls].emplace_back((int64_t)ca[cls].size() - 1, off);
      ent_a[cls].push_back(ne[i].k);
    }
    for (size_t i = 0; i < pe.size(); ++i) {
      if (i == 0 || pe[i].key != pe[i - 1].key) cb[cls].push_back((int32_t)pe[i].key);
      sb[cls].emplace_back((int64_t)cb[cls].size() - 1, pe[i].r);
      ent_b[cls].push_back(pe[i].k);
    }
    pa[cls].push_back((int64_t)ca[cls].size());
    pb[cls].push_back((int64_t)cb[cls].size());
  };
  std::vector<int64_t> rs(D);
  for (int64_t rb = 0; rb < b.nrb; ++rb) {
    const int64_t r0 = rb < lv.N2 ? D * rb : lv.off_u + D * (rb - lv.N2);
    b.nrow_off.push_back((int32_t)r0);
    for (int r = 0; r < D; ++r) rs[r] = r0 + r;
    add_row(0, rs, D);
  }
  for (int64_t p = 0; p < b.npr; ++p) {
    const int64_t row = p < lv.Nps ? lv.off_ps + p : lv.off_pf + (p - lv.Nps);
    b.prow_off.push_back((int32_t)row);
    rs[0] = row;
    add_row(1, rs, 1);
  }
  std::vector<int64_t> pos_a[2], pos_b[2];
  make_slices(b.nrb, pa[0], ca[0], pb[0], cb[0], b.node, pos_a[0], pos_b[0]);
  make_slices(b.npr, pa[1], ca[1], pb[1], cb[1], b.pres, pos_a[1], pos_b[1]);
  b.n_na = b.node.ea * D * D;
  b.n_nb = b.node.eb * D;
  b.n_pa = b.pres.ea * D;
  b.n_pb = b.pres.eb;
  const int64_t base_a[2] = {0, b.n_na + b.n_nb};
  const int64_t base_b[2] = {b.n_na, b.n_na + b.n_nb + b.n_pa};
  const int64_t per_a[2] = {(int64_t)D * D, (int64_t)D};
  const int64_t per_b[2] = {(int64_t)D, 1};
  for (int c = 0; c < 2; ++c) {
    for (size_t i = 0; i < sa[c].size(); ++i)
      b.map[ent_a[c][i]] = base_a[c] + pos_a[c][sa[c][i].first] * per_a[c] + sa[c][i].second;
    for (size_t i = 0; i < sb[c].size(); ++i)
      b.map[ent_b[c][i]] = base_b[c] + pos_b[c][sb[c][i].first] * per_b[c] + sb[c][i].second;
  }
  return b;
}

struct DevBOp {
  BOpView<double> v64{};
  BOpView<float> v32{};
  double* vals64 = nullptr;
  float* vals32 = nullptr;
  int64_t* map = nullptr;      // scalar entry of A -> value index
  int64_t nvals = 0;
  bool ready = false;
};

// Device factorization plan of one level's Schwarz blocks: the blocks in
// decreasing size, cut into chunks of at most 1 GiB of dense FP64 scratch
// (small and large blocks never share a chunk: the LDS of a launch is set by
// its largest block), with the per-chunk offsets uploaded once; the scratch
// stays allocated and each level is factored on its own stream.
// device memory allowed for one level's copies of its blocks' operator rows
// (read by the fused sweep form only)
constexpr size_t kRowCopyBudget = (size_t)4 << 30;

struct FactorPlan {
  struct Chunk {
    int64_t b0, b1, off;   // list range, position of its offsets in `offs`
    int max_n;
  };
  bool ready = false;
  std::vector<Chunk> chunks;
  std::vector<int32_t> order;    // host copy of jlist (blocks by size)
  std::vector<int64_t> hoffs;    // host copy of offs
  int32_t* jlist = nullptr;
  int64_t* offs = nullptr;
  double* dense = nullptr;
  int32_t* sigma = nullptr;
  int32_t* status = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  // levels of several chunks: a second scratch and stream, so that the
  // latency-bound panel launches of one chunk overlap the trailing updates
  // of the other
  double* dense2 = nullptr;
  int32_t* sigma2 = nullptr;
  hipStream_t stream2 = nullptr;
  hipEvent_t fork = nullptr, done2 = nullptr;
};

struct DLevel {
  int64_t N = 0, nnz = 0;
  DevBOp A, AT;
  // the field split's diagonal blocks of A (entries coupling [d, p^s] with
  // [u, p^f] removed), used by the cycle of the interchanged cascade; level 0
  // also keeps their CSR for its direct solve
  DevBOp Abd;
  bool use_bd = false;
  int64_t* bd_rp = nullptr;
  int32_t* bd_col = nullptr;
  double* bd_val = nullptr;
  FactorPlan fp;
  int64_t* rp = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  double* piece[4] = {nullptr, nullptr, nullptr, nullptr};
  uint8_t* flags = nullptr;
  TransferView<double> t64{};
  TransferView<float> t32{};
  BlocksView bv{};
  void* W = nullptr;
  int64_t W_elems = 0;
  double *b64 = nullptr, *x64 = nullptr, *r64 = nullptr, *tb64 = nullptr;
  float *b32 = nullptr, *x32 = nullptr, *r32 = nullptr, *tb32 = nullptr;
  // multiplicative sweep: correction e and the residual of the latest iterate
  double *e64 = nullptr, *rc64 = nullptr;
  float *e32 = nullptr, *rc32 = nullptr;
  // fused additive sweeps alternate between x and x2
  double* x2_64 = nullptr;
  float* x2_32 = nullptr;
  // several right-hand sides: K-column blocks (entry (i, c) at i * K + c)
  // of b, x, r in FP64 / FP32, sized for mcap64 / mcap32 columns
  int mcap64 = 0, mcap32 = 0;
  double *bm64 = nullptr, *xm64 = nullptr, *rm64 = nullptr, *tm64 = nullptr;
  float *bm32 = nullptr, *xm32 = nullptr, *rm32 = nullptr, *tm32 = nullptr;
  // transposed block inverses for the K-column transposed sweep (built on
  // first use after each factorization)
  void* Wt = nullptr;
  int64_t* wt_off = nullptr;
  bool wt_valid = false;
};

}  // namespace

struct fsgmg_hierarchy {
  // description
  fsgmg_mesh_desc mesh{};
  std::vector<double> breaks[3];
  std::vector<int8_t> region;
  Physics phys{};
  std::vector<double> w_finest;
  int L = 0, D = 2;
  int device = -1;
  hipStream_t stream = nullptr;
  std::string err;
  // device memory comes from the caller's allocator when one was given
  fsgmg_allocator alloc{nullptr, nullptr, nullptr};
  bool user_alloc() const { return alloc.alloc != nullptr; }
  // wall times of setup_hierarchy and of the last build_fs_as_blocks
  double t_setup_ms = 0, t_blocks_ms = 0;
  // debug_zero_block: the next factorization zeroes this block's matrix
  int zero_block_level = -1;
  int64_t zero_block = -1;
  // host setup data
  std::vector<Level> levels;
  std::vector<LevelOperator> ops;
  // re-assembly about a new advecting velocity (built at the first one)
  std::vector<AdvectionPlan> plans;
  // the same on the device (2D, additive smoother, not interchanged), per
  // level: the fluid elements and what their terms need, the per-element
  // term values, and the touched entries of the value arrays with their
  // velocity-independent sums and their terms (in the host's order)
  struct DevAdv {
    int64_t nfluid = 0;
    int per = 0;
    int32_t* elems = nullptr;
    int64_t* elem_nodes = nullptr;
    double* X = nullptr;
    int32_t* node_fine = nullptr;
    double* emit = nullptr;
    int64_t nt = 0;
    uint8_t* t_arr = nullptr;
    int64_t* t_slot = nullptr;
    double* t_stat = nullptr;
    int64_t* t_ptr = nullptr;
    int64_t* t_em = nullptr;
    int64_t* t_red = nullptr;
    int64_t nl = 0;   // finest: rows whose lift reads Dirichlet data
    int64_t* l_row = nullptr;
    int64_t* l_ptr = nullptr;
    int64_t* l_k = nullptr;
    double* l_g = nullptr;
  };
  std::vector<DevAdv> dadv;   // empty: not built
  double* adv_ref = nullptr;
  int32_t* adv_flag = nullptr;
  int64_t* loadT_perm_dev = nullptr;
  // the device's operator values are newer than the host copies (a device
  // re-assembly); the host copies are pulled when a host consumer needs them
  bool device_ahead = false;
  std::vector<int64_t> loadT_perm;   // entry of the load operator at each transpose entry
  std::vector<double> loadT_host;
  std::vector<Transfer> tr;      // tr[l] for l >= 1
  std::vector<BlockSet> blocks;  // blocks[l] for l >= 1
  bool have_blocks = false;      // index sets built
  bool factors_valid = false;    // block inverses match the current operator
  fsgmg_smoother_opts sopt{};
  // device data
  std::vector<void*> allocs;
  std::vector<DLevel> dl;
  double* coarse_inv = nullptr;
  hipEvent_t coarse_done = nullptr;   // end of a coarse rebuild not yet checked
  bool coarse_pending = false;
  // rebuilds after a parameter update or a re-assembly run on a stream of
  // their own, after the level-0 values are written (coarse_ready)
  hipStream_t coarse_stream = nullptr;
  hipEvent_t coarse_ready = nullptr;
  double* coarse_invT = nullptr;
  double* coarse_work = nullptr;
  int32_t* coarse_piv = nullptr;
  int64_t n0 = 0;
  int64_t coarse_np = 0;   // padded order of the coarse work matrix
  bool coarse_bd = false;  // the coarse inverse is that of level 0's diagonal blocks
  // host side of the diagonal-block operators: A's entries kept (in order)
  // and their value slots in the device layout, per level
  struct BdHost {
    std::vector<int64_t> keep, bmap;
    int64_t nvals = 0;
  };
  std::vector<BdHost> bd;
  bool bd_dirty = false;
  // finest-level extras
  int64_t* load_rp = nullptr;
  int32_t* load_col = nullptr;
  double* load_val = nullptr;
  int64_t* loadT_rp = nullptr;   // transpose of the load operator (adjoint of the load)
  int32_t* loadT_col = nullptr;
  double* loadT_val = nullptr;
  double* lift = nullptr;
  // finest-level time operator: the terms of the operator that carry 1/dt,
  // Dirichlet rows removed (set up with a finite dt only)
  int64_t* time_rp = nullptr;
  int32_t* time_col = nullptr;
  double* time_val = nullptr;
  double* time_piece[4] = {nullptr, nullptr, nullptr, nullptr};
  // period_solve: previous state, current and new iterate, right-hand side
  double* per_buf = nullptr;
  double* lift_piece[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t* full_rp = nullptr;
  int32_t* full_col = nullptr;
  double* full_piece[4] = {nullptr, nullptr, nullptr, nullptr};
  uint8_t* dir_mask = nullptr;
  // Krylov workspace
  int ws_restart = 0;
  int64_t ld = 0;
  double *V = nullptr, *Z = nullptr, *w = nullptr, *part = nullptr, *small = nullptr;
  // autotuned launch shapes per level: SpMV lanes per row (V-cycle precision),
  // smoother workgroup width; lanes of the outer FP64 products
  struct Tune {
    int spmv_lanes = 1;
    int smooth_threads = 0;
    int restrict_lanes = 8;   // transfers into this level's coarse neighbour
    int prolong_lanes = 2;    // transfers from it
    int fused = 0;            // smoother sweeps form their residual in-launch
    int split = 1;            // workgroups per block in the forward sweep
  };
  std::vector<Tune> tune;
  int outer_lanes = 1;
  bool tuned = false;
  // HIP graphs: one per Arnoldi step j (V-cycle included) and transposition,
  // one per V-cycle core; captured on a private stream, launched on `stream`
  std::vector<hipGraphExec_t> step_graph[2];
  hipGraphExec_t vcore_graph[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;
  bool capturing = false;
  void invalidate_graphs() {
    for (auto& v : step_graph) {
      for (hipGraphExec_t g : v)
        if (g) (void)hipGraphExecDestroy(g);
      v.clear();
    }
    for (auto& g : vcore_graph) {
      if (g) (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
  }
  double* tmp = nullptr;
  double* pinned = nullptr;
  double* pinned_dev = nullptr;   // device address of `pinned`
  hipEvent_t step_done[2] = {nullptr, nullptr};   // read-back of Arnoldi steps of each parity
  // K-column FGMRES workspace: basis / preconditioned vectors (ld_mc per
  // K-column block), work block, partial sums, small device arrays and their
  // pinned host mirror
  int mc_K = 0, mc_m = 0;
  int64_t ld_mc = 0;
  double *mc_V = nullptr, *mc_Z = nullptr, *mc_w = nullptr, *mc_part = nullptr;
  double *mc_small = nullptr, *mc_pinned = nullptr;
  // kernel timing: HIP events around selected launches on the handle stream
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_rec[4];

  bool host_only() const { return device < 0; }
  hipEvent_t next_event() {
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) throw Fail{FSGMG_EHIP, "hipEventCreate failed"};
      ev_pool.push_back(e);
    }
    return ev_pool[ev_used++];
  }

  // Device memory: the caller's allocator, else hipMalloc; nullptr when
  // neither has room (no exception).
  void* raw_alloc(size_t bytes) {
    void* p = nullptr;
    if (user_alloc()) {
      p = alloc.alloc(bytes, (void*)stream, alloc.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
    }
    return p;
  }
  void raw_free(void* p) {
    if (!p) return;
    if (user_alloc()) {
      // a caller's allocator may hand the memory out again at once on its
      // stream: every launch of this handle that may still use it ends first
      quiesce();
      alloc.free(p, (void*)stream, alloc.user);
    } else {
      (void)hipFree(p);
    }
  }
  void quiesce();
  void* dalloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    void* p = raw_alloc(bytes);
    if (!p)
      throw Fail{FSGMG_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
    allocs.push_back(p);
    return p;
  }
  // Copies and fills go through the handle's stream and are complete on
  // return: the handle may run on a non-blocking stream, which does not wait
  // for work on the null stream, and the new buffer may next be used on any
  // of the handle's streams.
  template <typename T>
  T* upload(const std::vector<T>& v) {
    T* p = (T*)dalloc(v.size() * sizeof(T));
    if (!v.empty()) {
      HIPCHECK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, stream));
      HIPCHECK(hipStreamSynchronize(stream));
    }
    return p;
  }
  template <typename T>
  T* zeros(int64_t n) {
    T* p = (T*)dalloc((size_t)n * sizeof(T));
    HIPCHECK(hipMemsetAsync(p, 0, (size_t)n * sizeof(T), stream));
    HIPCHECK(hipStreamSynchronize(stream));
    return p;
  }
  hipEvent_t factor_start = nullptr;
  // host copies of the level operators' values lag behind update_params on
  // a device handle until a host consumer needs them
  bool host_vals_stale = false;
  void pull_device_values();
  void ensure_host_values() {
    if (device_ahead) pull_device_values();
    if (!host_vals_stale) return;
    for (LevelOperator& op : ops)
      for (size_t k = 0; k < op.A.val.size(); ++k)
        op.A.val[k] = op.piece[0][k] + op.G * op.piece[1][k] + op.invlam * op.piece[2][k] +
                      op.mu * op.piece[3][k];
    host_vals_stale = false;
  }
  // release device memory obtained by dalloc before the handle ends
  void dfree(void* p) {
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), p);
    if (it != allocs.end()) {
      raw_free(p);
      allocs.erase(it);
    }
  }

  ~fsgmg_hierarchy() {
    if (device >= 0) {
      (void)hipSetDevice(device);
      // every stream drained while it still exists, then events and
      // streams destroyed, then memory freed
      if (coarse_pending && coarse_done) (void)hipEventSynchronize(coarse_done);
      quiesce();
      for (DLevel& d : dl) {
        if (d.fp.stream) (void)hipStreamDestroy(d.fp.stream);
        if (d.fp.done) (void)hipEventDestroy(d.fp.done);
        if (d.fp.stream2) (void)hipStreamDestroy(d.fp.stream2);
        if (d.fp.fork) (void)hipEventDestroy(d.fp.fork);
        if (d.fp.done2) (void)hipEventDestroy(d.fp.done2);
      }
      if (coarse_done) (void)hipEventDestroy(coarse_done);
      if (coarse_stream) (void)hipStreamDestroy(coarse_stream);
      if (coarse_ready) (void)hipEventDestroy(coarse_ready);
      if (factor_start) (void)hipEventDestroy(factor_start);
      for (hipEvent_t e : step_done)
        if (e) (void)hipEventDestroy(e);
      for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
      invalidate_graphs();
      if (cap_stream) (void)hipStreamDestroy(cap_stream);
      for (void* p : allocs) {
        if (user_alloc())
          alloc.free(p, (void*)stream, alloc.user);
        else
          (void)hipFree(p);
      }
      if (pinned) (void)hipHostFree(pinned);
      if (mc_pinned) (void)hipHostFree(mc_pinned);
    }
  }
};

// Wait for every stream this handle launches on (its own, the capture
// stream and the per-level factorization streams).
void fsgmg_hierarchy::quiesce() {
  if (device < 0) return;
  (void)hipStreamSynchronize(stream);
  if (cap_stream) (void)hipStreamSynchronize(cap_stream);
  if (coarse_stream) (void)hipStreamSynchronize(coarse_stream);
  for (DLevel& d : dl) {
    if (d.fp.stream) (void)hipStreamSynchronize(d.fp.stream);
    if (d.fp.stream2) (void)hipStreamSynchronize(d.fp.stream2);
  }
}

namespace {

template <typename F>
fsgmg_status guarded(fsgmg_h h, F&& f) {
  try {
    if (h && h->device >= 0) HIPCHECK(hipSetDevice(h->device));
    return f();
  } catch (const Fail& e) {
    if (h) h->err = e.msg;
    return e.st;
  } catch (const std::bad_alloc&) {
    if (h) h->err = "host allocation failed";
    return FSGMG_ENOMEM;
  } catch (const std::exception& e) {
    if (h) h->err = e.what();
    return FSGMG_EINVAL;
  }
}

// ---------------------------------------------------------------------------
// uploads
// ---------------------------------------------------------------------------
void upload_bop(fsgmg_hierarchy& h, const Level& lv, const CsrHost& A, DevBOp& d) {
  BOpHost b = build_bop(lv, A);
  std::vector<double> v(b.nvals(), 0.0);
  for (int64_t k = 0; k < A.nnz(); ++k) v[b.map[k]] = A.val[k];
  std::vector<float> v32(v.begin(), v.end());
  d.vals64 = h.upload(v);
  d.vals32 = h.upload(v32);
  d.map = h.upload(b.map);
  d.nvals = b.nvals();
  BOpView<double>& x = d.v64;
  x.nrb = b.nrb;
  x.npr = b.npr;
  x.nsn = b.node.nslices;
  x.nsp = b.pres.nslices;
  x.nrow_off = h.upload(b.nrow_off);
  x.prow_off = h.upload(b.prow_off);
  x.n_rows = h.upload(b.node.rows);
  x.n_wa = h.upload(b.node.wa);
  x.n_wb = h.upload(b.node.wb);
  x.n_oa = h.upload(b.node.oa);
  x.n_ob = h.upload(b.node.ob);
  x.n_ca = h.upload(b.node.ca);
  x.n_cb = h.upload(b.node.cb);
  x.p_rows = h.upload(b.pres.rows);
  x.p_wa = h.upload(b.pres.wa);
  x.p_wb = h.upload(b.pres.wb);
  x.p_oa = h.upload(b.pres.oa);
  x.p_ob = h.upload(b.pres.ob);
  x.p_ca = h.upload(b.pres.ca);
  x.p_cb = h.upload(b.pres.cb);
  auto set_vals = [&](auto& view, auto* base) {
    view.n_va = base;
    view.n_vb = base + b.n_na;
    view.p_va = base + b.n_na + b.n_nb;
    view.p_vb = base + b.n_na + b.n_nb + b.n_pa;
  };
  set_vals(x, d.vals64);
  BOpView<float>& y = d.v32;   // same index arrays, FP32 values
  y.nrb = x.nrb;
  y.npr = x.npr;
  y.nsn = x.nsn;
  y.nsp = x.nsp;
  y.nrow_off = x.nrow_off;
  y.prow_off = x.prow_off;
  y.n_rows = x.n_rows;
  y.n_wa = x.n_wa;
  y.n_wb = x.n_wb;
  y.n_oa = x.n_oa;
  y.n_ob = x.n_ob;
  y.n_ca = x.n_ca;
  y.n_cb = x.n_cb;
  y.p_rows = x.p_rows;
  y.p_wa = x.p_wa;
  y.p_wb = x.p_wb;
  y.p_oa = x.p_oa;
  y.p_ob = x.p_ob;
  y.p_ca = x.p_ca;
  y.p_cb = x.p_cb;
  set_vals(y, d.vals32);
  d.ready = true;
}

std::vector<uint8_t> node_flags(const Level& lv) {
  std::vector<uint8_t> f(lv.N2, 0);
  for (int64_t n = 0; n < lv.N2; ++n) {
    uint8_t v = lv.solid_side[n] ? 1 : 0;
    if (lv.dir[(int64_t)lv.D * n]) v |= 2;
    if (lv.dir[lv.off_u + (int64_t)lv.D * n]) v |= 4;
    f[n] = v;
  }
  return f;
}

std::vector<int32_t> ptr32(const std::vector<int64_t>& p) {
  std::vector<int32_t> o(p.size());
  for (size_t i = 0; i < p.size(); ++i) o[i] = (int32_t)p[i];
  return o;
}

template <typename T>
std::vector<T> conv(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

void upload_transfer(fsgmg_hierarchy& h, int l) {
  const Level& f = h.levels[l];
  const Level& c = h.levels[l - 1];
  const Transfer& t = h.tr[l];
  DLevel& d = h.dl[l];
  TransferView<double>& v = d.t64;
  v.N2f = f.N2;
  v.N2c = c.N2;
  v.Npsf = f.Nps;
  v.Npff = f.Npf;
  v.Npsc = c.Nps;
  v.Npfc = c.Npf;
  v.offu_f = f.off_u;
  v.offps_f = f.off_ps;
  v.offpf_f = f.off_pf;
  v.offu_c = c.off_u;
  v.offps_c = c.off_ps;
  v.offpf_c = c.off_pf;
  v.pn_ptr = h.upload(ptr32(t.Pn.rowptr));
  v.pn_col = h.upload(t.Pn.col);
  v.rn_ptr = h.upload(ptr32(t.Rn.rowptr));
  v.rn_col = h.upload(t.Rn.col);
  v.pps_ptr = h.upload(ptr32(t.Pps.rowptr));
  v.pps_col = h.upload(t.Pps.col);
  v.ppf_ptr = h.upload(ptr32(t.Ppf.rowptr));
  v.ppf_col = h.upload(t.Ppf.col);
  v.rps_ptr = h.upload(ptr32(t.Rps.rowptr));
  v.rps_col = h.upload(t.Rps.col);
  v.rpf_ptr = h.upload(ptr32(t.Rpf.rowptr));
  v.rpf_col = h.upload(t.Rpf.col);
  v.flags_f = h.dl[l].flags;
  v.flags_c = h.dl[l - 1].flags;
  TransferView<float>& u = d.t32;
  std::memcpy((void*)&u, (const void*)&v, sizeof(u));   // same layout: ints/pointers
  v.pn_val = h.upload(t.Pn.val);
  v.rn_val = h.upload(t.Rn.val);
  v.pps_val = h.upload(t.Pps.val);
  v.ppf_val = h.upload(t.Ppf.val);
  v.rps_val = h.upload(t.Rps.val);
  v.rpf_val = h.upload(t.Rpf.val);
  u.pn_val = h.upload(conv<float>(t.Pn.val));
  u.rn_val = h.upload(conv<float>(t.Rn.val));
  u.pps_val = h.upload(conv<float>(t.Pps.val));
  u.ppf_val = h.upload(conv<float>(t.Ppf.val));
  u.rps_val = h.upload(conv<float>(t.Rps.val));
  u.rpf_val = h.upload(conv<float>(t.Rpf.val));
}

// dense FP64 copy of the coarse-level matrix, inverted on the device; the
// transpose of the inverse is kept for the transposed V-cycle
// Wait for a coarse inverse enqueued by update_params and check that the
// coarse matrix was not singular (every cycle entry point calls this).
void ensure_coarse(fsgmg_hierarchy& h) {
  if (!h.coarse_pending) return;
  HIPCHECK(hipEventSynchronize(h.coarse_done));
  h.coarse_pending = false;
  int32_t st = 0;
  const int64_t np = h.coarse_np;
  HIPCHECK(hipMemcpyAsync(&st, h.coarse_piv + 2 * np, sizeof(int32_t), hipMemcpyDeviceToHost,
                          h.stream));
  HIPCHECK(hipStreamSynchronize(h.stream));
  if (st) throw Fail{FSGMG_ESINGULAR, "coarse-level matrix is singular"};
}

// Dense FP64 inverse of the level-0 operator from its device CSR.  With
// `async` the work is enqueued on a stream of its own after the level-0
// values (the column permutation formed on the device) and the call returns
// at once, so the block refactorization that follows a parameter update or
// a re-assembly runs beside it; ensure_coarse checks its status before the
// next cycle, and writers of level-0 values wait for it on the device.
// The handle's stream waits for a coarse rebuild still running on its own
// stream before level-0 values or the coarse buffers are written again.
void wait_coarse(fsgmg_hierarchy& h) {
  if (h.coarse_pending && h.coarse_done) HIPCHECK(hipStreamWaitEvent(h.stream, h.coarse_done, 0));
}

void build_coarse_inverse(fsgmg_hierarchy& h, bool async = false) {
  const int64_t n = h.ops[0].A.nrows;
  if (n > 20000) throw Fail{FSGMG_EINVAL, "coarse level too large for the dense inverse (n > 20000)"};
  wait_coarse(h);
  int64_t np = (n + 15) & ~(int64_t)15;
  int max_lds = 0;
  HIPCHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h.device));
  const int nb = coarse_panel_width(np, max_lds);
  const bool reg = coarse_register_path(np);
  const int64_t W = coarse_wide_panel();
  const bool wide = !reg && nb == W;
  if (wide) np = (n + W - 1) / W * W;   // whole strips on the wide-panel path
  // scratch after the work matrix: panel rows (LDS paths), or pivot rows,
  // staged interchanges, the pivot column and the scaled pivot row (wide)
  const int64_t scratch = wide ? (3 * W + 1) * np + 2 * W : 8 * np;
  if (!h.coarse_inv) {
    h.coarse_inv = (double*)h.dalloc((size_t)(n * n) * sizeof(double));
    h.coarse_invT = (double*)h.dalloc((size_t)(n * n) * sizeof(double));
    // work matrix + scratch, and the second work matrix of the register path
    h.coarse_work = (double*)h.dalloc((size_t)((reg ? 2 : 1) * np * np + scratch) * sizeof(double));
    // pivots, sigma, status, source rows
    h.coarse_piv = (int32_t*)h.dalloc((size_t)(3 * np + 1) * sizeof(int32_t));
  }
  h.coarse_np = np;
  int32_t* status = h.coarse_piv + 2 * np;
  int32_t* src = h.coarse_piv + 2 * np + 1;
  double* a2 = reg ? h.coarse_work + np * np + scratch : nullptr;
  const DLevel& C = h.dl[0];
  // device CSR of level 0 (current parameter values), or its field-split
  // diagonal blocks for the interchanged cascade
  const bool bd = C.use_bd;
  const int64_t* crp = bd ? C.bd_rp : C.rp;
  const int32_t* ccol = bd ? C.bd_col : C.col;
  const double* cval = bd ? C.bd_val : C.val;
  h.coarse_bd = bd;
  int32_t* dsig = h.coarse_piv + np;
  if (async && coarse_sigma_lds(np) <= (size_t)max_lds) {
    if (!h.coarse_done) HIPCHECK(hipEventCreateWithFlags(&h.coarse_done, hipEventDisableTiming));
    if (!h.coarse_ready) HIPCHECK(hipEventCreateWithFlags(&h.coarse_ready, hipEventDisableTiming));
    if (!h.coarse_stream) HIPCHECK(hipStreamCreateWithFlags(&h.coarse_stream, hipStreamNonBlocking));
    // after the level-0 values written on the handle's stream; the block
    // refactorization that follows a parameter update runs beside it
    HIPCHECK(hipEventRecord(h.coarse_ready, h.stream));
    HIPCHECK(hipStreamWaitEvent(h.coarse_stream, h.coarse_ready, 0));
    hipStream_t cs = h.coarse_stream;
    HIPCHECK(hipMemsetAsync(status, 0, sizeof(int32_t), cs));
    const double* res = launch_coarse_factor(n, np, crp, ccol, cval, h.coarse_work,
                                             h.coarse_work + np * np, a2, src, h.coarse_piv,
                                             status, nb, cs);
    launch_coarse_sigma(h.coarse_piv, np, status, dsig, cs);
    launch_coarse_finish(res, np, n, dsig, h.coarse_inv, h.coarse_invT, cs);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipEventRecord(h.coarse_done, cs));
    h.coarse_pending = true;
    h.n0 = n;
    return;
  }
  HIPCHECK(hipMemsetAsync(status, 0, sizeof(int32_t), h.stream));
  const double* res = launch_coarse_factor(n, np, crp, ccol, cval, h.coarse_work,
                                           h.coarse_work + np * np, a2, src, h.coarse_piv, status,
                                           nb, h.stream);
  HIPCHECK(hipGetLastError());
  std::vector<int32_t> piv(np + 1);
  HIPCHECK(hipMemcpyAsync(piv.data(), h.coarse_piv, np * sizeof(int32_t), hipMemcpyDeviceToHost,
                          h.stream));
  HIPCHECK(hipMemcpyAsync(piv.data() + np, status, sizeof(int32_t), hipMemcpyDeviceToHost, h.stream));
  HIPCHECK(hipStreamSynchronize(h.stream));
  if (piv[np]) throw Fail{FSGMG_ESINGULAR, "coarse-level matrix is singular"};
  // the row interchanges, undone in reverse order, as a column permutation
  std::vector<int32_t> sig(np);
  for (int64_t c = 0; c < np; ++c) sig[c] = (int32_t)c;
  for (int64_t c = np - 1; c >= 0; --c) std::swap(sig[c], sig[piv[c]]);
  HIPCHECK(hipMemcpyAsync(dsig, sig.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, h.stream));
  launch_coarse_finish(res, np, n, dsig, h.coarse_inv, h.coarse_invT, h.stream);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(h.stream));
  h.n0 = n;
}

// The field split's diagonal blocks of every level operator (entries that
// couple the groups [d, p^s] and [u, p^f] removed) on the device, for the
// interchanged cascade: built from the host values on first use; after
// update_params only their values are refreshed (the pattern is fixed).
// Level 0 also keeps their CSR for its direct solve.
void ensure_bd(fsgmg_hierarchy& h) {
  const bool first = h.bd.size() != (size_t)h.L;
  if (!first && !h.bd_dirty) return;
  wait_coarse(h);
  h.ensure_host_values();
  if (first) h.bd.resize(h.L);
  for (int l = 0; l < h.L; ++l) {
    DLevel& d = h.dl[l];
    const Level& lv = h.levels[l];
    const CsrHost& A = h.ops[l].A;
    fsgmg_hierarchy::BdHost& bh = h.bd[l];
    if (first) {
      CsrHost B;
      B.nrows = A.nrows;
      B.ncols = A.ncols;
      B.rowptr.assign(A.nrows + 1, 0);
      for (int64_t r = 0; r < A.nrows; ++r) {
        const bool gr = r >= lv.off_u;
        for (int64_t k = A.rowptr[r]; k < A.rowptr[r + 1]; ++k)
          if ((A.col[k] >= lv.off_u) == gr) {
            B.col.push_back(A.col[k]);
            B.val.push_back(A.val[k]);
            bh.keep.push_back(k);
          }
        B.rowptr[r + 1] = (int64_t)B.col.size();
      }
      const BOpHost bo = build_bop(lv, B);
      bh.bmap = bo.map;
      bh.nvals = bo.nvals();
      upload_bop(h, lv, B, d.Abd);
      if (l == 0) {
        d.bd_rp = h.upload(B.rowptr);
        d.bd_col = h.upload(B.col);
        d.bd_val = h.upload(B.val);
      }
      continue;
    }
    std::vector<double> v(bh.nvals, 0.0), kv(bh.keep.size());
    for (size_t i = 0; i < bh.keep.size(); ++i) kv[i] = A.val[bh.keep[i]];
    for (size_t i = 0; i < bh.keep.size(); ++i) v[bh.bmap[i]] = kv[i];
    const std::vector<float> v32(v.begin(), v.end());
    HIPCHECK(hipMemcpyAsync(d.Abd.vals64, v.data(), v.size() * sizeof(double),
                            hipMemcpyHostToDevice, h.stream));
    HIPCHECK(hipMemcpyAsync(d.Abd.vals32, v32.data(), v32.size() * sizeof(float),
                            hipMemcpyHostToDevice, h.stream));
    if (l == 0)
      HIPCHECK(hipMemcpyAsync(d.bd_val, kv.data(), kv.size() * sizeof(double),
                              hipMemcpyHostToDevice, h.stream));
    HIPCHECK(hipStreamSynchronize(h.stream));
  }
  h.bd_dirty = false;
}

// Entry of A at each position of its transpose as csr_transpose orders it
// (rows ascending within each column).
std::vector<int64_t> transpose_order(const CsrHost& A) {
  std::vector<int64_t> cur(A.ncols + 1, 0);
  for (int64_t k = 0; k < A.nnz(); ++k) cur[A.col[k] + 1]++;
  for (int64_t j = 0; j < A.ncols; ++j) cur[j + 1] += cur[j];
  std::vector<int64_t> perm(A.nnz());
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) perm[cur[A.col[k]]++] = k;
  return perm;
}

// The finest level's load operator (and its transpose) and time operator,
// patterns and values.
void upload_load_and_time(fsgmg_hierarchy& h) {
  const LevelOperator& op = h.ops[h.L - 1];
  h.loadT_perm = transpose_order(op.load);
  for (void* p : {(void*)h.load_rp, (void*)h.load_col, (void*)h.load_val, (void*)h.loadT_rp,
                  (void*)h.loadT_col, (void*)h.loadT_val, (void*)h.time_rp, (void*)h.time_col,
                  (void*)h.time_val})
    h.dfree(p);
  h.load_rp = h.upload(op.load.rowptr);
  h.load_col = h.upload(op.load.col);
  h.load_val = h.upload(op.load.val);
  CsrHost LT = csr_transpose(op.load);
  h.loadT_rp = h.upload(LT.rowptr);
  h.loadT_col = h.upload(LT.col);
  h.loadT_val = h.upload(LT.val);
  for (int p = 0; p < 4; ++p) h.dfree(h.time_piece[p]);
  h.time_rp = nullptr;
  h.time_col = nullptr;
  h.time_val = nullptr;
  for (int p = 0; p < 4; ++p) h.time_piece[p] = nullptr;
  if (h.phys.inv_dt != 0.0) {
    h.time_rp = h.upload(op.time.rowptr);
    h.time_col = h.upload(op.time.col);
    h.time_val = h.upload(op.time.val);
    for (int p = 0; p < 4; ++p) h.time_piece[p] = h.upload(op.time_piece[p]);
  }
}

// Their values only, on the patterns already on the device (re-assembly
// about a new advecting velocity keeps every pattern).  Asynchronous; the
// host staging stays valid until the next call.
void refresh_load_and_time(fsgmg_hierarchy& h) {
  const LevelOperator& op = h.ops[h.L - 1];
  HIPCHECK(hipMemcpyAsync(h.load_val, op.load.val.data(), op.load.val.size() * sizeof(double),
                          hipMemcpyHostToDevice, h.stream));
  h.loadT_host.resize(h.loadT_perm.size());
  for (size_t j = 0; j < h.loadT_perm.size(); ++j) h.loadT_host[j] = op.load.val[h.loadT_perm[j]];
  HIPCHECK(hipMemcpyAsync(h.loadT_val, h.loadT_host.data(), h.loadT_host.size() * sizeof(double),
                          hipMemcpyHostToDevice, h.stream));
  if (h.time_val) {
    const size_t n = op.time.val.size();
    HIPCHECK(hipMemcpyAsync(h.time_val, op.time.val.data(), n * sizeof(double),
                            hipMemcpyHostToDevice, h.stream));
    for (int p = 0; p < 4; ++p)
      HIPCHECK(hipMemcpyAsync(h.time_piece[p], op.time_piece[p].data(), n * sizeof(double),
                              hipMemcpyHostToDevice, h.stream));
  }
}

void upload_all(fsgmg_hierarchy& h) {
  h.dl.resize(h.L);
  h.tune.assign(h.L, {});
  for (int l = 0; l < h.L; ++l) {
    const Level& lv = h.levels[l];
    const LevelOperator& op = h.ops[l];
    DLevel& d = h.dl[l];
    d.N = lv.N;
    d.nnz = op.A.nnz();
    d.flags = h.upload(node_flags(lv));
    upload_bop(h, lv, op.A, d.A);
    d.rp = h.upload(op.A.rowptr);
    d.col = h.upload(op.A.col);
    d.val = h.upload(op.A.val);
    for (int p = 0; p < 4; ++p) d.piece[p] = h.upload(op.piece[p]);
    d.b64 = h.zeros<double>(lv.N);
    d.x64 = h.zeros<double>(lv.N);
    d.r64 = h.zeros<double>(lv.N);
    d.b32 = h.zeros<float>(lv.N);
    d.x32 = h.zeros<float>(lv.N);
    d.r32 = h.zeros<float>(lv.N);
  }
  for (int l = 1; l < h.L; ++l) upload_transfer(h, l);
  const Level& F = h.levels[h.L - 1];
  const LevelOperator& op = h.ops[h.L - 1];
  upload_load_and_time(h);
  for (int p = 0; p < 4; ++p) h.lift_piece[p] = h.upload(op.lift_piece[p]);
  std::vector<double> lift(F.N);
  for (int64_t i = 0; i < F.N; ++i)
    lift[i] = op.lift_piece[0][i] + op.G * op.lift_piece[1][i] + op.invlam * op.lift_piece[2][i] +
              op.mu * op.lift_piece[3][i];
  h.lift = h.upload(lift);
  h.full_rp = h.upload(op.full.rowptr);
  h.full_col = h.upload(op.full.col);
  for (int p = 0; p < 4; ++p) h.full_piece[p] = h.upload(op.full_piece[p]);
  h.dir_mask = h.upload(F.dir);
  h.tmp = h.zeros<double>(F.N);
  build_coarse_inverse(h);
}

void ensure_transposed(fsgmg_hierarchy& h) {
  for (int l = 0; l < h.L; ++l) {
    DLevel& d = h.dl[l];
    if (d.AT.ready) continue;
    h.ensure_host_values();
    const CsrHost& A = h.ops[l].A;
    CsrHost T = csr_transpose(A);
    upload_bop(h, h.levels[l], T, d.AT);
    // value map from A's entries into AT: position of (i,j) in T
    std::vector<int64_t> pos(A.nnz());
    std::vector<int64_t> cur(T.rowptr.begin(), T.rowptr.end() - 1);
    for (int64_t i = 0; i < A.nrows; ++i)
      for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) pos[k] = cur[A.col[k]]++;
    BOpHost bt = build_bop(h.levels[l], T);
    std::vector<int64_t> m(A.nnz());
    for (int64_t k = 0; k < A.nnz(); ++k) m[k] = bt.map[pos[k]];
    HIPCHECK(hipMemcpyAsync(d.AT.map, m.data(), m.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                            h.stream));
    HIPCHECK(hipStreamSynchronize(h.stream));
  }
}

// ---------------------------------------------------------------------------
// FS-AS block factors
// ---------------------------------------------------------------------------
int rows_per_vector(fsgmg_prec p) { return p == FSGMG_FP64 ? 2 : (p == FSGMG_FP32 ? 4 : 8); }
size_t w_bytes(fsgmg_prec p) { return p == FSGMG_FP64 ? 8 : (p == FSGMG_FP32 ? 4 : 2); }
WPrec wprec(fsgmg_prec p) {
  return p == FSGMG_FP64 ? WPrec::F64 : (p == FSGMG_FP32 ? WPrec::F32 : WPrec::BF16);
}

void upload_blocks(fsgmg_hierarchy& h, int l) {
  h.ensure_host_values();
  const Level& lv = h.levels[l];
  const BlockSet& bs = h.blocks[l];
  DLevel& d = h.dl[l];
  // release the previous index sets, inverses and sweep buffers of the level
  {
    BlocksView& o = d.bv;
    for (const void* q : {(const void*)o.dof_ptr, (const void*)o.dofs, (const void*)o.own_ptr,
                          (const void*)o.own_dof, (const void*)o.own_loc, (const void*)o.w_off,
                          (const void*)o.mpad, (const void*)o.jac, o.jac_inv,
                          (const void*)o.tpos_ptr, (const void*)o.tpos, (const void*)o.order,
                          (const void*)d.W, (const void*)d.tb64, (const void*)d.tb32,
                          (const void*)d.e64, (const void*)d.rc64, (const void*)d.e32,
                          (const void*)d.rc32, (const void*)o.rows_off, (const void*)o.rows_w,
                          (const void*)o.rows_col, o.rows_val, (const void*)o.jrow_col,
                          o.jrow_val, (const void*)d.x2_64, (const void*)d.x2_32, (const void*)d.Wt,
                          (const void*)d.wt_off})
      h.dfree(const_cast<void*>(q));
    o = BlocksView{};
    d.W = nullptr;
    d.tb64 = d.e64 = d.rc64 = d.x2_64 = nullptr;
    d.tb32 = d.e32 = d.rc32 = d.x2_32 = nullptr;
    d.Wt = nullptr;
    d.wt_off = nullptr;
    d.wt_valid = false;
    // K-column work blocks: the per-block rows depend on the index sets
    for (const void* q : {(const void*)d.bm64, (const void*)d.xm64, (const void*)d.rm64,
                          (const void*)d.tm64, (const void*)d.bm32, (const void*)d.xm32,
                          (const void*)d.rm32, (const void*)d.tm32})
      h.dfree(const_cast<void*>(q));
    d.bm64 = d.xm64 = d.rm64 = d.tm64 = nullptr;
    d.bm32 = d.xm32 = d.rm32 = d.tm32 = nullptr;
    d.mcap64 = d.mcap32 = 0;
  }
  const int RV = rows_per_vector(h.sopt.prec);
  const int64_t nb = bs.nblk();
  // multiplicative sweep: a block writes every one of its rows
  const bool all_rows = h.sopt.schwarz == FSGMG_SCHWARZ_MULTIPLICATIVE;
  std::vector<int32_t> own_ptr(1, 0), own_dof, own_loc, mpad(nb);
  std::vector<int64_t> w_off(nb + 1, 0);
  int max_n = 0, max_mpad = 0;
  for (int64_t j = 0; j < nb; ++j) {
    const int64_t b0 = bs.ptr[j], n = bs.ptr[j + 1] - b0;
    int m = 0;
    for (int64_t k = 0; k < n; ++k)
      if (all_rows || bs.owner[bs.dofs[b0 + k]] == (int32_t)j) {
        own_dof.push_back(bs.dofs[b0 + k]);
        own_loc.push_back((int32_t)k);
        ++m;
      }
    own_ptr.push_back((int32_t)own_dof.size());
    const int mp = std::max(RV, (m + RV - 1) / RV * RV);
    mpad[j] = mp;
    w_off[j + 1] = w_off[j] + n * mp;
    max_n = std::max(max_n, (int)n);
    max_mpad = std::max(max_mpad, mp);
  }
  // transposed apply: DOF -> positions (block order)
  std::vector<int32_t> tcnt(lv.N + 1, 0), tpos(bs.dofs.size());
  for (int32_t g : bs.dofs) tcnt[g + 1]++;
  for (int64_t i = 0; i < lv.N; ++i) tcnt[i + 1] += tcnt[i];
  {
    std::vector<int32_t> cur(tcnt.begin(), tcnt.end() - 1);
    for (int64_t p = 0; p < (int64_t)bs.dofs.size(); ++p) tpos[cur[bs.dofs[p]]++] = (int32_t)p;
  }
  // Jacobi inverse diagonal
  const CsrHost& A = h.ops[l].A;
  std::vector<double> jinv(bs.jac.size());
  for (size_t q = 0; q < bs.jac.size(); ++q) {
    const int32_t i = bs.jac[q];
    double dg = 0.0;
    for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
      if (A.col[k] == i) dg = A.val[k];
    if (dg == 0.0) throw Fail{FSGMG_ESINGULAR, "zero diagonal on a Jacobi row " + std::to_string(i)};
    jinv[q] = 1.0 / dg;
  }
  BlocksView& v = d.bv;
  v.nblk = nb;
  v.njac = (int64_t)bs.jac.size();
  v.dof_ptr = h.upload(bs.ptr);
  v.dofs = h.upload(bs.dofs);
  v.own_ptr = h.upload(own_ptr);
  v.own_dof = h.upload(own_dof);
  v.own_loc = h.upload(own_loc);
  v.w_off = h.upload(w_off);
  v.mpad = h.upload(mpad);
  v.jac = h.upload(bs.jac);
  v.jac_inv = h.sopt.prec == FSGMG_FP64 ? (const void*)h.upload(jinv)
                                        : (const void*)h.upload(conv<float>(jinv));
  v.max_n = max_n;
  v.max_mpad = max_mpad;
  v.tpos_ptr = h.upload(tcnt);
  v.tpos = h.upload(tpos);
  {
    // largest inverses first, inside each colour of a multiplicative sweep
    std::vector<int32_t> order(nb);
    for (int64_t j = 0; j < nb; ++j) order[j] = (int32_t)j;
    std::vector<int64_t> seg = all_rows ? bs.colour_ptr : std::vector<int64_t>{0, nb};
    for (size_t c = 0; c + 1 < seg.size(); ++c)
      std::stable_sort(order.begin() + seg[c], order.begin() + seg[c + 1],
                       [&](int32_t a, int32_t b) {
                         return w_off[a + 1] - w_off[a] > w_off[b + 1] - w_off[b];
                       });
    v.order = h.upload(order);
  }
  d.W_elems = w_off[nb];
  d.W = h.dalloc((size_t)d.W_elems * w_bytes(h.sopt.prec) + 64);
  const int64_t ntot = (int64_t)bs.dofs.size();
  if (h.sopt.prec == FSGMG_FP64)
    d.tb64 = h.zeros<double>(std::max<int64_t>(ntot, 1));
  else
    d.tb32 = h.zeros<float>(std::max<int64_t>(ntot, 1));
  if (all_rows) {
    if (h.sopt.prec == FSGMG_FP64) {
      d.e64 = h.zeros<double>(lv.N);
      d.rc64 = h.zeros<double>(lv.N);
    } else {
      d.e32 = h.zeros<float>(lv.N);
      d.rc32 = h.zeros<float>(lv.N);
    }
  }
  // operator rows of the blocks and of the Jacobi unknowns (fused sweeps);
  // the values are gathered on the device with every factorization
  {
    std::vector<int64_t> roff(nb + 1, 0);
    std::vector<int32_t> rw(nb, 0);
    for (int64_t j = 0; j < nb; ++j) {
      int w = 0;
      for (int64_t p = bs.ptr[j]; p < bs.ptr[j + 1]; ++p) {
        const int32_t g = bs.dofs[p];
        w = std::max(w, (int)(A.rowptr[g + 1] - A.rowptr[g]));
      }
      rw[j] = w;
      roff[j + 1] = roff[j] + (bs.ptr[j + 1] - bs.ptr[j]) * w;
    }
    int jw = 0;
    for (int32_t g : bs.jac) jw = std::max(jw, (int)(A.rowptr[g + 1] - A.rowptr[g]));
    const size_t vb = h.sopt.prec == FSGMG_FP64 ? 8 : 4;
    // the copies cost sum_j n_j * (longest row of block j) entries: in 3D
    // (rows of up to 125 node blocks) tens of GB, beyond what the fused form
    // can gain; such a level keeps the SpMV form only
    const size_t rows_bytes = ((size_t)roff[nb] + bs.jac.size() * (size_t)jw) * (4 + vb);
    if (rows_bytes <= kRowCopyBudget) {
      v.rows_off = h.upload(roff);
      v.rows_w = h.upload(rw);
      v.rows_col = (const int32_t*)h.dalloc((size_t)roff[nb] * sizeof(int32_t));
      v.rows_val = h.dalloc((size_t)roff[nb] * vb);
      v.jrow_w = jw;
      v.jrow_col = (const int32_t*)h.dalloc((size_t)bs.jac.size() * jw * sizeof(int32_t));
      v.jrow_val = h.dalloc((size_t)bs.jac.size() * jw * vb);
    }
    if (h.sopt.prec == FSGMG_FP64)
      d.x2_64 = h.zeros<double>(lv.N);
    else
      d.x2_32 = h.zeros<float>(lv.N);
  }
}

// FP32 and BF16 inverses are factored in FP32 (FP32 matrix cores, half the
// bytes and LDS of the FP64 factorization), FP64 inverses in FP64.
bool factor_f32(const fsgmg_hierarchy& h) { return h.sopt.prec != FSGMG_FP64; }

void plan_factor(fsgmg_hierarchy& h, int l) {
  const BlockSet& bs = h.blocks[l];
  DLevel& d = h.dl[l];
  FactorPlan& fp = d.fp;
  for (void* q : {(void*)fp.jlist, (void*)fp.offs, (void*)fp.dense, (void*)fp.sigma,
                  (void*)fp.status, (void*)fp.dense2, (void*)fp.sigma2})
    h.dfree(q);
  fp.ready = false;
  fp.dense2 = nullptr;
  fp.sigma2 = nullptr;
  fp.chunks.clear();
  fp.jlist = nullptr;
  fp.offs = nullptr;
  fp.dense = nullptr;
  fp.sigma = nullptr;
  fp.status = nullptr;
  const int64_t nb = bs.nblk();
  if (nb == 0) {
    fp.ready = true;
    return;
  }
  auto padded = [](int64_t n) { return (n + 15) & ~(int64_t)15; };
  int max_lds = 0;
  HIPCHECK(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, h.device));
  if (invert_blocks_lds((int)padded(d.bv.max_n), factor_f32(h)) > (size_t)max_lds)
    throw Fail{FSGMG_EINVAL, "Schwarz block of " + std::to_string(d.bv.max_n) +
                                 " unknowns exceeds the LDS of one workgroup"};
  // np <= 384: 55 KB of LDS, three workgroups per CU
  constexpr int64_t kSmallNp = 384;
  std::vector<int32_t> order(nb);
  for (int64_t j = 0; j < nb; ++j) order[j] = (int32_t)j;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return bs.ptr[a + 1] - bs.ptr[a] > bs.ptr[b + 1] - bs.ptr[b];
  });
  const size_t budget = (size_t)1 << 30;
  size_t maxchunk = 0, maxsig = 0;
  std::vector<int64_t> hoff;
  {
    size_t acc = 0, sacc = 0;
    int64_t b0 = 0;
    bool big = true;
    auto close = [&](int64_t b1) {
      const int64_t cnt = b1 - b0;
      FactorPlan::Chunk c{b0, b1, (int64_t)hoff.size(),
                          (int)(bs.ptr[order[b0] + 1] - bs.ptr[order[b0]])};
      const size_t base = hoff.size();
      hoff.resize(base + 2 * (cnt + 1), 0);
      for (int64_t b = 0; b < cnt; ++b) {
        const int32_t j = order[b0 + b];
        const int64_t np = padded(bs.ptr[j + 1] - bs.ptr[j]);
        hoff[base + b + 1] = hoff[base + b] + np * np;
        hoff[base + cnt + 1 + b + 1] = hoff[base + cnt + 1 + b] + np;
      }
      fp.chunks.push_back(c);
      maxchunk = std::max(maxchunk, acc);
      maxsig = std::max(maxsig, sacc);
      acc = sacc = 0;
      b0 = b1;
    };
    for (int64_t b = 0; b < nb; ++b) {
      const int64_t np = padded(bs.ptr[order[b] + 1] - bs.ptr[order[b]]);
      const bool isbig = np > kSmallNp;
      if (b > b0 && (acc + (size_t)(np * np * 8) > budget || isbig != big)) close(b);
      big = isbig;
      acc += (size_t)(np * np * 8);
      sacc += (size_t)np * 4;
    }
    close(nb);
  }
  fp.jlist = h.upload(order);
  fp.offs = h.upload(hoff);
  fp.order = order;
  fp.hoffs = hoff;
  fp.dense = (double*)h.dalloc(maxchunk);
  fp.sigma = (int32_t*)h.dalloc(maxsig);
  fp.status = (int32_t*)h.dalloc((size_t)nb * sizeof(int32_t));
  if (!fp.stream) HIPCHECK(hipStreamCreateWithFlags(&fp.stream, hipStreamNonBlocking));
  if (!fp.done) HIPCHECK(hipEventCreateWithFlags(&fp.done, hipEventDisableTiming));
  fp.dense2 = nullptr;
  fp.sigma2 = nullptr;
  if (fp.chunks.size() > 1) {
    fp.dense2 = (double*)h.dalloc(maxchunk);
    fp.sigma2 = (int32_t*)h.dalloc(maxsig);
    if (!fp.stream2) HIPCHECK(hipStreamCreateWithFlags(&fp.stream2, hipStreamNonBlocking));
    if (!fp.fork) HIPCHECK(hipEventCreateWithFlags(&fp.fork, hipEventDisableTiming));
    if (!fp.done2) HIPCHECK(hipEventCreateWithFlags(&fp.done2, hipEventDisableTiming));
  }
  fp.ready = true;
}

// Gather, invert and extract the blocks of every level l >= 1: each level on
// its own stream (the small coarse levels, one block per CU, overlap the fine
// one), joined back into the handle's stream.
void factor_blocks(fsgmg_hierarchy& h, bool retune) {
  if (!h.factor_start) HIPCHECK(hipEventCreateWithFlags(&h.factor_start, hipEventDisableTiming));
  HIPCHECK(hipEventRecord(h.factor_start, h.stream));
  for (int l = 1; l < h.L; ++l) {
    DLevel& d = h.dl[l];
    FactorPlan& fp = d.fp;
    if (!fp.ready) plan_factor(h, l);
    const int64_t nb = h.blocks[l].nblk();
    if (nb == 0) continue;
    HIPCHECK(hipStreamWaitEvent(fp.stream, h.factor_start, 0));
    HIPCHECK(hipMemsetAsync(fp.status, 0, (size_t)nb * sizeof(int32_t), fp.stream));
    d.wt_valid = false;
    // the blocks' copies of A's rows serve the fused sweep form only (and
    // the autotuner's trial of it)
    if ((retune || h.tune[l].fused) && d.bv.rows_col) {
      if (h.sopt.prec == FSGMG_FP64)
        launch_block_rows<double>(d.bv, d.rp, d.col, d.val, fp.stream);
      else
        launch_block_rows<float>(d.bv, d.rp, d.col, d.val, fp.stream);
    }
    // chunks alternate between the two scratch slots and streams (one slot
    // when the level has a single chunk)
    const bool two = fp.dense2 != nullptr;
    if (two) {
      HIPCHECK(hipEventRecord(fp.fork, fp.stream));
      HIPCHECK(hipStreamWaitEvent(fp.stream2, fp.fork, 0));
    }
    for (size_t ci = 0; ci < fp.chunks.size(); ++ci) {
      const FactorPlan::Chunk& c = fp.chunks[ci];
      const bool second = two && (ci & 1);
      hipStream_t cs = second ? fp.stream2 : fp.stream;
      double* dense = second ? fp.dense2 : fp.dense;
      int32_t* sigma = second ? fp.sigma2 : fp.sigma;
      const int64_t cnt = c.b1 - c.b0;
      const int32_t* jl = fp.jlist + c.b0;
      const int64_t* doff = fp.offs + c.off;
      const int64_t* soff = doff + cnt + 1;
      const bool f32 = factor_f32(h);
      launch_gather_blocks(jl, cnt, d.bv, d.rp, d.col, d.val, doff, dense, f32, c.max_n, cs);
      if (h.zero_block_level == l)
        for (int64_t b = 0; b < cnt; ++b)
          if (fp.order[c.b0 + b] == h.zero_block) {
            // test hook: a zero matrix, so the block's first pivot is zero
            const int64_t o = fp.hoffs[c.off + b], n2 = fp.hoffs[c.off + b + 1] - o;
            if (f32)
              launch_fill<float>(reinterpret_cast<float*>(dense) + o, 0.0f, n2, cs);
            else
              launch_fill<double>(dense + o, 0.0, n2, cs);
          }
      launch_invert_blocks(jl, cnt, d.bv.dof_ptr, doff, soff, dense, f32, sigma, fp.status,
                           c.max_n, cs);
      launch_extract_owned(jl, cnt, d.bv, doff, soff, dense, f32, sigma, wprec(h.sopt.prec),
                           d.W, cs);
      HIPCHECK(hipGetLastError());
    }
    if (two) {
      HIPCHECK(hipEventRecord(fp.done2, fp.stream2));
      HIPCHECK(hipStreamWaitEvent(fp.stream, fp.done2, 0));
    }
    HIPCHECK(hipEventRecord(fp.done, fp.stream));
  }
  for (int l = 1; l < h.L; ++l)
    if (h.blocks[l].nblk() > 0) HIPCHECK(hipStreamWaitEvent(h.stream, h.dl[l].fp.done, 0));
  HIPCHECK(hipStreamSynchronize(h.stream));
  for (int l = 1; l < h.L; ++l) {
    const int64_t nb = h.blocks[l].nblk();
    if (nb == 0) continue;
    std::vector<int32_t> st(nb);
    HIPCHECK(hipMemcpyAsync(st.data(), h.dl[l].fp.status, nb * sizeof(int32_t),
                            hipMemcpyDeviceToHost, h.stream));
    HIPCHECK(hipStreamSynchronize(h.stream));
    for (int64_t j = 0; j < nb; ++j)
      if (st[j])
        throw Fail{FSGMG_ESINGULAR, "singular Schwarz block " + std::to_string(j) + " on level " +
                                        std::to_string(l)};
  }
}

// ---------------------------------------------------------------------------
// optional event timing of selected launches (kinds: 0 finest smoother sweep,
// 1 finest residual SpMV of the V-cycle, 2 outer FP64 SpMV, 3 finest-level
// restriction + prolongation)
// ---------------------------------------------------------------------------
struct TimedLaunch {
  fsgmg_hierarchy& h;
  int kind;
  hipEvent_t b = nullptr;
  TimedLaunch(fsgmg_hierarchy& hh, int k, bool on) : h(hh), kind(k) {
    if (on && h.timing) {
      b = h.next_event();
      HIPCHECK(hipEventRecord(b, h.stream));
    }
  }
  ~TimedLaunch() noexcept(false) {
    if (b) {
      hipEvent_t e = h.next_event();
      HIPCHECK(hipEventRecord(e, h.stream));
      h.ev_rec[kind].emplace_back(b, e);
    }
  }
};

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------
template <typename TV>
struct Vec;
template <>
struct Vec<double> {
  static double* b(DLevel& d) { return d.b64; }
  static double* x(DLevel& d) { return d.x64; }
  static double* r(DLevel& d) { return d.r64; }
  static double* t(DLevel& d) { return d.tb64; }
  static double* e(DLevel& d) { return d.e64; }
  static double* rc(DLevel& d) { return d.rc64; }
  static double* x2(DLevel& d) { return d.x2_64; }
  static double* bm(DLevel& d) { return d.bm64; }
  static double* xm(DLevel& d) { return d.xm64; }
  static double* rm(DLevel& d) { return d.rm64; }
  static double* tm(DLevel& d) { return d.tm64; }
  static const BOpView<double>& op(DLevel& d, bool tr) {
    return tr ? d.AT.v64 : (d.use_bd ? d.Abd.v64 : d.A.v64);
  }
  static const TransferView<double>& tv(DLevel& d) { return d.t64; }
};
template <>
struct Vec<float> {
  static float* b(DLevel& d) { return d.b32; }
  static float* x(DLevel& d) { return d.x32; }
  static float* r(DLevel& d) { return d.r32; }
  static float* t(DLevel& d) { return d.tb32; }
  static float* e(DLevel& d) { return d.e32; }
  static float* rc(DLevel& d) { return d.rc32; }
  static float* x2(DLevel& d) { return d.x2_32; }
  static float* bm(DLevel& d) { return d.bm32; }
  static float* xm(DLevel& d) { return d.xm32; }
  static float* rm(DLevel& d) { return d.rm32; }
  static float* tm(DLevel& d) { return d.tm32; }
  static const BOpView<float>& op(DLevel& d, bool tr) {
    return tr ? d.AT.v32 : (d.use_bd ? d.Abd.v32 : d.A.v32);
  }
  static const TransferView<float>& tv(DLevel& d) { return d.t32; }
};

// Multiplicative sweeps on level l (Section 3.2): from r0 = b - A x (b when
// starting from zero) the correction e is built colour by colour, each colour
// on the residual r0 - A e of the latest correction, the Jacobi unknowns last;
// then x += omega e.  Transposed: A^T, the Jacobi unknowns first, colours in
// reverse order, transposed block solves.
template <typename TV>
void smooth_level_mult(fsgmg_hierarchy& h, int l, int nsweeps, bool transpose, bool from_zero) {
  DLevel& d = h.dl[l];
  const BlockSet& bs = h.blocks[l];
  const int D = h.D;
  const WPrec wp = wprec(h.sopt.prec);
  TV* b = Vec<TV>::b(d);
  TV* x = Vec<TV>::x(d);
  TV* r0 = Vec<TV>::r(d);
  TV* e = Vec<TV>::e(d);
  TV* rc = Vec<TV>::rc(d);
  const bool fin = l == h.L - 1;
  const int64_t ncol = (int64_t)bs.colour_ptr.size() - 1;
  const BOpView<TV>& A = Vec<TV>::op(d, transpose);
  const int lanes = h.tune[l].spmv_lanes;
  if (!transpose && h.tune[l].fused) {
    // in-place colour steps on y (a copy of x, or 0), residuals formed in-launch
    for (int s = 0; s < nsweeps; ++s) {
      const bool first = s == 0 && from_zero;
      if (first)
        launch_fill<TV>(e, TV(0), d.N, h.stream);
      else
        launch_add_scaled<TV>(d.N, 1.0, x, e, true, h.stream);
      for (int64_t c = 0; c < ncol; ++c) {
        BlocksView v = d.bv;
        v.order = d.bv.order + bs.colour_ptr[c];
        v.nblk = bs.colour_ptr[c + 1] - bs.colour_ptr[c];
        v.njac = 0;
        TimedLaunch t(h, 0, fin);
        // the first colour of a sweep from zero: y = 0, the residual is b
        launch_smooth_fused<TV>(v, wp, d.W, b, e, e, 1.0, first && c == 0, h.stream,
                                h.tune[l].smooth_threads);
      }
      launch_mult_finish<TV>(d.bv, b, e, x, d.N, h.sopt.omega, first, h.stream);
    }
    return;
  }
  for (int s = 0; s < nsweeps; ++s) {
    const bool first = s == 0 && from_zero;
    const TV* rs = b;
    if (!first) {
      TimedLaunch t(h, 1, fin);
      launch_spmv<TV>(A, D, x, b, r0, true, h.stream, lanes);
      rs = r0;
    }
    launch_fill<TV>(e, TV(0), d.N, h.stream);
    bool fresh = true;   // e == 0: the residual of the latest iterate is rs
    auto step = [&](const BlocksView& v, int64_t p0, int64_t p1) {
      if (v.nblk == 0 && v.njac == 0) return;
      const TV* rr = rs;
      if (!fresh) {
        TimedLaunch t(h, 1, fin);
        launch_spmv<TV>(A, D, e, rs, rc, true, h.stream, lanes);
        rr = rc;
      }
      TimedLaunch t(h, 0, fin);
      launch_smooth_colour<TV>(v, wp, d.W, rr, e, Vec<TV>::t(d), p0, p1, transpose, h.stream,
                               h.tune[l].smooth_threads, h.tune[l].split);
      fresh = false;
    };
    BlocksView jv = d.bv;
    jv.nblk = 0;
    auto colour = [&](int64_t c) {
      BlocksView v = d.bv;
      v.order = d.bv.order + bs.colour_ptr[c];
      v.nblk = bs.colour_ptr[c + 1] - bs.colour_ptr[c];
      v.njac = 0;
      step(v, bs.ptr[bs.colour_ptr[c]], bs.ptr[bs.colour_ptr[c + 1]]);
    };
    if (transpose) {
      step(jv, 0, 0);
      for (int64_t c = ncol - 1; c >= 0; --c) colour(c);
    } else {
      for (int64_t c = 0; c < ncol; ++c) colour(c);
      step(jv, 0, 0);
    }
    launch_add_scaled<TV>(d.N, h.sopt.omega, e, x, first, h.stream);
  }
}

template <typename TV>
void smooth_level(fsgmg_hierarchy& h, int l, int nsweeps, bool transpose, bool from_zero) {
  if (h.sopt.schwarz == FSGMG_SCHWARZ_MULTIPLICATIVE) {
    smooth_level_mult<TV>(h, l, nsweeps, transpose, from_zero);
    return;
  }
  DLevel& d = h.dl[l];
  const int D = h.D;
  const WPrec wp = wprec(h.sopt.prec);
  TV* b = Vec<TV>::b(d);
  TV* x = Vec<TV>::x(d);
  TV* r = Vec<TV>::r(d);
  const bool fin = l == h.L - 1;
  if (!transpose && h.tune[l].fused) {
    // every sweep reads one buffer and writes all of the other
    TV* cur = x;
    for (int s = 0; s < nsweeps; ++s) {
      TV* out = cur == x ? Vec<TV>::x2(d) : x;
      TimedLaunch t(h, 0, fin);
      launch_smooth_fused<TV>(d.bv, wp, d.W, b, cur, out, h.sopt.omega, s == 0 && from_zero,
                              h.stream, h.tune[l].smooth_threads);
      cur = out;
    }
    if (cur != x) launch_add_scaled<TV>(d.N, 1.0, cur, x, true, h.stream);
    return;
  }
  for (int s = 0; s < nsweeps; ++s) {
    if (s == 0 && from_zero) {
      TimedLaunch t(h, 0, fin);
      launch_smooth<TV>(d.bv, wp, d.W, b, x, Vec<TV>::t(d), h.sopt.omega, true, transpose, d.N,
                        h.stream, h.tune[l].smooth_threads, h.tune[l].split);
    } else {
      {
        TimedLaunch t(h, 1, fin);
        launch_spmv<TV>(Vec<TV>::op(d, transpose), D, x, b, r, true, h.stream, h.tune[l].spmv_lanes);
      }
      TimedLaunch t(h, 0, fin);
      launch_smooth<TV>(d.bv, wp, d.W, r, x, Vec<TV>::t(d), h.sopt.omega, false, transpose, d.N,
                        h.stream, h.tune[l].smooth_threads, h.tune[l].split);
    }
  }
}

// V-cycle from the finest right-hand side buffer b to the finest x buffer
// One multigrid cycle on level l for the right-hand side in b_l, result in
// x_l (zero_init: from x_l = 0, else from the iterate already in x_l).  The
// coarse correction runs one cycle on level l-1 (V), two W-cycles (W), or an
// F-cycle then a V-cycle (F; transposed: V then F, the transpose of that
// composition); every coarse cycle after the first starts from the previous
// result.  Level 0 is the direct solve.
template <typename TV>
void cycle_level(fsgmg_hierarchy& h, int l, int kind, bool transpose, bool zero_init) {
  const int L = h.L, D = h.D;
  if (l == 0) {
    DLevel& C = h.dl[0];
    launch_dense_gemv<TV>(h.n0, transpose ? h.coarse_invT : h.coarse_inv, false, Vec<TV>::b(C),
                          Vec<TV>::x(C), h.stream);
    return;
  }
  const int npre = transpose ? h.sopt.nu_post : h.sopt.nu_pre;
  const int npost = transpose ? h.sopt.nu_pre : h.sopt.nu_post;
  DLevel& d = h.dl[l];
  if (npre == 0 && zero_init) launch_fill<TV>(Vec<TV>::x(d), TV(0), d.N, h.stream);
  smooth_level<TV>(h, l, npre, transpose, zero_init);
  {
    TimedLaunch t(h, 1, l == L - 1);
    launch_spmv<TV>(Vec<TV>::op(d, transpose), D, Vec<TV>::x(d), Vec<TV>::b(d), Vec<TV>::r(d),
                    true, h.stream, h.tune[l].spmv_lanes);
  }
  {
    TimedLaunch t(h, 3, l == L - 1);
    launch_transfer<TV>(Vec<TV>::tv(d), D, transpose ? 2 : (d.use_bd ? 4 : 0), Vec<TV>::r(d),
                        Vec<TV>::b(h.dl[l - 1]),
                        h.stream, h.tune[l].restrict_lanes);
  }
  int seq[2] = {FSGMG_CYCLE_V, FSGMG_CYCLE_V};
  int nseq = 1;
  if (kind == FSGMG_CYCLE_W) {
    seq[0] = seq[1] = FSGMG_CYCLE_W;
    nseq = 2;
  } else if (kind == FSGMG_CYCLE_F) {
    seq[0] = transpose ? FSGMG_CYCLE_V : FSGMG_CYCLE_F;
    seq[1] = transpose ? FSGMG_CYCLE_F : FSGMG_CYCLE_V;
    nseq = 2;
  }
  for (int i = 0; i < nseq; ++i) cycle_level<TV>(h, l - 1, seq[i], transpose, i == 0);
  {
    TimedLaunch t(h, 3, l == L - 1);
    launch_transfer<TV>(Vec<TV>::tv(d), D, transpose ? 3 : 1, Vec<TV>::x(h.dl[l - 1]),
                        Vec<TV>::x(d), h.stream, h.tune[l].prolong_lanes);
  }
  smooth_level<TV>(h, l, npost, transpose, false);
}

template <typename TV>
void vcycle_core(fsgmg_hierarchy& h, bool transpose) {
  cycle_level<TV>(h, h.L - 1, h.sopt.cycle, transpose, true);
}

bool graphs_on(const fsgmg_hierarchy& h) { return h.sopt.use_graph && !h.timing && !h.capturing; }

// Capture whatever `enqueue` puts on the handle stream into an executable graph.
// Captures are serialized over the process, so that handles driven from
// several host threads never capture at the same time (a run with several
// threads and unserialized captures ended one with "unjoined work").
std::mutex capture_mutex;

template <typename F>
hipGraphExec_t capture(fsgmg_hierarchy& h, F&& enqueue) {
  const std::lock_guard<std::mutex> lock(capture_mutex);
  if (!h.cap_stream) HIPCHECK(hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking));
  hipStream_t saved = h.stream;
  h.stream = h.cap_stream;
  h.capturing = true;
  HIPCHECK(hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeThreadLocal));
  hipGraph_t g = nullptr;
  try {
    enqueue();
  } catch (...) {
    (void)hipStreamEndCapture(h.cap_stream, &g);
    if (g) (void)hipGraphDestroy(g);
    h.stream = saved;
    h.capturing = false;
    throw;
  }
  h.stream = saved;
  h.capturing = false;
  HIPCHECK(hipStreamEndCapture(h.cap_stream, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) throw Fail{FSGMG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
  return ex;
}

template <typename TV>
void vcycle_impl(fsgmg_hierarchy& h, const double* rin, double* zout, bool transpose) {
  DLevel& F = h.dl[h.L - 1];
  launch_cast<double, TV>(rin, Vec<TV>::b(F), F.N, h.stream);
  if (graphs_on(h)) {
    hipGraphExec_t& g = h.vcore_graph[transpose ? 1 : 0];
    if (!g) g = capture(h, [&] { vcycle_core<TV>(h, transpose); });
    HIPCHECK(hipGraphLaunch(g, h.stream));
  } else {
    vcycle_core<TV>(h, transpose);
  }
  launch_cast<TV, double>(Vec<TV>::x(F), zout, F.N, h.stream);
}

void vcycle(fsgmg_hierarchy& h, const double* r, double* z, bool transpose) {
  if (h.L == 1) {
    launch_dense_gemv<double>(h.n0, transpose ? h.coarse_invT : h.coarse_inv, false, r, z, h.stream);
    return;
  }
  if (h.sopt.prec == FSGMG_FP64)
    vcycle_impl<double>(h, r, z, transpose);
  else
    vcycle_impl<float>(h, r, z, transpose);
}

// ---------------------------------------------------------------------------
// Several right-hand sides on the same operator: the cycle of each column is
// the one-column cycle (same operators, smoother, transfers, coarse solve),
// every launch works on all K columns, so each matrix and block inverse is
// read once per K columns and the block apply runs on the matrix cores.
// ---------------------------------------------------------------------------
template <typename TV>
void ensure_mc_buffers(fsgmg_hierarchy& h, int K) {
  for (int l = 0; l < h.L; ++l) {
    DLevel& d = h.dl[l];
    const int64_t n = d.N * (int64_t)K;
    // per-block rows of the transposed sweep: one K-column row per block entry
    const int64_t nt = (l > 0 ? (int64_t)h.blocks[l].dofs.size() : 0) * K;
    if (sizeof(TV) == 8) {
      if (d.mcap64 >= K) continue;
      for (void* q : {(void*)d.bm64, (void*)d.xm64, (void*)d.rm64, (void*)d.tm64}) h.dfree(q);
      d.bm64 = d.xm64 = d.rm64 = d.tm64 = nullptr;
      d.mcap64 = 0;
      d.bm64 = h.zeros<double>(n);
      d.xm64 = h.zeros<double>(n);
      d.rm64 = h.zeros<double>(n);
      d.tm64 = h.zeros<double>(std::max<int64_t>(nt, 1));
      d.mcap64 = K;
    } else {
      if (d.mcap32 >= K) continue;
      for (void* q : {(void*)d.bm32, (void*)d.xm32, (void*)d.rm32, (void*)d.tm32}) h.dfree(q);
      d.bm32 = d.xm32 = d.rm32 = d.tm32 = nullptr;
      d.mcap32 = 0;
      d.bm32 = h.zeros<float>(n);
      d.xm32 = h.zeros<float>(n);
      d.rm32 = h.zeros<float>(n);
      d.tm32 = h.zeros<float>(std::max<int64_t>(nt, 1));
      d.mcap32 = K;
    }
  }
}

// transposed inverses of level l's blocks (after the latest factorization)
void ensure_wt(fsgmg_hierarchy& h, int l) {
  DLevel& d = h.dl[l];
  if (d.wt_valid) return;
  const BlockSet& bs = h.blocks[l];
  const int RV = rows_per_vector(h.sopt.prec);
  if (!d.Wt) {
    const int64_t nb = bs.nblk();
    std::vector<int64_t> off(nb + 1, 0);
    for (int64_t j = 0; j < nb; ++j) {
      const int64_t n = bs.ptr[j + 1] - bs.ptr[j];
      int64_t m = 0;
      for (int64_t p = bs.ptr[j]; p < bs.ptr[j + 1]; ++p) m += bs.owner[bs.dofs[p]] == (int32_t)j;
      off[j + 1] = off[j] + m * ((n + RV - 1) / RV * RV);
    }
    d.wt_off = h.upload(off);
    d.Wt = h.dalloc((size_t)off[nb] * w_bytes(h.sopt.prec) + 64);
  }
  launch_transpose_blocks(d.bv, wprec(h.sopt.prec), d.W, d.wt_off, d.Wt, h.stream);
  HIPCHECK(hipGetLastError());
  d.wt_valid = true;
}

template <typename TV>
void smooth_level_mc(fsgmg_hierarchy& h, int l, int nsweeps, bool from_zero, int K,
                     bool transpose = false) {
  DLevel& d = h.dl[l];
  const WPrec wp = wprec(h.sopt.prec);
  TV* b = Vec<TV>::bm(d);
  TV* x = Vec<TV>::xm(d);
  TV* r = Vec<TV>::rm(d);
  const bool fin = l == h.L - 1;
  if (transpose) {
    ensure_wt(h, l);
    for (int s = 0; s < nsweeps; ++s) {
      const bool first = s == 0 && from_zero;
      if (!first) {
        TimedLaunch t(h, 1, fin);
        launch_spmm<TV>(Vec<TV>::op(d, true), h.D, x, b, r, K, true, h.stream);
      }
      TimedLaunch t(h, 0, fin);
      launch_smooth_mc_t<TV>(d.bv, wp, d.Wt, d.wt_off, first ? b : r, x, Vec<TV>::tm(d), d.N, K,
                             h.sopt.omega, first, h.stream);
    }
    return;
  }
  for (int s = 0; s < nsweeps; ++s) {
    if (s == 0 && from_zero) {
      TimedLaunch t(h, 0, fin);
      launch_smooth_mc<TV>(d.bv, wp, d.W, b, x, K, h.sopt.omega, true, h.stream);
    } else {
      {
        TimedLaunch t(h, 1, fin);
        launch_spmm<TV>(Vec<TV>::op(d, false), h.D, x, b, r, K, true, h.stream);
      }
      TimedLaunch t(h, 0, fin);
      launch_smooth_mc<TV>(d.bv, wp, d.W, r, x, K, h.sopt.omega, false, h.stream);
    }
  }
}

template <typename TV>
void cycle_level_mc(fsgmg_hierarchy& h, int l, int kind, bool zero_init, int K,
                    bool transpose = false) {
  if (l == 0) {
    DLevel& C = h.dl[0];
    launch_dense_mc<TV>(h.n0, transpose ? h.coarse_invT : h.coarse_inv, Vec<TV>::bm(C),
                        Vec<TV>::xm(C), K, h.stream);
    return;
  }
  DLevel& d = h.dl[l];
  const int64_t nk = d.N * (int64_t)K;
  const int npre = transpose ? h.sopt.nu_post : h.sopt.nu_pre;
  const int npost = transpose ? h.sopt.nu_pre : h.sopt.nu_post;
  if (npre == 0 && zero_init) launch_fill<TV>(Vec<TV>::xm(d), TV(0), nk, h.stream);
  smooth_level_mc<TV>(h, l, npre, zero_init, K, transpose);
  launch_spmm<TV>(Vec<TV>::op(d, transpose), h.D, Vec<TV>::xm(d), Vec<TV>::bm(d), Vec<TV>::rm(d),
                  K, true, h.stream);
  launch_transfer_mc<TV>(Vec<TV>::tv(d), h.D, transpose ? 2 : 0, Vec<TV>::rm(d),
                         Vec<TV>::bm(h.dl[l - 1]), K, h.stream);
  int seq[2] = {FSGMG_CYCLE_V, FSGMG_CYCLE_V};
  int nseq = 1;
  if (kind == FSGMG_CYCLE_W) {
    seq[0] = seq[1] = FSGMG_CYCLE_W;
    nseq = 2;
  } else if (kind == FSGMG_CYCLE_F) {
    seq[0] = transpose ? FSGMG_CYCLE_V : FSGMG_CYCLE_F;
    seq[1] = transpose ? FSGMG_CYCLE_F : FSGMG_CYCLE_V;
    nseq = 2;
  }
  for (int i = 0; i < nseq; ++i) cycle_level_mc<TV>(h, l - 1, seq[i], i == 0, K, transpose);
  launch_transfer_mc<TV>(Vec<TV>::tv(d), h.D, transpose ? 3 : 1, Vec<TV>::xm(h.dl[l - 1]),
                         Vec<TV>::xm(d), K, h.stream);
  smooth_level_mc<TV>(h, l, npost, false, K, transpose);
}
void vcycle_mc(fsgmg_hierarchy& h, const double* r, double* z, int K, bool transpose = false) {
  if (h.L == 1) {
    launch_dense_mc<double>(h.n0, transpose ? h.coarse_invT : h.coarse_inv, r, z, K, h.stream);
    return;
  }
  auto run = [&](auto tag) {
    using TV = decltype(tag);
    ensure_mc_buffers<TV>(h, K);
    DLevel& F = h.dl[h.L - 1];
    const int64_t nk = F.N * (int64_t)K;
    launch_cast<double, TV>(r, Vec<TV>::bm(F), nk, h.stream);
    cycle_level_mc<TV>(h, h.L - 1, h.sopt.cycle, true, K, transpose);
    launch_cast<TV, double>(Vec<TV>::xm(F), z, nk, h.stream);
  };
  if (h.sopt.prec == FSGMG_FP64)
    run(double{});
  else
    run(float{});
}

// ---------------------------------------------------------------------------
// FGMRES
// ---------------------------------------------------------------------------
void ensure_reduction_buffers(fsgmg_hierarchy& h) {
  if (!h.part) h.part = h.zeros<double>(krylov_partials());
  if (!h.small) h.small = h.zeros<double>(256);
  for (hipEvent_t& e : h.step_done)
    if (!e) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  if (!h.pinned) {
    HIPCHECK(hipHostMalloc((void**)&h.pinned, 256 * sizeof(double), hipHostMallocMapped));
    HIPCHECK(hipHostGetDevicePointer((void**)&h.pinned_dev, h.pinned, 0));
  }
}

void ensure_workspace(fsgmg_hierarchy& h, int m) {
  if (h.ws_restart >= m) return;
  const int64_t N = h.dl[h.L - 1].N;
  h.invalidate_graphs();
  h.ld = (N + 63) / 64 * 64;
  h.V = h.zeros<double>((int64_t)(m + 1) * h.ld);
  h.Z = h.zeros<double>((int64_t)m * h.ld);
  h.w = h.zeros<double>(h.ld);
  ensure_reduction_buffers(h);
  h.ws_restart = m;
}

double device_norm(fsgmg_hierarchy& h, const double* v, int64_t N) {
  ensure_reduction_buffers(h);
  launch_norm2(v, N, h.part, h.small + 128, h.stream);
  HIPCHECK(hipMemcpyAsync(h.pinned, h.small + 128, sizeof(double), hipMemcpyDeviceToHost, h.stream));
  HIPCHECK(hipStreamSynchronize(h.stream));
  return h.pinned[0];
}

// Enqueue Arnoldi step j: v_j = w / ||w|| (j > 0), z_j = M^{-1} v_j,
// w = A z_j, two classical Gram-Schmidt passes and ||w||; the Hessenberg
// column pieces [h1 | h2 | ||w||] are copied to pinned host memory.
// Step j leaves h1, h2 and ||w|| in the device / pinned area of its parity
// (small and pinned at step_area(j)), so step j + 1 can be queued before the
// host has read step j's values; v_j is normalized with ||w|| of step j - 1.
constexpr int kStepArea = 160;
inline int step_area(int j) { return (j & 1) ? kStepArea : 0; }

void arnoldi_step(fsgmg_hierarchy& h, int j, bool transpose) {
  DLevel& F = h.dl[h.L - 1];
  const int64_t N = F.N, ld = h.ld;
  const BOpView<double>& A = transpose ? F.AT.v64 : F.A.v64;
  double* const h1 = h.small + step_area(j);
  double* const h2 = h1 + 32;
  double* const nr = h1 + 64;
  double* vj = h.V + (int64_t)j * ld;
  double* zj = h.Z + (int64_t)j * ld;
  if (j > 0) launch_scale_copy(h.w, h.small + step_area(j - 1) + 64, vj, N, h.stream);
  vcycle(h, vj, zj, transpose);
  {
    TimedLaunch t(h, 2, true);
    launch_spmv<double>(A, h.D, zj, nullptr, h.w, false, h.stream, h.outer_lanes);
  }
  launch_mdot(h.V, ld, j + 1, h.w, N, h.part, h1, h.stream);
  launch_maxpy_mdot(h.V, ld, j + 1, h1, h.w, N, h.part, h2, h.stream);
  launch_maxpy_norm(h.V, ld, j + 1, h2, h.w, N, h.part, nr, h.stream);
  launch_store_host(h1, h.pinned_dev + step_area(j), 65, h.stream);
}

void run_arnoldi_step(fsgmg_hierarchy& h, int j, bool transpose) {
  if (!graphs_on(h)) {
    arnoldi_step(h, j, transpose);
    return;
  }
  auto& v = h.step_graph[transpose ? 1 : 0];
  if ((int)v.size() <= j) v.resize(j + 1, nullptr);
  if (!v[j]) v[j] = capture(h, [&] { arnoldi_step(h, j, transpose); });
  HIPCHECK(hipGraphLaunch(v[j], h.stream));
}

// ---------------------------------------------------------------------------
// FGMRES on K right-hand sides in lockstep: every column has its own Krylov
// basis, Hessenberg matrix, Givens rotations and convergence test (the
// one-column algorithm of fgmres, column by column); every operator product,
// K-column cycle and Gram-Schmidt pass works on all K columns at once.  A
// column that has converged (or met a breakdown) in the current restart
// cycle gets a zero next basis vector, so it stays zero through the rest of
// the cycle's launches.
// ---------------------------------------------------------------------------
// mc_small layout (doubles): h1 [kMaxMcK * 32], h2 [kMaxMcK * 32], norms
// [kMaxMcK], scale [kMaxMcK], y [32 * kMaxMcK]
constexpr int kMaxMcK = kMaxRhs;
constexpr int kMcH1 = 0, kMcH2 = 32 * kMaxMcK, kMcNrm = 64 * kMaxMcK, kMcScale = 65 * kMaxMcK,
              kMcY = 66 * kMaxMcK, kMcSmall = 98 * kMaxMcK;

void ensure_mc_workspace(fsgmg_hierarchy& h, int K, int m) {
  if (h.mc_K >= K && h.mc_m >= m) return;
  for (void* q : {(void*)h.mc_V, (void*)h.mc_Z, (void*)h.mc_w, (void*)h.mc_part,
                  (void*)h.mc_small})
    h.dfree(q);
  h.mc_V = h.mc_Z = h.mc_w = h.mc_part = h.mc_small = nullptr;
  h.mc_K = h.mc_m = 0;
  const int64_t N = h.dl[h.L - 1].N;
  h.ld_mc = (N * K + 63) / 64 * 64;
  h.mc_V = h.zeros<double>((int64_t)(m + 1) * h.ld_mc);
  h.mc_Z = h.zeros<double>((int64_t)m * h.ld_mc);
  h.mc_w = h.zeros<double>(h.ld_mc);
  h.mc_part = h.zeros<double>(krylov_mc_partials());
  h.mc_small = h.zeros<double>(kMcSmall);
  if (!h.mc_pinned)
    HIPCHECK(hipHostMalloc((void**)&h.mc_pinned, kMcSmall * sizeof(double), hipHostMallocDefault));
  h.mc_K = K;
  h.mc_m = m;
}

fsgmg_status fgmres_batch(fsgmg_hierarchy& h, const double* b, double* x, int K,
                          const fsgmg_krylov_opts& o, fsgmg_solve_info* infos,
                          bool transpose = false) {
  const auto t0 = std::chrono::steady_clock::now();
  if (o.restart < 1 || o.restart > 31 || o.rtol <= 0 || o.max_restarts < 0)
    throw Fail{FSGMG_EINVAL, "krylov options out of range (restart 1..31, rtol > 0)"};
  if (!h.factors_valid) throw Fail{FSGMG_ESTATE, "build_fs_as_blocks has not been called"};
  const int m = o.restart;
  ensure_mc_workspace(h, K, m);
  if (transpose) ensure_transposed(h);
  DLevel& F = h.dl[h.L - 1];
  const int64_t N = F.N, ld = h.ld_mc;
  const BOpView<double>& A = transpose ? F.AT.v64 : F.A.v64;
  double* dsm = h.mc_small;
  double* hp = h.mc_pinned;
  auto norms = [&](const double* v, std::vector<double>& out) {
    launch_mc_maxpy_norm(nullptr, ld, 0, nullptr, const_cast<double*>(v), N, K, h.mc_part,
                         dsm + kMcNrm, h.stream);
    HIPCHECK(hipMemcpyAsync(hp + kMcNrm, dsm + kMcNrm, K * sizeof(double), hipMemcpyDeviceToHost,
                            h.stream));
    HIPCHECK(hipStreamSynchronize(h.stream));
    out.assign(hp + kMcNrm, hp + kMcNrm + K);
  };
  auto upload_scale = [&](const std::vector<double>& sc) {
    for (int c = 0; c < K; ++c) hp[kMcScale + c] = sc[c];
    HIPCHECK(hipMemcpyAsync(dsm + kMcScale, hp + kMcScale, K * sizeof(double),
                            hipMemcpyHostToDevice, h.stream));
  };
  std::vector<double> bnorm, beta, nrm, scale(K);
  norms(b, bnorm);
  for (int c = 0; c < K; ++c)
    if (!std::isfinite(bnorm[c])) throw Fail{FSGMG_EINVAL, "right-hand side contains NaN or Inf"};
  launch_fill<double>(x, 0.0, N * K, h.stream);
  std::vector<int> iters(K, 0), restarts(K, 0), conv(K, 0);
  std::vector<double> true_rel(K, NAN);
  for (int c = 0; c < K; ++c)
    if (bnorm[c] == 0.0) {
      conv[c] = 1;
      true_rel[c] = 0.0;
    }
  std::vector<double> H((size_t)K * (m + 1) * m), cs((size_t)K * m), sn((size_t)K * m),
      g((size_t)K * (m + 1)), y((size_t)m * K);
  std::vector<int> jc(K), done(K);
  auto all_conv = [&] {
    for (int c = 0; c < K; ++c)
      if (!conv[c]) return false;
    return true;
  };
  for (int cycle = 0; !all_conv() && cycle <= o.max_restarts; ++cycle) {
    launch_spmm<double>(A, h.D, x, b, h.mc_w, K, true, h.stream);
    norms(h.mc_w, beta);
    for (int c = 0; c < K; ++c) {
      if (!conv[c] && beta[c] <= o.rtol * bnorm[c]) {
        conv[c] = 1;
        true_rel[c] = beta[c] / bnorm[c];
      }
      done[c] = conv[c];
      jc[c] = 0;
      scale[c] = done[c] ? 0.0 : 1.0 / beta[c];
      std::fill(H.begin() + (size_t)c * (m + 1) * m, H.begin() + (size_t)(c + 1) * (m + 1) * m, 0.0);
      std::fill(g.begin() + (size_t)c * (m + 1), g.begin() + (size_t)(c + 1) * (m + 1), 0.0);
      g[(size_t)c * (m + 1)] = beta[c];
    }
    if (all_conv()) break;
    upload_scale(scale);
    launch_mc_scale(N, K, dsm + kMcScale, h.mc_w, h.mc_V, h.stream);
    for (int j = 0; j < m; ++j) {
      bool any = false;
      for (int c = 0; c < K; ++c) any |= !done[c];
      if (!any) break;
      double* Vj = h.mc_V + (int64_t)j * ld;
      double* Zj = h.mc_Z + (int64_t)j * ld;
      vcycle_mc(h, Vj, Zj, K, transpose);
      launch_spmm<double>(A, h.D, Zj, nullptr, h.mc_w, K, false, h.stream);
      launch_mc_mdot(h.mc_V, ld, j + 1, h.mc_w, N, K, h.mc_part, dsm + kMcH1, h.stream);
      launch_mc_maxpy_mdot(h.mc_V, ld, j + 1, dsm + kMcH1, h.mc_w, N, K, h.mc_part, dsm + kMcH2,
                           h.stream);
      launch_mc_maxpy_norm(h.mc_V, ld, j + 1, dsm + kMcH2, h.mc_w, N, K, h.mc_part, dsm + kMcNrm,
                           h.stream);
      HIPCHECK(hipMemcpyAsync(hp, dsm, (size_t)(kMcNrm + K) * sizeof(double),
                              hipMemcpyDeviceToHost, h.stream));
      HIPCHECK(hipStreamSynchronize(h.stream));
      for (int c = 0; c < K; ++c) {
        scale[c] = 0.0;
        if (done[c]) continue;
        double* Hc = H.data() + (size_t)c * (m + 1) * m;
        double* csc = cs.data() + (size_t)c * m;
        double* snc = sn.data() + (size_t)c * m;
        double* gc = g.data() + (size_t)c * (m + 1);
        const double hn = hp[kMcNrm + c];
        for (int i = 0; i <= j; ++i) Hc[i * m + j] = hp[kMcH1 + i * K + c] + hp[kMcH2 + i * K + c];
        Hc[(j + 1) * m + j] = hn;
        for (int i = 0; i < j; ++i) {
          const double t = csc[i] * Hc[i * m + j] + snc[i] * Hc[(i + 1) * m + j];
          Hc[(i + 1) * m + j] = -snc[i] * Hc[i * m + j] + csc[i] * Hc[(i + 1) * m + j];
          Hc[i * m + j] = t;
        }
        const double den = std::hypot(Hc[j * m + j], Hc[(j + 1) * m + j]);
        csc[j] = Hc[j * m + j] / den;
        snc[j] = Hc[(j + 1) * m + j] / den;
        Hc[j * m + j] = den;
        Hc[(j + 1) * m + j] = 0.0;
        gc[j + 1] = -snc[j] * gc[j];
        gc[j] = csc[j] * gc[j];
        ++iters[c];
        jc[c] = j + 1;
        const double est = std::fabs(gc[j + 1]);
        if (!std::isfinite(est)) throw Fail{FSGMG_EINVAL, "non-finite residual estimate"};
        if (est <= o.rtol * bnorm[c] || hn == 0.0)
          done[c] = 1;
        else
          scale[c] = 1.0 / hn;
      }
      if (j + 1 < m) {
        upload_scale(scale);
        launch_mc_scale(N, K, dsm + kMcScale, h.mc_w, h.mc_V + (int64_t)(j + 1) * ld, h.stream);
      }
    }
    // per-column least squares, then one K-column update of x
    int kmax = 0;
    std::fill(y.begin(), y.end(), 0.0);
    for (int c = 0; c < K; ++c) {
      if (conv[c]) continue;
      const int k = jc[c];
      kmax = std::max(kmax, k);
      const double* Hc = H.data() + (size_t)c * (m + 1) * m;
      const double* gc = g.data() + (size_t)c * (m + 1);
      for (int i = k - 1; i >= 0; --i) {
        double sum = gc[i];
        for (int q = i + 1; q < k; ++q) sum -= Hc[i * m + q] * y[(size_t)q * K + c];
        y[(size_t)i * K + c] = sum / Hc[i * m + i];
      }
    }
    for (int i = 0; i < kmax; ++i)
      for (int c = 0; c < K; ++c) hp[kMcY + i * K + c] = y[(size_t)i * K + c];
    HIPCHECK(hipMemcpyAsync(dsm + kMcY, hp + kMcY, (size_t)kmax * K * sizeof(double),
                            hipMemcpyHostToDevice, h.stream));
    launch_mc_update(h.mc_Z, ld, kmax, dsm + kMcY, x, N, K, h.stream);
    launch_spmm<double>(A, h.D, x, b, h.mc_w, K, true, h.stream);
    std::vector<double> tn;
    norms(h.mc_w, tn);
    for (int c = 0; c < K; ++c) {
      if (conv[c]) continue;
      true_rel[c] = tn[c] / bnorm[c];
      if (true_rel[c] <= o.rtol)
        conv[c] = 1;
      else
        ++restarts[c];
    }
  }
  HIPCHECK(hipGetLastError());
  bool ok = true;
  const double ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int c = 0; c < K; ++c) {
    ok &= conv[c] != 0;
    if (infos) {
      infos[c].iters = iters[c];
      infos[c].restarts = restarts[c];
      infos[c].converged = conv[c];
      infos[c].rel_res_true = true_rel[c];
      infos[c].history_len = 0;
      infos[c].t_solve_ms = ms;
      infos[c].vcycles = iters[c];
      infos[c].t_setup_ms = h.t_setup_ms;
      infos[c].t_blocks_ms = h.t_blocks_ms;
    }
  }
  return ok ? FSGMG_OK : FSGMG_NOT_CONVERGED;
}

// An Arnoldi step is queued ahead of the host's read-back of the previous one
// while the last residual estimate exceeds kSpeculate times the target.
constexpr double kSpeculate = 1e3;

fsgmg_status fgmres(fsgmg_hierarchy& h, const double* b, double* x, const fsgmg_krylov_opts& o,
                    fsgmg_solve_info* info, bool transpose) {
  const auto t0 = std::chrono::steady_clock::now();
  if (o.restart < 1 || o.restart > 31 || o.rtol <= 0 || o.max_restarts < 0)
    throw Fail{FSGMG_EINVAL, "krylov options out of range (restart 1..31, rtol > 0)"};
  if (!h.factors_valid) throw Fail{FSGMG_ESTATE, "build_fs_as_blocks has not been called"};
  if (transpose) ensure_transposed(h);
  const int m = o.restart;
  ensure_workspace(h, m);
  DLevel& F = h.dl[h.L - 1];
  const int64_t N = F.N, ld = h.ld;
  const BOpView<double>& A = transpose ? F.AT.v64 : F.A.v64;
  double* const yv = h.small + 96;  // 32 (h1, h2, ||w|| live in small[0..64])
  std::vector<double> hist;
  const double bnorm = device_norm(h, b, N);
  if (!std::isfinite(bnorm)) throw Fail{FSGMG_EINVAL, "right-hand side contains NaN or Inf"};
  launch_fill<double>(x, 0.0, N, h.stream);
  int iters = 0, restarts = 0;
  bool converged = false;
  double true_rel = NAN;
  if (bnorm == 0.0) {
    converged = true;
    true_rel = 0.0;
  }
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  for (int cycle = 0; !converged && cycle <= o.max_restarts; ++cycle) {
    launch_spmv<double>(A, h.D, x, b, h.w, true, h.stream, h.outer_lanes);
    const double beta = device_norm(h, h.w, N);
    if (cycle == 0) hist.push_back(beta / bnorm);
    if (beta <= o.rtol * bnorm) {
      converged = true;
      true_rel = beta / bnorm;
      break;
    }
    launch_scale_copy(h.w, h.small + 128, h.V, N, h.stream);
    std::fill(H.begin(), H.end(), 0.0);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    int queued = -1;          // last Arnoldi step enqueued
    double last_est = beta;   // latest residual estimate known on the host
    for (int j = 0; j < m; ++j) {
      if (queued < j) {
        run_arnoldi_step(h, j, transpose);
        queued = j;
      }
      HIPCHECK(hipEventRecord(h.step_done[j & 1], h.stream));
      // queue step j + 1 before reading step j back while convergence is
      // still far off (a step queued past convergence is wasted work only)
      if (j + 1 < m && last_est > kSpeculate * o.rtol * bnorm) {
        run_arnoldi_step(h, j + 1, transpose);
        queued = j + 1;
      }
      HIPCHECK(hipEventSynchronize(h.step_done[j & 1]));
      const double* pv = h.pinned + step_area(j);
      const double hn = pv[64];
      for (int i = 0; i <= j; ++i) H[i * m + j] = pv[i] + pv[32 + i];
      H[(j + 1) * m + j] = hn;
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
        H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t;
      }
      const double den = std::hypot(H[j * m + j], H[(j + 1) * m + j]);
      cs[j] = H[j * m + j] / den;
      sn[j] = H[(j + 1) * m + j] / den;
      H[j * m + j] = den;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++iters;
      k = j + 1;
      const double est = std::fabs(g[j + 1]);
      hist.push_back(est / bnorm);
      if (!std::isfinite(est)) throw Fail{FSGMG_EINVAL, "non-finite residual estimate"};
      last_est = est;
      if (est <= o.rtol * bnorm || hn == 0.0) break;
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int q = i + 1; q < k; ++q) s -= H[i * m + q] * y[q];
      y[i] = s / H[i * m + i];
    }
    HIPCHECK(hipMemcpyAsync(yv, y.data(), k * sizeof(double), hipMemcpyHostToDevice, h.stream));
    launch_gemv_update(h.Z, ld, k, yv, x, N, h.stream);
    launch_spmv<double>(A, h.D, x, b, h.w, true, h.stream, h.outer_lanes);
    true_rel = device_norm(h, h.w, N) / bnorm;
    if (true_rel <= o.rtol) {
      converged = true;
      break;
    }
    ++restarts;
  }
  HIPCHECK(hipGetLastError());
  if (info) {
    info->iters = iters;
    info->restarts = restarts;
    info->converged = converged ? 1 : 0;
    info->rel_res_true = true_rel;
    info->history_len = (int)hist.size();
    if (info->history && info->history_cap > 0)
      for (int i = 0; i < std::min(info->history_cap, (int)hist.size()); ++i) info->history[i] = hist[i];
    info->t_solve_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    info->vcycles = iters;
    info->t_setup_ms = h.t_setup_ms;
    info->t_blocks_ms = h.t_blocks_ms;
  }
  return converged ? FSGMG_OK : FSGMG_NOT_CONVERGED;
}

// Launch-shape autotuner: for every level time the V-cycle SpMV with 1 to 16
// lanes per row, the transfers' lanes, the smoother sweep with 256, 512 and
// 1024-thread workgroups (and several workgroups per block where blocks are
// few), the fused against the SpMV form of a sweep, and the outer FP64
// product's lanes.  Each candidate is timed cold: a read pass over a buffer
// larger than the last-level cache runs before every timed launch, as the
// finer levels' sweeps evict a coarse level's data inside a cycle (with the
// data cached, launch shapes with long chains of dependent loads look
// cheaper than they are there).  HIP events on the handle's stream around
// the launch alone; the median of five after one warm-up.
struct Flush {
  static constexpr int64_t kBytes = int64_t(512) << 20;   // twice the 256 MB cache
  fsgmg_hierarchy& h;
  void* buf = nullptr;
  uint32_t* sink = nullptr;
  explicit Flush(fsgmg_hierarchy& hh) : h(hh) {
    buf = h.raw_alloc(kBytes + 256);
    if (!buf) return;   // no room: the candidates are timed warm
    if (hipMemsetAsync(buf, 0, kBytes + 256, h.stream) != hipSuccess ||
        hipStreamSynchronize(h.stream) != hipSuccess) {
      (void)hipGetLastError();
      h.raw_free(buf);
      buf = nullptr;
      return;
    }
    sink = reinterpret_cast<uint32_t*>(static_cast<char*>(buf) + kBytes);
  }
  ~Flush() {
    if (buf) h.raw_free(buf);
  }
  Flush(const Flush&) = delete;
  Flush& operator=(const Flush&) = delete;
};

template <typename F>
float time_launch(fsgmg_hierarchy& h, const Flush& fl, F&& f) {
  constexpr int kReps = 5;
  hipEvent_t a = h.next_event(), b = h.next_event();
  f();
  float t[kReps];
  for (int i = 0; i < kReps; ++i) {
    if (fl.buf) launch_flush(fl.buf, Flush::kBytes, fl.sink, h.stream);
    HIPCHECK(hipEventRecord(a, h.stream));
    f();
    HIPCHECK(hipEventRecord(b, h.stream));
    HIPCHECK(hipEventSynchronize(b));
    HIPCHECK(hipEventElapsedTime(&t[i], a, b));
  }
  h.ev_used -= 2;
  std::sort(t, t + kReps);
  return t[kReps / 2];
}

template <typename TV>
void autotune_impl(fsgmg_hierarchy& h) {
  const Flush fl(h);
  const bool was_timing = h.timing;
  h.timing = false;
  h.tune.assign(h.L, {});
  const WPrec wp = wprec(h.sopt.prec);
  const int lanes[5] = {1, 2, 4, 8, 16}, threads[6] = {256, 512, 1024, -256, -512, -1024};
  for (int l = 0; l < h.L; ++l) {
    DLevel& d = h.dl[l];
    float best = 1e30f;
    for (int lg : lanes) {
      const float t = time_launch(h, fl, [&] {
        launch_spmv<TV>(Vec<TV>::op(d, false), h.D, Vec<TV>::x(d), Vec<TV>::b(d), Vec<TV>::r(d),
                        true, h.stream, lg);
      });
      if (t < best) {
        best = t;
        h.tune[l].spmv_lanes = lg;
      }
    }
    if (l == 0) continue;
    // transfers: restriction into level l-1 (coarse outputs, ~9-25 weights
    // each) and prolongation from it (fine outputs, 1-4 weights each)
    best = 1e30f;
    for (int lg : lanes) {
      const float t = time_launch(h, fl, [&] {
        launch_transfer<TV>(Vec<TV>::tv(d), h.D, 0, Vec<TV>::r(d), Vec<TV>::b(h.dl[l - 1]),
                            h.stream, lg);
      });
      if (t < best) {
        best = t;
        h.tune[l].restrict_lanes = lg;
      }
    }
    best = 1e30f;
    for (int lg : lanes) {
      const float t = time_launch(h, fl, [&] {
        launch_transfer<TV>(Vec<TV>::tv(d), h.D, 1, Vec<TV>::x(h.dl[l - 1]), Vec<TV>::r(d),
                            h.stream, lg);
      });
      if (t < best) {
        best = t;
        h.tune[l].prolong_lanes = lg;
      }
    }
    best = 1e30f;
    // multiplicative sweep: time the first colour (disjoint blocks, no Jacobi)
    BlocksView tv = d.bv;
    const BlockSet& bs = h.blocks[l];
    if (h.sopt.schwarz == FSGMG_SCHWARZ_MULTIPLICATIVE && bs.colour_ptr.size() > 1) {
      tv.nblk = bs.colour_ptr[1];
      tv.njac = 0;
    }
    // workgroups per block: more than one only where the blocks leave CUs idle
    const int splits[4] = {1, 2, 4, 8};
    const int nsplit = tv.nblk < 1024 ? 4 : 1;
    for (int th : threads)
      for (int q = 0; q < nsplit; ++q) {
        const float t = time_launch(h, fl, [&] {
          launch_smooth<TV>(tv, wp, d.W, Vec<TV>::b(d), Vec<TV>::x(d), Vec<TV>::t(d), 1.0, true,
                            false, d.N, h.stream, th, splits[q]);
        });
        if (t < best) {
          best = t;
          h.tune[l].smooth_threads = th;
          h.tune[l].split = splits[q];
        }
      }
    // a sweep after the first: residual SpMV + sweep, or one fused launch
    // that forms the blocks' residual rows itself (fewer launches, but every
    // block reads its own copy of its operator rows)
    {
      const float t_sep = time_launch(h, fl, [&] {
        launch_spmv<TV>(Vec<TV>::op(d, false), h.D, Vec<TV>::x(d), Vec<TV>::b(d), Vec<TV>::r(d),
                        true, h.stream, h.tune[l].spmv_lanes);
        launch_smooth<TV>(tv, wp, d.W, Vec<TV>::r(d), Vec<TV>::x(d), Vec<TV>::t(d), 1.0, false,
                          false, d.N, h.stream, h.tune[l].smooth_threads, h.tune[l].split);
      });
      float t_fused = 1e30f;
      int th_fused = h.tune[l].smooth_threads;
      if (h.sopt.sweep_form == 2 && !tv.rows_col)
        throw Fail{FSGMG_EINVAL, "the fused sweep form is not available on level " +
                                     std::to_string(l) +
                                     " (its blocks' operator-row copies exceed the budget)"};
      for (int th : threads) {
        if (!tv.rows_col) break;   // no operator-row copies: no fused form
        const float t = time_launch(h, fl, [&] {
          launch_smooth_fused<TV>(tv, wp, d.W, Vec<TV>::b(d), Vec<TV>::x(d), Vec<TV>::x2(d), 1.0,
                                  false, h.stream, th);
        });
        if (t < t_fused) {
          t_fused = t;
          th_fused = th;
        }
      }
      // the fused form reads the blocks' copies of A's rows, so the
      // interchanged cascade (its cycle uses the diagonal blocks of A) keeps
      // the SpMV form
      const int form = h.sopt.sweep_form;
      if (!h.sopt.interchange && (form == 2 || (form == 0 && t_fused < t_sep))) {
        h.tune[l].fused = 1;
        h.tune[l].smooth_threads = th_fused;
        h.tune[l].split = 1;
      }
    }
  }
  DLevel& F = h.dl[h.L - 1];
  float best = 1e30f;
  for (int lg : lanes) {
    const float t = time_launch(h, fl, [&] {
      launch_spmv<double>(F.A.v64, h.D, F.x64, F.b64, F.r64, true, h.stream, lg);
    });
    if (t < best) {
      best = t;
      h.outer_lanes = lg;
    }
  }
  HIPCHECK(hipGetLastError());
  h.timing = was_timing;
}

void autotune(fsgmg_hierarchy& h) {
  if (h.sopt.prec == FSGMG_FP64)
    autotune_impl<double>(h);
  else
    autotune_impl<float>(h);
}

// the checks shared by the several-right-hand-side entry points
void check_mc(fsgmg_hierarchy& h, int k) {
  if (k < 1 || k > kMaxRhs) throw Fail{FSGMG_EINVAL, "k must be in 1..64"};
  if (h.sopt.schwarz != FSGMG_SCHWARZ_ADDITIVE)
    throw Fail{FSGMG_EINVAL, "several right-hand sides need the additive smoother"};
  if (h.sopt.interchange)
    throw Fail{FSGMG_EINVAL, "several right-hand sides: not built for the interchanged cascade"};
  for (int l = 1; l < h.L; ++l)
    if (h.dl[l].bv.max_n > kMaxRhsBlock)
      throw Fail{FSGMG_EINVAL, "several right-hand sides: a Schwarz block exceeds " +
                                   std::to_string(kMaxRhsBlock) + " unknowns"};
}

void check_device(fsgmg_hierarchy& h) {
  if (h.host_only()) throw Fail{FSGMG_ESTATE, "device call on a host-only handle"};
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
static fsgmg_status build_fs_as_blocks_impl(fsgmg_h h, const fsgmg_smoother_opts* opts);

extern "C" {

// The finest-level advecting velocity injected at the nodes of level l.
static std::vector<double> level_velocity(const fsgmg_hierarchy& h, int l) {
  const Level& Fl = h.levels[h.L - 1];
  const Level& lv = h.levels[l];
  std::vector<double> wl;
  if (h.w_finest.empty()) return wl;
  const int step = 1 << (h.L - 1 - l);
  wl.resize(lv.N2 * h.D);
  for (int64_t n = 0; n < lv.N2; ++n) {
    int ix[kMaxDim] = {0, 0, 0};
    lv.node_ijk(n, ix);
    int fx[kMaxDim] = {0, 0, 0};
    for (int a = 0; a < h.D; ++a) fx[a] = ix[a] * step;
    const int64_t fn = Fl.node_index(fx);
    for (int c = 0; c < h.D; ++c) wl[n * h.D + c] = h.w_finest[fn * h.D + c];
  }
  return wl;
}

// Run f(l) for every level, one host thread each.
static void for_levels(int L, const std::function<void(int)>& f) {
  std::vector<std::thread> pool;
  std::vector<std::exception_ptr> errs(L);
  for (int l = 0; l < L; ++l)
    pool.emplace_back([&, l]() {
      try {
        f(l);
      } catch (...) {
        errs[l] = std::current_exception();
      }
    });
  for (std::thread& t : pool) t.join();
  for (const std::exception_ptr& e : errs)
    if (e) std::rethrow_exception(e);
}

// Assemble every level operator about the handle's physics and finest-level
// advecting velocity (injected at each level's nodes: the meshes are nested
// and Q2 nodes of a coarse level are nodes of every finer one); the levels
// are independent and are assembled on one host thread each.  plans !=
// nullptr also keeps each level's re-assembly plan.
static void assemble_all(fsgmg_hierarchy& h, std::vector<LevelOperator>& ops,
                         std::vector<AdvectionPlan>* plans = nullptr) {
  const std::vector<double> cvol = element_volumes(h.levels[0]);
  ops.clear();
  ops.resize(h.L);
  if (plans) {
    plans->clear();
    plans->resize(h.L);
  }
  for_levels(h.L, [&](int l) {
    const std::vector<double> wl = level_velocity(h, l);
    assemble_level(h.levels[l], h.phys, cvol, wl.empty() ? nullptr : &wl, l == h.L - 1, ops[l],
                   plans ? &(*plans)[l] : nullptr);
  });
}

// Re-assemble the values of every level operator in place about the
// handle's current advecting velocity, from the plans.
static void reassemble_all(fsgmg_hierarchy& h) {
  for_levels(h.L, [&](int l) {
    reassemble_level(h.levels[l], h.phys, h.plans[l], level_velocity(h, l), l == h.L - 1,
                     h.ops[l]);
  });
}

fsgmg_status setup_hierarchy(const fsgmg_mesh_desc* mesh, const fsgmg_physics* phys,
                             const fsgmg_allocator* alloc, int device, void* stream, fsgmg_h* out) {
  if (!mesh || !phys || !out) return FSGMG_EINVAL;
  *out = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  auto h = std::make_unique<fsgmg_hierarchy>();
  h->device = device;
  h->stream = (hipStream_t)stream;
  fsgmg_status st = guarded(h.get(), [&]() -> fsgmg_status {
    if (alloc && (!alloc->alloc) != (!alloc->free))
      throw Fail{FSGMG_EINVAL, "an allocator needs both alloc and free"};
    if (alloc && alloc->alloc) h->alloc = *alloc;
    if (mesh->dim != 2 && mesh->dim != 3) throw Fail{FSGMG_EINVAL, "dim must be 2 or 3"};
    if (mesh->n_levels < 1 || mesh->n_levels > 12) throw Fail{FSGMG_EINVAL, "n_levels out of range"};
    int64_t nce = 1;
    for (int a = 0; a < mesh->dim; ++a) {
      if (mesh->nc[a] < 1 || !mesh->breaks[a]) throw Fail{FSGMG_EINVAL, "bad coarse mesh"};
      nce *= mesh->nc[a];
    }
    if (!mesh->region) throw Fail{FSGMG_EINVAL, "region tags missing"};
    if (!(phys->E > 0) || !(phys->nu > 0 && phys->nu <= 0.5) || !(phys->mu > 0) ||
        !(phys->rho > 0) || !std::isfinite(phys->E) || !std::isfinite(phys->mu) ||
        !std::isfinite(phys->rho))
      throw Fail{FSGMG_EINVAL, "physical parameters out of range"};
    if (!(phys->theta >= 0 && phys->theta <= 1))
      throw Fail{FSGMG_EINVAL, "theta must lie in (0, 1] (0 selects 1)"};
    h->mesh = *mesh;
    for (int a = 0; a < mesh->dim; ++a) {
      h->breaks[a].assign(mesh->breaks[a], mesh->breaks[a] + mesh->nc[a] + 1);
      h->mesh.breaks[a] = h->breaks[a].data();
    }
    h->region.assign(mesh->region, mesh->region + nce);
    h->mesh.region = h->region.data();
    h->L = mesh->n_levels;
    h->D = mesh->dim;
    h->levels.resize(h->L);
    for (int l = 0; l < h->L; ++l) build_level(h->mesh, l, h->levels[l]);
    const Level& Fl = h->levels[h->L - 1];
    if (phys->w) h->w_finest.assign(phys->w, phys->w + Fl.N2 * h->D);
    h->phys = Physics{phys->E, phys->nu, phys->mu, phys->rho,
                      (phys->dt > 0 && std::isfinite(phys->dt)) ? 1.0 / phys->dt : 0.0,
                      phys->theta > 0 ? phys->theta : 1.0, phys->supg, phys->ale_k, phys->k_mass,
                      h->w_finest.empty() ? nullptr : h->w_finest.data(), h->L};
    assemble_all(*h, h->ops);
    h->tr.resize(h->L);
    for (int l = 1; l < h->L; ++l) build_transfer(h->levels[l], h->levels[l - 1], h->tr[l]);
    h->blocks.resize(h->L);
    if (device >= 0) {
      int ndev = 0;
      HIPCHECK(hipGetDeviceCount(&ndev));
      if (device >= ndev) throw Fail{FSGMG_EINVAL, "device index out of range"};
      HIPCHECK(hipSetDevice(device));
      upload_all(*h);
      HIPCHECK(hipStreamSynchronize(h->stream));
    }
    h->t_setup_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return FSGMG_OK;
  });
  // on failure the handle is still returned so that last_error() can be read;
  // the caller destroys it
  *out = h.release();
  return st;
}

fsgmg_status build_fs_as_blocks(fsgmg_h h, const fsgmg_smoother_opts* opts) {
  if (!h || !opts) return FSGMG_EINVAL;
  const auto t0 = std::chrono::steady_clock::now();
  const fsgmg_status st = build_fs_as_blocks_impl(h, opts);
  if (st == FSGMG_OK)
    h->t_blocks_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

static fsgmg_status build_fs_as_blocks_impl(fsgmg_h h, const fsgmg_smoother_opts* opts) {
  return guarded(h, [&]() -> fsgmg_status {
    if (opts->halo < 0 || opts->nu_pre < 0 || opts->nu_post < 0 || !(opts->omega > 0))
      throw Fail{FSGMG_EINVAL, "smoother options out of range"};
    for (int a = 0; a < h->D; ++a)
      if (opts->core[a] < 1) throw Fail{FSGMG_EINVAL, "core sizes must be >= 1"};
    if (opts->prec < FSGMG_FP64 || opts->prec > FSGMG_BF16) throw Fail{FSGMG_EINVAL, "bad precision"};
    if (opts->cycle < FSGMG_CYCLE_V || opts->cycle > FSGMG_CYCLE_F)
      throw Fail{FSGMG_EINVAL, "cycle must be FSGMG_CYCLE_V, _W or _F"};
    if (opts->iface_mult < 0) throw Fail{FSGMG_EINVAL, "iface_mult must be >= 0"};
    if (opts->schwarz != FSGMG_SCHWARZ_ADDITIVE && opts->schwarz != FSGMG_SCHWARZ_MULTIPLICATIVE)
      throw Fail{FSGMG_EINVAL, "schwarz must be FSGMG_SCHWARZ_ADDITIVE or _MULTIPLICATIVE"};
    if (opts->sweep_form < 0 || opts->sweep_form > 2)
      throw Fail{FSGMG_EINVAL, "sweep_form must be 0 (autotuned), 1 (SpMV) or 2 (fused)"};
    if (opts->interchange && opts->sweep_form == 2)
      throw Fail{FSGMG_EINVAL, "the interchanged cascade runs its sweeps in the SpMV form"};
    const int mult = std::max(1, opts->iface_mult);
    const bool same_sets = h->have_blocks && h->sopt.halo == opts->halo &&
                           h->sopt.core[0] == opts->core[0] && h->sopt.core[1] == opts->core[1] &&
                           h->sopt.core[2] == opts->core[2] &&
                           std::max(1, h->sopt.iface_mult) == mult &&
                           (h->sopt.monolithic != 0) == (opts->monolithic != 0) &&
                           h->sopt.schwarz == opts->schwarz && h->sopt.prec == opts->prec;
    const int prev_form = h->sopt.sweep_form;
    // The captured graphs hold buffer addresses, launch shapes and the
    // options' scalars only.  A rebuild that keeps the index sets, the
    // precision, every other option and the tuning refactors into the same
    // buffers (update_params likewise rewrites values in place), so its
    // graphs stay valid and are not captured again.
    const fsgmg_smoother_opts& o = h->sopt;
    const bool keep_graphs = same_sets && h->tuned && o.nu_pre == opts->nu_pre &&
                             o.nu_post == opts->nu_post && o.omega == opts->omega &&
                             o.use_graph == opts->use_graph && o.cycle == opts->cycle &&
                             o.sweep_form == opts->sweep_form &&
                             (o.interchange != 0) == (opts->interchange != 0);
    h->sopt = *opts;
    h->factors_valid = false;
    if (!keep_graphs) h->invalidate_graphs();
    if (!same_sets) {
      h->ensure_host_values();   // the colouring reads the operator's values
      try {
        for (int l = 1; l < h->L; ++l) {
          build_blocks(h->levels[l], opts->core, opts->halo, mult, opts->monolithic != 0,
                       h->blocks[l]);
          if (opts->schwarz == FSGMG_SCHWARZ_MULTIPLICATIVE)
            colour_blocks(h->ops[l].A, h->ops[l].piece, 4, h->blocks[l]);
        }
      } catch (const std::invalid_argument& e) {
        h->have_blocks = false;
        throw Fail{FSGMG_EINVAL, e.what()};
      }
      h->have_blocks = true;
      if (!h->host_only())
        for (int l = 1; l < h->L; ++l) {
          upload_blocks(*h, l);
          h->dl[l].fp.ready = false;   // new index sets: new factorization plan
        }
    }
    if (h->host_only()) return FSGMG_OK;
    // the cycle's operators: A, or the field split's diagonal blocks of A
    // for the interchanged cascade (whose level-0 direct solve is then that
    // of level 0's diagonal blocks)
    if (opts->interchange) ensure_bd(*h);
    for (DLevel& d : h->dl) d.use_bd = opts->interchange != 0;
    if (h->coarse_bd != (opts->interchange != 0)) {
      ensure_coarse(*h);
      build_coarse_inverse(*h);
    }
    struct ClearHook {
      fsgmg_hierarchy* h;
      ~ClearHook() { h->zero_block_level = -1, h->zero_block = -1; }
    } clear_hook{h};
    // launch shapes depend on the block structure only: keep them while the
    // index sets and precision are unchanged, so rebuilds stay reproducible
    const bool retune = !same_sets || !h->tuned || prev_form != opts->sweep_form;
    factor_blocks(*h, retune);
    if (retune) autotune(*h);
    h->tuned = true;
    h->factors_valid = true;
    return FSGMG_OK;
  });
}

fsgmg_status vcycle_apply(fsgmg_h h, const double* r, double* z, int transpose) {
  if (!h || !r || !z || r == z) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    if (!h->factors_valid) throw Fail{FSGMG_ESTATE, "build_fs_as_blocks has not been called"};
    if (transpose && h->sopt.interchange)
      throw Fail{FSGMG_EINVAL, "the interchanged cascade has no transposed cycle"};
    if (transpose) ensure_transposed(*h);
    ensure_coarse(*h);
    vcycle(*h, r, z, transpose != 0);
    HIPCHECK(hipGetLastError());
    return FSGMG_OK;
  });
}

fsgmg_status vcycle_apply_batch(fsgmg_h h, const double* r, double* z, int k, int transpose) {
  if (!h || !r || !z || r == z) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    if (!h->factors_valid) throw Fail{FSGMG_ESTATE, "build_fs_as_blocks has not been called"};
    check_mc(*h, k);
    ensure_coarse(*h);
    if (transpose) ensure_transposed(*h);
    vcycle_mc(*h, r, z, k, transpose != 0);
    HIPCHECK(hipGetLastError());
    return FSGMG_OK;
  });
}

fsgmg_status gmres_solve_batch(fsgmg_h h, const double* b, double* x, int k,
                               const fsgmg_krylov_opts* opts, fsgmg_solve_info* infos) {
  if (!h || !b || !x || !opts || b == x) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    check_mc(*h, k);
    ensure_coarse(*h);
    return fgmres_batch(*h, b, x, k, *opts, infos);
  });
}

fsgmg_status adjoint_solve_batch(fsgmg_h h, const double* c, double* lam, int k,
                                 const fsgmg_krylov_opts* opts, fsgmg_solve_info* infos) {
  if (!h || !c || !lam || !opts || c == lam) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    check_mc(*h, k);
    ensure_coarse(*h);
    return fgmres_batch(*h, c, lam, k, *opts, infos, true);
  });
}

fsgmg_status gmres_solve(fsgmg_h h, const double* b, double* x, const fsgmg_krylov_opts* opts,
                         fsgmg_solve_info* info) {
  if (!h || !b || !x || !opts || b == x) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    ensure_coarse(*h);
    return fgmres(*h, b, x, *opts, info, false);
  });
}

fsgmg_status adjoint_solve(fsgmg_h h, const double* c, double* lam, const fsgmg_krylov_opts* opts,
                           fsgmg_solve_info* info) {
  if (!h || !c || !lam || !opts || c == lam) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    if (h->sopt.interchange)
      throw Fail{FSGMG_EINVAL, "the interchanged cascade has no transposed cycle for the adjoint"};
    ensure_coarse(*h);
    return fgmres(*h, c, lam, *opts, info, true);
  });
}

fsgmg_status assemble_load(fsgmg_h h, const double* f, double* b) {
  if (!h || !f || !b) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    launch_load_rhs(h->dl[h->L - 1].N, h->load_rp, h->load_col, h->load_val, f, h->lift, b, h->stream);
    HIPCHECK(hipGetLastError());
    return FSGMG_OK;
  });
}

fsgmg_status load_adjoint(fsgmg_h h, const double* lam, double* gf) {
  if (!h || !lam || !gf || (const void*)lam == (void*)gf) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    const Level& F = h->levels[h->L - 1];
    launch_csr_spmv((int64_t)F.D * F.N2, h->loadT_rp, h->loadT_col, h->loadT_val, lam, gf, 0.0,
                    h->stream);
    HIPCHECK(hipGetLastError());
    return FSGMG_OK;
  });
}

fsgmg_status apply_operator(fsgmg_h h, int level, const double* x, double* y, int transpose) {
  if (!h || !x || !y || x == y) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    if (level < 0 || level >= h->L) throw Fail{FSGMG_EINVAL, "level out of range"};
    if (transpose) ensure_transposed(*h);
    DLevel& d = h->dl[level];
    launch_spmv<double>(transpose ? d.AT.v64 : d.A.v64, h->D, x, nullptr, y, false, h->stream);
    HIPCHECK(hipGetLastError());
    return FSGMG_OK;
  });
}

fsgmg_status param_grad(fsgmg_h h, const double* lam, const double* x, double out[2]) {
  if (!h || !lam || !x || !out) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    const Level& F = h->levels[h->L - 1];
    const LevelOperator& op = h->ops[h->L - 1];
    double s[3];
    const int pieces[3] = {1, 2, 3};
    for (int q = 0; q < 3; ++q) {
      launch_csr_spmv(F.N, h->full_rp, h->full_col, h->full_piece[pieces[q]], x, h->tmp, 0.0, h->stream);
      ensure_reduction_buffers(*h);
      launch_masked_dot(lam, h->dir_mask, h->tmp, F.N, h->part, h->small + 200, h->stream);
      HIPCHECK(hipMemcpyAsync(h->pinned, h->small + 200, sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIPCHECK(hipStreamSynchronize(h->stream));
      s[q] = h->pinned[0];
    }
    const double nu = h->phys.nu, E = h->phys.E;
    const double dG = 1.0 / (2.0 * (1.0 + nu));
    const double dI = nu >= 0.5 ? 0.0 : -(1.0 + nu) * (1.0 - 2.0 * nu) / (nu * E * E);
    (void)op;
    out[0] = -(dG * s[0] + dI * s[1]);
    out[1] = -s[2];
    return FSGMG_OK;
  });
}

fsgmg_status param_grad_noalloc(fsgmg_h h, const double* lam, const double* x, double out[2]) {
  if (!h || !lam || !x || !out) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    const Level& F = h->levels[h->L - 1];
    // scratch layout: dA/dtheta x (N doubles) | reduction partials | 3 sums
    auto up256 = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t off_part = up256((size_t)F.N * sizeof(double));
    const size_t off_sum = off_part + up256((size_t)krylov_partials() * sizeof(double));
    const size_t need = off_sum + 3 * sizeof(double);
    if (need > kNoAllocScratchBytes)
      throw Fail{FSGMG_EINVAL, "param_grad_noalloc: " + std::to_string(F.N) +
                                   " unknowns need " + std::to_string(need) +
                                   " bytes of scratch, more than its " +
                                   std::to_string(kNoAllocScratchBytes)};
    const char* err = "";
    char* base = static_cast<char*>(noalloc_scratch(h->device, &err));
    if (!base) throw Fail{FSGMG_EHIP, err};
    double* tmp = reinterpret_cast<double*>(base);
    double* part = reinterpret_cast<double*>(base + off_part);
    double* sum = reinterpret_cast<double*>(base + off_sum);
    // every scratch word read below is written first in the same call (the
    // product with beta = 0, each workgroup's partial, each sum)
    const int pieces[3] = {1, 2, 3};
    for (int q = 0; q < 3; ++q) {
      launch_csr_spmv(F.N, h->full_rp, h->full_col, h->full_piece[pieces[q]], x, tmp, 0.0, h->stream);
      launch_masked_dot(lam, h->dir_mask, tmp, F.N, part, sum + q, h->stream);
    }
    double s[3];
    HIPCHECK(hipMemcpyAsync(s, sum, sizeof(s), hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    const double nu = h->phys.nu, E = h->phys.E;
    const double dG = 1.0 / (2.0 * (1.0 + nu));
    const double dI = nu >= 0.5 ? 0.0 : -(1.0 + nu) * (1.0 - 2.0 * nu) / (nu * E * E);
    out[0] = -(dG * s[0] + dI * s[1]);
    out[1] = -s[2];
    return FSGMG_OK;
  });
}

fsgmg_status update_params(fsgmg_h h, double E, double mu) {
  if (!h) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    if (!(E > 0) || !(mu > 0) || !std::isfinite(E) || !std::isfinite(mu))
      throw Fail{FSGMG_EINVAL, "parameters must be positive and finite"};
    h->phys.E = E;
    h->phys.mu = mu;
    double G, invlam;
    lame(E, h->phys.nu, G, invlam);
    for (int l = 0; l < h->L; ++l) {
      LevelOperator& op = h->ops[l];
      op.G = G;
      op.invlam = invlam;
      op.mu = mu;
    }
    h->host_vals_stale = true;
    h->factors_valid = false;
    if (h->host_only()) {
      h->ensure_host_values();
      return FSGMG_OK;
    }
    wait_coarse(*h);
    for (int l = 0; l < h->L; ++l) {
      DLevel& d = h->dl[l];
      launch_recombine(d.nnz, d.piece[0], d.piece[1], d.piece[2], d.piece[3], G, invlam, mu, d.val,
                       nullptr, h->stream);
      launch_scatter(d.nnz, d.val, d.A.map, d.A.vals64, d.A.vals32, h->stream);
      if (d.AT.ready) launch_scatter(d.nnz, d.val, d.AT.map, d.AT.vals64, d.AT.vals32, h->stream);
    }
    const int64_t NF = h->dl[h->L - 1].N;
    launch_recombine(NF, h->lift_piece[0], h->lift_piece[1], h->lift_piece[2], h->lift_piece[3], G,
                     invlam, mu, h->lift, nullptr, h->stream);
    if (h->time_val) {   // the explicit part of a theta step carries G and mu
      const LevelOperator& F = h->ops[h->L - 1];
      launch_recombine((int64_t)F.time.col.size(), h->time_piece[0], h->time_piece[1],
                       h->time_piece[2], h->time_piece[3], G, invlam, mu, h->time_val, nullptr,
                       h->stream);
    }
    HIPCHECK(hipGetLastError());
    if (!h->bd.empty()) h->bd_dirty = true;      // the diagonal blocks follow the values
    if (h->dl[0].use_bd) ensure_bd(*h);
    build_coarse_inverse(*h, true);
    return FSGMG_OK;
  });
}

// Values of every level operator, the Dirichlet lift's pieces and the
// finest level's unreduced pieces from freshly assembled host operators with
// the patterns already on the device, recombined for the current (E, mu) as
// update_params does.
static void upload_operator_values(fsgmg_hierarchy& h) {
  wait_coarse(h);
  for (int l = 0; l < h.L; ++l) {
    DLevel& d = h.dl[l];
    const LevelOperator& op = h.ops[l];
    for (int p = 0; p < 4; ++p)
      HIPCHECK(hipMemcpyAsync(d.piece[p], op.piece[p].data(), op.piece[p].size() * sizeof(double),
                              hipMemcpyHostToDevice, h.stream));
    launch_recombine(d.nnz, d.piece[0], d.piece[1], d.piece[2], d.piece[3], op.G, op.invlam, op.mu,
                     d.val, nullptr, h.stream);
    launch_scatter(d.nnz, d.val, d.A.map, d.A.vals64, d.A.vals32, h.stream);
    if (d.AT.ready) launch_scatter(d.nnz, d.val, d.AT.map, d.AT.vals64, d.AT.vals32, h.stream);
  }
  const LevelOperator& F = h.ops[h.L - 1];
  const int64_t NF = h.dl[h.L - 1].N;
  for (int p = 0; p < 4; ++p) {
    HIPCHECK(hipMemcpyAsync(h.lift_piece[p], F.lift_piece[p].data(), NF * sizeof(double),
                            hipMemcpyHostToDevice, h.stream));
    HIPCHECK(hipMemcpyAsync(h.full_piece[p], F.full_piece[p].data(),
                            F.full_piece[p].size() * sizeof(double), hipMemcpyHostToDevice,
                            h.stream));
  }
  launch_recombine(NF, h.lift_piece[0], h.lift_piece[1], h.lift_piece[2], h.lift_piece[3], F.G,
                   F.invlam, F.mu, h.lift, nullptr, h.stream);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(h.stream));
}

// Host copies of every value array a device re-assembly wrote: the level
// operators' pieces (the values follow on the host when needed), and on the
// finest level the unreduced pieces, the lift pieces, the load operator
// and the time operator's pieces.
void fsgmg_hierarchy::pull_device_values() {
  auto pull = [&](std::vector<double>& to, const double* from) {
    if (!to.empty() && from)
      HIPCHECK(hipMemcpyAsync(to.data(), from, to.size() * sizeof(double), hipMemcpyDeviceToHost,
                              stream));
  };
  for (int l = 0; l < L; ++l)
    for (int p = 0; p < 4; ++p) pull(ops[l].piece[p], dl[l].piece[p]);
  LevelOperator& F = ops[L - 1];
  for (int p = 0; p < 4; ++p) {
    pull(F.full_piece[p], full_piece[p]);
    pull(F.lift_piece[p], lift_piece[p]);
    if (time_val) pull(F.time_piece[p], time_piece[p]);
  }
  pull(F.load.val, load_val);
  HIPCHECK(hipStreamSynchronize(stream));
  if (time_val)
    for (size_t k = 0; k < F.time.val.size(); ++k)
      F.time.val[k] = F.time_piece[0][k] + F.G * F.time_piece[1][k] +
                      F.invlam * F.time_piece[2][k] + F.mu * F.time_piece[3][k];
  device_ahead = false;
  host_vals_stale = true;
}

static bool dev_adv_eligible(const fsgmg_hierarchy& h) {
  if (h.host_only() || h.D != 2 || h.plans.size() != (size_t)h.L) return false;
  if (h.sopt.schwarz == FSGMG_SCHWARZ_MULTIPLICATIVE || h.sopt.interchange) return false;
  for (const AdvectionPlan& P : h.plans)
    if (!P.ready || (!P.elems.empty() && P.slots.empty())) return false;
  return true;
}

static void run_dev_adv(fsgmg_hierarchy& h, const double* x);

// Upload what the device re-assembly needs, from the plans (the term slots
// recorded by the host assembly, in its order), then check once that every
// element emits the number of terms the host recorded.
static void build_dev_adv(fsgmg_hierarchy& h, const double* x) {
  const std::vector<double> ref = reference_tables(h.D);
  if (ref.size() != (size_t)kRefSize) throw Fail{FSGMG_ESTATE, "reference table layout"};
  h.adv_ref = h.upload(ref);
  h.adv_flag = h.zeros<int32_t>(1);
  h.loadT_perm_dev = h.upload(h.loadT_perm);
  std::vector<fsgmg_hierarchy::DevAdv> dadv(h.L);
  const Level& Fl = h.levels[h.L - 1];
  for (int l = 0; l < h.L; ++l) {
    const Level& lv = h.levels[l];
    const AdvectionPlan& P = h.plans[l];
    const LevelOperator& op = h.ops[l];
    const bool finest = l == h.L - 1;
    fsgmg_hierarchy::DevAdv& a = dadv[l];
    a.nfluid = (int64_t)P.elems.size();
    a.per = P.per;
    if (a.nfluid == 0) continue;
    if ((int64_t)P.slots.size() != a.nfluid * a.per || P.dest.size() != P.slots.size())
      throw Fail{FSGMG_ESTATE, "re-assembly plan sizes"};
    a.elems = h.upload(P.elems);
    a.elem_nodes = h.upload(lv.elem_nodes);
    a.X = h.upload(lv.X);
    std::vector<int32_t> nf(lv.N2);
    const int step = 1 << (h.L - 1 - l);
    for (int64_t n = 0; n < lv.N2; ++n) {
      int ix[kMaxDim] = {0, 0, 0}, fx[kMaxDim] = {0, 0, 0};
      lv.node_ijk(n, ix);
      for (int c = 0; c < h.D; ++c) fx[c] = ix[c] * step;
      nf[n] = (int32_t)Fl.node_index(fx);
    }
    a.node_fine = h.upload(nf);
    a.emit = (double*)h.dalloc((size_t)(a.nfluid * a.per) * sizeof(double));
    // the reduced entry of every unreduced one (finest level), -1 for the
    // entries of Dirichlet rows and columns
    std::vector<int64_t> red_of_full;
    if (finest) {
      red_of_full.assign(op.full.nnz(), -1);
      for (int64_t i = 0; i < lv.N; ++i) {
        if (lv.dir[i]) continue;
        int64_t o = op.A.rowptr[i];
        for (int64_t k = op.full.rowptr[i]; k < op.full.rowptr[i + 1]; ++k)
          if (!lv.dir[op.full.col[k]]) red_of_full[k] = o++;
      }
    }
    // touched entries: the terms grouped by (array, entry), in term order
    std::vector<std::pair<uint64_t, int64_t>> keyed;
    keyed.reserve(P.slots.size());
    for (int64_t k = 0; k < (int64_t)P.slots.size(); ++k)
      if (P.slots[k] >= 0) keyed.emplace_back(((uint64_t)P.dest[k] << 40) | (uint64_t)P.slots[k], k);
    std::sort(keyed.begin(), keyed.end());
    std::vector<uint8_t> arr;
    std::vector<int64_t> slot, ptr{0}, em, red;
    std::vector<double> stat;
    for (size_t q = 0; q < keyed.size(); ++q) {
      if (q == 0 || keyed[q].first != keyed[q - 1].first) {
        const int d = (int)(keyed[q].first >> 40);
        const int64_t sl = (int64_t)(keyed[q].first & ((uint64_t(1) << 40) - 1));
        const int tgt = d / 4, p = d % 4;
        if (tgt > 2 || (tgt == 2 && p != 0) || (tgt > 0 && !finest) ||
            (tgt == 1 && !h.time_piece[p]))
          throw Fail{FSGMG_ESTATE, "re-assembly plan destinations"};
        const std::vector<double>& sv = tgt == 0 ? P.stat[p] : (tgt == 1 ? P.tstat[p] : P.lstat);
        if (sl >= (int64_t)sv.size()) throw Fail{FSGMG_ESTATE, "re-assembly plan slots"};
        if (q > 0) ptr.push_back((int64_t)em.size());
        arr.push_back((uint8_t)d);
        slot.push_back(sl);
        stat.push_back(sv[sl]);
        red.push_back(finest && tgt == 0 ? red_of_full[sl] : -1);
      }
      em.push_back(keyed[q].second);
    }
    ptr.push_back((int64_t)em.size());
    a.nt = (int64_t)arr.size();
    a.t_arr = h.upload(arr);
    a.t_slot = h.upload(slot);
    a.t_stat = h.upload(stat);
    a.t_ptr = h.upload(ptr);
    a.t_em = h.upload(em);
    a.t_red = finest ? h.upload(red) : nullptr;
    if (finest) {   // rows whose lift reads nonzero Dirichlet data, and those entries
      std::vector<int64_t> lrow, lptr{0}, lk;
      std::vector<double> lg;
      for (int64_t i = 0; i < lv.N; ++i) {
        if (lv.dir[i]) continue;
        const size_t before = lk.size();
        for (int64_t k = op.full.rowptr[i]; k < op.full.rowptr[i + 1]; ++k) {
          const int32_t j = op.full.col[k];
          if (!lv.dir[j] || lv.dir_val[j] == 0.0) continue;
          lk.push_back(k);
          lg.push_back(lv.dir_val[j]);
        }
        if (lk.size() > before) {
          lrow.push_back(i);
          lptr.push_back((int64_t)lk.size());
        }
      }
      a.nl = (int64_t)lrow.size();
      a.l_row = h.upload(lrow);
      a.l_ptr = h.upload(lptr);
      a.l_k = h.upload(lk);
      a.l_g = h.upload(lg);
    }
  }
  h.dadv = std::move(dadv);
  // one run: every element must emit the number of terms the host recorded
  run_dev_adv(h, x);
  int32_t flag = 0;
  HIPCHECK(hipMemcpyAsync(&flag, h.adv_flag, sizeof(int32_t), hipMemcpyDeviceToHost, h.stream));
  HIPCHECK(hipStreamSynchronize(h.stream));
  if (flag & 2) {
    h.dadv.clear();
    throw Fail{FSGMG_ESTATE, "device re-assembly emits another number of terms than the host"};
  }
}

// The advective terms of every level about the velocity part of the device
// vector x, added on the device to the velocity-independent sums; then the
// lift, the load operator's transpose, the time operator's values and every
// level operator's values and device layouts follow.  Asynchronous.
static void run_dev_adv(fsgmg_hierarchy& h, const double* x) {
  const Level& F = h.levels[h.L - 1];
  wait_coarse(h);
  HIPCHECK(hipMemsetAsync(h.adv_flag, 0, sizeof(int32_t), h.stream));
  for (int l = 0; l < h.L; ++l) {
    const fsgmg_hierarchy::DevAdv& a = h.dadv[l];
    if (a.nfluid == 0) continue;
    const bool finest = l == h.L - 1;
    AdvElemView v;
    v.nfluid = a.nfluid;
    v.per = a.per;
    v.elems = a.elems;
    v.elem_nodes = a.elem_nodes;
    v.X = a.X;
    v.node_fine = a.node_fine;
    v.x = x;
    v.off_u = F.off_u;
    v.ref = h.adv_ref;
    v.rho = h.phys.rho;
    v.mu = h.phys.mu;
    v.inv_dt = h.phys.inv_dt;
    v.theta = h.phys.theta;
    v.supg = h.phys.supg;
    v.finest = finest ? 1 : 0;
    v.emit = a.emit;
    v.flag = h.adv_flag;
    launch_adv_elements(v, h.stream);
    AdvGatherView g;
    g.n = a.nt;
    g.arr = a.t_arr;
    g.slot = a.t_slot;
    g.stat = a.t_stat;
    g.ptr = a.t_ptr;
    g.em = a.t_em;
    g.red = a.t_red;
    g.emit = a.emit;
    DLevel& d = h.dl[l];
    for (int p = 0; p < 4; ++p) {
      if (finest) {
        g.dst[p] = h.full_piece[p];
        g.dst_red[p] = d.piece[p];
        g.dst[4 + p] = h.time_piece[p];
      } else {
        g.dst[p] = d.piece[p];
      }
    }
    if (finest) g.dst[8] = h.load_val;
    launch_adv_gather(g, h.stream);
    if (finest) {
      launch_adv_lift(a.nl, a.l_row, a.l_ptr, a.l_k, a.l_g, h.full_piece[0], h.full_piece[1],
                      h.full_piece[2], h.full_piece[3], h.lift_piece[0], h.lift_piece[1],
                      h.lift_piece[2], h.lift_piece[3], h.stream);
    }
  }
  const LevelOperator& Fo = h.ops[h.L - 1];
  launch_permute_values((int64_t)h.loadT_perm.size(), h.loadT_perm_dev, h.load_val, h.loadT_val,
                        h.stream);
  launch_recombine(F.N, h.lift_piece[0], h.lift_piece[1], h.lift_piece[2], h.lift_piece[3], Fo.G,
                   Fo.invlam, Fo.mu, h.lift, nullptr, h.stream);
  if (h.time_val)
    launch_recombine((int64_t)Fo.time.col.size(), h.time_piece[0], h.time_piece[1],
                     h.time_piece[2], h.time_piece[3], Fo.G, Fo.invlam, Fo.mu, h.time_val,
                     nullptr, h.stream);
  for (int l = 0; l < h.L; ++l) {
    DLevel& d = h.dl[l];
    const LevelOperator& op = h.ops[l];
    launch_recombine(d.nnz, d.piece[0], d.piece[1], d.piece[2], d.piece[3], op.G, op.invlam, op.mu,
                     d.val, nullptr, h.stream);
    launch_scatter(d.nnz, d.val, d.A.map, d.A.vals64, d.A.vals32, h.stream);
    if (d.AT.ready) launch_scatter(d.nnz, d.val, d.AT.map, d.AT.vals64, d.AT.vals32, h.stream);
  }
  HIPCHECK(hipGetLastError());
  h.device_ahead = true;
}

static bool same_pattern(const CsrHost& a, const CsrHost& b) {
  return a.rowptr == b.rowptr && a.col == b.col;
}

// Re-assemble every level about the advecting velocity w = the velocity
// part of the finest-level vector x (the Picard step of the nonlinear
// loop): operators, lift, load and time operators.  The first call keeps a
// plan per level (the sums of the terms that do not depend on w); later
// calls add only the advective terms to them, on the fixed patterns, and
// upload values only.  The blocks and the coarse inverse follow as after
// update_params.
static void reassemble_about(fsgmg_hierarchy& h, const double* x) {
  const Level& F = h.levels[h.L - 1];
  const size_t nw = (size_t)F.N2 * h.D;
  if (!h.dadv.empty() && dev_adv_eligible(h)) {
    // device re-assembly: the velocity is checked first, as on the host
    HIPCHECK(hipMemsetAsync(h.adv_flag, 0, sizeof(int32_t), h.stream));
    launch_nonfinite_flag((int64_t)nw, x + F.off_u, h.adv_flag, h.stream);
    int32_t flag = 0;
    HIPCHECK(hipMemcpyAsync(&flag, h.adv_flag, sizeof(int32_t), hipMemcpyDeviceToHost, h.stream));
    HIPCHECK(hipStreamSynchronize(h.stream));
    if (flag & 1) throw Fail{FSGMG_EINVAL, "the velocity contains NaN or Inf"};
    run_dev_adv(h, x);
    h.factors_valid = false;
    if (!h.bd.empty()) h.bd_dirty = true;
    build_coarse_inverse(h, true);
    return;
  }
  if (h.host_only()) {
    std::memcpy(h.w_finest.data(), x + F.off_u, nw * sizeof(double));
  } else {
    HIPCHECK(hipMemcpyAsync(h.w_finest.data(), x + F.off_u, nw * sizeof(double),
                            hipMemcpyDeviceToHost, h.stream));
    HIPCHECK(hipStreamSynchronize(h.stream));
  }
  for (double v : h.w_finest)
    if (!std::isfinite(v)) throw Fail{FSGMG_EINVAL, "the velocity contains NaN or Inf"};
  if (h.plans.size() != (size_t)h.L) {
    std::vector<LevelOperator> ops;
    std::vector<AdvectionPlan> plans;
    assemble_all(h, ops, &plans);
    const LevelOperator &Fo = h.ops[h.L - 1], &Fn = ops[h.L - 1];
    for (int l = 0; l < h.L; ++l)
      if (!same_pattern(ops[l].A, h.ops[l].A))
        throw Fail{FSGMG_ESTATE, "operator pattern changed with the advecting velocity"};
    if (!same_pattern(Fn.full, Fo.full) || !same_pattern(Fn.load, Fo.load) ||
        !same_pattern(Fn.time, Fo.time))
      throw Fail{FSGMG_ESTATE, "operator pattern changed with the advecting velocity"};
    h.ops = std::move(ops);
    h.plans = std::move(plans);
  } else {
    reassemble_all(h);
  }
  h.host_vals_stale = false;
  h.device_ahead = false;
  h.factors_valid = false;
  // the multiplicative colouring reads the operator's values: recolour
  if (h.sopt.schwarz == FSGMG_SCHWARZ_MULTIPLICATIVE) h.have_blocks = false;
  if (h.host_only()) return;
  refresh_load_and_time(h);
  upload_operator_values(h);
  // the next re-assemblies run on the device where they can
  if (h.dadv.empty() && dev_adv_eligible(h)) build_dev_adv(h, x);
  if (!h.bd.empty()) h.bd_dirty = true;
  if (h.dl[0].use_bd) ensure_bd(h);
  build_coarse_inverse(h, true);
}

fsgmg_status update_advection(fsgmg_h h, const double* x) {
  if (!h || !x) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    if (h->w_finest.empty())
      throw Fail{FSGMG_EINVAL, "the hierarchy was set up without an advecting velocity"};
    reassemble_about(*h, x);
    return FSGMG_OK;
  });
}

fsgmg_status time_rhs(fsgmg_h h, const double* f, double g, const double* x_prev, double* b) {
  if (!h || !f || !x_prev || !b || (const void*)b == (const void*)x_prev ||
      (const void*)b == (const void*)f || !std::isfinite(g))
    return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    if (!h->time_val) throw Fail{FSGMG_EINVAL, "time_rhs needs a hierarchy set up with a finite dt"};
    launch_time_rhs(h->dl[h->L - 1].N, h->load_rp, h->load_col, h->load_val, f, h->lift, g,
                    h->time_rp, h->time_col, h->time_val, x_prev, b, h->stream);
    HIPCHECK(hipGetLastError());
    return FSGMG_OK;
  });
}

fsgmg_status period_solve(fsgmg_h h, const fsgmg_period_opts* po, const fsgmg_krylov_opts* ko,
                          const double* f, double* x, int32_t* iters, double* changes,
                          fsgmg_period_info* info) {
  if (!h || !po || !ko || !f || !x || (const void*)f == (const void*)x) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    if (po->steps < 1 || po->picard_max < 1 || !(po->picard_tol >= 0) ||
        !std::isfinite(po->picard_tol) || !std::isfinite(po->t0) || !std::isfinite(po->inflow_amp))
      throw Fail{FSGMG_EINVAL, "period options out of range"};
    if (!h->time_val) throw Fail{FSGMG_EINVAL, "period_solve needs a hierarchy set up with a finite dt"};
    if (h->w_finest.empty())
      throw Fail{FSGMG_EINVAL, "the hierarchy was set up without an advecting velocity"};
    if (!h->tuned) throw Fail{FSGMG_ESTATE, "build_fs_as_blocks has not been called"};
    const auto t_start = std::chrono::steady_clock::now();
    auto ms_since = [](std::chrono::steady_clock::time_point t) {
      return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t).count();
    };
    const int64_t N = h->dl[h->L - 1].N;
    if (!h->per_buf) h->per_buf = (double*)h->dalloc((size_t)4 * N * sizeof(double));
    double* xprev = h->per_buf;
    double* xcur = h->per_buf + N;
    double* xnew = h->per_buf + 2 * N;
    double* b = h->per_buf + 3 * N;
    HIPCHECK(hipMemcpyAsync(xprev, x, N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    if (iters)
      for (int k = 0; k < po->steps * po->picard_max; ++k) iters[k] = -1;
    if (changes)
      for (int k = 0; k < po->steps * po->picard_max; ++k) changes[k] = NAN;
    const fsgmg_smoother_opts so = h->sopt;
    const double dt = 1.0 / h->phys.inv_dt;
    const double two_pi = 6.283185307179586;
    fsgmg_period_info acc{};
    double sum_iters = 0, sum_rate = 0, t_asm = 0, t_fac = 0, t_sol = 0;
    fsgmg_status st = FSGMG_OK;
    for (int i = 1; i <= po->steps && st == FSGMG_OK; ++i) {
      const double g = 1.0 + po->inflow_amp * std::sin(two_pi * (po->t0 + i * dt));
      HIPCHECK(hipMemcpyAsync(xcur, xprev, N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
      int taken = 0;
      for (int s = 0; s < po->picard_max; ++s) {
        auto t0 = std::chrono::steady_clock::now();
        reassemble_about(*h, xcur);
        t_asm += ms_since(t0);
        t0 = std::chrono::steady_clock::now();
        const fsgmg_status bs = build_fs_as_blocks_impl(h, &so);
        if (bs != FSGMG_OK) return bs;
        HIPCHECK(hipStreamSynchronize(h->stream));
        t_fac += ms_since(t0);
        t0 = std::chrono::steady_clock::now();
        launch_time_rhs(N, h->load_rp, h->load_col, h->load_val, f, h->lift, g, h->time_rp,
                        h->time_col, h->time_val, xprev, b, h->stream);
        HIPCHECK(hipGetLastError());
        fsgmg_solve_info si{};
        const fsgmg_status fs = fgmres(*h, b, xnew, *ko, &si, false);
        // relative change of the iterate: ||x_new - x_cur|| / ||x_new||
        launch_add_scaled<double>(N, -1.0, xnew, xcur, false, h->stream);
        const double dn = device_norm(*h, xcur, N);
        const double nn = device_norm(*h, xnew, N);
        t_sol += ms_since(t0);
        std::swap(xcur, xnew);
        const double change = nn > 0 ? dn / nn : dn;
        const int k = (i - 1) * po->picard_max + s;
        if (iters) iters[k] = si.iters;
        if (changes) changes[k] = change;
        ++taken;
        ++acc.solves;
        sum_iters += si.iters;
        acc.max_iters = std::max(acc.max_iters, si.iters);
        sum_rate += si.iters > 0 ? std::pow(si.rel_res_true, 1.0 / si.iters) : 0.0;
        if (fs != FSGMG_OK) {
          st = fs;
          break;
        }
        if (po->picard_tol > 0 && change <= po->picard_tol) break;
      }
      HIPCHECK(hipMemcpyAsync(xprev, xcur, N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
      acc.steps = i;
      acc.s_max += taken;
    }
    HIPCHECK(hipMemcpyAsync(x, xprev, N * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    if (info) {
      *info = acc;
      info->s_max = acc.steps ? acc.s_max / acc.steps : 0.0;
      info->N = acc.solves ? sum_iters / acc.solves : 0.0;
      info->rho = acc.solves ? sum_rate / acc.solves : 0.0;
      info->t_assemble_ms = t_asm;
      info->t_factor_ms = t_fac;
      info->t_solve_ms = t_sol;
      info->t_total_ms = ms_since(t_start);
    }
    return st;
  });
}

fsgmg_status debug_zero_block(fsgmg_h h, int level, int64_t block) {
  if (!h) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    if (block < 0) {
      h->zero_block_level = -1;
      h->zero_block = -1;
      return FSGMG_OK;
    }
    if (level < 1 || level >= h->L) throw Fail{FSGMG_EINVAL, "level out of range (1 .. L-1)"};
    h->zero_block_level = level;
    h->zero_block = block;
    return FSGMG_OK;
  });
}

fsgmg_status level_info(fsgmg_h h, int level, int64_t out[9]) {
  if (!h || !out) return FSGMG_EINVAL;
  if (level < 0 || level >= h->L) return FSGMG_EINVAL;
  const Level& lv = h->levels[level];
  out[0] = lv.N;
  out[1] = lv.N2;
  out[2] = lv.Nps;
  out[3] = lv.Npf;
  out[4] = lv.off_ps;
  out[5] = lv.off_u;
  out[6] = lv.off_pf;
  out[7] = h->ops[level].A.nnz();
  out[8] = lv.D;
  return FSGMG_OK;
}

fsgmg_status dof_map(fsgmg_h h, int level, int64_t* n, int32_t* field, int32_t* comp,
                     int32_t* node, double* xyz) {
  if (!h || !n) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    if (level < 0 || level >= h->L) throw Fail{FSGMG_EINVAL, "level out of range"};
    const Level& lv = h->levels[level];
    const int64_t cap = *n;
    *n = lv.N;
    if (!field && !comp && !node && !xyz) return FSGMG_OK;
    if (cap < lv.N) throw Fail{FSGMG_EINVAL, "output arrays shorter than the level's unknowns"};
    const int D = lv.D;
    auto put = [&](int64_t i, int f, int c, int64_t nd, int64_t q2) {
      if (field) field[i] = f;
      if (comp) comp[i] = c;
      if (node) node[i] = (int32_t)nd;
      if (xyz)
        for (int a = 0; a < 3; ++a) xyz[3 * i + a] = a < D ? lv.X[q2 * D + a] : 0.0;
    };
    for (int64_t q = 0; q < lv.N2; ++q)
      for (int c = 0; c < D; ++c) {
        put(D * q + c, 0, c, q, q);
        put(lv.off_u + D * q + c, 2, c, q, q);
      }
    for (int64_t v = 0; v < lv.NV; ++v) {
      const int64_t q2 = lv.vertex_node(v);
      if (lv.ps_of_vert[v] >= 0) put(lv.ps_of_vert[v], 1, 0, v, q2);
      if (lv.pf_of_vert[v] >= 0) put(lv.pf_of_vert[v], 3, 0, v, q2);
    }
    return FSGMG_OK;
  });
}

fsgmg_status export_csr(fsgmg_h h, int level, int which, int64_t dims[3], int64_t* rowptr,
                        int32_t* col, double* val) {
  if (!h || !dims) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    if (level < 0 || level >= h->L) throw Fail{FSGMG_EINVAL, "level out of range"};
    h->ensure_host_values();
    CsrHost tmp;
    const CsrHost* M = nullptr;
    if (which == 0) {
      h->ensure_host_values();
      M = &h->ops[level].A;
    } else if (which == 1 || which == 2) {
      if (level < 1) throw Fail{FSGMG_EINVAL, "transfers exist for level >= 1"};
      tmp = which == 1 ? prolongation_full(h->levels[level], h->levels[level - 1], h->tr[level])
                       : restriction_full(h->levels[level], h->levels[level - 1], h->tr[level]);
      M = &tmp;
    } else if (which == 3) {
      if (level != h->L - 1) throw Fail{FSGMG_EINVAL, "load operator exists on the finest level"};
      M = &h->ops[level].load;
    } else if (which == 4) {
      if (level != h->L - 1) throw Fail{FSGMG_EINVAL, "time operator exists on the finest level"};
      if (h->phys.inv_dt == 0.0) throw Fail{FSGMG_EINVAL, "steady hierarchy: no time operator"};
      const LevelOperator& op = h->ops[level];
      tmp = op.time;
      for (size_t k = 0; k < tmp.val.size(); ++k)
        tmp.val[k] = op.time_piece[0][k] + op.G * op.time_piece[1][k] +
                     op.invlam * op.time_piece[2][k] + op.mu * op.time_piece[3][k];
      M = &tmp;
    } else {
      throw Fail{FSGMG_EINVAL, "unknown matrix"};
    }
    dims[0] = M->nrows;
    dims[1] = M->ncols;
    dims[2] = M->nnz();
    if (rowptr) std::memcpy(rowptr, M->rowptr.data(), M->rowptr.size() * sizeof(int64_t));
    if (col) std::memcpy(col, M->col.data(), M->col.size() * sizeof(int32_t));
    if (val) std::memcpy(val, M->val.data(), M->val.size() * sizeof(double));
    return FSGMG_OK;
  });
}

fsgmg_status export_vector(fsgmg_h h, int level, int which, double* out) {
  if (!h || !out) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    if (level < 0 || level >= h->L) throw Fail{FSGMG_EINVAL, "level out of range"};
    const Level& lv = h->levels[level];
    if (which == 0) {
      if (level != h->L - 1) throw Fail{FSGMG_EINVAL, "lift exists on the finest level"};
      h->ensure_host_values();
      const LevelOperator& op = h->ops[level];
      for (int64_t i = 0; i < lv.N; ++i)
        out[i] = op.lift_piece[0][i] + op.G * op.lift_piece[1][i] + op.invlam * op.lift_piece[2][i] +
                 op.mu * op.lift_piece[3][i];
    } else if (which == 1) {
      for (int64_t i = 0; i < lv.N; ++i) out[i] = lv.dir[i] ? 1.0 : 0.0;
    } else {
      throw Fail{FSGMG_EINVAL, "unknown vector"};
    }
    return FSGMG_OK;
  });
}

fsgmg_status export_blocks(fsgmg_h h, int level, int64_t sizes[2], int64_t* ptr, int32_t* dofs,
                           int32_t* owner) {
  if (!h || !sizes) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    if (!h->have_blocks) throw Fail{FSGMG_ESTATE, "blocks not built"};
    if (level < 1 || level >= h->L) throw Fail{FSGMG_EINVAL, "blocks exist on levels >= 1"};
    const BlockSet& bs = h->blocks[level];
    sizes[0] = bs.nblk();
    sizes[1] = (int64_t)bs.dofs.size();
    if (ptr) std::memcpy(ptr, bs.ptr.data(), bs.ptr.size() * sizeof(int64_t));
    if (dofs) std::memcpy(dofs, bs.dofs.data(), bs.dofs.size() * sizeof(int32_t));
    if (owner) std::memcpy(owner, bs.owner.data(), bs.owner.size() * sizeof(int32_t));
    return FSGMG_OK;
  });
}

fsgmg_status block_colours(fsgmg_h h, int level, int64_t* ncolours, int64_t* colour_ptr) {
  if (!h || !ncolours) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    if (!h->have_blocks) throw Fail{FSGMG_ESTATE, "blocks not built"};
    if (level < 1 || level >= h->L) throw Fail{FSGMG_EINVAL, "blocks exist on levels >= 1"};
    const BlockSet& bs = h->blocks[level];
    const bool mult = h->sopt.schwarz == FSGMG_SCHWARZ_MULTIPLICATIVE;
    *ncolours = mult ? (int64_t)bs.colour_ptr.size() - 1 : 0;
    if (mult && colour_ptr)
      std::memcpy(colour_ptr, bs.colour_ptr.data(), bs.colour_ptr.size() * sizeof(int64_t));
    return FSGMG_OK;
  });
}

fsgmg_status stream_read_ceiling(fsgmg_h h, int64_t bytes, int reps, double* gbs) {
  if (!h || !gbs || bytes < (int64_t)(1 << 20) || reps < 1) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    bytes &= ~(int64_t)255;
    void* buf = h->raw_alloc((size_t)bytes + 256);
    if (!buf) throw Fail{FSGMG_ENOMEM, "no room for the streaming buffer"};
    struct Release {
      fsgmg_hierarchy* h;
      void* p;
      ~Release() { h->raw_free(p); }
    } rel{h, buf};
    uint32_t* sink = reinterpret_cast<uint32_t*>(static_cast<char*>(buf) + bytes);
    HIPCHECK(hipMemsetAsync(buf, 0, (size_t)bytes + 256, h->stream));
    launch_flush(buf, bytes, sink, h->stream);   // warm-up
    std::vector<float> ms;
    hipEvent_t a = h->next_event(), b = h->next_event();
    for (int r = 0; r < reps; ++r) {
      HIPCHECK(hipEventRecord(a, h->stream));
      launch_flush(buf, bytes, sink, h->stream);
      HIPCHECK(hipEventRecord(b, h->stream));
      HIPCHECK(hipEventSynchronize(b));
      float t = 0;
      HIPCHECK(hipEventElapsedTime(&t, a, b));
      ms.push_back(t);
    }
    h->ev_used -= 2;
    std::sort(ms.begin(), ms.end());
    *gbs = (double)bytes / (ms[ms.size() / 2] * 1e-3) / 1e9;
    return FSGMG_OK;
  });
}

fsgmg_status kernel_timing(fsgmg_h h, int enable, int64_t counts[4], double total_ms[4]) {
  if (!h) return FSGMG_EINVAL;
  return guarded(h, [&]() -> fsgmg_status {
    check_device(*h);
    if (enable) {
      for (auto& v : h->ev_rec) v.clear();
      h->ev_used = 0;
      h->timing = true;
      return FSGMG_OK;
    }
    h->timing = false;
    HIPCHECK(hipStreamSynchronize(h->stream));
    for (int k = 0; k < 4; ++k) {
      double tot = 0.0;
      for (auto& p : h->ev_rec[k]) {
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, p.first, p.second));
        tot += ms;
      }
      if (counts) counts[k] = (int64_t)h->ev_rec[k].size();
      if (total_ms) total_ms[k] = tot;
      h->ev_rec[k].clear();
    }
    h->ev_used = 0;
    return FSGMG_OK;
  });
}

fsgmg_status tuning_info(fsgmg_h h, int level, int32_t out[7]) {
  // out[1] < 0 means non-temporal loads of the block inverses
  if (!h || !out) return FSGMG_EINVAL;
  if (level < 0 || level >= h->L || (int)h->tune.size() != h->L) return FSGMG_ESTATE;
  out[0] = h->tune[level].spmv_lanes;
  out[1] = h->tune[level].smooth_threads;
  out[2] = h->outer_lanes;
  out[3] = level > 0 ? h->tune[level].restrict_lanes : 0;
  out[4] = level > 0 ? h->tune[level].prolong_lanes : 0;
  out[5] = level > 0 ? h->tune[level].fused : 0;
  out[6] = level > 0 ? h->tune[level].split : 0;
  return FSGMG_OK;
}

const char* last_error(fsgmg_h h) { return h ? h->err.c_str() : "null handle"; }

void hierarchy_destroy(fsgmg_h h) { delete h; }

}  // extern "C"
