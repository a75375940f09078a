// C ABI of libsccs (include/sccs.h): handle management, workspace carving,
// setup and the cooperative launches of the persistent CCD kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "sccs.h"
#include "sccs_device.hpp"
#include "sccs_kernels.hpp"
#include "sccs_batch.hpp"
#include "sccs_valued.hpp"
#include "sccs_layout.hpp"

using namespace sccs;

struct sccs_handle {
  std::string err;
  int32_t N = 0, J = 0, G = 0, T = 0, prec = 0;
  int32_t device = 0;   // HIP device current at sccs_create
  int64_t K = 0, nnz = 0;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  bool owns_ws = false;
  bool failed = false;
  int32_t prior_kind = -1;
  double var = 1.0;
  int32_t refresh_period = 0;
  size_t lds_bytes = 0;
  int32_t nbits = 0;
  int32_t mv_words = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed = false;
  KArgs args{};
  // device pointers kept for setup and copies
  int64_t* d_col_ptr = nullptr;
  int32_t* d_count = nullptr;
  int32_t* d_weight = nullptr;
  std::vector<int32_t> gcol;  // host copy of the column groups
  Ctrl* h_ctrl = nullptr;  // pinned host mirror of the control block
  uint32_t gseq0[kSlotClasses] = {};  // reduction sequence numbers before the last sweep launch
  int last_mode = -1;              // kind of the last launch
  int32_t passes = 0, rejects = 0, zero_steps = 0;  // schedule statistics of the last sweep launch
  bool swept = false;
  bool use_merge = false;          // the next sweep launch takes the merged-pass form
  bool valued = false;             // covariate values: k_ccd_val / k_diag_val
  bool last_merged = false;        // the last sweep launch used the merged-pass form
  bool group_timing = false;       // sweep launches stamp each column group (sccs_group_timing)
  bool last_stamped = false;       // the last sweep launch stamped its column groups
  int32_t n_classes = 0;           // grouped prior: classes (their sums take n_classes doubles of LDS)
  double class_var = 0.0;
  std::vector<int32_t> perm;       // perm[k]: the column visited k-th (empty: the given order)
  // the internal position of each column (inverse of perm); set with perm
  std::vector<int32_t> pos;
};

static thread_local std::string g_create_error;

namespace {

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base((char*)b) {}
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct Plan {
  uint2* rp;
  int32_t *tile_start, *own, *gcol, *pb, *pptr, *era_ptr, *era_col, *offset, *count, *weight;
  double *val, *era_val;
  int32_t* pclass;
  double* pkappa;
  uint64_t* group_ticks;
  uint32_t* gdesc;
  uint64_t* moved;
  int64_t* col_ptr;
  void* w;
  double2* pat;
  double *ytx, *beta, *trust;
  uint64_t *slots, *slots2, *oslots, *oslots2;
  Ctrl* ctrl;
};

size_t carve(void* base, const Layout& L, int prec, bool has_weight, bool has_val, Plan& P) {
  Carver c(base);
  P.rp = c.take<uint2>((size_t)L.nnz + 1);
  P.tile_start = c.take<int32_t>((size_t)L.tiles_cap);
  P.own = c.take<int32_t>((size_t)L.J * (L.G + 1));
  P.gcol = c.take<int32_t>((size_t)L.J + 1);
  P.gdesc = c.take<uint32_t>((size_t)L.J);
  P.moved = c.take<uint64_t>(((size_t)L.J + 63) / 64);
  P.pb = c.take<int32_t>((size_t)L.G + 1);
  P.pptr = c.take<int32_t>((size_t)L.N + 1);
  P.era_ptr = c.take<int32_t>((size_t)L.K + 1);
  P.era_col = c.take<int32_t>((size_t)L.nnz + 1);
  P.offset = c.take<int32_t>((size_t)L.K);
  P.count = c.take<int32_t>((size_t)L.K);
  P.weight = has_weight ? c.take<int32_t>((size_t)L.N) : nullptr;
  P.val = has_val ? c.take<double>((size_t)L.nnz + 1) : nullptr;
  P.pclass = c.take<int32_t>((size_t)L.J);
  P.group_ticks = c.take<uint64_t>((size_t)L.J + 1);
  P.pkappa = c.take<double>((size_t)L.J);
  P.era_val = has_val ? c.take<double>((size_t)L.nnz + 1) : nullptr;
  P.col_ptr = c.take<int64_t>((size_t)L.J + 1);
  P.w = prec == SCCS_PREC_FP64 ? (void*)c.take<double>((size_t)L.K) : (void*)c.take<float>((size_t)L.K);
  P.pat = c.take<double2>((size_t)L.N);
  P.ytx = c.take<double>((size_t)L.J);
  P.beta = c.take<double>((size_t)L.J);
  P.trust = c.take<double>((size_t)L.J);
  const size_t n1 = kSlots1Words, n2 = (size_t)2 * kReplicas * kGroups * kSlotWords;
  P.slots = c.take<uint64_t>(kSlotClasses * kSlots1PerClass);
  P.slots2 = c.take<uint64_t>(kSlotClasses * kSlots2PerClass);
  P.oslots = c.take<uint64_t>(n1);
  P.oslots2 = c.take<uint64_t>(n2);
  P.ctrl = c.take<Ctrl>(1);
  return (c.off + 255) & ~(size_t)255;
}

sccs_status check_options(const sccs_options* o, std::string& err) {
  if (!o) return SCCS_OK;
  if (o->precision != SCCS_PREC_FP64 && o->precision != SCCS_PREC_MIXED) {
    err = "options.precision must be SCCS_PREC_FP64 or SCCS_PREC_MIXED";
    return SCCS_ERR_INVALID_ARG;
  }
  if (o->n_workgroups < 0 || o->n_workgroups > kMaxWorkgroups) {
    err = "options.n_workgroups must be in [0, 256]";
    return SCCS_ERR_INVALID_ARG;
  }
  if (o->refresh_period < -1) {
    err = "options.refresh_period must be >= -1";
    return SCCS_ERR_INVALID_ARG;
  }
  if (o->tile_nnz != 0 && (o->tile_nnz < 8 || o->tile_nnz > kTile)) {
    err = "options.tile_nnz must be 0 (64) or in [8, 64]";
    return SCCS_ERR_INVALID_ARG;
  }
  if (o->max_group < 0 || o->max_group > kMaxGroup) {
    err = "options.max_group must be 0 (4) or in [1, 4]";
    return SCCS_ERR_INVALID_ARG;
  }
  if (o->merge_passes != 0 && o->merge_passes != 1) {
    err = "options.merge_passes must be 0 or 1";
    return SCCS_ERR_INVALID_ARG;
  }
  if (o->column_order != SCCS_ORDER_GIVEN && o->column_order != SCCS_ORDER_INDEPENDENT) {
    err = "options.column_order must be SCCS_ORDER_GIVEN or SCCS_ORDER_INDEPENDENT";
    return SCCS_ERR_INVALID_ARG;
  }
  if (o->batch_engine != 0 && o->batch_engine != 1) {
    err = "options.batch_engine must be 0 (partitioned) or 1 (lockstep)";
    return SCCS_ERR_INVALID_ARG;
  }
  return SCCS_OK;
}

sccs_status pick_workgroups(const sccs_options* o, int32_t& G, std::string& err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { err = "hipGetDevice failed"; return SCCS_ERR_HIP; }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
    err = "cannot query the compute-unit count";
    return SCCS_ERR_HIP;
  }
  G = (o && o->n_workgroups > 0) ? o->n_workgroups : cus;
  if (G > kMaxWorkgroups) G = kMaxWorkgroups;
  if (G > cus) { err = "n_workgroups exceeds the number of compute units"; return SCCS_ERR_INVALID_ARG; }
  return SCCS_OK;
}

// The sweep kernel in its merged-pass form, or in the one-pass-per-group
// form, which carries less state per pass; problems with covariate values
// take the valued sweep (no merged passes) and its diagnostic kernel.
const void* ccd_kernel(int prec, int mode, bool merge = false, bool valued = false) {
  if (valued) {
    if (mode == kModeSweep) return prec == SCCS_PREC_FP64 ? (const void*)k_ccd_val<double> : (const void*)k_ccd_val<float>;
    if (mode == kModeGradHess)
      return prec == SCCS_PREC_FP64 ? (const void*)k_diag_val<double> : (const void*)k_diag_val<float>;
  }
  if (mode == kModeSweep) {
    if (merge) return prec == SCCS_PREC_FP64 ? (const void*)k_ccd<double, true> : (const void*)k_ccd<float, true>;
    return prec == SCCS_PREC_FP64 ? (const void*)k_ccd<double, false> : (const void*)k_ccd<float, false>;
  }
  return prec == SCCS_PREC_FP64 ? (const void*)k_diag<double> : (const void*)k_diag<float>;
}

#define HIPCHK(h, call)                                                        \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      (h)->err = std::string(#call) + ": " + hipGetErrorString(e_);            \
      return SCCS_ERR_HIP;                                                     \
    }                                                                          \
  } while (0)

sccs_status usable(sccs_handle* h) {
  if (!h) return SCCS_ERR_INVALID_ARG;
  if (h->failed) {
    h->err = "handle unusable after a failed device reduction; destroy it";
    return SCCS_ERR_STATE;
  }
  return SCCS_OK;
}

sccs_status read_ctrl(sccs_handle* h) {
  HIPCHK(h, hipMemcpyAsync(h->h_ctrl, h->args.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (h->last_mode == kModeSweep) {
    // one reduction per pass, each on the sequence of its width class
    uint32_t n = 0;
    for (int c = 0; c < kSlotClasses; ++c) n += h->h_ctrl->gseq[c] - h->gseq0[c];
    h->passes = (int32_t)n;
    h->rejects = h->h_ctrl->rejects;
    h->zero_steps = h->h_ctrl->zero_steps;
    h->swept = true;
    // Merged passes pay off once many coordinates take exactly zero steps
    // (coordinates held at zero by the Laplace prior, and converged ones,
    // whose FP64 step rounds to zero); they cost a little more per pass
    // otherwise.  The next launch follows this launch's share, with
    // hysteresis.
    const double visits = (double)h->J * (h->h_ctrl->sweeps > 0 ? h->h_ctrl->sweeps : 1);
    const double zf = h->zero_steps / visits;
    if (!h->use_merge && zf >= 0.5) h->use_merge = true;
    else if (h->use_merge && zf < 0.35) h->use_merge = false;
  }
  if (h->h_ctrl->status == SCCS_ERR_SYNC) {
    h->failed = true;
    h->err = "device-wide reduction timed out (workgroups not co-resident?)";
    return SCCS_ERR_SYNC;
  }
  if (h->h_ctrl->status == SCCS_ERR_NUMERIC) {
    h->err = "non-finite gradient, Hessian or coefficient; last finite beta kept";
    return SCCS_ERR_NUMERIC;
  }
  return SCCS_OK;
}

// Dynamic LDS of a sweep or diagnostic launch: beta, trust, the sweep-start
// beta, the patient bitmaps and the moved bits, then the class sums of the
// grouped prior when it is in use.
size_t ssum_offset(const sccs_handle* h) { return (h->lds_bytes + 7) / 8; }   // in doubles
size_t launch_lds(const sccs_handle* h, int prior_kind) {
  return prior_kind == SCCS_PRIOR_GROUPED ? ssum_offset(h) * 8 + (size_t)h->n_classes * 8 : h->lds_bytes;
}

sccs_status launch(sccs_handle* h, int mode, int n_sweeps, int criterion, double tol, int want_obj, int diag_j) {
  KArgs a = h->args;
  if (mode == kModeGradHess) {
    // group of column diag_j, and its index within the group
    const int g = (int)(std::upper_bound(h->gcol.begin(), h->gcol.end(), diag_j) - h->gcol.begin()) - 1;
    a.diag_g = g;
    a.diag_c = diag_j - h->gcol[g];
  }
  a.prior_kind = h->prior_kind < 0 ? SCCS_PRIOR_NONE : h->prior_kind;
  a.var = h->var;
  a.inv_var = 1.0 / h->var;
  a.lambda = (a.prior_kind == SCCS_PRIOR_LAPLACE) ? std::sqrt(2.0 / h->var) : 0.0;
  a.n_classes = a.prior_kind == SCCS_PRIOR_GROUPED ? h->n_classes : 0;
  a.n_sweeps = n_sweeps;
  a.criterion = criterion;
  a.tol = tol;
  a.refresh_period = h->refresh_period;
  a.want_objective = want_obj;
  a.mode = mode;
  a.diag_j = diag_j;
  a.stamp = mode == kModeSweep && h->group_timing ? 1 : 0;
  void* params[] = {&a};
  HIPCHK(h, hipMemsetAsync(&h->args.ctrl->status, 0, sizeof(int32_t), h->stream));
  HIPCHK(h, hipEventRecord(h->ev0, h->stream));
  const bool merge = a.merge && h->use_merge && !h->valued && a.prior_kind != SCCS_PRIOR_GROUPED && h->perm.empty();
  if (mode == kModeSweep) {   // the mirror holds the state after the previous launch
    for (int c = 0; c < kSlotClasses; ++c) h->gseq0[c] = h->h_ctrl->gseq[c];
    h->last_merged = merge;
    h->last_stamped = a.stamp && !merge;
  }
  h->last_mode = mode;
  HIPCHK(h, hipLaunchCooperativeKernel(ccd_kernel(h->prec, mode, merge, h->valued), dim3(h->G), dim3(kBlock), params,
                                        (unsigned)launch_lds(h, a.prior_kind), h->stream));
  HIPCHK(h, hipEventRecord(h->ev1, h->stream));
  h->timed = true;
  return SCCS_OK;
}

sccs_status refresh_all(sccs_handle* h) {
  KArgs a = h->args;
  int grid = (h->N + 255) / 256;
  if (grid > 4096) grid = 4096;
  if (h->prec == SCCS_PREC_FP64)
    hipLaunchKernelGGL(k_refresh<double>, dim3(grid), dim3(256), 0, h->stream, a);
  else
    hipLaunchKernelGGL(k_refresh<float>, dim3(grid), dim3(256), 0, h->stream, a);
  HIPCHK(h, hipGetLastError());
  // the maintained state is exact again
  HIPCHK(h, hipMemsetAsync(&h->args.ctrl->since_refresh, 0, sizeof(int32_t), h->stream));
  return SCCS_OK;
}

// Forget which columns took zero steps (a new beta makes the prediction of
// merged passes stale; it is only a prediction either way, and a new prior
// keeps it: the steps of a warm-started chain change gradually).
sccs_status reset_moved(sccs_handle* h) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, h->stream, (uint64_t*)h->args.moved,
                     (size_t)h->mv_words / 2, ~0ull);
  HIPCHK(h, hipGetLastError());
  return SCCS_OK;
}

// ------------------------------------------------ allocation-free sweep
//
// sccs_sweep_static runs the sweep kernel with its device-wide reduction
// slots and its control block in `scratch`, a file-scope device array, in
// place of the handle's workspace copies.  The array holds one set of slots
// for up to kMaxWorkgroups workgroups (every reduction class of the sweep and
// the objective) plus one control block: 480 KiB, held by every device the
// library runs on until the process ends.  Every call on a device shares
// that device's copy; each call first refills it (tags, sequence numbers),
// so calls that overlap on one device race.
constexpr size_t kScrSlots1 = (size_t)kSlotClasses * kSlots1PerClass;
constexpr size_t kScrSlots2 = (size_t)kSlotClasses * kSlots2PerClass;
constexpr size_t kScrO1 = kSlots1Words;
constexpr size_t kScrO2 = (size_t)2 * kReplicas * kGroups * kSlotWords;
constexpr size_t kScrTagWords = kScrSlots1 + kScrSlots2 + kScrO1 + kScrO2;   // filled with the start tag
constexpr size_t kScrCtrlWords = (sizeof(Ctrl) + 255) / 256 * 32;
constexpr size_t kScratchWords = kScrTagWords + kScrCtrlWords;
constexpr int32_t kScratchMaxWorkgroups = kMaxWorkgroups;
static_assert(kScrSlots1 % 32 == 0 && kScrSlots2 % 32 == 0 && kScrO1 % 32 == 0 && kScrO2 % 32 == 0,
              "every part of the scratch array starts on a 256-byte boundary");

static __device__ __align__(256) uint64_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the array's name is only a
// host-side stand-in); looked up once per device, with that device current.
sccs_status scratch_address(int dev, uint64_t** out, std::string& err) {
  if (dev < 0 || dev >= kMaxDevices) { err = "device index beyond the scratch table"; return SCCS_ERR_STATE; }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return SCCS_ERR_HIP;
    }
    g_scratch_ptr[dev] = (uint64_t*)p;
  }
  *out = g_scratch_ptr[dev];
  return SCCS_OK;
}

// Start of a static sweep: every slot word gets the tag that reductions 0 and
// 1 do not expect, and the scratch control block starts from the handle's
// state with every sequence number at zero (a fill kernel, not a memset, so
// that the sequence can be captured in a graph).
__global__ void k_scratch_prep(uint64_t* slots, size_t n, Ctrl* sc, const Ctrl* hc) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    slots[i] = kSign;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctrl c{};
    c.since_refresh = hc->since_refresh;
    *sc = c;
  }
}

// End of a static sweep: results go back to the handle's control block; the
// handle keeps its own sequence numbers (its own slots were not touched).
__global__ void k_scratch_post(const Ctrl* sc, Ctrl* hc) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  uint32_t n = 0;
  for (int c = 0; c < kSlotClasses; ++c) n += sc->gseq[c];
  hc->passes = (int32_t)n;
  hc->status = sc->status;
  hc->sweeps = sc->sweeps;
  hc->converged = sc->converged;
  hc->since_refresh = sc->since_refresh;
  hc->loglik = sc->loglik;
  hc->logpost = sc->logpost;
  hc->rejects = sc->rejects;
  hc->zero_steps = sc->zero_steps;
}

}  // namespace

extern "C" {

void sccs_default_options(sccs_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->precision = SCCS_PREC_FP64;
  o->n_workgroups = 0;
  o->refresh_period = -1;
  o->tile_nnz = 0;
  o->max_group = 0;
  o->merge_passes = 1;
  o->stream = nullptr;
  o->batch_engine = 0;
  o->column_order = SCCS_ORDER_GIVEN;
}

sccs_status sccs_query_workspace(const sccs_problem* prob, const sccs_options* opts, size_t* bytes) {
  std::string err;
  if (!bytes) { g_create_error = "bytes is NULL"; return SCCS_ERR_INVALID_ARG; }
  sccs_status st = check_options(opts, err);
  if (st == SCCS_OK) st = validate_problem(prob, err);
  int32_t G = 0;
  if (st == SCCS_OK) st = pick_workgroups(opts, G, err);
  if (st != SCCS_OK) { g_create_error = err; return st; }
  if (prob->n_cols > kMaxJ) { g_create_error = "n_cols exceeds 6144"; return SCCS_ERR_INVALID_ARG; }
  Layout L;
  layout_dims(prob, G, opts && opts->tile_nnz ? opts->tile_nnz : kTile, L);
  Plan P;
  *bytes = carve(nullptr, L, opts ? opts->precision : SCCS_PREC_FP64, prob->patient_weight != nullptr,
                 prob->value != nullptr, P);
  return SCCS_OK;
}

sccs_status sccs_create(const sccs_problem* prob, const sccs_options* opts_in, void* workspace,
                        size_t workspace_bytes, sccs_handle** out) {
  if (!out) { g_create_error = "out is NULL"; return SCCS_ERR_INVALID_ARG; }
  *out = nullptr;
  sccs_options opts;
  sccs_default_options(&opts);
  if (opts_in) opts = *opts_in;
  std::string err;
  sccs_status st = check_options(&opts, err);
  if (st == SCCS_OK) st = validate_problem(prob, err);
  int32_t G = 0;
  if (st == SCCS_OK) st = pick_workgroups(&opts, G, err);
  if (st == SCCS_OK && prob->n_cols > kMaxJ) { err = "n_cols exceeds 6144"; st = SCCS_ERR_INVALID_ARG; }
  if (st != SCCS_OK) { g_create_error = err; return st; }
  if (workspace && ((uintptr_t)workspace & 255u)) {
    g_create_error = "workspace must be 256-byte aligned";
    return SCCS_ERR_WORKSPACE;
  }

  sccs_handle* h = new (std::nothrow) sccs_handle();
  if (!h) { g_create_error = "out of host memory"; return SCCS_ERR_INVALID_ARG; }
  // relabelled columns: the handle works on a copy of the problem with its
  // columns in sweep order, and maps column indices at the ABI
  PermutedProblem pp;
  if (opts.column_order == SCCS_ORDER_INDEPENDENT) {
    try {
      independent_order(prob, opts.max_group ? opts.max_group : kMaxGroup, h->perm);
      permute_columns(prob, h->perm, pp);
    } catch (const std::bad_alloc&) {
      delete h;
      g_create_error = "host out of memory while relabelling the columns";
      return SCCS_ERR_INVALID_ARG;
    }
    h->pos.assign(h->perm.size(), 0);
    for (size_t k = 0; k < h->perm.size(); ++k) h->pos[h->perm[k]] = (int32_t)k;
    prob = &pp.p;
  }
  Layout L;
  const int32_t tile_nnz = opts.tile_nnz ? opts.tile_nnz : kTile;
  const int32_t max_group = opts.max_group ? opts.max_group : kMaxGroup;
  std::vector<double> ytx;
  try {
    build_layout(prob, G, L, tile_nnz, max_group);
    host_ytx(prob, prob->patient_weight, ytx);
  } catch (const std::bad_alloc&) {
    delete h;
    g_create_error = "host out of memory while building the layout";
    return SCCS_ERR_INVALID_ARG;
  }
  L.tiles_cap = tile_bound(L.nnz, L.J, G, tile_nnz) + 1;
  if ((int64_t)L.tile_start.size() > L.tiles_cap) {
    delete h;
    g_create_error = "internal: tile count exceeds its bound";
    return SCCS_ERR_INVALID_ARG;
  }
  const bool has_w = prob->patient_weight != nullptr;
  const bool has_v = prob->value != nullptr;
  Plan P;
  size_t need = carve(nullptr, L, opts.precision, has_w, has_v, P);
  if (workspace && workspace_bytes < need) {
    delete h;
    g_create_error = "workspace too small";
    return SCCS_ERR_WORKSPACE;
  }
  h->N = L.N; h->J = L.J; h->G = G; h->T = L.n_tiles(); h->K = L.K; h->nnz = L.nnz;
  h->prec = opts.precision;
  h->valued = has_v;
  h->stream = (hipStream_t)opts.stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    g_create_error = "hipGetDevice failed";
    return SCCS_ERR_HIP;
  }
  h->refresh_period = opts.refresh_period >= 0 ? opts.refresh_period : (opts.precision == SCCS_PREC_MIXED ? kMixedRefresh : 0);
  {
    int32_t maxrange = 1;
    for (int32_t b = 0; b < G; ++b) maxrange = std::max(maxrange, L.pb[b + 1] - L.pb[b]);
    h->nbits = (maxrange + 31) / 32;
  }
  h->mv_words = 2 * ((L.J + 63) / 64);
  h->lds_bytes = (size_t)3 * L.J * sizeof(double) + (size_t)2 * h->nbits * sizeof(uint32_t) +
                 (size_t)h->mv_words * sizeof(uint32_t);
  if (h->lds_bytes > 150 * 1024) {
    delete h;
    g_create_error = "too many columns or patients per workgroup for the LDS budget";
    return SCCS_ERR_INVALID_ARG;
  }

  auto bail = [&](const std::string& m, sccs_status code) {
    g_create_error = m;
    if (h->owns_ws && h->ws) (void)hipFree(h->ws);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->h_ctrl) (void)hipHostFree(h->h_ctrl);
    delete h;
    return code;
  };

  if (workspace) {
    h->ws = workspace;
    h->ws_bytes = workspace_bytes;
  } else {
    if (hipMalloc(&h->ws, need) != hipSuccess) return bail("hipMalloc of the workspace failed", SCCS_ERR_HIP);
    h->owns_ws = true;
    h->ws_bytes = need;
  }
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
    return bail("hipEventCreate failed", SCCS_ERR_HIP);
  if (hipHostMalloc((void**)&h->h_ctrl, sizeof(Ctrl), hipHostMallocDefault) != hipSuccess)
    return bail("hipHostMalloc failed", SCCS_ERR_HIP);
  std::memset(h->h_ctrl, 0, sizeof(Ctrl));   // mirrors the zeroed device block

  // occupancy: every workgroup must be resident at once
  for (const void* k : {ccd_kernel(h->prec, kModeSweep, false), ccd_kernel(h->prec, kModeSweep, true),
                         ccd_kernel(h->prec, kModeObjective), ccd_kernel(h->prec, kModeSweep, false, true),
                         ccd_kernel(h->prec, kModeGradHess, false, true)}) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, h->lds_bytes) != hipSuccess || per_cu < 1)
      return bail("the persistent kernel cannot be resident (registers or LDS)", SCCS_ERR_HIP);
  }

  carve(h->ws, L, opts.precision, has_w, has_v, P);
  hipStream_t s = h->stream;
  auto cp = [&](void* dst, const void* src, size_t bytes) {
    return bytes == 0 || hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) == hipSuccess;
  };
  bool ok = cp(P.rp, L.rp.data(), L.rp.size() * 4) && cp(P.tile_start, L.tile_start.data(), L.tile_start.size() * 4) &&
            cp(P.own, L.own.data(), L.own.size() * 4) && cp(P.gcol, L.gcol.data(), L.gcol.size() * 4) &&
            cp(P.gdesc, L.gdesc.data(), L.gdesc.size() * 4) &&
            cp(P.pb, L.pb.data(), L.pb.size() * 4) && cp(P.ytx, ytx.data(), ytx.size() * 8) &&
            cp(P.pptr, L.pptr.data(), L.pptr.size() * 4) && cp(P.era_ptr, L.era_ptr.data(), L.era_ptr.size() * 4) &&
            cp(P.era_col, L.era_col.data(), L.era_col.size() * 4) &&
            cp(P.offset, prob->offset, (size_t)L.K * 4) && cp(P.count, prob->count, (size_t)L.K * 4) &&
            cp(P.col_ptr, prob->col_ptr, ((size_t)L.J + 1) * 8) &&
            (!has_w || cp(P.weight, prob->patient_weight, (size_t)L.N * 4)) &&
            (!has_v || (cp(P.val, L.val.data(), L.val.size() * 8) && cp(P.era_val, L.era_val.data(), L.era_val.size() * 8)));
  if (!ok) return bail("copy of the problem to the device failed", SCCS_ERR_HIP);
  std::vector<double> ones((size_t)L.J, 1.0);
  ok = hipMemsetAsync(P.beta, 0, (size_t)L.J * 8, s) == hipSuccess && cp(P.trust, ones.data(), (size_t)L.J * 8) &&
       hipMemsetAsync(P.ctrl, 0, sizeof(Ctrl), s) == hipSuccess;
  if (!ok) return bail("state initialisation failed", SCCS_ERR_HIP);
  // reduction slots start with the tag that reductions 0 and 1 do not expect
  {
    const size_t n1 = kSlots1Words, n2 = (size_t)2 * kReplicas * kGroups * kSlotWords;
    hipLaunchKernelGGL(k_fill_u64, dim3(64), dim3(256), 0, s, P.slots, kSlotClasses * kSlots1PerClass, kSign);
    hipLaunchKernelGGL(k_fill_u64, dim3(16), dim3(256), 0, s, P.slots2, kSlotClasses * kSlots2PerClass, kSign);
    hipLaunchKernelGGL(k_fill_u64, dim3(16), dim3(256), 0, s, P.oslots, n1, kSign);
    hipLaunchKernelGGL(k_fill_u64, dim3(4), dim3(256), 0, s, P.oslots2, n2, kSign);
  }
  // no column has a known zero step yet: no pass is merged in the first sweep
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(256), 0, s, P.moved, ((size_t)L.J + 63) / 64, ~0ull);
  int gp = (L.N + 255) / 256;
  if (gp > 4096) gp = 4096;
  hipLaunchKernelGGL(k_setup_patients, dim3(gp), dim3(256), 0, s, P.pptr, P.count, P.weight, P.pat, L.N);
  if (hipGetLastError() != hipSuccess) return bail("setup kernel launch failed", SCCS_ERR_HIP);

  KArgs& a = h->args;
  a.rp = P.rp; a.tile_start = P.tile_start; a.own = P.own; a.gcol = P.gcol; a.n_groups = L.n_groups;
  a.pb = P.pb; a.pptr = P.pptr;
  a.era_ptr = P.era_ptr; a.era_col = P.era_col; a.offset = P.offset; a.w = P.w; a.pat = P.pat;
  a.val = P.val; a.era_val = P.era_val;
  a.pclass = P.pclass; a.pkappa = P.pkappa; a.group_ticks = P.group_ticks; a.n_classes = 0; a.ssum_off = (int32_t)ssum_offset(h);
  a.ytx = P.ytx; a.beta = P.beta; a.trust = P.trust; a.slots = P.slots; a.slots2 = P.slots2;
  a.oslots = P.oslots; a.oslots2 = P.oslots2;
  a.ctrl = P.ctrl; a.N = L.N; a.J = L.J; a.G = G; a.nbits = h->nbits;
  a.gdesc = P.gdesc; a.moved = (uint32_t*)P.moved; a.mv_words = h->mv_words; a.merge = opts.merge_passes;
  h->d_col_ptr = P.col_ptr; h->d_count = P.count; h->d_weight = P.weight;
  h->gcol = L.gcol;
  if (refresh_all(h) != SCCS_OK) return bail(h->err, SCCS_ERR_HIP);
  if (hipStreamSynchronize(s) != hipSuccess) return bail("setup failed on the device", SCCS_ERR_HIP);
  *out = h;
  return SCCS_OK;
}

sccs_status sccs_destroy(sccs_handle* h) {
  if (!h) return SCCS_OK;
  (void)hipStreamSynchronize(h->stream);
  if (h->owns_ws && h->ws) (void)hipFree(h->ws);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->h_ctrl) (void)hipHostFree(h->h_ctrl);
  delete h;
  return SCCS_OK;
}

sccs_status sccs_set_prior(sccs_handle* h, int32_t kind, double variance) {
  sccs_status st = usable(h);
  if (st) return st;
  if (kind != SCCS_PRIOR_NONE && kind != SCCS_PRIOR_NORMAL && kind != SCCS_PRIOR_LAPLACE) {
    h->err = kind == SCCS_PRIOR_GROUPED ? "the grouped prior is set by sccs_set_prior_grouped" : "unknown prior kind";
    return SCCS_ERR_INVALID_ARG;
  }
  if (kind != SCCS_PRIOR_NONE && !(variance > 0.0 && std::isfinite(variance))) {
    h->err = "prior variance must be positive and finite";
    return SCCS_ERR_INVALID_ARG;
  }
  h->prior_kind = kind;
  h->var = kind == SCCS_PRIOR_NONE ? 1.0 : variance;
  return SCCS_OK;
}

sccs_status sccs_set_prior_grouped(sccs_handle* h, double variance, double class_variance, int32_t n_classes,
                                   const int32_t* class_of) {
  sccs_status st = usable(h);
  if (st) return st;
  if (!(variance > 0.0 && std::isfinite(variance)) || !(class_variance >= 0.0 && std::isfinite(class_variance))) {
    h->err = "grouped prior: variance must be positive and class_variance >= 0, both finite";
    return SCCS_ERR_INVALID_ARG;
  }
  if (!class_of || n_classes < 1 || n_classes > h->J) {
    h->err = "grouped prior: class_of must be given and 1 <= n_classes <= n_cols";
    return SCCS_ERR_INVALID_ARG;
  }
  std::vector<int32_t> members((size_t)n_classes, 0);
  for (int32_t j = 0; j < h->J; ++j) {
    if (class_of[j] < 0 || class_of[j] >= n_classes) {
      h->err = "grouped prior: class_of values must be in [0, n_classes)";
      return SCCS_ERR_INVALID_ARG;
    }
    ++members[class_of[j]];
  }
  // the class sums live in LDS next to beta and trust
  {
    const size_t lds = ssum_offset(h) * 8 + (size_t)n_classes * 8;
    int per_cu = 0;
    const void* k = ccd_kernel(h->prec, kModeSweep, false, h->valued);
    if (lds > 160 * 1024 || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, lds) != hipSuccess ||
        per_cu < 1) {
      h->err = "grouped prior: too many classes for the LDS budget";
      return SCCS_ERR_INVALID_ARG;
    }
  }
  std::vector<double> kappa((size_t)n_classes);
  for (int32_t c = 0; c < n_classes; ++c) kappa[c] = class_variance / (variance + (double)members[c] * class_variance);
  std::vector<int32_t> cls(class_of, class_of + h->J);
  if (!h->perm.empty())
    for (int32_t k = 0; k < h->J; ++k) cls[k] = class_of[h->perm[k]];
  HIPCHK(h, hipMemcpyAsync((void*)h->args.pclass, cls.data(), (size_t)h->J * 4, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync((void*)h->args.pkappa, kappa.data(), (size_t)n_classes * 8, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->prior_kind = SCCS_PRIOR_GROUPED;
  h->var = variance;
  h->class_var = class_variance;
  h->n_classes = n_classes;
  return SCCS_OK;
}

sccs_status sccs_set_beta(sccs_handle* h, const double* beta, const double* trust) {
  sccs_status st = usable(h);
  if (st) return st;
  if (!beta) { h->err = "beta is NULL"; return SCCS_ERR_INVALID_ARG; }
  for (int32_t j = 0; j < h->J; ++j) {
    if (!std::isfinite(beta[j]) || (trust && !(trust[j] > 0.0 && std::isfinite(trust[j])))) {
      h->err = "beta must be finite and trust positive";
      return SCCS_ERR_INVALID_ARG;
    }
  }
  std::vector<double> b(beta, beta + h->J), t((size_t)h->J, 1.0);
  if (trust) t.assign(trust, trust + h->J);
  if (!h->perm.empty())
    for (int32_t k = 0; k < h->J; ++k) {
      b[k] = beta[h->perm[k]];
      t[k] = trust ? trust[h->perm[k]] : 1.0;
    }
  HIPCHK(h, hipMemcpyAsync(h->args.beta, b.data(), (size_t)h->J * 8, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(h->args.trust, t.data(), (size_t)h->J * 8, hipMemcpyHostToDevice, h->stream));
  if (refresh_all(h) != SCCS_OK) return SCCS_ERR_HIP;
  h->use_merge = false;
  st = reset_moved(h);
  if (st) return st;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return SCCS_OK;
}

sccs_status sccs_get_beta(sccs_handle* h, double* beta, double* trust) {
  sccs_status st = usable(h);
  if (st) return st;
  if (!beta) { h->err = "beta is NULL"; return SCCS_ERR_INVALID_ARG; }
  std::vector<double> b((size_t)h->J), t(trust ? (size_t)h->J : 0);
  HIPCHK(h, hipMemcpyAsync(b.data(), h->args.beta, (size_t)h->J * 8, hipMemcpyDeviceToHost, h->stream));
  if (trust) HIPCHK(h, hipMemcpyAsync(t.data(), h->args.trust, (size_t)h->J * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int32_t k = 0; k < h->J; ++k) {
    const int32_t j = h->perm.empty() ? k : h->perm[k];
    beta[j] = b[k];
    if (trust) trust[j] = t[k];
  }
  return SCCS_OK;
}

sccs_status sccs_sweep(sccs_handle* h, int32_t n_sweeps, double* logpost) {
  sccs_status st = usable(h);
  if (st) return st;
  if (h->prior_kind < 0) { h->err = "set a prior before sweeping"; return SCCS_ERR_STATE; }
  if (n_sweeps < 0) { h->err = "n_sweeps must be >= 0"; return SCCS_ERR_INVALID_ARG; }
  if (n_sweeps == 0 && !logpost) return SCCS_OK;
  if (n_sweeps == 0) {
    double L;
    return sccs_objective(h, &L, logpost);
  }
  st = launch(h, kModeSweep, n_sweeps, SCCS_CRIT_FIXED, 0.0, logpost != nullptr, 0);
  if (st) return st;
  st = read_ctrl(h);
  if (st) return st;
  if (logpost) *logpost = h->h_ctrl->logpost;
  return SCCS_OK;
}

sccs_status sccs_sweep_static(sccs_handle* h, int32_t n_sweeps, double* logpost) {
  sccs_status st = usable(h);
  if (st) return st;
  if (h->prior_kind < 0) { h->err = "set a prior before sweeping"; return SCCS_ERR_STATE; }
  if (n_sweeps < 1) { h->err = "n_sweeps must be >= 1"; return SCCS_ERR_INVALID_ARG; }
  if (h->G > kScratchMaxWorkgroups) {
    h->err = "the static scratch array holds reduction slots for at most 256 workgroups";
    return SCCS_ERR_INVALID_ARG;
  }
  int dev = -1;
  HIPCHK(h, hipGetDevice(&dev));
  if (dev != h->device) { h->err = "make the handle's device current before sccs_sweep_static"; return SCCS_ERR_STATE; }
  uint64_t* base = nullptr;
  st = scratch_address(dev, &base, h->err);
  if (st) return st;
  KArgs a = h->args;
  a.slots = base;
  a.slots2 = base + kScrSlots1;
  a.oslots = a.slots2 + kScrSlots2;
  a.oslots2 = a.oslots + kScrO1;
  a.ctrl = (Ctrl*)(base + kScrTagWords);
  a.prior_kind = h->prior_kind;
  a.var = h->var;
  a.inv_var = 1.0 / h->var;
  a.lambda = (a.prior_kind == SCCS_PRIOR_LAPLACE) ? std::sqrt(2.0 / h->var) : 0.0;
  a.n_classes = a.prior_kind == SCCS_PRIOR_GROUPED ? h->n_classes : 0;
  a.n_sweeps = n_sweeps;
  a.criterion = SCCS_CRIT_FIXED;
  a.tol = 0.0;
  a.refresh_period = h->refresh_period;
  a.want_objective = logpost != nullptr;
  a.mode = kModeSweep;
  a.diag_j = 0;
  a.stamp = 0;
  hipLaunchKernelGGL(k_scratch_prep, dim3(64), dim3(256), 0, h->stream, base, kScrTagWords, a.ctrl,
                     (const Ctrl*)h->args.ctrl);
  HIPCHK(h, hipGetLastError());
  void* params[] = {&a};
  const bool merge = a.merge && h->use_merge && !h->valued && a.prior_kind != SCCS_PRIOR_GROUPED && h->perm.empty();
  HIPCHK(h, hipEventRecord(h->ev0, h->stream));
  HIPCHK(h, hipLaunchCooperativeKernel(ccd_kernel(h->prec, kModeSweep, merge, h->valued), dim3(h->G), dim3(kBlock), params,
                                        (unsigned)launch_lds(h, a.prior_kind), h->stream));
  HIPCHK(h, hipEventRecord(h->ev1, h->stream));
  h->timed = true;
  hipLaunchKernelGGL(k_scratch_post, dim3(1), dim3(64), 0, h->stream, (const Ctrl*)a.ctrl, h->args.ctrl);
  HIPCHK(h, hipGetLastError());
  // the handle's control block kept its own sequence numbers, so the host
  // mirror stays valid for the next sccs_sweep
  HIPCHK(h, hipMemcpyAsync(h->h_ctrl, h->args.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->last_mode = -1;
  h->passes = h->h_ctrl->passes;
  h->rejects = h->h_ctrl->rejects;
  h->zero_steps = h->h_ctrl->zero_steps;
  h->swept = true;
  {
    const double visits = (double)h->J * (h->h_ctrl->sweeps > 0 ? h->h_ctrl->sweeps : 1);
    const double zf = h->zero_steps / visits;
    if (!h->use_merge && zf >= 0.5) h->use_merge = true;
    else if (h->use_merge && zf < 0.35) h->use_merge = false;
  }
  if (h->h_ctrl->status == SCCS_ERR_SYNC) {
    h->failed = true;
    h->err = "device-wide reduction timed out (workgroups not co-resident?)";
    return SCCS_ERR_SYNC;
  }
  if (h->h_ctrl->status == SCCS_ERR_NUMERIC) {
    h->err = "non-finite gradient, Hessian or coefficient; last finite beta kept";
    return SCCS_ERR_NUMERIC;
  }
  if (logpost) *logpost = h->h_ctrl->logpost;
  return SCCS_OK;
}

sccs_status sccs_fit(sccs_handle* h, const sccs_fit_opts* fo, sccs_fit_result* res) {
  sccs_status st = usable(h);
  if (st) return st;
  if (!fo || !res) { h->err = "fit options and result must not be NULL"; return SCCS_ERR_INVALID_ARG; }
  if (h->prior_kind < 0) { h->err = "set a prior before fitting"; return SCCS_ERR_STATE; }
  if (fo->max_sweeps < 1 || fo->criterion < SCCS_CRIT_FIXED || fo->criterion > SCCS_CRIT_ABS_DXBETA ||
      !(fo->tol >= 0.0)) {
    h->err = "invalid fit options";
    return SCCS_ERR_INVALID_ARG;
  }
  st = launch(h, kModeSweep, fo->max_sweeps, fo->criterion, fo->tol, 1, 0);
  if (st) return st;
  st = read_ctrl(h);
  if (st) return st;
  res->sweeps = h->h_ctrl->sweeps;
  res->converged = h->h_ctrl->converged;
  res->loglik = h->h_ctrl->loglik;
  res->logpost = h->h_ctrl->logpost;
  if (fo->criterion == SCCS_CRIT_FIXED) return SCCS_OK;
  return res->converged ? SCCS_OK : SCCS_NOT_CONVERGED;
}

sccs_status sccs_grad_hess(sccs_handle* h, int32_t j, double* g, double* hess) {
  sccs_status st = usable(h);
  if (st) return st;
  if (j < 0 || j >= h->J || !g || !hess) { h->err = "invalid column or NULL output"; return SCCS_ERR_INVALID_ARG; }
  st = launch(h, kModeGradHess, 0, SCCS_CRIT_FIXED, 0.0, 0, h->pos.empty() ? j : h->pos[j]);
  if (st) return st;
  st = read_ctrl(h);
  if (st) return st;
  *g = h->h_ctrl->g;
  *hess = h->h_ctrl->h;
  return SCCS_OK;
}

sccs_status sccs_objective(sccs_handle* h, double* loglik, double* logpost) {
  sccs_status st = usable(h);
  if (st) return st;
  if (!loglik || !logpost) { h->err = "NULL output"; return SCCS_ERR_INVALID_ARG; }
  st = launch(h, kModeObjective, 0, SCCS_CRIT_FIXED, 0.0, 1, 0);
  if (st) return st;
  st = read_ctrl(h);
  if (st) return st;
  *loglik = h->h_ctrl->loglik;
  *logpost = h->h_ctrl->logpost;
  return SCCS_OK;
}

sccs_status sccs_pass_stats(sccs_handle* h, int32_t* passes, int32_t* rejects, int32_t* zero_steps) {
  if (!h || !passes || !rejects || !zero_steps) return SCCS_ERR_INVALID_ARG;
  if (!h->swept) { h->err = "no sweep run yet"; return SCCS_ERR_STATE; }
  *passes = h->passes;
  *rejects = h->rejects;
  *zero_steps = h->zero_steps;
  return SCCS_OK;
}

sccs_status sccs_group_timing(sccs_handle* h, int32_t on) {
  if (!h || (on != 0 && on != 1)) return SCCS_ERR_INVALID_ARG;
  h->group_timing = on != 0;
  return SCCS_OK;
}

sccs_status sccs_group_times(sccs_handle* h, int32_t max_groups, double* t_us, int32_t* first_col, int32_t* n_groups) {
  if (!h || !t_us || !first_col || !n_groups) return SCCS_ERR_INVALID_ARG;
  if (!h->swept || h->last_mode != kModeSweep || h->last_merged || h->valued || !h->last_stamped) {
    h->err = "group times need a preceding sccs_sweep / sccs_fit launch in the one-pass-per-group form, "
             "with sccs_group_timing on";
    return SCCS_ERR_STATE;
  }
  const int32_t NG = (int32_t)h->gcol.size() - 1;
  *n_groups = NG;
  if (max_groups < NG) { h->err = "max_groups is smaller than the number of column groups"; return SCCS_ERR_INVALID_ARG; }
  std::vector<uint64_t> ticks((size_t)NG + 1);
  HIPCHK(h, hipMemcpyAsync(ticks.data(), h->args.group_ticks, ticks.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  int khz = 0;
  HIPCHK(h, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device));
  if (khz <= 0) { h->err = "wall-clock rate unknown"; return SCCS_ERR_HIP; }
  for (int32_t g = 0; g < NG; ++g) t_us[g] = (double)(int64_t)(ticks[g] - ticks[NG]) * 1e3 / khz;
  for (int32_t g = 0; g <= NG; ++g) first_col[g] = h->gcol[g];
  return SCCS_OK;
}

sccs_status sccs_last_kernel_ms(sccs_handle* h, double* ms) {
  if (!h || !ms) return SCCS_ERR_INVALID_ARG;
  if (!h->timed) { h->err = "no kernel launched yet"; return SCCS_ERR_STATE; }
  HIPCHK(h, hipEventSynchronize(h->ev1));
  float f = 0.f;
  HIPCHK(h, hipEventElapsedTime(&f, h->ev0, h->ev1));
  *ms = f;
  return SCCS_OK;
}

sccs_status sccs_tune(const sccs_problem* prob, const sccs_options* base, int32_t prior_kind, double variance,
                      int32_t n_sweeps, sccs_options* best, sccs_tune_result* result) {
  if (!prob || !best || !result || n_sweeps < 1) {
    g_create_error = "sccs_tune: NULL argument or n_sweeps < 1";
    return SCCS_ERR_INVALID_ARG;
  }
  sccs_options o;
  sccs_default_options(&o);
  if (base) o = *base;
  std::string err;
  int32_t G = 0;
  sccs_status st = check_options(&o, err);
  if (st == SCCS_OK) {
    sccs_options all = o;
    all.n_workgroups = 0;
    st = pick_workgroups(&all, G, err);
  }
  if (st) { g_create_error = err; return st; }
  std::memset(result, 0, sizeof *result);
  const int gs[4] = {G, (3 * G) / 4, G / 2, G / 4};
  const int ts[3] = {16, 32, 64};
  double best_ms = 1e300;
  for (int gi = 0; gi < 4; ++gi) {
    if (gs[gi] < 1 || (gi > 0 && gs[gi] == gs[gi - 1])) continue;
    for (int ti = 0; ti < 3; ++ti) {
      if (result->n_candidates >= SCCS_TUNE_MAX) break;
      sccs_options c = o;
      c.n_workgroups = gs[gi];
      c.tile_nnz = ts[ti];
      sccs_handle* h = nullptr;
      st = sccs_create(prob, &c, nullptr, 0, &h);
      if (st) return st;
      double ms = 0.0;
      st = sccs_set_prior(h, prior_kind, variance);
      if (!st) st = sccs_sweep(h, 1, nullptr);
      if (!st) st = sccs_sweep(h, n_sweeps, nullptr);
      if (!st) st = sccs_last_kernel_ms(h, &ms);
      if (st) {
        g_create_error = std::string("sccs_tune: ") + h->err;
        sccs_destroy(h);
        return st;
      }
      sccs_destroy(h);
      const int k = result->n_candidates++;
      result->n_workgroups[k] = gs[gi];
      result->tile_nnz[k] = ts[ti];
      result->ms_per_sweep[k] = ms / n_sweeps;
      if (ms < best_ms) {
        best_ms = ms;
        result->best = k;
      }
    }
  }
  *best = o;
  best->n_workgroups = result->n_workgroups[result->best];
  best->tile_nnz = result->tile_nnz[result->best];
  return SCCS_OK;
}

sccs_status sccs_column_order(const sccs_problem* prob, int32_t width, int32_t* order) {
  std::string err;
  if (!order) { g_create_error = "order is NULL"; return SCCS_ERR_INVALID_ARG; }
  if (width < 1 || width > kMaxGroup) { g_create_error = "width must be in [1, 4]"; return SCCS_ERR_INVALID_ARG; }
  sccs_status st = validate_problem(prob, err);
  if (st) { g_create_error = err; return st; }
  std::vector<int32_t> o;
  try {
    independent_order(prob, width, o);
  } catch (const std::bad_alloc&) {
    g_create_error = "host out of memory";
    return SCCS_ERR_INVALID_ARG;
  }
  std::copy(o.begin(), o.end(), order);
  return SCCS_OK;
}

sccs_status sccs_get_column_order(sccs_handle* h, int32_t* order) {
  if (!h || !order) return SCCS_ERR_INVALID_ARG;
  for (int32_t k = 0; k < h->J; ++k) order[k] = h->perm.empty() ? k : h->perm[k];
  return SCCS_OK;
}

const char* sccs_last_error(const sccs_handle* h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"

#include "sccs_batch_api.inc"
