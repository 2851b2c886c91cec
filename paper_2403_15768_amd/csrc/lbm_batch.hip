// lbm_batch.hip -- batches of channels advanced by one kernel launch per step
// and group.
//
// A batch groups existing contexts (same lattice, storage precision and wall
// kind; any sizes and parameters).  Its work list holds, per wave, 64 lanes
// of one member (a 64-cell x-segment, or two 32-cell chunks of interior
// columns), and every item carries its column's record so that a wave's
// set-up is one chain of two scalar loads (item, member).  Members keep their
// own buffers, parameters and step counters: a member's step number decides
// which of its two buffers is current and which stochastic-rounding bits it
// uses, so a channel advanced inside a batch is bit-identical to the same
// channel advanced alone.  On the device the batch keeps one counter, the
// steps taken since its member table was written; a member's step is its base
// step plus that counter.
//
// Members are independent, so they need not advance in lockstep: the batch
// is cut into groups whose state fits the 256 MB last-level cache, and each
// group runs a whole 64-step graph before the next group starts.  A group's
// populations then stay in that cache from one step to the next instead of
// streaming from HBM every step.  Groups are dealt round-robin to two
// streams (the batch's own and one of the batch's making, both at default
// priority) so that one group's launch tails overlap another group's work;
// the streams join before the device counter advances.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_internal.h"

using lbm::MemberDesc;
using lbm::WorkItem;
using namespace lbm_host;

constexpr int kMaxStreams = 4;

struct lbm_batch {
  std::vector<lbm_ctx*> m;
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  int Q = 0, prec = 0;
  bool bouz = false;
  int th = 0;  // every member's thermal-noise form (0: none)
  int64_t nitems = 0;
  struct Group {
    int64_t first, nwall, last;  // items [first, last), wall items [first, nwall)
  };
  std::vector<Group> groups;
  size_t group_bytes = 0;
  int wpb = 4;  // waves (work items) per workgroup, set by lbm_batch_tune
  int64_t k = 0;                  // steps since the member table was written
  std::vector<int64_t> base;      // each member's step when the table was written
  std::vector<double> th_amp;     // each member's noise amplitude and key in the table
  std::vector<uint64_t> th_seed;
  std::vector<std::array<double, 6>> th_fac;  // and noise-closure factors
  int64_t max_items = 0;  // capacity of the item arrays (largest list over the shapes)
  size_t off_desc = 0, off_items = 0, off_cols = 0, off_order = 0, off_mstart = 0, off_partials = 0,
         off_out = 0, off_bstep = 0, total = 0;
  std::vector<hipGraph_t> graph;  // per group: kGraphSteps steps
  std::vector<hipGraphExec_t> gexec;
  int graph_wpb = 0;
  int nstreams = 2;                       // streams the groups are dealt to
  hipStream_t side[kMaxStreams - 1] = {};  // streams 1.. (stream 0 is the batch stream)
  hipEvent_t fork = nullptr, join[kMaxStreams - 1] = {};
  bool graphs_ok = true;
  std::string err;

  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(arena + off);
  }
  lbm_status fail(lbm_status s, const char* msg) {
    err = msg;
    return s;
  }
  lbm_status hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return LBM_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EDEVICE;
  }
};

#define BCHK(b, call)                               \
  do {                                              \
    lbm_status _s = (b)->hip((call), #call);        \
    if (_s != LBM_OK) return _s;                    \
  } while (0)

namespace {

struct Lists {
  std::vector<WorkItem> items;
  std::vector<int32_t> cols;  // column ids of the runs the items cover
  std::vector<lbm_batch::Group> groups;
  std::vector<int32_t> order;
  std::vector<int64_t> mstart;
};

// Default group size: with two groups in flight at a time their state (both
// buffers of every member) fills most of the 256 MB last-level cache.  Half
// storage does best with somewhat smaller groups (measured on 256 uneven
// ducts: 96 MiB 681 us/step against 719 with 128 MiB).
size_t default_group_bytes(int precision) {
  return precision == LBM_F16S ? (size_t)96 << 20 : (size_t)128 << 20;
}

// The work list, in units of one workgroup (wpb items, one per wave; a
// workgroup never shares a column with another, so the partly covered cache
// lines at the ends of a column's x-lines are completed inside one L2):
//  * general columns (wall links or periodic wrap): as many whole columns as
//    fit in wpb waves, ceil(nxp/64) waves each; a longer column in segments
//    of 64 wpb cells (its x-lines are then padded, so segments start on
//    whole lines);
//  * plain columns of a member whose lines fit 64-bit-free addressing: runs
//    of k = floor(64 wpb / nxp) whole columns, their cells taken in order
//    and 64 to a wave (a wave may span up to three columns);
//  * unused waves of a workgroup get empty items (member -1).
// cols[] holds the column ids of each run, items point into it.
bool packs(const lbm_ctx* c) {
  const Plan& pl = c->pl;
  return pl.nxp >= 32 && pl.pop_bytes < ((size_t)1 << 31);
}

struct Builder {
  Lists* L;
  std::vector<std::vector<int32_t>>* mine;
  int wpb;
  int used = 0;  // items in the current workgroup
  void push(const WorkItem& w) {
    if (w.member >= 0) (*mine)[w.member].push_back((int32_t)L->items.size());
    L->items.push_back(w);
    used = (used + 1) % wpb;
  }
  void close_group() {  // pad the current workgroup with empty items
    while (used != 0) push(WorkItem{-1, 0, 0, 0, 0, -1, 0u, 0});
  }
  // a run of columns (ids ascending) covering ncols * nxp cells
  void run(int m, const std::vector<int32_t>& ids, int nxp, int32_t wallcol, uint32_t mask) {
    const int32_t cbase = (int32_t)L->cols.size();
    L->cols.insert(L->cols.end(), ids.begin(), ids.end());
    const int64_t cells = (int64_t)ids.size() * nxp;
    for (int64_t e0 = 0; e0 < cells; e0 += 64)
      push(WorkItem{m, cbase, (int32_t)ids.size(), (int32_t)(e0 / nxp), (int32_t)(e0 % nxp), wallcol,
                    mask, 0});
  }
};

void member_items(Builder& B, lbm_ctx* c, int m, int pass) {
  const Plan& pl = c->pl;
  const int wpb = B.wpb, nxp = pl.nxp;
  const int wpc = (nxp + 63) / 64;  // waves per column
  std::vector<int32_t> ids;
  if (pass == 1 && packs(c) && nxp <= 64 * wpb) {
    const int k = std::max(1, 64 * wpb / nxp);
    for (const lbm::ColSlot& cs : pl.slots) {
      if (cs.mask != 0u) continue;
      ids.push_back(cs.col);
      if ((int)ids.size() == k) {
        B.run(m, ids, nxp, -1, 0u);
        B.close_group();
        ids.clear();
      }
    }
    if (!ids.empty()) {
      B.run(m, ids, nxp, -1, 0u);
      B.close_group();
    }
    return;
  }
  for (const lbm::ColSlot& cs : pl.slots) {
    if ((pass == 0) != (cs.mask != 0u)) continue;
    ids.assign(1, cs.col);
    if (wpc > wpb) {  // long (padded) x-lines: segments of whole workgroups
      const int32_t cbase = (int32_t)B.L->cols.size();
      B.L->cols.push_back(cs.col);
      B.close_group();
      for (int x0 = 0; x0 < nxp; x0 += 64) B.push(WorkItem{m, cbase, 1, 0, x0, cs.wallcol, cs.mask, 0});
      B.close_group();
      continue;
    }
    if (B.used + wpc > wpb) B.close_group();
    B.run(m, ids, nxp, cs.wallcol, cs.mask);
  }
  B.close_group();
}

// Members in order, cut into groups of at most group_bytes of state (a
// larger member forms a group of its own; 0: one group).  Within a group,
// the general columns of every member first (they do more work), then the
// plain ones; `order` lists each member's items contiguously for the
// reductions.
int64_t count_items(lbm_ctx* const* ctxs, int n, int wpb);

void make_lists(lbm_ctx* const* ctxs, int n, size_t group_bytes, int wpb, Lists* L) {
  L->items.clear();
  L->cols.clear();
  L->groups.clear();
  int64_t ncol = 0;
  for (int m = 0; m < n; m++) ncol += (int64_t)ctxs[m]->pl.slots.size();
  L->cols.reserve(ncol);
  L->items.reserve(count_items(ctxs, n, wpb));
  std::vector<std::vector<int32_t>> mine(n);
  Builder B{L, &mine, wpb};
  for (int m0 = 0; m0 < n;) {
    int m1 = m0 + 1;
    size_t bytes = 2 * ctxs[m0]->pl.pop_bytes;
    while (group_bytes && m1 < n && bytes + 2 * ctxs[m1]->pl.pop_bytes <= group_bytes)
      bytes += 2 * ctxs[m1++]->pl.pop_bytes;
    if (!group_bytes) m1 = n;
    lbm_batch::Group g{(int64_t)L->items.size(), 0, 0};
    for (int m = m0; m < m1; m++) member_items(B, ctxs[m], m, 0);
    g.nwall = (int64_t)L->items.size();
    for (int m = m0; m < m1; m++) member_items(B, ctxs[m], m, 1);
    g.last = (int64_t)L->items.size();
    L->groups.push_back(g);
    m0 = m1;
  }
  L->order.clear();
  L->mstart.assign(n + 1, 0);
  for (int m = 0; m < n; m++) {
    L->mstart[m] = (int64_t)L->order.size();
    L->order.insert(L->order.end(), mine[m].begin(), mine[m].end());
  }
  L->mstart[n] = (int64_t)L->order.size();
}

lbm_status check_members(lbm_ctx* const* ctxs, int n) {
  if (!ctxs || n < 1) return LBM_EINVAL;
  for (int m = 0; m < n; m++) {
    if (!ctxs[m]) return LBM_EINVAL;
    for (int k = 0; k < m; k++)
      if (ctxs[k] == ctxs[m]) return LBM_EINVAL;
    const lbm_params &a = ctxs[0]->p, &b = ctxs[m]->p;
    if (a.lattice != b.lattice || a.precision != b.precision ||
        (a.geometry == LBM_TUBE) != (b.geometry == LBM_TUBE))
      return LBM_EINVAL;
    // one noise form for the whole batch (each member its own kT and seed);
    // the batch kernel has no electron sheets, masked walls or open ends
    if (ctxs[m]->args.th_mode != ctxs[0]->args.th_mode || ctxs[m]->elec || ctxs[m]->pl.masked ||
        ctxs[m]->args.open)
      return LBM_EINVAL;
  }
  return LBM_OK;
}

void layout(lbm_batch* b, int n, int64_t nitems, int64_t ncols) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  b->off_desc = take(n * sizeof(MemberDesc));
  b->off_items = take(nitems * sizeof(WorkItem));
  b->off_cols = take(ncols * sizeof(int32_t));
  b->off_order = take(nitems * sizeof(int32_t));
  b->off_mstart = take((n + 1) * sizeof(int64_t));
  b->off_partials = take(nitems * 2 * sizeof(double));
  b->off_out = take(n * 2 * sizeof(double));
  b->off_bstep = take(sizeof(int64_t));
  b->total = off;
}

// workgroup shapes (waves per workgroup) the autotuner tries
constexpr int kShapes[3] = {2, 4, 8};

// items make_lists gives a member's pass, counted without building them
int64_t member_count(const lbm_ctx* c, int wpb, int pass) {
  const Plan& pl = c->pl;
  const int64_t nxp = pl.nxp, wpc = (nxp + 63) / 64;
  int64_t g = 0;
  for (const lbm::ColSlot& cs : pl.slots) g += (pass == 0) == (cs.mask != 0u);
  if (g == 0) return 0;
  if (pass == 1 && packs(c) && nxp <= 64 * wpb) {
    const int64_t k = std::max<int64_t>(1, 64 * wpb / nxp);
    return (g + k - 1) / k * wpb;
  }
  if (wpc > wpb) return g * ((wpc + wpb - 1) / wpb) * wpb;
  const int64_t kw = wpb / wpc;
  return (g + kw - 1) / kw * wpb;
}

int64_t count_items(lbm_ctx* const* ctxs, int n, int wpb) {
  int64_t t = 0;
  for (int m = 0; m < n; m++) t += member_count(ctxs[m], wpb, 0) + member_count(ctxs[m], wpb, 1);
  return t;
}

// item capacity: the longest list over every shape (the length does not
// depend on the grouping: each member's items are whole workgroups)
int64_t max_items(lbm_ctx* const* ctxs, int n) {
  int64_t t = 0;
  for (int w : {1, 2, 4, 8}) t = std::max(t, count_items(ctxs, n, w));
  return t;
}

int64_t count_cols(lbm_ctx* const* ctxs, int n) {
  int64_t t = 0;
  for (int m = 0; m < n; m++) t += (int64_t)ctxs[m]->pl.slots.size();
  return t;
}

// one step (step_off steps past the device counter) of group gi
lbm_status launch_batch(lbm_batch* b, size_t gi, int64_t step_off, int wpb,
                        hipStream_t st = nullptr) {
  const void* fn = lbm::batch_step_kernel_ptr(b->Q, b->prec, b->bouz, b->th);
  const MemberDesc* md = b->at<MemberDesc>(b->off_desc);
  const WorkItem* items = b->at<WorkItem>(b->off_items);
  const int32_t* cols = b->at<int32_t>(b->off_cols);
  lbm_batch::Group g = b->groups[gi];
  const int64_t* bstep = b->at<int64_t>(b->off_bstep);
  void* args[9] = {(void*)&md,     (void*)&items, (void*)&cols,     (void*)&g.first, (void*)&g.nwall,
                   (void*)&g.last, (void*)&bstep, (void*)&step_off, (void*)&wpb};
  const dim3 grid((unsigned)((g.last - g.first + wpb - 1) / wpb)), block(64 * wpb);
  BCHK(b, hipLaunchKernel(fn, grid, block, args, 0, st ? st : b->stream));
  return LBM_OK;
}

hipStream_t group_stream(const lbm_batch* b, size_t gi) {
  const int k = (int)(gi % (size_t)b->nstreams);
  return k ? b->side[k - 1] : b->stream;
}

// the other streams start after the work queued so far on the batch stream
lbm_status fork_streams(lbm_batch* b) {
  if (b->nstreams < 2) return LBM_OK;
  BCHK(b, hipEventRecord(b->fork, b->stream));
  for (int k = 1; k < b->nstreams; k++) BCHK(b, hipStreamWaitEvent(b->side[k - 1], b->fork, 0));
  return LBM_OK;
}

// the batch stream continues after everything queued on the others
lbm_status join_streams(lbm_batch* b) {
  for (int k = 1; k < b->nstreams; k++) {
    BCHK(b, hipEventRecord(b->join[k - 1], b->side[k - 1]));
    BCHK(b, hipStreamWaitEvent(b->stream, b->join[k - 1], 0));
  }
  return LBM_OK;
}

void drop_streams(lbm_batch* b) {
  for (int k = 0; k < kMaxStreams - 1; k++) {
    if (b->side[k]) {
      (void)hipStreamSynchronize(b->side[k]);
      (void)hipStreamDestroy(b->side[k]);
      b->side[k] = nullptr;
    }
    if (b->join[k]) {
      (void)hipEventDestroy(b->join[k]);
      b->join[k] = nullptr;
    }
  }
  if (b->fork) {
    (void)hipEventDestroy(b->fork);
    b->fork = nullptr;
  }
}

void drop_graphs(lbm_batch* b) {
  for (hipGraphExec_t e : b->gexec)
    if (e) (void)hipGraphExecDestroy(e);
  for (hipGraph_t g : b->graph)
    if (g) (void)hipGraphDestroy(g);
  b->gexec.clear();
  b->graph.clear();
}

lbm_status launch_bump(lbm_batch* b, int64_t v) {
  const void* fn = lbm::add_step_kernel_ptr();
  int64_t* d = b->at<int64_t>(b->off_bstep);
  void* args[2] = {(void*)&d, (void*)&v};
  BCHK(b, hipLaunchKernel(fn, dim3(1), dim3(64), args, 0, b->stream));
  return LBM_OK;
}

// the members' own device step bases are not advanced by batch steps
constexpr int64_t kStale = INT64_MIN;

void advance_members(lbm_batch* b, int64_t k) {
  b->k += k;
  for (lbm_ctx* c : b->m) {
    c->step += k;
    c->dstep_value = kStale;
    if (k & 1) c->cur = 1 - c->cur;
  }
}

MemberDesc describe(const lbm_ctx* c, int64_t k) {
  MemberDesc d;
  std::memset(&d, 0, sizeof d);
  d.a = c->args;
  d.a.dstep = nullptr;
  d.a.step_off = 0;
  d.pop[0] = c->pop[0];
  d.pop[1] = c->pop[1];
  d.base_step = c->step - k;
  d.cur_base = (int32_t)((c->cur + k) & 1);  // (cur_base + k) & 1 == cur
  return d;
}

// A member stepped, restored or overwritten outside the batch no longer sits
// at base + k: rewrite its table entry (after its own queued work).
lbm_status resync(lbm_batch* b) {
  for (size_t m = 0; m < b->m.size(); m++) {
    lbm_ctx* c = b->m[m];
    if (c->step == b->base[m] + b->k && c->args.th_amp == b->th_amp[m] &&
        c->args.th_seed == b->th_seed[m] &&
        std::equal(b->th_fac[m].begin(), b->th_fac[m].end(), c->args.th_fac))
      continue;
    lbm_status s = sync(c);
    if (s != LBM_OK) return b->fail(s, "member stream failed");
    const MemberDesc d = describe(c, b->k);
    BCHK(b, hipMemcpyAsync(b->at<MemberDesc>(b->off_desc) + m, &d, sizeof d,
                           hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipStreamSynchronize(b->stream));
    b->base[m] = d.base_step;
    b->th_amp[m] = c->args.th_amp;
    b->th_seed[m] = c->args.th_seed;
    std::copy(c->args.th_fac, c->args.th_fac + 6, b->th_fac[m].begin());
  }
  return LBM_OK;
}

// kGraphSteps steps of group gi, step k at (device counter + k); the
// counter itself is advanced once all groups have run
lbm_status build_graph(lbm_batch* b, size_t gi, hipGraph_t* gout, hipGraphExec_t* xout) {
  hipGraph_t g = nullptr;
  BCHK(b, hipGraphCreate(&g, 0));
  const void* fn = lbm::batch_step_kernel_ptr(b->Q, b->prec, b->bouz, b->th);
  const MemberDesc* md = b->at<MemberDesc>(b->off_desc);
  const WorkItem* items = b->at<WorkItem>(b->off_items);
  const int32_t* cols = b->at<int32_t>(b->off_cols);
  const int64_t* bstep = b->at<int64_t>(b->off_bstep);
  lbm_batch::Group grp = b->groups[gi];
  int wpb = b->wpb;
  hipGraphNode_t prev = nullptr;
  int64_t offs[kGraphSteps];
  for (int k = 0; k < kGraphSteps; k++) {
    offs[k] = k;
    void* args[9] = {(void*)&md,       (void*)&items,       (void*)&cols,
                     (void*)&grp.first, (void*)&grp.nwall,  (void*)&grp.last,
                     (void*)&bstep,     (void*)&offs[k],    (void*)&wpb};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = dim3((unsigned)((grp.last - grp.first + wpb - 1) / wpb));
    kp.blockDim = dim3(64 * wpb);
    kp.kernelParams = args;
    hipGraphNode_t node = nullptr;
    hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return b->hip(e, "hipGraphAddKernelNode");
    }
    prev = node;
  }
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return b->hip(e, "hipGraphInstantiate");
  }
  *gout = g;
  *xout = ex;
  return LBM_OK;
}

lbm_status build_graphs(lbm_batch* b) {
  drop_graphs(b);
  for (size_t gi = 0; gi < b->groups.size(); gi++) {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    lbm_status s = build_graph(b, gi, &g, &x);
    if (s != LBM_OK) {
      drop_graphs(b);
      return s;
    }
    b->graph.push_back(g);
    b->gexec.push_back(x);
  }
  b->graph_wpb = b->wpb;
  return LBM_OK;
}

// (re)write the work list for the current group size and shape; synchronous
lbm_status upload_lists(lbm_batch* b) {
  Lists L;
  make_lists(b->m.data(), (int)b->m.size(), b->group_bytes, b->wpb, &L);
  if ((int64_t)L.items.size() != count_items(b->m.data(), (int)b->m.size(), b->wpb) ||
      (int64_t)L.items.size() > b->max_items)
    return b->fail(LBM_EINVAL, "internal: item count");
  BCHK(b, hipStreamSynchronize(b->stream));  // no launch may still read the old list
  drop_graphs(b);
  b->groups = L.groups;
  b->nitems = (int64_t)L.items.size();
  BCHK(b, hipMemcpyAsync(b->at<void>(b->off_items), L.items.data(),
                         L.items.size() * sizeof(WorkItem), hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemcpyAsync(b->at<void>(b->off_cols), L.cols.data(),
                         L.cols.size() * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemcpyAsync(b->at<void>(b->off_order), L.order.data(),
                         L.order.size() * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemcpyAsync(b->at<void>(b->off_mstart), L.mstart.data(),
                         L.mstart.size() * sizeof(int64_t), hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_footprint(lbm_ctx* const* ctxs, int n, size_t* bytes) {
  if (!bytes) return LBM_EINVAL;
  lbm_status s = check_members(ctxs, n);
  if (s != LBM_OK) return s;
  lbm_batch tmp;
  layout(&tmp, n, max_items(ctxs, n), count_cols(ctxs, n));
  *bytes = tmp.total;
  return LBM_OK;
}

lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int n, void* arena, size_t arena_bytes,
                            void* hip_stream, lbm_batch** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  lbm_status s = check_members(ctxs, n);
  if (s != LBM_OK) return s;
  if (!arena || reinterpret_cast<uintptr_t>(arena) % kAlign) return LBM_EINVAL;
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ENOMEM;
  b->m.assign(ctxs, ctxs + n);
  b->Q = ctxs[0]->p.lattice;
  b->prec = ctxs[0]->p.precision;
  b->bouz = ctxs[0]->p.geometry == LBM_TUBE;
  Lists L;
  b->group_bytes = default_group_bytes(b->prec);
  make_lists(ctxs, n, b->group_bytes, b->wpb, &L);
  b->nitems = (int64_t)L.items.size();
  b->groups = L.groups;
  b->max_items = max_items(ctxs, n);
  layout(b, n, b->max_items, count_cols(ctxs, n));
  if (b->nitems != count_items(ctxs, n, b->wpb)) {
    delete b;
    return LBM_EINVAL;  // internal: the counted and the built lists differ
  }
  if (arena_bytes < b->total || b->max_items >= ((int64_t)1 << 31)) {
    const lbm_status e = arena_bytes < b->total ? LBM_ENOMEM : LBM_EINVAL;
    delete b;
    return e;
  }
  b->arena = static_cast<char*>(arena);
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  // extra streams at the default priority, and the events that order them
  bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; ok && k < kMaxStreams - 1; k++)
    ok = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    drop_streams(b);
    delete b;
    return LBM_EDEVICE;
  }
  std::vector<MemberDesc> desc(n);
  b->base.assign(n, 0);
  b->th_amp.assign(n, 0.0);
  b->th_seed.assign(n, 0);
  b->th_fac.assign(n, std::array<double, 6>{});
  b->th = ctxs[0]->args.th_mode;
  for (int m = 0; m < n; m++) {
    lbm_ctx* c = ctxs[m];
    if ((s = sync(c)) != LBM_OK) {
      drop_streams(b);
      delete b;
      return s;
    }
    desc[m] = describe(c, 0);
    b->base[m] = c->step;
    b->th_amp[m] = c->args.th_amp;
    b->th_seed[m] = c->args.th_seed;
    std::copy(c->args.th_fac, c->args.th_fac + 6, b->th_fac[m].begin());
  }
  const int64_t zero = 0;
  lbm_status st = LBM_OK;
  do {
    if ((st = b->hip(hipMemcpyAsync(b->at<void>(b->off_desc), desc.data(), n * sizeof(MemberDesc),
                                    hipMemcpyHostToDevice, b->stream), "upload")) != LBM_OK) break;
    if ((st = b->hip(hipMemcpyAsync(b->at<void>(b->off_items), L.items.data(),
                                    L.items.size() * sizeof(WorkItem), hipMemcpyHostToDevice,
                                    b->stream), "upload")) != LBM_OK) break;
    if ((st = b->hip(hipMemcpyAsync(b->at<void>(b->off_cols), L.cols.data(),
                                    L.cols.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                    b->stream), "upload")) != LBM_OK) break;
    if ((st = b->hip(hipMemcpyAsync(b->at<void>(b->off_order), L.order.data(),
                                    L.order.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                                    b->stream), "upload")) != LBM_OK) break;
    if ((st = b->hip(hipMemcpyAsync(b->at<void>(b->off_mstart), L.mstart.data(),
                                    L.mstart.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                                    b->stream), "upload")) != LBM_OK) break;
    if ((st = b->hip(hipMemcpyAsync(b->at<void>(b->off_bstep), &zero, sizeof zero,
                                    hipMemcpyHostToDevice, b->stream), "upload")) != LBM_OK) break;
    st = b->hip(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  } while (0);
  if (st != LBM_OK) {
    drop_streams(b);
    delete b;
    return st;
  }
  *out = b;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  drop_graphs(b);
  drop_streams(b);
  delete b;
}

lbm_status lbm_batch_items(const lbm_batch* b, int64_t* nitems) {
  if (!b || !nitems) return LBM_EINVAL;
  *nitems = b->nitems;
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return LBM_EINVAL;
  if (nsteps == 0) return LBM_OK;
  for (lbm_ctx* c : b->m)
    if (c->args.th_mode != b->th || c->elec || c->args.open) {
      b->err = "a member's noise form changed or its electron sheets or open ends are on; "
               "rebuild the batch";
      return LBM_EINVAL;
    }
  lbm_status rs = resync(b);
  if (rs != LBM_OK) return rs;
  // each group runs its kGraphSteps steps before the next group starts; the
  // device counter advances once all groups have
  while (nsteps >= kGraphSteps && b->graphs_ok) {
    if (b->gexec.empty() || b->graph_wpb != b->wpb) {
      if (build_graphs(b) != LBM_OK) {
        b->graphs_ok = false;  // fall back to plain launches
        (void)hipGetLastError();
        break;
      }
    }
    lbm_status s = fork_streams(b);
    if (s != LBM_OK) return s;
    for (size_t gi = 0; gi < b->gexec.size(); gi++)
      BCHK(b, hipGraphLaunch(b->gexec[gi], group_stream(b, gi)));
    if ((s = join_streams(b)) != LBM_OK) return s;
    s = launch_bump(b, kGraphSteps);
    if (s != LBM_OK) return s;
    advance_members(b, kGraphSteps);
    nsteps -= kGraphSteps;
  }
  if (nsteps > 0) {
    lbm_status s = fork_streams(b);
    if (s != LBM_OK) return s;
    for (size_t gi = 0; gi < b->groups.size(); gi++)
      for (int64_t j = 0; j < nsteps; j++)
        if ((s = launch_batch(b, gi, j, b->wpb, group_stream(b, gi))) != LBM_OK) return s;
    if ((s = join_streams(b)) != LBM_OK) return s;
    s = launch_bump(b, nsteps);
    if (s != LBM_OK) return s;
    advance_members(b, nsteps);
  }
  return LBM_OK;
}

lbm_status lbm_batch_invariants(lbm_batch* b, double* out) {
  if (!b || !out) return LBM_EINVAL;
  const int n = (int)b->m.size();
  double* dout = b->at<double>(b->off_out);
  lbm_status rs = resync(b);
  if (rs != LBM_OK) return rs;
  BCHK(b, lbm::launch_batch_moments(b->Q, b->prec, b->at<MemberDesc>(b->off_desc),
                                    b->at<WorkItem>(b->off_items), b->at<int32_t>(b->off_cols),
                                    b->nitems,
                                    b->at<int64_t>(b->off_bstep), b->at<double>(b->off_partials), b->at<int32_t>(b->off_order),
                                    b->at<int64_t>(b->off_mstart), n, dout, b->bouz, b->stream));
  std::vector<double> h(2 * n);
  BCHK(b, hipMemcpyAsync(h.data(), dout, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                         b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  bool finite = true;
  for (int m = 0; m < n; m++) {
    const lbm_ctx* c = b->m[m];
    out[3 * m] = h[2 * m] / c->pl.nx;
    out[3 * m + 1] = (double)c->pl.nfluid * c->p.rho0 + h[2 * m + 1];
    out[3 * m + 2] = h[2 * m + 1];
    finite = finite && std::isfinite(out[3 * m]) && std::isfinite(out[3 * m + 1]);
  }
  return finite ? LBM_OK : b->fail(LBM_EDIVERGED, "a member's flux or mass is not finite");
}

lbm_status lbm_batch_tune(lbm_batch* b, int* chosen) {
  if (!b) return LBM_EINVAL;
  lbm_status rs = resync(b);
  if (rs != LBM_OK) return rs;
  // time each candidate shape (the work list is rebuilt for it) on launches
  // whose results land in the buffers the next step overwrites anyway
  // (state and counters unchanged)
  hipEvent_t e0, e1;
  BCHK(b, hipEventCreate(&e0));
  BCHK(b, hipEventCreate(&e1));
  float best = 1e30f;
  int pick = b->wpb;
  lbm_status s = LBM_OK;
  for (int w : kShapes) {
    b->wpb = w;
    if ((s = upload_lists(b)) != LBM_OK) break;
    const size_t ng = b->groups.size();
    for (int r = 0; r < 2 && s == LBM_OK; r++)
      for (size_t gi = 0; gi < ng && s == LBM_OK; gi++) s = launch_batch(b, gi, 0, w);
    if (s != LBM_OK) break;
    if ((s = b->hip(hipEventRecord(e0, b->stream), "hipEventRecord")) != LBM_OK) break;
    for (int r = 0; r < 5 && s == LBM_OK; r++)
      for (size_t gi = 0; gi < ng && s == LBM_OK; gi++) s = launch_batch(b, gi, 0, w);
    if (s != LBM_OK) break;
    if ((s = b->hip(hipEventRecord(e1, b->stream), "hipEventRecord")) != LBM_OK) break;
    if ((s = b->hip(hipEventSynchronize(e1), "hipEventSynchronize")) != LBM_OK) break;
    float ms = 0;
    if ((s = b->hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) != LBM_OK) break;
    if (ms < best) {
      best = ms;
      pick = w;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->wpb = pick;
  lbm_status u = upload_lists(b);
  if (s != LBM_OK) return s;
  if (u != LBM_OK) return u;
  if (chosen) *chosen = pick;
  return LBM_OK;
}

lbm_status lbm_batch_set_shape(lbm_batch* b, int waves_per_group) {
  if (!b || !(waves_per_group == 1 || waves_per_group == 2 || waves_per_group == 4 ||
              waves_per_group == 8))
    return LBM_EINVAL;
  if (waves_per_group == b->wpb) return LBM_OK;
  b->wpb = waves_per_group;
  return upload_lists(b);
}

lbm_status lbm_batch_set_group_bytes(lbm_batch* b, size_t bytes) {
  if (!b) return LBM_EINVAL;
  if (bytes == b->group_bytes) return LBM_OK;
  b->group_bytes = bytes;
  return upload_lists(b);
}

lbm_status lbm_batch_set_streams(lbm_batch* b, int nstreams) {
  if (!b || nstreams < 1 || nstreams > kMaxStreams) return LBM_EINVAL;
  b->nstreams = nstreams;
  return LBM_OK;
}

lbm_status lbm_batch_groups(const lbm_batch* b, int* ngroups) {
  if (!b || !ngroups) return LBM_EINVAL;
  *ngroups = (int)b->groups.size();
  return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
