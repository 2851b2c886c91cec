// lbm_batch.hip -- batches of channels advanced by one kernel launch per step
// and group, whose members join and leave while the others run.
//
// A batch holds contexts of one lattice, storage precision, wall kind and
// noise form (any sizes and parameters) in member slots.  Its work list
// holds, per wave, 64 lanes of one member (a 64-cell x-segment, or cells of
// several plain columns of that member), and every item carries its
// column's record so that a wave's set-up is one chain of two scalar loads
// (item, member).  Members keep their own buffers, parameters and step
// counters: a member's step number decides which of its two buffers is
// current and which stochastic-rounding bits it uses, so a channel advanced
// inside a batch is bit-identical to the same channel advanced alone.  On
// the device the batch keeps one counter, the steps taken since the batch
// was made; a member's step is its base step (written when it joined or was
// last taken up) plus that counter.
//
// Members are independent, so they need not advance in lockstep: the
// members are cut into groups whose state fits the 256 MB last-level cache,
// and each group runs a whole 64-step graph before the next group starts.  A
// group's populations then stay in that cache from one step to the next
// instead of streaming from HBM every step.  Groups are dealt round-robin to
// streams (the batch's own and ones of the batch's making, all at default
// priority) so that one group's launch tails overlap another group's work;
// the streams join before the device counter advances.
//
// Joining and leaving (continuous batching): every group owns a region of
// the item array and of the column-id array.  A member that joins goes to
// the first group with room (or a new group); a member that leaves frees its
// slot.  Only the groups that changed get their lists rebuilt (a few
// thousand items each), written into their region in place when they fit
// or into a fresh region at the end of the arrays; when the arrays run out
// every group is packed again from the start.  A changed group's graph is
// rebuilt before its next launch; the others keep theirs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "lbm_internal.h"

using lbm::MemberDesc;
using lbm::WorkItem;
using namespace lbm_host;

constexpr int kMaxStreams = 4;

struct lbm_batch {
  hipStream_t stream = nullptr;
  char* arena = nullptr;
  int Q = 0, prec = 0;
  bool bouz = false;
  int th = 0;         // every member's thermal-noise form (0: none)
  bool open = false;  // every member's x ends open (else periodic)
  bool elec = false;  // every member has electron lines (else none)
  int cap_members = 0;
  int64_t cap_items = 0, cap_cols = 0;
  // member slots (nullptr: free) and what the member table on the device
  // holds for each
  std::vector<lbm_ctx*> m;
  std::vector<int64_t> base;  // step of the member when the device counter was 0
  std::vector<double> th_amp;
  std::vector<uint64_t> th_seed;
  std::vector<std::array<double, 6>> th_fac;
  std::vector<std::array<double, 2>> ends;  // the open ends' densities (rho - rho0)
  std::vector<lbm::ElecArgs> eargs;         // the electron lines' arguments
  std::vector<int> gof;                // group of each slot (-1: free)
  std::vector<int64_t> mstart, mcount;  // each slot's entries in the order array
  struct Group {
    std::vector<int> slots;  // members, in the order they joined
    size_t bytes = 0;        // their state (both buffers)
    int64_t istart = 0, icap = 0, n = 0, nwall = 0;  // items [istart, istart + n), wall ones first
    int64_t cstart = 0, ccap = 0;                    // column ids [cstart, cstart + ccap)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool stale = true;  // lists changed since the graph was built
  };
  std::vector<Group> groups;
  int64_t ibump = 0, cbump = 0;  // first free item / column-id index
  size_t group_bytes = 0;
  int wpb = 4;     // waves (work items) per workgroup
  int64_t k = 0;   // steps since the batch was made (the device counter)
  int nstreams = 2;
  hipStream_t side[kMaxStreams - 1] = {};  // streams 1.. (stream 0 is the batch stream)
  hipEvent_t fork = nullptr, join[kMaxStreams - 1] = {};
  bool graphs_ok = true;
  int64_t repacks = 0;  // times every group was laid out again
  std::string err;
  size_t off_desc = 0, off_items = 0, off_cols = 0, off_order = 0, off_mstart = 0, off_mcount = 0,
         off_partials = 0, off_out = 0, off_bstep = 0, total = 0;

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
  int nslots() const {  // highest used slot + 1
    int n = (int)m.size();
    while (n > 0 && !m[n - 1]) n--;
    return n;
  }
};

#define BCHK(b, call)                               \
  do {                                              \
    lbm_status _s = (b)->hip((call), #call);        \
    if (_s != LBM_OK) return _s;                    \
  } while (0)

namespace {

// Default group size: with two groups in flight at a time their state (both
// buffers of every member) fills most of the 256 MB last-level cache.  Half
// storage does best with somewhat smaller groups (measured on 256 uneven
// ducts: 96 MiB 681 us/step against 719 with 128 MiB).
size_t default_group_bytes(int precision) {
  return precision == LBM_F16S ? (size_t)96 << 20 : (size_t)128 << 20;
}

size_t member_bytes(const lbm_ctx* c) { return 2 * c->pl.pop_bytes; }

// The work list of a group, in units of one workgroup (wpb items, one per
// wave; a workgroup never shares a column with another, so the partly
// covered cache lines at the ends of a column's x-lines are completed inside
// one L2):
//  * general columns (wall links or periodic wrap): as many whole columns as
//    fit in wpb waves, ceil(nxp/64) waves each; a longer column in segments
//    of 64 wpb cells (its x-lines are then padded, so segments start on
//    whole lines);
//  * plain columns of a member whose lines fit 64-bit-free addressing: runs
//    of k = floor(64 wpb / nxp) whole columns, their cells taken in order
//    and 64 to a wave (a wave may span up to three columns);
//  * unused waves of a workgroup get empty items (member -1).
// The general columns of every member of the group come first (they do more
// work), then the plain ones.  cols[] holds the column ids of each run,
// items point into it.
bool packs(const lbm_ctx* c) {
  const Plan& pl = c->pl;
  return pl.nxp >= 32 && pl.pop_bytes < ((size_t)1 << 31);
}

struct Lists {
  std::vector<WorkItem> items;
  std::vector<int32_t> cols;
  int64_t nwall = 0;
  std::vector<std::vector<int32_t>> mine;  // per member of the group: its item indices (local)
  std::vector<int32_t> order;              // each member's items contiguous (batch indices)
};

struct Builder {
  Lists* L;
  int64_t cbase0;  // index of the group's first column id in the batch's array
  int wpb;
  int used = 0;    // items in the current workgroup
  int who = -1;    // index of the member within the group
  void push(const WorkItem& w) {
    if (w.member >= 0) L->mine[who].push_back((int32_t)L->items.size());
    L->items.push_back(w);
    used = (used + 1) % wpb;
  }
  void close_group() {  // pad the current workgroup with empty items
    while (used != 0) push(WorkItem{-1, 0, 0, 0, 0, -1, 0u, 0});
  }
  // a run of columns (ids ascending) covering ncols * nxp cells
  void run(int m, const std::vector<int32_t>& ids, int nxp, int32_t wallcol, uint32_t mask) {
    const int32_t cbase = (int32_t)(cbase0 + (int64_t)L->cols.size());
    L->cols.insert(L->cols.end(), ids.begin(), ids.end());
    const int64_t cells = (int64_t)ids.size() * nxp;
    for (int64_t e0 = 0; e0 < cells; e0 += 64)
      push(WorkItem{m, cbase, (int32_t)ids.size(), (int32_t)(e0 / nxp), (int32_t)(e0 % nxp),
                    wallcol, mask, 0});
  }
};

void member_items(Builder& B, const lbm_ctx* c, int m, int pass) {
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
      const int32_t cbase = (int32_t)(B.cbase0 + (int64_t)B.L->cols.size());
      B.L->cols.push_back(cs.col);
      B.close_group();
      for (int x0 = 0; x0 < nxp; x0 += 64)
        B.push(WorkItem{m, cbase, 1, 0, x0, cs.wallcol, cs.mask, 0});
      B.close_group();
      continue;
    }
    if (B.used + wpc > wpb) B.close_group();
    B.run(m, ids, nxp, cs.wallcol, cs.mask);
  }
  B.close_group();
}

// items member_items gives a member's pass, counted without building them
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

int64_t member_items_count(const lbm_ctx* c, int wpb) {
  return member_count(c, wpb, 0) + member_count(c, wpb, 1);
}

// the most items a member needs over every workgroup shape
int64_t member_items_max(const lbm_ctx* c) {
  int64_t t = 0;
  for (int w : {1, 2, 4, 8}) t = std::max(t, member_items_count(c, w));
  return t;
}

void build_lists(const lbm_batch* b, const lbm_batch::Group& g, int64_t cbase0, Lists* L) {
  L->items.clear();
  L->cols.clear();
  L->mine.assign(g.slots.size(), {});
  Builder B{L, cbase0, b->wpb};
  for (int pass = 0; pass < 2; pass++) {
    for (size_t j = 0; j < g.slots.size(); j++) {
      B.who = (int)j;
      member_items(B, b->m[g.slots[j]], g.slots[j], pass);
    }
    if (pass == 0) L->nwall = (int64_t)L->items.size();
  }
}

lbm_status check_member(const lbm_batch* b, const lbm_ctx* c) {
  if (!c) return LBM_EINVAL;
  if (c->p.lattice != b->Q || c->p.precision != b->prec ||
      (c->p.geometry == LBM_TUBE) != b->bouz)
    return LBM_EINVAL;
  // one noise form, one kind of x ends and electron lines on all or none
  // (each member its own kT, seed, end densities and line parameters); the
  // batch kernel has no masked walls
  if (c->args.th_mode != b->th || (c->args.open != 0) != b->open || c->elec != b->elec ||
      c->pl.masked)
    return LBM_EINVAL;
  return LBM_OK;
}

void layout(lbm_batch* b) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return o;
  };
  const size_t nm = (size_t)b->cap_members, ni = (size_t)b->cap_items;
  b->off_desc = take(nm * sizeof(MemberDesc));
  b->off_items = take(ni * sizeof(WorkItem));
  b->off_cols = take((size_t)b->cap_cols * sizeof(int32_t));
  b->off_order = take(ni * sizeof(int32_t));
  b->off_mstart = take(nm * sizeof(int64_t));
  b->off_mcount = take(nm * sizeof(int64_t));
  b->off_partials = take(ni * 2 * sizeof(double));
  b->off_out = take(nm * 2 * sizeof(double));
  b->off_bstep = take(sizeof(int64_t));
  b->total = off;
}

// one step (step_off steps past the device counter) of group gi
// The group's members with electron lines, in launches of at most
// kEGroupMax: (member slots, grid) of each.
struct ELaunch {
  lbm::EGroup eg;
  dim3 grid;
};
std::vector<ELaunch> electron_launches(const lbm_batch* b, const lbm_batch::Group& g) {
  std::vector<ELaunch> out;
  if (!b->elec) return out;
  for (size_t j = 0; j < g.slots.size(); j += lbm::kEGroupMax) {
    ELaunch l{};
    int64_t most = 0;
    for (size_t t = j; t < g.slots.size() && l.eg.n < lbm::kEGroupMax; t++) {
      const lbm_ctx* c = b->m[g.slots[t]];
      l.eg.slot[l.eg.n++] = g.slots[t];
      most = std::max<int64_t>(most, c->pl.nsheet);
    }
    l.grid = dim3((unsigned)((most + 255) / 256), (unsigned)l.eg.n);
    out.push_back(l);
  }
  return out;
}

// one step (step_off steps past the device counter) of group gi: with
// electron lines their step first (the water step reads their velocity);
// water_only: the water step alone (the autotuner's timings)
lbm_status launch_batch(lbm_batch* b, size_t gi, int64_t step_off, hipStream_t st,
                        bool water_only = false) {
  const lbm_batch::Group& g = b->groups[gi];
  if (g.n == 0) return LBM_OK;
  const MemberDesc* mde = b->at<MemberDesc>(b->off_desc);
  const int64_t* bse = b->at<int64_t>(b->off_bstep);
  if (!water_only)
    for (ELaunch& l : electron_launches(b, g)) {
      void* eargs[4] = {(void*)&mde, (void*)&l.eg, (void*)&bse, (void*)&step_off};
      BCHK(b, hipLaunchKernel(lbm::batch_electron_kernel_ptr(b->Q, b->prec), l.grid, dim3(256),
                              eargs, 0, st));
    }
  const void* fn = lbm::batch_step_kernel_ptr(b->Q, b->prec, b->bouz, b->th, b->open, b->elec);
  const MemberDesc* md = b->at<MemberDesc>(b->off_desc);
  const WorkItem* items = b->at<WorkItem>(b->off_items);
  const int32_t* cols = b->at<int32_t>(b->off_cols);
  int64_t first = g.istart, nwall = g.istart + g.nwall, last = g.istart + g.n;
  const int64_t* bstep = b->at<int64_t>(b->off_bstep);
  int wpb = b->wpb;
  void* args[9] = {(void*)&md,   (void*)&items, (void*)&cols,     (void*)&first, (void*)&nwall,
                   (void*)&last, (void*)&bstep, (void*)&step_off, (void*)&wpb};
  const dim3 grid((unsigned)((last - first + wpb - 1) / wpb)), block(64 * wpb);
  BCHK(b, hipLaunchKernel(fn, grid, block, args, 0, st));
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

// the caller has synchronised the batch stream (no graph may be running)
void drop_graph(lbm_batch::Group& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
  g.stale = true;
}

void drop_graphs(lbm_batch* b) {
  for (lbm_batch::Group& g : b->groups) drop_graph(g);
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
    if (!c) continue;
    c->step += k;
    c->dstep_value = kStale;
    if (k & 1) c->cur = 1 - c->cur;
    c->checked_step = -1;
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
  d.bmom[0] = end_records(const_cast<lbm_ctx*>(c), 0);
  d.bmom[1] = end_records(const_cast<lbm_ctx*>(c), 1);
  if (c->elec) {
    d.ea = c->ea;
    d.eline[0] = c->at<double>(c->pl.off_e[0]);
    d.eline[1] = c->at<double>(c->pl.off_e[1]);
    d.uel = c->at<double>(c->pl.off_ue);
  }
  d.base_step = c->step - k;
  d.cur_base = (int32_t)((c->cur + k) & 1);  // (cur_base + k) & 1 == cur
  return d;
}

// write slot s's member-table entry for the member's current step (after
// its own queued work)
lbm_status write_desc(lbm_batch* b, int s) {
  lbm_ctx* c = b->m[s];
  // open ends: the records of the buffer the member's next step reads
  lbm_status st = c->args.open ? ensure_end_records(c) : LBM_OK;
  if (st == LBM_OK) st = sync(c);
  if (st != LBM_OK) return b->fail(st, "member stream failed");
  const MemberDesc d = describe(c, b->k);
  BCHK(b, hipMemcpyAsync(b->at<MemberDesc>(b->off_desc) + s, &d, sizeof d, hipMemcpyHostToDevice,
                         b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  b->base[s] = d.base_step;
  b->th_amp[s] = c->args.th_amp;
  b->th_seed[s] = c->args.th_seed;
  std::copy(c->args.th_fac, c->args.th_fac + 6, b->th_fac[s].begin());
  b->ends[s] = {c->args.drho_in, c->args.drho_out};
  b->eargs[s] = c->ea;
  return LBM_OK;
}

// the electron lines' parameters as the member table holds them
bool same_lines(const lbm::ElecArgs& a, const lbm::ElecArgs& e) {
  return a.nshell == e.nshell && a.rwall == e.rwall && a.swc == e.swc && a.tube == e.tube &&
         a.bz == e.bz && a.rho0 == e.rho0 && a.omega_e == e.omega_e && a.rho_e0 == e.rho_e0 &&
         a.gamma_e == e.gamma_e && a.force_e == e.force_e && a.phon == e.phon &&
         a.omega_p == e.omega_p && a.rho_p0 == e.rho_p0 && a.gamma_pc == e.gamma_pc &&
         a.gamma_ep == e.gamma_ep;
}

// A member stepped, restored or overwritten outside the batch no longer sits
// at base + k: rewrite its table entry.
lbm_status resync(lbm_batch* b) {
  for (size_t s = 0; s < b->m.size(); s++) {
    const lbm_ctx* c = b->m[s];
    if (!c) continue;
    if (c->step == b->base[s] + b->k && c->args.th_amp == b->th_amp[s] &&
        c->args.th_seed == b->th_seed[s] &&
        std::equal(b->th_fac[s].begin(), b->th_fac[s].end(), c->args.th_fac) &&
        c->args.drho_in == b->ends[s][0] && c->args.drho_out == b->ends[s][1] &&
        (!c->args.open || c->bmom_ok) &&
        (!c->elec || same_lines(c->ea, b->eargs[s])))
      continue;
    lbm_status st = write_desc(b, (int)s);
    if (st != LBM_OK) return st;
  }
  return LBM_OK;
}

// kGraphSteps steps of group gi, step j at (device counter + j); the
// counter itself is advanced once all groups have run
lbm_status build_graph(lbm_batch* b, size_t gi) {
  lbm_batch::Group& grp = b->groups[gi];
  hipGraph_t g = nullptr;
  BCHK(b, hipGraphCreate(&g, 0));
  const void* fn = lbm::batch_step_kernel_ptr(b->Q, b->prec, b->bouz, b->th, b->open, b->elec);
  const void* fe = lbm::batch_electron_kernel_ptr(b->Q, b->prec);
  const MemberDesc* md = b->at<MemberDesc>(b->off_desc);
  const WorkItem* items = b->at<WorkItem>(b->off_items);
  const int32_t* cols = b->at<int32_t>(b->off_cols);
  const int64_t* bstep = b->at<int64_t>(b->off_bstep);
  int64_t first = grp.istart, nwall = grp.istart + grp.nwall, last = grp.istart + grp.n;
  int wpb = b->wpb;
  std::vector<ELaunch> el = electron_launches(b, grp);
  hipGraphNode_t prev = nullptr;
  int64_t offs[kGraphSteps];
  for (int j = 0; j < kGraphSteps; j++) {
    offs[j] = j;
    for (ELaunch& l : el) {  // the electron lines' step before the water's
      void* eargs[4] = {(void*)&md, (void*)&l.eg, (void*)&bstep, (void*)&offs[j]};
      hipKernelNodeParams ep{};
      ep.func = const_cast<void*>(fe);
      ep.gridDim = l.grid;
      ep.blockDim = dim3(256);
      ep.kernelParams = eargs;
      hipGraphNode_t node = nullptr;
      hipError_t e = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &ep);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return b->hip(e, "hipGraphAddKernelNode");
      }
      prev = node;
    }
    void* args[9] = {(void*)&md,   (void*)&items, (void*)&cols,    (void*)&first, (void*)&nwall,
                     (void*)&last, (void*)&bstep, (void*)&offs[j], (void*)&wpb};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = dim3((unsigned)((last - first + wpb - 1) / wpb));
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
  grp.graph = g;
  grp.exec = ex;
  grp.stale = false;
  return LBM_OK;
}

// upload the order-array offsets of every slot
lbm_status upload_slot_tables(lbm_batch* b) {
  const size_t n = (size_t)b->cap_members;
  BCHK(b, hipMemcpyAsync(b->at<int64_t>(b->off_mstart), b->mstart.data(), n * sizeof(int64_t),
                         hipMemcpyHostToDevice, b->stream));
  BCHK(b, hipMemcpyAsync(b->at<int64_t>(b->off_mcount), b->mcount.data(), n * sizeof(int64_t),
                         hipMemcpyHostToDevice, b->stream));
  return LBM_OK;
}

// Lists of group gi into its regions (a fresh region at the end of the
// arrays if they outgrew theirs, with a quarter of headroom if `headroom`
// and there is room for it).  Returns LBM_ENOMEM when the arrays have no
// room left for it (the caller packs every group again).  Uploads go on the
// batch stream, after every launch queued there; the caller synchronises.
lbm_status place_group(lbm_batch* b, size_t gi, std::vector<Lists>* keep, bool headroom = true) {
  lbm_batch::Group& g = b->groups[gi];
  Lists L;
  build_lists(b, g, 0, &L);  // column ids local to the group for now
  const int64_t ni = (int64_t)L.items.size(), nc = (int64_t)L.cols.size();
  if (ni > g.icap || nc > g.ccap) {
    int64_t ic = headroom ? ni + ni / 4 + b->wpb : ni, cc = headroom ? nc + nc / 4 + 1 : nc;
    if (b->ibump + ic > b->cap_items || b->cbump + cc > b->cap_cols) {
      ic = ni;
      cc = nc;
    }
    if (b->ibump + ic > b->cap_items || b->cbump + cc > b->cap_cols) return LBM_ENOMEM;
    g.istart = b->ibump;
    g.icap = ic;
    g.cstart = b->cbump;
    g.ccap = cc;
    b->ibump += ic;
    b->cbump += cc;
  }
  for (WorkItem& w : L.items)
    if (w.member >= 0) w.cbase += (int32_t)g.cstart;
  g.n = ni;
  g.nwall = L.nwall;
  // the order array: each member's items contiguous, in the group's region
  std::vector<int32_t>& order = L.order;
  order.reserve(ni);
  for (size_t j = 0; j < g.slots.size(); j++) {
    const int s = g.slots[j];
    b->mstart[s] = g.istart + (int64_t)order.size();
    b->mcount[s] = (int64_t)L.mine[j].size();
    for (int32_t it : L.mine[j]) order.push_back((int32_t)(g.istart + it));
  }
  if (ni) {
    BCHK(b, hipMemcpyAsync(b->at<WorkItem>(b->off_items) + g.istart, L.items.data(),
                           ni * sizeof(WorkItem), hipMemcpyHostToDevice, b->stream));
    BCHK(b, hipMemcpyAsync(b->at<int32_t>(b->off_order) + g.istart, order.data(),
                           order.size() * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
  }
  if (nc)
    BCHK(b, hipMemcpyAsync(b->at<int32_t>(b->off_cols) + g.cstart, L.cols.data(),
                           nc * sizeof(int32_t), hipMemcpyHostToDevice, b->stream));
  g.stale = true;
  // the host buffers must live until the caller synchronises the batch
  // stream (moving the vectors keeps their storage)
  keep->push_back(std::move(L));
  return LBM_OK;
}

// Every group laid out again from the start of the arrays (on running out
// of room, or after the shape changed), each with a quarter of headroom for
// members to come if the arrays hold that for every group, else packed tight.
lbm_status repack(lbm_batch* b) {
  BCHK(b, hipStreamSynchronize(b->stream));
  drop_graphs(b);
  b->ibump = b->cbump = 0;
  int64_t ni = 0, nc = 0;
  for (lbm_batch::Group& g : b->groups) {
    g.icap = g.ccap = 0;
    for (int s : g.slots) {
      const int64_t i = member_items_count(b->m[s], b->wpb);
      const int64_t c = (int64_t)b->m[s]->pl.slots.size();
      ni += i;
      nc += c;
    }
  }
  const int64_t ng = (int64_t)b->groups.size();
  const bool headroom = ni + ni / 4 + ng * (b->wpb + 1) <= b->cap_items &&
                        nc + nc / 4 + ng * 2 <= b->cap_cols;
  std::vector<Lists> keep;
  for (size_t gi = 0; gi < b->groups.size(); gi++) {
    lbm_status s = place_group(b, gi, &keep, headroom);
    if (s == LBM_ENOMEM) {
      (void)hipStreamSynchronize(b->stream);
      char msg[256];
      snprintf(msg, sizeof msg,
               "the batch's work-list capacity is too small: group %zu of %zu at items %lld "
               "of %lld (%lld counted in all), column ids %lld of %lld (%lld)",
               gi, b->groups.size(), (long long)b->ibump, (long long)b->cap_items,
               (long long)ni, (long long)b->cbump, (long long)b->cap_cols, (long long)nc);
      return b->fail(LBM_ENOMEM, msg);
    }
    if (s != LBM_OK) return s;
  }
  lbm_status s = upload_slot_tables(b);
  BCHK(b, hipStreamSynchronize(b->stream));
  b->repacks++;
  return s;
}

// Groups changed: lists of those groups placed anew (everything repacked
// when the arrays run out), slot tables uploaded; synchronous.
lbm_status update_groups(lbm_batch* b, const std::vector<size_t>& changed) {
  BCHK(b, hipStreamSynchronize(b->stream));  // no launch still reads the old lists
  std::vector<Lists> keep;
  for (size_t gi : changed) {
    drop_graph(b->groups[gi]);
    lbm_status s = place_group(b, gi, &keep);
    if (s == LBM_ENOMEM) {
      BCHK(b, hipStreamSynchronize(b->stream));
      return repack(b);
    }
    if (s != LBM_OK) return s;
  }
  lbm_status s = upload_slot_tables(b);
  BCHK(b, hipStreamSynchronize(b->stream));
  return s;
}

void recompute_gof(lbm_batch* b) {
  std::fill(b->gof.begin(), b->gof.end(), -1);
  for (size_t gi = 0; gi < b->groups.size(); gi++)
    for (int s : b->groups[gi].slots) b->gof[s] = (int)gi;
}

// Members in slot order cut into consecutive groups of at most group_bytes
// of state (a larger member forms a group of its own; 0: one group).
void regroup(lbm_batch* b) {
  drop_graphs(b);
  b->groups.clear();
  for (size_t s = 0; s < b->m.size(); s++) {
    const lbm_ctx* c = b->m[s];
    if (!c) continue;
    const size_t mb = member_bytes(c);
    if (b->groups.empty() ||
        (b->group_bytes && b->groups.back().bytes + mb > b->group_bytes))
      b->groups.emplace_back();
    b->groups.back().slots.push_back((int)s);
    b->groups.back().bytes += mb;
  }
  recompute_gof(b);
}

lbm_status init_batch(lbm_batch* b, void* arena, size_t arena_bytes, void* hip_stream) {
  if (arena_bytes < b->total || b->cap_items >= ((int64_t)1 << 31) ||
      b->cap_cols >= ((int64_t)1 << 31))
    return arena_bytes < b->total ? LBM_ENOMEM : LBM_EINVAL;
  b->arena = static_cast<char*>(arena);
  b->stream = reinterpret_cast<hipStream_t>(hip_stream);
  b->m.assign(b->cap_members, nullptr);
  b->base.assign(b->cap_members, 0);
  b->th_amp.assign(b->cap_members, 0.0);
  b->th_seed.assign(b->cap_members, 0);
  b->th_fac.assign(b->cap_members, std::array<double, 6>{});
  b->ends.assign(b->cap_members, std::array<double, 2>{});
  b->eargs.assign(b->cap_members, lbm::ElecArgs{});
  b->gof.assign(b->cap_members, -1);
  b->mstart.assign(b->cap_members, 0);
  b->mcount.assign(b->cap_members, 0);
  b->group_bytes = default_group_bytes(b->prec);
  // extra streams at the default priority, and the events that order them
  bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; ok && k < kMaxStreams - 1; k++)
    ok = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) == hipSuccess;
  if (!ok) return LBM_EDEVICE;
  const int64_t zero = 0;
  BCHK(b, hipMemcpyAsync(b->at<void>(b->off_bstep), &zero, sizeof zero, hipMemcpyHostToDevice,
                         b->stream));
  lbm_status s = upload_slot_tables(b);
  if (s != LBM_OK) return s;
  BCHK(b, hipStreamSynchronize(b->stream));
  return LBM_OK;
}

// take member c into free slot s (table entry written; groups untouched)
lbm_status take_member(lbm_batch* b, int s, lbm_ctx* c) {
  b->m[s] = c;
  lbm_status st = write_desc(b, s);
  if (st != LBM_OK) b->m[s] = nullptr;
  return st;
}

// ------------------------------------------------------------ autotuner
// Settings the tuner chose, per kind of batch: lattice, storage, wall kind,
// noise form and the size bucket (log2 of the fluid cells, log2 of the
// members).  Shared by every batch of the process.
struct TuneKey {
  int Q, prec, bouz, th, open, elec, cells_log2, members_log2;
  bool operator<(const TuneKey& o) const {
    return std::tie(Q, prec, bouz, th, open, elec, cells_log2, members_log2) <
           std::tie(o.Q, o.prec, o.bouz, o.th, o.open, o.elec, o.cells_log2, o.members_log2);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, lbm_batch_tuning> g_tune;

int ilog2(int64_t v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    r++;
  }
  return r;
}

TuneKey tune_key(const lbm_batch* b) {
  int64_t cells = 0, n = 0;
  for (const lbm_ctx* c : b->m)
    if (c) {
      cells += c->pl.nfluid;
      n++;
    }
  return TuneKey{b->Q, b->prec,         b->bouz ? 1 : 0, b->th, b->open ? 1 : 0,
                 b->elec ? 1 : 0, ilog2(cells), ilog2(n)};
}

// Time `reps` steps of every group with the current shape, grouping and
// stream count, each group taking kTuneRun steps in a row as it does inside
// its graph (so that what a group keeps in the last-level cache from one of
// its steps to the next counts): launches whose results land in the buffers
// the next step overwrites anyway (state and counters unchanged).  Returns
// microseconds per step.
constexpr int kTuneRun = 8;
lbm_status time_steps(lbm_batch* b, int reps, hipEvent_t e0, hipEvent_t e1, double* us) {
  auto round = [&]() -> lbm_status {
    lbm_status s = fork_streams(b);
    if (s != LBM_OK) return s;
    for (size_t gi = 0; gi < b->groups.size(); gi++)
      for (int j = 0; j < kTuneRun; j++)
        if ((s = launch_batch(b, gi, 0, group_stream(b, gi), true)) != LBM_OK) return s;
    return join_streams(b);
  };
  lbm_status s0 = round();  // warm
  if (s0 != LBM_OK) return s0;
  BCHK(b, hipEventRecord(e0, b->stream));
  for (int r = 0; r < reps; r++) {
    lbm_status s = round();
    if (s != LBM_OK) return s;
  }
  BCHK(b, hipEventRecord(e1, b->stream));
  BCHK(b, hipEventSynchronize(e1));
  float ms = 0;
  BCHK(b, hipEventElapsedTime(&ms, e0, e1));
  *us = 1e3 * ms / (reps * kTuneRun);
  return LBM_OK;
}

lbm_status apply_setting(lbm_batch* b, int wpb, size_t gbytes, int nstreams) {
  const bool relayout = wpb != b->wpb || gbytes != b->group_bytes;
  b->wpb = wpb;
  b->group_bytes = gbytes;
  b->nstreams = nstreams;
  if (!relayout) return LBM_OK;
  BCHK(b, hipStreamSynchronize(b->stream));
  regroup(b);
  return repack(b);
}

}  // namespace

extern "C" {

lbm_status lbm_batch_member_cost(const lbm_ctx* c, int64_t* items, int64_t* columns) {
  if (!c) return LBM_EINVAL;
  if (items) *items = member_items_max(c);
  if (columns) *columns = (int64_t)c->pl.slots.size();
  return LBM_OK;
}

lbm_status lbm_batch_spec_footprint(const lbm_batch_spec* sp, size_t* bytes) {
  if (!sp || !bytes || sp->max_members < 1 || sp->max_items < 0 || sp->max_columns < 0)
    return LBM_EINVAL;
  lbm_batch tmp;
  tmp.cap_members = sp->max_members;
  tmp.cap_items = sp->max_items;
  tmp.cap_cols = sp->max_columns;
  layout(&tmp);
  *bytes = tmp.total;
  return LBM_OK;
}

lbm_status lbm_batch_create_spec(const lbm_batch_spec* sp, void* arena, size_t arena_bytes,
                                 void* hip_stream, lbm_batch** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!sp || (sp->lattice != 9 && sp->lattice != 19) || sp->precision < 0 || sp->precision > 2 ||
      sp->noise < 0 || sp->noise > 2 || (sp->open_ends != 0 && sp->open_ends != 1) ||
      (sp->electrons != 0 && sp->electrons != 1) || (sp->open_ends && sp->electrons) ||
      sp->max_members < 1 || sp->max_items < 0 || sp->max_columns < 0)
    return LBM_EINVAL;
  if (!arena || reinterpret_cast<uintptr_t>(arena) % kAlign) return LBM_EINVAL;
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ENOMEM;
  b->Q = sp->lattice;
  b->prec = sp->precision;
  b->bouz = sp->tube != 0;
  b->th = sp->noise;
  b->open = sp->open_ends != 0;
  b->elec = sp->electrons != 0;
  b->cap_members = sp->max_members;
  b->cap_items = sp->max_items;
  b->cap_cols = sp->max_columns;
  layout(b);
  lbm_status s = init_batch(b, arena, arena_bytes, hip_stream);
  if (s != LBM_OK) {
    drop_streams(b);
    delete b;
    return s;
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_footprint(lbm_ctx* const* ctxs, int n, size_t* bytes) {
  if (!bytes || !ctxs || n < 1 || !ctxs[0]) return LBM_EINVAL;
  lbm_batch_spec sp{};
  sp.max_members = n;
  lbm_batch kind;  // the members must be of one kind
  kind.Q = ctxs[0]->p.lattice;
  kind.prec = ctxs[0]->p.precision;
  kind.bouz = ctxs[0]->p.geometry == LBM_TUBE;
  kind.th = ctxs[0]->args.th_mode;
  kind.open = ctxs[0]->args.open != 0;
  kind.elec = ctxs[0]->elec;
  for (int i = 0; i < n; i++) {
    if (!ctxs[i] || check_member(&kind, ctxs[i]) != LBM_OK) return LBM_EINVAL;
    sp.max_items += member_items_max(ctxs[i]);
    sp.max_columns += (int64_t)ctxs[i]->pl.slots.size();
  }
  return lbm_batch_spec_footprint(&sp, bytes);
}

lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int n, void* arena, size_t arena_bytes,
                            void* hip_stream, lbm_batch** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!ctxs || n < 1 || !ctxs[0]) return LBM_EINVAL;
  lbm_batch_spec sp{};
  sp.lattice = ctxs[0]->p.lattice;
  sp.precision = ctxs[0]->p.precision;
  sp.tube = ctxs[0]->p.geometry == LBM_TUBE;
  sp.noise = ctxs[0]->args.th_mode;
  sp.open_ends = ctxs[0]->args.open != 0;
  sp.electrons = ctxs[0]->elec ? 1 : 0;
  sp.max_members = n;
  for (int i = 0; i < n; i++) {
    if (!ctxs[i]) return LBM_EINVAL;
    for (int j = 0; j < i; j++)
      if (ctxs[j] == ctxs[i]) return LBM_EINVAL;
    sp.max_items += member_items_max(ctxs[i]);
    sp.max_columns += (int64_t)ctxs[i]->pl.slots.size();
  }
  lbm_batch* b = nullptr;
  lbm_status s = lbm_batch_create_spec(&sp, arena, arena_bytes, hip_stream, &b);
  if (s != LBM_OK) return s;
  for (int i = 0; i < n && s == LBM_OK; i++) {
    s = check_member(b, ctxs[i]);
    if (s == LBM_OK) s = take_member(b, i, ctxs[i]);
  }
  if (s == LBM_OK) {
    regroup(b);
    s = repack(b);
  }
  if (s != LBM_OK) {
    lbm_batch_destroy(b);
    return s;
  }
  *out = b;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  drop_graphs(b);
  drop_streams(b);
  delete b;
}

lbm_status lbm_batch_add(lbm_batch* b, lbm_ctx* c, int* slot) {
  if (!b || !c) return LBM_EINVAL;
  for (const lbm_ctx* x : b->m)
    if (x == c) return b->fail(LBM_EINVAL, "the context is a member already");
  if (check_member(b, c) != LBM_OK)
    return b->fail(LBM_EINVAL, "the context differs from the batch in lattice, precision, wall "
                               "kind, noise form, kind of x ends or electron lines, or has masked "
                               "walls");
  int s = -1;
  for (int i = 0; i < b->cap_members && s < 0; i++)
    if (!b->m[i]) s = i;
  if (s < 0) return b->fail(LBM_ENOMEM, "every member slot is taken");
  // a synchronised batch stream: the member's table entry is written for the
  // steps the batch has queued so far
  BCHK(b, hipStreamSynchronize(b->stream));
  lbm_status st = take_member(b, s, c);
  if (st != LBM_OK) return st;
  // the first group with room, else a new one
  const size_t mb = member_bytes(c);
  size_t gi = b->groups.size();
  for (size_t i = 0; i < b->groups.size(); i++)
    if (!b->group_bytes || b->groups[i].bytes + mb <= b->group_bytes) {
      gi = i;
      break;
    }
  if (gi == b->groups.size()) b->groups.emplace_back();
  b->groups[gi].slots.push_back(s);
  b->groups[gi].bytes += mb;
  b->gof[s] = (int)gi;
  st = update_groups(b, {gi});
  if (st != LBM_OK) {  // undo: the member leaves again
    std::vector<int>& v = b->groups[gi].slots;
    v.erase(std::find(v.begin(), v.end(), s));
    b->groups[gi].bytes -= mb;
    if (v.empty()) b->groups.erase(b->groups.begin() + (long)gi);
    b->m[s] = nullptr;
    recompute_gof(b);
    (void)update_groups(b, {});
    return st;
  }
  if (slot) *slot = s;
  return LBM_OK;
}

lbm_status lbm_batch_remove(lbm_batch* b, lbm_ctx* c) {
  if (!b || !c) return LBM_EINVAL;
  int s = -1;
  for (size_t i = 0; i < b->m.size(); i++)
    if (b->m[i] == c) s = (int)i;
  if (s < 0) return b->fail(LBM_EINVAL, "the context is not a member");
  BCHK(b, hipStreamSynchronize(b->stream));  // the member's last steps are done
  const size_t gi = (size_t)b->gof[s];
  lbm_batch::Group& g = b->groups[gi];
  g.slots.erase(std::find(g.slots.begin(), g.slots.end(), s));
  g.bytes -= member_bytes(c);
  b->m[s] = nullptr;
  b->mstart[s] = 0;
  b->mcount[s] = 0;
  if (g.slots.empty()) {
    drop_graph(g);
    b->groups.erase(b->groups.begin() + (long)gi);
    recompute_gof(b);
    return update_groups(b, {});
  }
  b->gof[s] = -1;
  // a group that lost members merges into another one with room for them,
  // so that members leaving do not leave many small groups (each a launch
  // of little work) behind
  for (size_t gj = 0; gj < b->groups.size(); gj++) {
    if (gj == gi || !b->group_bytes ||
        b->groups[gj].bytes + b->groups[gi].bytes > b->group_bytes)
      continue;
    lbm_batch::Group& src = b->groups[gi];
    lbm_batch::Group& dst = b->groups[gj];
    dst.slots.insert(dst.slots.end(), src.slots.begin(), src.slots.end());
    dst.bytes += src.bytes;
    drop_graph(src);
    b->groups.erase(b->groups.begin() + (long)gi);
    recompute_gof(b);
    return update_groups(b, {gj > gi ? gj - 1 : gj});
  }
  return update_groups(b, {gi});
}

lbm_status lbm_batch_size(const lbm_batch* b, int* members, int* slots) {
  if (!b) return LBM_EINVAL;
  if (members) {
    int n = 0;
    for (const lbm_ctx* c : b->m) n += c != nullptr;
    *members = n;
  }
  if (slots) *slots = b->nslots();
  return LBM_OK;
}

lbm_status lbm_batch_items(const lbm_batch* b, int64_t* nitems) {
  if (!b || !nitems) return LBM_EINVAL;
  int64_t n = 0;
  for (const lbm_batch::Group& g : b->groups) n += g.n;
  *nitems = n;
  return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch* b, int64_t nsteps) {
  if (!b || nsteps < 0) return LBM_EINVAL;
  if (nsteps == 0 || b->groups.empty()) return LBM_OK;
  for (const lbm_ctx* c : b->m)
    if (c && (c->args.th_mode != b->th || c->elec != b->elec ||
              (c->args.open != 0) != b->open)) {
      b->err = "a member's noise form, kind of x ends or electron lines changed; "
               "remove it from the batch";
      return LBM_EINVAL;
    }
  lbm_status rs = resync(b);
  if (rs != LBM_OK) return rs;
  // each group runs its kGraphSteps steps before the next group starts; the
  // device counter advances once all groups have
  while (nsteps >= kGraphSteps && b->graphs_ok) {
    bool ok = true;
    for (size_t gi = 0; gi < b->groups.size() && ok; gi++)
      if (b->groups[gi].stale || !b->groups[gi].exec) {
        BCHK(b, hipStreamSynchronize(b->stream));
        drop_graph(b->groups[gi]);
        ok = build_graph(b, gi) == LBM_OK;
      }
    if (!ok) {
      b->graphs_ok = false;  // fall back to plain launches
      (void)hipGetLastError();
      break;
    }
    lbm_status s = fork_streams(b);
    if (s != LBM_OK) return s;
    for (size_t gi = 0; gi < b->groups.size(); gi++)
      BCHK(b, hipGraphLaunch(b->groups[gi].exec, group_stream(b, gi)));
    if ((s = join_streams(b)) != LBM_OK) return s;
    s = launch_bump(b, kGraphSteps);
    if (s != LBM_OK) return s;
    advance_members(b, kGraphSteps);
    nsteps -= kGraphSteps;
  }
  while (nsteps > 0) {
    const int64_t n = b->graphs_ok ? nsteps : std::min<int64_t>(nsteps, kGraphSteps);
    lbm_status s = fork_streams(b);
    if (s != LBM_OK) return s;
    for (size_t gi = 0; gi < b->groups.size(); gi++)
      for (int64_t j = 0; j < n; j++)
        if ((s = launch_batch(b, gi, j, group_stream(b, gi))) != LBM_OK) return s;
    if ((s = join_streams(b)) != LBM_OK) return s;
    s = launch_bump(b, n);
    if (s != LBM_OK) return s;
    advance_members(b, n);
    nsteps -= n;
  }
  return LBM_OK;
}

lbm_status lbm_batch_invariants(lbm_batch* b, double* out) {
  if (!b || !out) return LBM_EINVAL;
  const int ns = b->nslots();
  if (ns == 0) return LBM_OK;
  lbm_status rs = resync(b);
  if (rs != LBM_OK) return rs;
  double* partials = b->at<double>(b->off_partials);
  for (const lbm_batch::Group& g : b->groups)
    BCHK(b, lbm::launch_batch_moments(b->Q, b->prec, b->at<MemberDesc>(b->off_desc),
                                      b->at<WorkItem>(b->off_items), b->at<int32_t>(b->off_cols),
                                      g.istart, g.n, b->at<int64_t>(b->off_bstep), partials,
                                      b->bouz, b->stream));
  double* dout = b->at<double>(b->off_out);
  BCHK(b, lbm::launch_batch_reduce(partials, b->at<int32_t>(b->off_order),
                                   b->at<int64_t>(b->off_mstart), b->at<int64_t>(b->off_mcount),
                                   ns, dout, b->stream));
  std::vector<double> h(2 * (size_t)ns);
  BCHK(b, hipMemcpyAsync(h.data(), dout, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                         b->stream));
  BCHK(b, hipStreamSynchronize(b->stream));
  bool finite = true;
  for (int s = 0; s < ns; s++) {
    const lbm_ctx* c = b->m[s];
    if (!c) {
      out[3 * s] = out[3 * s + 1] = out[3 * s + 2] = NAN;
      continue;
    }
    out[3 * s] = h[2 * s] / c->pl.nx;
    out[3 * s + 1] = (double)c->pl.nfluid * c->p.rho0 + h[2 * s + 1];
    out[3 * s + 2] = h[2 * s + 1];
    finite = finite && std::isfinite(out[3 * s]) && std::isfinite(out[3 * s + 1]);
  }
  return finite ? LBM_OK : b->fail(LBM_EDIVERGED, "a member's flux or mass is not finite");
}

lbm_status lbm_batch_tune(lbm_batch* b, int flags, lbm_batch_tuning* chosen) {
  if (!b) return LBM_EINVAL;
  if (b->groups.empty()) return b->fail(LBM_ESTATE, "the batch has no members");
  lbm_status rs = resync(b);
  if (rs != LBM_OK) return rs;
  const TuneKey key = tune_key(b);
  if (!(flags & LBM_TUNE_RETIME)) {
    lbm_batch_tuning t{};
    bool hit = false;
    {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        t = it->second;
        hit = true;
      }
    }
    if (hit) {
      lbm_status s = apply_setting(b, t.waves_per_group, t.group_bytes, t.streams);
      if (s != LBM_OK) return s;
      t.cached = 1;
      if (chosen) *chosen = t;
      return LBM_OK;
    }
  }
  // the search: waves per workgroup x group size x streams; every
  // candidate's work list is built and timed on this batch
  hipEvent_t e0, e1;
  BCHK(b, hipEventCreate(&e0));
  BCHK(b, hipEventCreate(&e1));
  const size_t dflt = default_group_bytes(b->prec);
  const int shapes[3] = {2, 4, 8};
  const size_t gsizes[4] = {(size_t)64 << 20, (size_t)96 << 20, (size_t)128 << 20,
                            (size_t)192 << 20};
  const int nst[3] = {1, 2, 3};
  double best = 1e300, at_default = 0;
  lbm_batch_tuning pick{b->wpb, b->group_bytes, b->nstreams, 0, 0, 0, 0};
  lbm_status s = LBM_OK;
  for (int w : shapes) {
    for (size_t gb : gsizes) {
      for (int ns : nst) {
        if ((s = apply_setting(b, w, gb, ns)) != LBM_OK) break;
        double us = 0;
        if ((s = time_steps(b, 2, e0, e1, &us)) != LBM_OK) break;
        if (w == 4 && gb == dflt && ns == 2) at_default = us;
        if (us < best) {
          best = us;
          pick = lbm_batch_tuning{w, gb, ns, us, 0, 0, 0};
        }
      }
      if (s != LBM_OK) break;
    }
    if (s != LBM_OK) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (s != LBM_OK) return s;
  // the default setting stays unless another is faster by more than 1 %
  // (the spread of repeated timings of one setting)
  if (at_default > 0 && best > 0.99 * at_default)
    pick = lbm_batch_tuning{4, dflt, 2, at_default, 0, 0, 0};
  pick.us_per_step_default = at_default;
  if ((s = apply_setting(b, pick.waves_per_group, pick.group_bytes, pick.streams)) != LBM_OK)
    return s;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[key] = pick;
  }
  if (chosen) *chosen = pick;
  return LBM_OK;
}

lbm_status lbm_batch_set_shape(lbm_batch* b, int waves_per_group) {
  if (!b || !(waves_per_group == 1 || waves_per_group == 2 || waves_per_group == 4 ||
              waves_per_group == 8))
    return LBM_EINVAL;
  if (waves_per_group == b->wpb) return LBM_OK;
  return apply_setting(b, waves_per_group, b->group_bytes, b->nstreams);
}

lbm_status lbm_batch_set_group_bytes(lbm_batch* b, size_t bytes) {
  if (!b) return LBM_EINVAL;
  if (bytes == b->group_bytes) return LBM_OK;
  return apply_setting(b, b->wpb, bytes, b->nstreams);
}

lbm_status lbm_batch_groups(const lbm_batch* b, int* ngroups) {
  if (!b || !ngroups) return LBM_EINVAL;
  *ngroups = (int)b->groups.size();
  return LBM_OK;
}

lbm_status lbm_batch_set_streams(lbm_batch* b, int nstreams) {
  if (!b || nstreams < 1 || nstreams > kMaxStreams) return LBM_EINVAL;
  b->nstreams = nstreams;
  return LBM_OK;
}

lbm_status lbm_batch_settings(const lbm_batch* b, lbm_batch_tuning* now) {
  if (!b || !now) return LBM_EINVAL;
  *now = lbm_batch_tuning{b->wpb, b->group_bytes, b->nstreams, 0, 0, 0, b->repacks};
  return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
