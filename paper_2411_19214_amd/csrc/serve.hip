// Serving: continuous batching of many independent markets on one device.
//
// A scheduler thread owns every device-side action of the server. Requests
// wait in a queue and are admitted smallest first (by log2(N M), less their
// waiting time over an aging constant) while the footprint fits the arena
// (one device slab with a first-fit allocator), a control-block slot is free
// and the lane of the request's size class holds fewer reduction workgroups
// than a fill target: a lane that already fills the chip gains nothing from
// another market but would share its time with it. Admission packs the market
// on its lane's stream. Each lane runs rounds: a round is `chunk` sweeps over all markets
// resident on the lane, each sweep being four grouped launches (row pass, row
// combine with the exact fallback and each market's convergence check, column
// pass, column combine) whose grids concatenate the markets' single-market
// grids, followed by one copy of the
// control blocks to the host. After a round the scheduler retires the markets
// whose device loop has stopped (copying a, b and the residual history out)
// and lets newly admitted markets join. Lanes run concurrently, so small
// markets are not held to the pace of large ones.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>

#include "handle.h"

using namespace ipfp;

namespace {

constexpr int kMaxLanes = 4;

// First-fit allocator over [0, cap) with coalescing; 256-byte granules.
class Arena {
 public:
  void init(size_t cap) {
    cap_ = cap;
    free_.clear();
    free_[0] = cap;
    used_ = peak_ = 0;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes, 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, start = it->first + bytes;
      free_.erase(it);
      if (rest) free_[start] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes, 256);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t cap() const { return cap_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  std::map<size_t, size_t> free_;   // offset -> length
  size_t cap_ = 0, used_ = 0, peak_ = 0;
};

// kAdmitting: taken off the queue by the scheduler, being placed.
enum ReqState { kQueued = 0, kAdmitting = 1, kRunning = 2, kRetiring = 3, kFinished = 4 };

struct Req {
  uint64_t ticket = 0;
  ipfp_market mk{};
  ipfp_options opt{};
  ipfp_result* res = nullptr;
  size_t bytes = 0;
  int64_t blocks = 0;       // workgroups of its row pass
  int lane_hint = 0;        // lane of its size class
  int state = kQueued;      // guarded by the server mutex
  int code = IPFP_OK;
  int lane = -1;
  double t_submit = 0, t_admit = 0, t_done = 0;
  std::atomic<bool> cancel{false};
  // scheduler-thread state
  ipfp_handle* h = nullptr;
  size_t off = 0;
  int slot = -1;
  hipEvent_t ready = nullptr;   // inputs complete on the submitter's stream
  hipEvent_t fin = nullptr;
  Ctl last{};               // control block as last read

  ~Req() {
    if (ready) (void)hipEventDestroy(ready);
    if (fin) (void)hipEventDestroy(fin);
  }
};

// Host-side description of one grouped pass launch (markets sharing kpad).
struct PassKey {
  int64_t kpad;
  int cnt = 0;
  int idx_off = 0;          // into the idx arrays
  int first_off = 0;        // into the pass-first arrays
  int row_total = 0, col_total = 0;
};

struct Lane {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  bool dirty = true;
  std::vector<Req*> active, joining;
  // grouped-launch table: pinned staging and its device copy
  char* htab = nullptr;
  char* dtab = nullptr;
  size_t tab_cap = 0;
  Ctl* hctl = nullptr;      // pinned mirror of the control-block pool
  // device addresses inside dtab of the current table
  const GroupHalf *row = nullptr, *col = nullptr;
  const int32_t *row_idx = nullptr, *col_idx = nullptr;
  const int32_t *row_pf = nullptr, *col_pf = nullptr;
  const int32_t *row_cf = nullptr, *col_cf = nullptr;
  int row_ctot = 0, col_ctot = 0;
  std::vector<PassKey> keys;
  int64_t blocks = 0;       // row-pass workgroups of active + joining markets
};

}  // namespace

struct ipfp_server {
  ipfp_ctx* ctx = nullptr;
  ipfp_server_options opt{};
  double bounds[kMaxLanes - 1] = {0, 0, 0};
  // device resources
  char* slab = nullptr;
  Ctl* ctl_pool = nullptr;
  double* hist_stage = nullptr;   // pinned, max_active x kHistCap
  Arena arena;
  std::vector<int> free_slots;
  Lane lanes[kMaxLanes];
  std::vector<Req*> retiring;
  // shared with the API threads
  std::mutex mu;
  std::condition_variable cv;        // wakes the scheduler
  std::condition_variable done_cv;   // wakes waiters
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  ipfp_server_stats stats{};
  std::thread th;
  int resident = 0;                  // scheduler thread only
};

namespace {

// Offsets of the grouped-launch table of `count` markets with `nk` distinct
// kpads: two GroupHalf arrays, then int32 arrays -- pass market indices (row,
// column), pass block starts (count + nk each), combine block starts (count +
// 1 each).
struct TableLayout {
  size_t row, col, ridx, cidx, rpf, cpf, rcf, ccf, total;
};

TableLayout table_layout(int count, int nk) {
  TableLayout t;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = align_up(off, 256);
    const size_t o = off;
    off += bytes;
    return o;
  };
  t.row = take(sizeof(GroupHalf) * count);
  t.col = take(sizeof(GroupHalf) * count);
  t.ridx = take(sizeof(int32_t) * count);
  t.cidx = take(sizeof(int32_t) * count);
  t.rpf = take(sizeof(int32_t) * (count + nk));
  t.cpf = take(sizeof(int32_t) * (count + nk));
  t.rcf = take(sizeof(int32_t) * (count + 1));
  t.ccf = take(sizeof(int32_t) * (count + 1));
  t.total = align_up(off, 256);
  return t;
}

int lane_for(const ipfp_server* srv, int64_t N, int64_t M) {
  const double pairs = (double)N * (double)M;
  for (int k = 0; k + 1 < srv->opt.lanes; ++k)
    if (pairs <= srv->bounds[k]) return k;
  return srv->opt.lanes - 1;
}

GroupHalf half_of(const ipfp_handle* h, bool row) {
  return fused_half(row ? h->rowp : h->colp, h->ctl, row ? h->u2 : h->v, row ? 1 : 0, h->hist,
                    handle_sweep_params(h));
}

int64_t pass_blocks(const FusedPass& fp) {
  int64_t blocks = 0;
  int tps = 0;
  fused_pass_grid(fp, &blocks, &tps);
  return blocks;
}

// Lays the lane's grouped-launch table out in its pinned staging buffer and
// copies it to the device (the lane is idle, so the previous copy is done).
hipError_t build_table(Lane& L) {
  const int count = (int)L.active.size();
  // distinct kpads, in first-seen order
  L.keys.clear();
  std::vector<int> key_of(count);
  for (int j = 0; j < count; ++j) {
    const int64_t kp = L.active[j]->h->kpad;
    int k = 0;
    while (k < (int)L.keys.size() && L.keys[k].kpad != kp) ++k;
    if (k == (int)L.keys.size()) {
      PassKey pk;
      pk.kpad = kp;
      L.keys.push_back(pk);
    }
    key_of[j] = k;
    L.keys[k].cnt += 1;
  }
  const int nk = (int)L.keys.size();
  const TableLayout t = table_layout(count, nk);
  if (t.total > L.tab_cap) {
    if (L.htab) (void)hipHostFree(L.htab);
    if (L.dtab) (void)hipFree(L.dtab);
    L.htab = L.dtab = nullptr;
    L.tab_cap = 0;
    const int grow = std::max(2 * count, 32);
    const size_t cap = table_layout(grow, grow).total;
    hipError_t e = hipHostMalloc((void**)&L.htab, cap, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    e = hipMalloc((void**)&L.dtab, cap);
    if (e != hipSuccess) return e;
    L.tab_cap = cap;
  }
  const size_t o_row = t.row, o_col = t.col, o_ridx = t.ridx, o_cidx = t.cidx,
               o_rpf = t.rpf, o_cpf = t.cpf, o_rcf = t.rcf, o_ccf = t.ccf, used = t.total;

  GroupHalf* row = (GroupHalf*)(L.htab + o_row);
  GroupHalf* col = (GroupHalf*)(L.htab + o_col);
  int32_t* ridx = (int32_t*)(L.htab + o_ridx);
  int32_t* cidx = (int32_t*)(L.htab + o_cidx);
  int32_t* rpf = (int32_t*)(L.htab + o_rpf);
  int32_t* cpf = (int32_t*)(L.htab + o_cpf);
  int32_t* rcf = (int32_t*)(L.htab + o_rcf);
  int32_t* ccf = (int32_t*)(L.htab + o_ccf);

  int io = 0, fo = 0;
  for (int k = 0; k < nk; ++k) {
    L.keys[k].idx_off = io;
    L.keys[k].first_off = fo;
    io += L.keys[k].cnt;
    fo += L.keys[k].cnt + 1;
    L.keys[k].cnt = 0;   // refilled below
  }
  int rc_acc = 0, cc_acc = 0;
  for (int j = 0; j < count; ++j) {
    const ipfp_handle* h = L.active[j]->h;
    row[j] = half_of(h, true);
    col[j] = half_of(h, false);
    PassKey& pk = L.keys[key_of[j]];
    ridx[pk.idx_off + pk.cnt] = j;
    cidx[pk.idx_off + pk.cnt] = j;
    rpf[pk.first_off + pk.cnt] = pk.row_total;
    cpf[pk.first_off + pk.cnt] = pk.col_total;
    pk.row_total += (int)pass_blocks(h->rowp);
    pk.col_total += (int)pass_blocks(h->colp);
    pk.cnt += 1;
    rcf[j] = rc_acc;
    ccf[j] = cc_acc;
    rc_acc += h->row_combine_blocks;
    cc_acc += h->col_combine_blocks;
  }
  for (int k = 0; k < nk; ++k) {
    rpf[L.keys[k].first_off + L.keys[k].cnt] = L.keys[k].row_total;
    cpf[L.keys[k].first_off + L.keys[k].cnt] = L.keys[k].col_total;
  }
  rcf[count] = rc_acc;
  ccf[count] = cc_acc;
  L.row_ctot = rc_acc;
  L.col_ctot = cc_acc;
  L.row = (const GroupHalf*)(L.dtab + o_row);
  L.col = (const GroupHalf*)(L.dtab + o_col);
  L.row_idx = (const int32_t*)(L.dtab + o_ridx);
  L.col_idx = (const int32_t*)(L.dtab + o_cidx);
  L.row_pf = (const int32_t*)(L.dtab + o_rpf);
  L.col_pf = (const int32_t*)(L.dtab + o_cpf);
  L.row_cf = (const int32_t*)(L.dtab + o_rcf);
  L.col_cf = (const int32_t*)(L.dtab + o_ccf);
  return hipMemcpyAsync(L.dtab, L.htab, used, hipMemcpyHostToDevice, L.s);
}

#define TRY(expr)                    \
  do {                               \
    hipError_t e_ = (expr);          \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// One sweep of every market on the lane.
hipError_t enqueue_group_unit(ipfp_server* srv, Lane& L) {
  const int count = (int)L.active.size();
  const ipfp_dtype cd = srv->opt.compute;
  auto tr = [&](int64_t kpad) {
    return srv->opt.tile_rows > 0 ? srv->opt.tile_rows : fused_default_tile_rows(kpad, cd);
  };
  for (const PassKey& k : L.keys)
    TRY(launch_group_pass(L.row, L.row_idx + k.idx_off, L.row_pf + k.first_off, k.cnt,
                          k.row_total, k.kpad, cd, tr(k.kpad), L.s));
  TRY(launch_group_combine(L.row, L.row_cf, count, L.row_ctot, cd, L.s));
  for (const PassKey& k : L.keys)
    TRY(launch_group_pass(L.col, L.col_idx + k.idx_off, L.col_pf + k.first_off, k.cnt,
                          k.col_total, k.kpad, cd, tr(k.kpad), L.s));
  return launch_group_combine(L.col, L.col_cf, count, L.col_ctot, cd, L.s);
}

hipError_t start_round(ipfp_server* srv, Lane& L) {
  if (!L.joining.empty()) {
    L.active.insert(L.active.end(), L.joining.begin(), L.joining.end());
    L.joining.clear();
    L.dirty = true;
  }
  if (L.active.empty()) return hipSuccess;
  if (L.dirty) {
    TRY(build_table(L));
    L.dirty = false;
  }
  for (int k = 0; k < srv->opt.chunk; ++k) TRY(enqueue_group_unit(srv, L));
  TRY(hipMemcpyAsync(L.hctl, srv->ctl_pool, sizeof(Ctl) * srv->opt.max_active,
                     hipMemcpyDeviceToHost, L.s));
  TRY(hipEventRecord(L.ev, L.s));
  L.busy = true;
  std::lock_guard<std::mutex> g(srv->mu);
  srv->stats.rounds += 1;
  return hipSuccess;
}

int final_code(const Req* r) {
  if (r->cancel.load()) return IPFP_ECANCELLED;
  const Ctl& c = r->last;
  if (c.bad_margin) return IPFP_EINVAL;
  if (c.nonfinite) return IPFP_ENONFINITE;
  if (r->opt.tol > 0.0 && !(c.last_res < r->opt.tol)) return IPFP_NOT_CONVERGED;
  return IPFP_OK;
}

void release_req(ipfp_server* srv, Req* r) {
  if (r->h) {
    srv->arena.release(r->off, r->bytes);
    delete r->h;   // arena memory: the handle frees nothing on the device
    r->h = nullptr;
  }
  if (r->slot >= 0) {
    srv->free_slots.push_back(r->slot);
    r->slot = -1;
    srv->resident -= 1;
  }
  if (r->fin) {
    (void)hipEventDestroy(r->fin);
    r->fin = nullptr;
  }
  if (r->ready) {
    (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
  }
}

void mark_finished(ipfp_server* srv, Req* r, int code) {
  std::lock_guard<std::mutex> g(srv->mu);
  srv->stats.arena_used = srv->arena.used();
  r->code = code;
  r->state = kFinished;
  r->t_done = now_ms();
  srv->stats.finished += 1;
  if (r->lane >= 0) srv->stats.active -= 1;
  if (code == IPFP_OK || code == IPFP_NOT_CONVERGED) {
    const double sweeps = r->res ? r->res->sweeps : 0;
    srv->stats.pair_evals += 2.0 * (double)r->mk.N * (double)r->mk.M * sweeps;
  }
  srv->done_cv.notify_all();
}

// The market's device loop has stopped (or it was cancelled): enqueue the
// output copies on its lane and wait for them before releasing its memory.
void retire(ipfp_server* srv, Lane& L, Req* r) {
  L.blocks -= r->blocks;
  const Ctl& c = r->last;
  const int code = final_code(r);
  const ipfp_handle* h = r->h;
  hipError_t e = hipSuccess;
  if (code != IPFP_ECANCELLED) {
    const int state = c.done ? c.stop_sweep : c.sweep;
    const double* u = h->u2 + (int64_t)(state & 1) * h->N;
    ipfp_result* res = r->res;
    e = hipMemcpyAsync(res->a, u, h->N * sizeof(double), hipMemcpyDeviceToDevice, L.s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(res->b, h->v, h->M * sizeof(double), hipMemcpyDeviceToDevice, L.s);
    const int ncopy = std::min(std::min(c.n_checks, res->res_cap), kHistCap);
    if (e == hipSuccess && res->res_hist && ncopy > 0)
      e = hipMemcpyAsync(srv->hist_stage + (size_t)r->slot * kHistCap, h->hist,
                         ncopy * sizeof(double), hipMemcpyDeviceToHost, L.s);
    res->sweeps = state;
    res->n_res = c.n_checks;
    res->final_res = c.n_checks ? c.last_res : NAN;
    res->fixups = c.fix_total;
    res->pass_ms = 0.0;
    res->pass_launches = 0;
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&r->fin, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(r->fin, L.s);
  {
    std::lock_guard<std::mutex> g(srv->mu);
    r->code = e == hipSuccess ? code : IPFP_EHIP;
    r->state = kRetiring;
  }
  srv->retiring.push_back(r);
}

void finish_retired(ipfp_server* srv, Req* r, bool copy_failed) {
  int code;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (copy_failed) r->code = IPFP_EHIP;
    code = r->code;
  }
  if (code != IPFP_ECANCELLED && code != IPFP_EHIP && r->res) {
    ipfp_result* res = r->res;
    const int ncopy = std::min(std::min(r->last.n_checks, res->res_cap), kHistCap);
    if (res->res_hist && ncopy > 0)
      memcpy(res->res_hist, srv->hist_stage + (size_t)r->slot * kHistCap,
             ncopy * sizeof(double));
    res->setup_ms = 0.0;
    res->loop_ms = now_ms() - r->t_admit;
  }
  release_req(srv, r);
  mark_finished(srv, r, code);
}

// A launch or copy on the lane failed: its markets finish with IPFP_EHIP.
void fail_lane(ipfp_server* srv, Lane& L) {
  (void)hipStreamSynchronize(L.s);
  std::vector<Req*> all;
  all.swap(L.active);
  for (Req* r : all) {
    L.blocks -= r->blocks;
    release_req(srv, r);
    mark_finished(srv, r, IPFP_EHIP);   // r may be freed by a poller from here on
  }
  L.dirty = true;
}

void after_round(ipfp_server* srv, Lane& L) {
  std::vector<Req*> keep;
  for (Req* r : L.active) {
    r->last = L.hctl[r->slot];
    if (r->last.done || r->cancel.load()) {
      retire(srv, L, r);
      L.dirty = true;
    } else {
      keep.push_back(r);
    }
  }
  L.active.swap(keep);
}

// Places a request taken off the queue if it fits; false: it goes back.
bool admit(ipfp_server* srv, Req* r) {
  if (srv->free_slots.empty()) return false;
  size_t off = 0;
  if (!srv->arena.alloc(r->bytes, &off)) return false;
  const int slot = srv->free_slots.back();
  srv->free_slots.pop_back();
  srv->resident += 1;
  ipfp_handle* h = new ipfp_handle;
  h->ctx = srv->ctx;
  h->mk = r->mk;
  h->opt = r->opt;
  h->plain = false;
  h->N = r->mk.N;
  h->M = r->mk.M;
  h->arena = true;
  h->ext_ctl = srv->ctl_pool + slot;
  h->mem = srv->slab + off;
  h->bytes = r->bytes;
  r->h = h;
  r->off = off;
  r->slot = slot;
  const int lane = r->lane_hint;
  Lane& L = srv->lanes[lane];
  L.blocks += r->blocks;
  // the layout is carved here, on the scheduler thread: check that it fits the
  // slice sized at submission before any buffer is placed
  Carver size_only;
  handle_layout(h, size_only);
  hipError_t e = align_up(size_only.off, 256) <= r->bytes ? hipSuccess : hipErrorInvalidValue;
  if (e == hipSuccess) {
    Carver cv;
    cv.base = h->mem;
    handle_layout(h, cv);
    e = hipStreamWaitEvent(L.s, r->ready, 0);
  }
  if (e == hipSuccess) e = handle_setup(h, nullptr, IPFP_F32, 0, L.s);
  {
    std::lock_guard<std::mutex> g(srv->mu);
    r->lane = lane;
    r->t_admit = now_ms();
    r->state = kRunning;
    srv->stats.admitted += 1;
    srv->stats.active += 1;
    srv->stats.arena_used = srv->arena.used();
    srv->stats.arena_peak = srv->arena.peak();
  }
  if (e != hipSuccess) {
    // nothing of this market is in flight beyond what failed to enqueue:
    // wait for the lane before handing the memory back
    (void)hipStreamSynchronize(L.s);
    L.blocks -= r->blocks;
    release_req(srv, r);
    mark_finished(srv, r, IPFP_EHIP);
    return true;
  }
  L.joining.push_back(r);
  return true;
}

void scheduler(ipfp_server* srv) {
  (void)hipSetDevice(srv->ctx->device);
  for (;;) {
    bool progress = false;
    // rounds that have completed
    for (int k = 0; k < srv->opt.lanes; ++k) {
      Lane& L = srv->lanes[k];
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.ev);
      if (q == hipErrorNotReady) continue;
      L.busy = false;
      progress = true;
      if (q != hipSuccess) {
        fail_lane(srv, L);
        continue;
      }
      after_round(srv, L);
    }
    // retired markets whose output copies are done
    for (size_t i = 0; i < srv->retiring.size();) {
      Req* r = srv->retiring[i];
      const hipError_t q = r->fin ? hipEventQuery(r->fin) : hipSuccess;
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      srv->retiring[i] = srv->retiring.back();
      srv->retiring.pop_back();
      finish_retired(srv, r, q != hipSuccess);
      progress = true;
    }
    // admission: smallest aged size first, among requests whose lane has room
    for (;;) {
      Req* head = nullptr;
      {
        std::lock_guard<std::mutex> g(srv->mu);
        const double now = now_ms();
        double best = INFINITY;
        size_t at = 0;
        for (size_t q = 0; q < srv->queue.size(); ++q) {
          Req* r = srv->queue[q];
          const Lane& L = srv->lanes[r->lane_hint];
          if (L.blocks > 0 && L.blocks + r->blocks > srv->opt.lane_blocks) continue;
          const double key = log2((double)r->mk.N * (double)r->mk.M) -
                             (now - r->t_submit) / srv->opt.aging_ms;
          if (key < best) {
            best = key;
            head = r;
            at = q;
          }
        }
        if (head) {
          srv->queue.erase(srv->queue.begin() + at);
          head->state = kAdmitting;
          srv->stats.queued -= 1;
        }
      }
      if (!head) break;
      if (admit(srv, head)) {
        progress = true;
        continue;
      }
      std::lock_guard<std::mutex> g(srv->mu);
      if (head->cancel.load()) {          // cancelled while being placed
        head->state = kFinished;
        head->code = IPFP_ECANCELLED;
        head->t_done = now_ms();
        srv->stats.finished += 1;
        srv->done_cv.notify_all();
        continue;
      }
      head->state = kQueued;      // waits for memory or a slot
      srv->stats.queued += 1;
      srv->queue.push_back(head);
      break;
    }
    // new rounds on idle lanes
    bool any_work = !srv->retiring.empty();
    for (int k = 0; k < srv->opt.lanes; ++k) {
      Lane& L = srv->lanes[k];
      if (!L.busy && (!L.active.empty() || !L.joining.empty())) {
        const hipError_t e = start_round(srv, L);
        progress = true;
        if (e != hipSuccess) fail_lane(srv, L);
      }
      any_work = any_work || L.busy || !L.active.empty() || !L.joining.empty();
    }
    std::unique_lock<std::mutex> g(srv->mu);
    if (srv->stop) {
      // cancel everything still queued; running markets stop at round end
      for (Req* r : srv->queue) {
        r->state = kFinished;
        r->code = IPFP_ECANCELLED;
        r->t_done = now_ms();
        srv->stats.queued -= 1;
        srv->stats.finished += 1;
      }
      srv->queue.clear();
      srv->done_cv.notify_all();
      if (!any_work && srv->resident == 0) break;
    }
    if (!progress) {
      const bool idle = !any_work && srv->queue.empty();
      if (idle)
        srv->cv.wait_for(g, std::chrono::milliseconds(50));
      else
        srv->cv.wait_for(g, std::chrono::microseconds(50));
    }
  }
  srv->done_cv.notify_all();
}

void fill_info(const Req* r, ipfp_request_info* info) {
  if (!info) return;
  info->state = r->state == kQueued ? IPFP_REQ_QUEUED
                : r->state == kFinished ? IPFP_REQ_FINISHED
                                        : IPFP_REQ_RUNNING;
  info->code = r->state == kFinished ? r->code : IPFP_EBUSY;
  info->lane = r->lane;
  info->t_submit = r->t_submit;
  info->t_admit = r->t_admit;
  info->t_done = r->t_done;
}

void free_server(ipfp_server* srv) {
  for (int k = 0; k < kMaxLanes; ++k) {
    Lane& L = srv->lanes[k];
    if (L.s) (void)hipStreamSynchronize(L.s);
    if (L.ev) (void)hipEventDestroy(L.ev);
    if (L.s) (void)hipStreamDestroy(L.s);
    if (L.htab) (void)hipHostFree(L.htab);
    if (L.dtab) (void)hipFree(L.dtab);
    if (L.hctl) (void)hipHostFree(L.hctl);
  }
  if (srv->hist_stage) (void)hipHostFree(srv->hist_stage);
  if (srv->ctl_pool) (void)hipFree(srv->ctl_pool);
  if (srv->slab) (void)hipFree(srv->slab);
  if (srv->ctx) ctx_release(srv->ctx, srv->arena.cap());
  for (auto& kv : srv->reqs) delete kv.second;
  delete srv;
}

}  // namespace

extern "C" {

double ipfp_clock_ms(void) { return now_ms(); }

void ipfp_default_server_options(ipfp_server_options* opt) {
  memset(opt, 0, sizeof(*opt));
  opt->arena_bytes = (size_t)1 << 30;
  opt->max_active = 256;
  opt->lanes = 3;
  opt->chunk = 4;
  opt->compute = IPFP_BF16;
  opt->tile_rows = 0;
  opt->lane_blocks = 2048;
  opt->aging_ms = 4000.0;
}

int ipfp_server_create(ipfp_ctx* ctx, const ipfp_server_options* opt, ipfp_server** out) {
  if (!ctx || !out) return IPFP_EINVAL;
  *out = nullptr;
  ipfp_server_options o;
  ipfp_default_server_options(&o);
  if (opt) {
    if (opt->arena_bytes) o.arena_bytes = opt->arena_bytes;
    if (opt->max_active) o.max_active = opt->max_active;
    if (opt->lanes) o.lanes = opt->lanes;
    if (opt->chunk) o.chunk = opt->chunk;
    o.compute = opt->compute;
    o.tile_rows = opt->tile_rows;
    for (int k = 0; k < 3; ++k) o.lane_pairs[k] = opt->lane_pairs[k];
    if (opt->lane_blocks) o.lane_blocks = opt->lane_blocks;
    if (opt->aging_ms != 0.0) o.aging_ms = opt->aging_ms;
  }
  if (o.max_active < 1 || o.max_active > 1024 || o.lanes < 1 || o.lanes > kMaxLanes ||
      o.chunk < 1 || o.chunk > 64)
    return IPFP_EINVAL;
  if (o.compute != IPFP_BF16 && o.compute != IPFP_FP8E4M3) return IPFP_EINVAL;
  if (o.lane_blocks < 1 || !(o.aging_ms > 0.0)) return IPFP_EINVAL;
  if (o.tile_rows != 0 && o.tile_rows != 128 && o.tile_rows != 256 && o.tile_rows != 512)
    return IPFP_EINVAL;
  ipfp_server* srv = new ipfp_server;
  srv->opt = o;
  for (int k = 0; k + 1 < o.lanes; ++k) {
    double b = o.lane_pairs[k];
    if (!(b > 0.0)) b = exp2(20.0 + 16.0 * (k + 1) / o.lanes);
    if (k > 0 && !(b > srv->bounds[k - 1])) {
      delete srv;
      return IPFP_EINVAL;
    }
    srv->bounds[k] = b;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) {
    delete srv;
    return IPFP_EHIP;
  }
  const size_t cap = align_up(o.arena_bytes, 256);
  int rc = ctx_reserve(ctx, cap);
  if (rc != IPFP_OK) {
    delete srv;
    return rc;
  }
  srv->ctx = ctx;
  srv->arena.init(cap);
  bool ok = hipMalloc((void**)&srv->slab, cap) == hipSuccess;
  ok = ok && hipMalloc((void**)&srv->ctl_pool, sizeof(Ctl) * o.max_active) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&srv->hist_stage,
                           sizeof(double) * kHistCap * o.max_active,
                           hipHostMallocDefault) == hipSuccess;
  for (int k = 0; ok && k < o.lanes; ++k) {
    Lane& L = srv->lanes[k];
    ok = hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) == hipSuccess &&
         hipHostMalloc((void**)&L.hctl, sizeof(Ctl) * o.max_active,
                       hipHostMallocDefault) == hipSuccess;
  }
  if (!ok) {
    free_server(srv);
    return IPFP_EHIP;
  }
  for (int k = o.max_active - 1; k >= 0; --k) srv->free_slots.push_back(k);
  srv->stats.arena_bytes = cap;
  srv->th = std::thread(scheduler, srv);
  *out = srv;
  return IPFP_OK;
}

void ipfp_server_destroy(ipfp_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    for (auto& kv : srv->reqs) kv.second->cancel.store(true);
  }
  srv->cv.notify_all();
  if (srv->th.joinable()) srv->th.join();
  free_server(srv);
}

int ipfp_submit(ipfp_server* srv, const ipfp_market* mk, const ipfp_options* opt,
                ipfp_result* res, uint64_t* ticket, void* stream) {
  if (!srv || !mk || !opt || !res || !res->a || !res->b || !ticket) return IPFP_EINVAL;
  ipfp_options o = *opt;
  if (o.path != IPFP_PATH_FUSED || o.compute != srv->opt.compute) return IPFP_EINVAL;
  if (o.tile_rows == 0) o.tile_rows = srv->opt.tile_rows;
  if (o.tile_rows != srv->opt.tile_rows) return IPFP_EINVAL;
  o.use_graph = 0;
  o.time_passes = 0;
  int rc = validate_market(mk, &o, true);
  if (rc != IPFP_OK) return rc;
  // the layout's split counts depend on the current device's compute units and
  // occupancy: size it with the server's device current, as admission will
  if (hipSetDevice(srv->ctx->device) != hipSuccess) return IPFP_EHIP;
  size_t bytes = 0;
  rc = ipfp_footprint(mk, &o, &bytes);
  if (rc != IPFP_OK) return rc;
  if (bytes > srv->arena.cap()) return IPFP_EBUDGET;
  const int64_t kpad = fused_kpad(mk->d, o.compute);
  const int tr = o.tile_rows > 0 ? o.tile_rows : fused_default_tile_rows(kpad, o.compute);
  const int rx = fused_rows_per_wg(kpad, o.compute, tr);
  const int sx = o.splits > 0 ? o.splits : fused_pass_splits(mk->N, mk->M, kpad, o.compute, tr);
  hipEvent_t ready = nullptr;
  if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess) return IPFP_EHIP;
  if (hipEventRecord(ready, (hipStream_t)stream) != hipSuccess) {
    (void)hipEventDestroy(ready);
    return IPFP_EHIP;
  }
  Req* r = new Req;
  r->ready = ready;
  r->mk = *mk;
  r->opt = o;
  r->res = res;
  r->bytes = bytes;
  r->blocks = (mk->N + rx - 1) / rx * sx;
  r->lane_hint = lane_for(srv, mk->N, mk->M);
  r->t_submit = now_ms();
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->stop) {
      (void)hipEventDestroy(ready);
      delete r;
      return IPFP_ECANCELLED;
    }
    r->ticket = srv->next_ticket++;
    srv->reqs[r->ticket] = r;
    srv->queue.push_back(r);
    srv->stats.submitted += 1;
    srv->stats.queued += 1;
    *ticket = r->ticket;
  }
  srv->cv.notify_all();
  return IPFP_OK;
}

static int poll_locked(ipfp_server* srv, uint64_t ticket, ipfp_request_info* info) {
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return IPFP_ENOTFOUND;
  Req* r = it->second;
  fill_info(r, info);
  if (r->state != kFinished) return IPFP_EBUSY;
  const int code = r->code;
  srv->reqs.erase(it);
  delete r;
  return code;
}

int ipfp_poll(ipfp_server* srv, uint64_t ticket, ipfp_request_info* info) {
  if (!srv) return IPFP_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  return poll_locked(srv, ticket, info);
}

int ipfp_wait(ipfp_server* srv, uint64_t ticket, double timeout_ms, ipfp_request_info* info) {
  if (!srv) return IPFP_EINVAL;
  std::unique_lock<std::mutex> g(srv->mu);
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::microseconds((int64_t)(timeout_ms * 1000.0));
  for (;;) {
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return IPFP_ENOTFOUND;
    if (it->second->state == kFinished) return poll_locked(srv, ticket, info);
    if (timeout_ms < 0) {
      srv->done_cv.wait(g);
    } else if (srv->done_cv.wait_until(g, deadline) == std::cv_status::timeout) {
      return poll_locked(srv, ticket, info);
    }
  }
}

int ipfp_cancel(ipfp_server* srv, uint64_t ticket) {
  if (!srv) return IPFP_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return IPFP_ENOTFOUND;
  Req* r = it->second;
  if (r->state == kFinished) return IPFP_EINVAL;
  r->cancel.store(true);
  if (r->state == kQueued) {
    srv->queue.erase(std::find(srv->queue.begin(), srv->queue.end(), r));
    r->state = kFinished;
    r->code = IPFP_ECANCELLED;
    r->t_done = now_ms();
    srv->stats.queued -= 1;
    srv->stats.finished += 1;
    srv->done_cv.notify_all();
  }
  srv->cv.notify_all();
  return IPFP_OK;
}

int ipfp_server_get_stats(ipfp_server* srv, ipfp_server_stats* out) {
  if (!srv || !out) return IPFP_EINVAL;
  std::lock_guard<std::mutex> g(srv->mu);
  *out = srv->stats;
  return IPFP_OK;
}

}  // extern "C"
