// Continuous-batching server over a resident index.
//
// The paper's query process is online (Section 2.3); this loop keeps one
// shard's tables resident in HBM and serves a stream of queries and inserts:
//   - submit calls copy the request and append it to a FIFO (E_BUSY when the
//     FIFO is full);
//   - a scheduler thread owns staging slots (device and pinned host memory
//     for one batch each).  As soon as a slot is free it takes the longest
//     run of queries at the head of the FIFO that fits the slot (continuous
//     batching: no waiting for a full batch while the device has room),
//     runs slash_query on them (a small batch is read in place from
//     host-coherent memory, a larger one copied in first);
//   - query batches and the table-writing kernels of inserts go to one
//     device stream in FIFO order, so a query admitted in epoch e sees
//     exactly the inserts submitted before it: an insert at the head of the
//     FIFO (with the inserts queued right behind it, merged into one launch
//     while they fit its staging) writes the tables after the batches before
//     it and before the batches after it;
//   - an insert is prepared ahead, as soon as it is queued and an insert
//     slot is free (inserts in FIFO order, so ids follow submission order):
//     its rows are hashed (read in place from host-coherent staging up to
//     1 MB, else copied in first) and grouped by bucket into the slot's own
//     scratch on a second stream, beside the query batches before it, and
//     the grouping kernel's last block writes the slot's sequence number to
//     host-coherent memory.  When the insert reaches the head, the scheduler
//     sees that word (it has usually long been written) and launches the
//     table writes on the batch stream.  No event joins the two streams: a
//     cross-stream event wait costs the launching thread about 20 us per
//     insert on this runtime;
//   - a small query batch followed in the FIFO by an insert whose
//     preparation is done shares one launch with that insert: the batch's
//     queries only gather their slots (ids kept in device memory) and the
//     insert's table writers start once they have; the batch is ranked in
//     the next launch, beside the next batch's gathers, or on its own when
//     none follows soon.  So an epoch costs one launch of about a gather and
//     an insert's writes, not a whole query's ranking as well;
//   - query results are written by the query kernel straight into pinned,
//     host-coherent memory (no copy back);
//   - batch slots are allocated at start, up to max_inflight, as far as the
//     HBM budget and the device's free memory allow (a slot that did not fit
//     then is added later, while work is waiting, if memory has freed up);
//   - with max_wait_us > 0, a batch that is neither full nor followed by an
//     insert is held back until its oldest query has waited that long;
//   - finished work is detected with one event per launch, recorded into
//     one of the slots the launch finishes (polled without
//     sleeping while work is in flight; every event is recorded on the batch
//     stream, so they complete in launch order and only the oldest
//     outstanding one is polled) and turned into completions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "slash_internal.h"

using namespace slash;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Insert staging slots a server keeps at most (inserts queued on the device
// behind the one running).
constexpr size_t kInsertSlots = 8;
// Device memory a server leaves free when it adds a batch slot.
constexpr uint64_t kFreeReserve = uint64_t(1) << 30;

struct Request {
  uint64_t ticket = 0;
  uint32_t kind = 0;  // 0 query, 1 insert
  uint32_t k = 0;
  uint32_t n_rows = 0;
  std::vector<int32_t> idx;
  std::vector<int64_t> indptr;  // inserts
  double t_submit = 0;
  int32_t prep = -1;  // inserts: the insert slot preparing it
};

struct Slot {
  hipEvent_t done = nullptr;  // everything the slot launched has finished
  bool busy = false;
  uint32_t kind = 0;
  uint64_t epoch = 0;  // queries: the epoch they see; inserts: the first request's epoch
  std::vector<Request> reqs;
  // request data of one launch, packed so that it moves in one copy:
  // indptr [n + 1] (int64), k [n] (queries only), then the indices (int32)
  // from a 256-byte boundary
  char* d_in = nullptr;
  char* h_in = nullptr;  // pinned
  // query results of one launch, written by the kernel: ids [n][k_max] then
  // scores [n][k_max] (pinned, host-coherent)
  uint32_t* h_out = nullptr;
  uint32_t cap_q = 0;
  uint64_t cap_nnz = 0;
  uint32_t first_id = 0;
  // inserts: the prepared rows, their bucket ids and runs, and the
  // host-coherent word the preparation stream sets to prep_seq when done
  uint32_t rows = 0;
  size_t in_bytes = 0, idx_off = 0;
  InsertScratch sc;
  uint32_t* counter = nullptr;  // the grouping kernel's block counter (device)
  uint64_t* flag = nullptr;
  uint64_t prep_seq = 0;
  bool prep_failed = false;
  // query slots: the slot ids of a batch gathered in one launch and ranked
  // in a later one ([n][L * R], device), and the batch as packed
  uint32_t* slot_ids = nullptr;
  ServeBatch batch;
};

// One launch on the batch stream and the slots it finishes: one event,
// recorded into the first slot's.
struct Launch {
  uint32_t n = 0;
  std::pair<bool, uint32_t> slot[3];  // (insert slot?, index)
};

}  // namespace

struct slash_server {
  slash_index* ix = nullptr;
  slash_serve_config cfg{};
  slash_index_info info{};
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request> pending;
  std::deque<slash_completion> done;
  std::vector<Slot> slots;  // query batch staging
  std::vector<Slot> ins;    // insert staging
  hipStream_t stream = nullptr;  // query batches and table writes, in FIFO order
  hipStream_t prep = nullptr;    // insert preparation
  FuseSync fuse;                 // counters of query launches that also write an insert
  uint64_t prep_seq = 0;         // preparations launched
  size_t prep_scan = 0;          // FIFO entries from the head already looked at for preparation
  uint32_t cap_q = 0;
  uint64_t cap_nnz = 0, per_slot = 0;
  // launches in flight, in launch order (the scheduler thread's only)
  std::deque<Launch> inflight;
  int32_t gathered = -1;       // batch slot gathered and waiting to be ranked
  double prep_wait_since = -1.0;  // the head insert's preparation was first found unfinished
  size_t slot_ids_bytes = 0;   // per batch slot (0: batches are never split)
  uint64_t epoch = 0;
  uint64_t next_ticket = 0;
  uint64_t next_id = 0;  // id of the next inserted row
  bool stopping = false;
  bool closed = false;
  std::thread th;
  slash_serve_stats stats{};
  uint64_t hbm_used = 0;
  double grow_retry_at = 0;  // a slot that did not fit is retried after this time
  int device = 0;
  hipError_t dev_err = hipSuccess;
};

namespace {

void free_slot(Slot& s) {
  if (s.done) (void)hipEventSynchronize(s.done);
  if (s.done) (void)hipEventDestroy(s.done);
  (void)hipFree(s.d_in);
  (void)hipFree(s.sc.keys);
  (void)hipFree(s.sc.runs);
  (void)hipFree(s.slot_ids);
  (void)hipFree(s.counter);
  (void)hipHostFree(s.h_in);
  (void)hipHostFree(s.h_out);
  (void)hipHostFree(s.flag);
  s = Slot();
}

// Offsets of one launch's packed request data (see Slot::d_in).
struct InLayout {
  size_t k, idx, bytes;
};
InLayout in_layout(uint64_t n, uint64_t nnz, bool with_k) {
  InLayout l;
  l.k = (n + 1) * 8;
  l.idx = (l.k + (with_k ? n * 4 : 0) + 255) & ~(size_t)255;
  l.bytes = l.idx + nnz * 4;
  return l;
}

// Device + pinned staging for up to cap_q queries / rows and cap_nnz indices
// (query slots: plus host-coherent result memory the kernel writes; insert
// slots: plus insert scratch of keys_b + runs_b bytes and the
// host-coherent preparation word and the device counter that sets it).
bool alloc_slot(Slot& s, uint32_t cap_q, uint64_t cap_nnz, uint32_t k_max, bool with_out, size_t keys_b = 0,
                size_t runs_b = 0, size_t slot_ids_b = 0) {
  s.cap_q = cap_q;
  s.cap_nnz = cap_nnz;
  const size_t in_bytes = in_layout(cap_q, cap_nnz, with_out).bytes;
  // The slot's event only has to say that its launch has ended: what the
  // host reads then (results, the give-up word) is host-coherent memory the
  // kernels write directly, not lines held in the device's L2, and device
  // buffers are reused only by later device work.  So it is recorded without
  // the system-scope cache writeback and invalidation (1.8 us less between
  // launches on one stream, measured with 64 groups per launch).
  if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming | hipEventDisableSystemFence) != hipSuccess) return false;
  if (hipMalloc(&s.d_in, in_bytes) != hipSuccess) return false;
  // staging is host-coherent: small batches and inserts are read by the
  // kernels in place (no stale lines when the slot is reused)
  if (hipHostMalloc(&s.h_in, in_bytes, hipHostMallocCoherent) != hipSuccess) return false;
  if (with_out && hipHostMalloc(&s.h_out, (size_t)cap_q * k_max * 8, hipHostMallocCoherent) != hipSuccess)
    return false;
  if (slot_ids_b && hipMalloc(&s.slot_ids, slot_ids_b) != hipSuccess) return false;
  if (!with_out) {
    if (hipMalloc(&s.sc.keys, keys_b) != hipSuccess || hipMalloc(&s.sc.runs, runs_b) != hipSuccess) return false;
    if (hipMalloc(&s.counter, 256) != hipSuccess || hipMemset(s.counter, 0, 256) != hipSuccess) return false;
    if (hipHostMalloc(&s.flag, 64, hipHostMallocCoherent) != hipSuccess) return false;
    *(volatile uint64_t*)s.flag = 0;
    s.sc.rows = cap_q;
  }
  return true;
}


__global__ void k_touch(int64_t* p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = 0;
}

// Run each transfer the slot will make once, at full size, and one kernel,
// and wait: the runtime sets up the stream's hardware queue and copy engines
// on first use, which would otherwise stall the first requests by
// milliseconds.
bool warm_slot(hipStream_t st, Slot& s, bool with_out) {
  hipLaunchKernelGGL(k_touch, dim3(1), dim3(64), 0, st, (int64_t*)s.d_in);
  if (hipGetLastError() != hipSuccess) return false;
  const size_t in_bytes = in_layout(s.cap_q, s.cap_nnz, with_out).bytes;
  if (hipMemcpyAsync(s.d_in, s.h_in, in_bytes, hipMemcpyHostToDevice, st) != hipSuccess) return false;
  if (hipEventRecord(s.done, st) != hipSuccess) return false;
  return hipStreamSynchronize(st) == hipSuccess;
}

// Device bytes of one batch slot (its request data; results go to host memory).
uint64_t slot_bytes(uint32_t cap_q, uint64_t cap_nnz) { return in_layout(cap_q, cap_nnz, true).bytes; }

// Turn a finished slot into completions (called with the lock held); status
// is SLASH_E_DEVICE when the slot's work failed on the device.
void finish_slot(slash_server* srv, Slot& s, int32_t status) {
  const uint32_t km = srv->info.params.k_max;
  double t = now_s();
  if (s.kind == 0) {
    for (size_t q = 0; q < s.reqs.size(); ++q) {
      const Request& r = s.reqs[q];
      slash_completion c;
      memset(&c, 0, sizeof c);
      c.ticket = r.ticket;
      c.epoch = s.epoch;
      c.status = status;
      c.kind = 0;
      c.k = r.k;
      const uint32_t* oi = s.h_out + q * km;
      const uint32_t* os = s.h_out + s.reqs.size() * km + q * km;
      memcpy(c.ids, oi, r.k * 4);
      memcpy(c.scores, os, r.k * 4);
      c.t_submit_s = r.t_submit;
      c.t_done_s = t;
      srv->done.push_back(c);
    }
    srv->stats.queries_done += s.reqs.size();
  } else {
    // merged inserts: each request closes its own epoch and gets its own ids
    uint32_t first = s.first_id;
    for (size_t i = 0; i < s.reqs.size(); ++i) {
      const Request& r = s.reqs[i];
      slash_completion c;
      memset(&c, 0, sizeof c);
      c.ticket = r.ticket;
      c.epoch = s.epoch + i;
      c.status = status;
      c.kind = 1;
      c.n_ids = r.n_rows;
      c.first_id = first;
      c.t_submit_s = r.t_submit;
      c.t_done_s = t;
      srv->done.push_back(c);
      srv->stats.inserts_done += 1;
      srv->stats.rows_inserted += r.n_rows;
      first += r.n_rows;
    }
  }
  s.reqs.clear();
  s.busy = false;
}

// Request bytes up to which a query batch is read by the kernel straight
// from host-coherent memory: a copy would add a blit kernel and its launch
// gap to the ordered stream, longer than the kernel's few reads over the
// host link.
constexpr size_t kZeroCopyBytes = size_t(64) << 10;

hipError_t wait_prepared(slash_server* srv, const Slot& s);

// Pack query batch slot s's requests into its staging (lock not held) and
// set s.batch: request data read by the kernels in place (host-coherent)
// when small, else copied in on the batch stream; results to host-coherent
// memory.
hipError_t pack_queries(slash_server* srv, Slot& s) {
  const double t0 = now_s();
  const uint32_t n = (uint32_t)s.reqs.size();
  const uint32_t km = srv->info.params.k_max;
  uint64_t nnz = 0;
  for (const Request& r : s.reqs) nnz += r.idx.size();
  const InLayout l = in_layout(n, nnz, true);
  int64_t* h_ip = (int64_t*)s.h_in;
  uint32_t* h_k = (uint32_t*)(s.h_in + l.k);
  int32_t* h_ix = (int32_t*)(s.h_in + l.idx);
  uint64_t off = 0;
  h_ip[0] = 0;
  for (uint32_t q = 0; q < n; ++q) {
    const Request& r = s.reqs[q];
    memcpy(h_ix + off, r.idx.data(), r.idx.size() * 4);
    off += r.idx.size();
    h_ip[q + 1] = (int64_t)off;
    h_k[q] = r.k;
  }
  srv->stats.pack_s += now_s() - t0;
  const char* in = s.h_in;
  if (l.bytes > kZeroCopyBytes) {
    const hipError_t e = hipMemcpyAsync(s.d_in, s.h_in, l.bytes, hipMemcpyHostToDevice, srv->stream);
    if (e != hipSuccess) return e;
    in = s.d_in;
  }
  s.batch.q = slash_csr{(const int64_t*)in, (const int32_t*)(in + l.idx), n};
  s.batch.host_indptr = h_ip;
  s.batch.kq = (const uint32_t*)(in + l.k);
  s.batch.ids = s.h_out;
  s.batch.scores = s.h_out + (size_t)n * km;
  s.batch.slot_ids = s.slot_ids;
  return hipSuccess;
}

// One launch on the batch stream (lock not held): rank the gathered batch
// `agg`, answer (or, with gather_only, gather) the batch `cur`, commit the
// prepared insert `ins`; each may be null.  A serving-step kernel does all
// of it when one fits, else `cur` runs as slash_query and `ins` as its own
// commit (agg and gather_only need the step kernel).  One event, recorded
// into ev_slot's.  *fused is set when cur and ins shared the kernel.
hipError_t launch_step(slash_server* srv, Slot* agg, Slot* cur, bool gather_only, Slot* ins, Slot& ev_slot,
                       bool* fused) {
  hipStream_t st = srv->stream;
  hipError_t e;
  *fused = false;
  if (cur && (e = pack_queries(srv, *cur)) != hipSuccess) return e;
  if (ins && (e = wait_prepared(srv, *ins)) != hipSuccess) return e;
  const bool step = srv->slot_ids_bytes && (agg || gather_only || (cur && ins)) &&
                    (!cur || serve_step_ok(srv->ix, cur->reqs.size()));
  if (step) {
    const ServeBatch none;
    if (serve_step(srv->ix, agg ? agg->batch : none, cur ? cur->batch : none, gather_only, ins ? &ins->sc : nullptr,
                   ins ? ins->rows : 0, srv->fuse, st) != SLASH_OK)
      return hipErrorLaunchFailure;
    *fused = cur && ins;
  } else {
    if (agg || gather_only) return hipErrorInvalidValue;
    if (cur && slash_query(srv->ix, cur->batch.q, cur->batch.kq, 0, SLASH_FLAG_TRUSTED, cur->batch.ids,
                           cur->batch.scores, st) != SLASH_OK)
      return hipErrorLaunchFailure;
    if (ins && insert_commit(srv->ix, ins->sc, ins->rows, st) != SLASH_OK) return hipErrorLaunchFailure;
  }
  return hipEventRecord(ev_slot.done, st);
}

// Pack inserts `rs` into insert slot s's staging.  Called without the lock:
// the requests stay in the FIFO, whose other thread only appends (which
// moves no element).
void pack_inserts(Slot& s, const std::vector<const Request*>& rs) {
  uint32_t rows = 0;
  uint64_t nnz = 0;
  for (const Request* r : rs) {
    rows += r->n_rows;
    nnz += r->idx.size();
  }
  const InLayout l = in_layout(rows, nnz, false);
  int64_t* h_ip = (int64_t*)s.h_in;
  int32_t* h_ix = (int32_t*)(s.h_in + l.idx);
  uint32_t row = 0;
  uint64_t off = 0;
  h_ip[0] = 0;
  for (const Request* rp : rs) {
    const Request& r = *rp;
    for (uint32_t k = 0; k < r.n_rows; ++k) h_ip[row + k + 1] = (int64_t)off + r.indptr[k + 1];
    memcpy(h_ix + off, r.idx.data(), r.idx.size() * 4);
    off += r.idx.size();
    row += r.n_rows;
  }
  s.rows = rows;
  s.in_bytes = l.bytes;
  s.idx_off = l.idx;
}

// Rows up to which an insert is hashed straight from host-coherent staging
// (larger ones are copied in first).
constexpr size_t kZeroCopyInsertBytes = size_t(1) << 20;

// Prepare insert slot s on the preparation stream (lock not held): (copy,)
// hash, group into the slot's scratch (the ids are taken here); the grouping
// kernel's last block sets the slot's word.
hipError_t prepare_insert(slash_server* srv, Slot& s) {
  hipStream_t pst = srv->prep;
  hipError_t e;
  const char* in = s.h_in;
  if (s.in_bytes > kZeroCopyInsertBytes) {
    if ((e = hipMemcpyAsync(s.d_in, s.h_in, s.in_bytes, hipMemcpyHostToDevice, pst)) != hipSuccess) return e;
    in = s.d_in;
  }
  slash_csr csr{(const int64_t*)in, (const int32_t*)(in + s.idx_off), s.rows};
  s.prep_seq = ++srv->prep_seq;
  const GroupSignal sig{s.counter, s.flag, s.prep_seq};
  if (insert_prepare(srv->ix, csr, s.sc, pst, &s.first_id, sig) != SLASH_OK) return hipErrorLaunchFailure;
  return hipSuccess;
}

// A preparation that has not set its word after this long is taken as a
// device failure.
constexpr double kPrepTimeout = 10.0;

// Wait (bounded) until insert slot s's preparation has set its word.
hipError_t wait_prepared(slash_server* srv, const Slot& s) {
  if (s.prep_failed) return hipErrorLaunchFailure;
  const volatile uint64_t* f = s.flag;
  if (*f < s.prep_seq) {
    const double t0 = now_s();
    while (*f < s.prep_seq)
      if (now_s() - t0 > kPrepTimeout) return hipErrorLaunchTimeOut;
    srv->stats.wait_s += now_s() - t0;
  }
  return hipSuccess;
}

// Whether insert slot s's preparation has set its word (no wait).
bool is_prepared(const Slot& s) { return !s.prep_failed && *(const volatile uint64_t*)s.flag >= s.prep_seq; }

// Remove the FIFO's head (lock held).
void pop_head(slash_server* srv) {
  srv->pending.pop_front();
  if (srv->prep_scan) --srv->prep_scan;
}

// Move the prepared inserts at the FIFO's head (those sharing the head's
// insert slot) into that slot; each closes its own epoch.  Lock held.
Slot& take_insert(slash_server* srv) {
  const int32_t idx = srv->pending.front().prep;
  Slot& s = srv->ins[idx];
  s.reqs.clear();
  while (!srv->pending.empty() && srv->pending.front().kind == 1 && srv->pending.front().prep == idx) {
    s.reqs.push_back(std::move(srv->pending.front()));
    pop_head(srv);
  }
  s.epoch = srv->epoch + 1;
  srv->epoch += s.reqs.size();
  return s;
}

// Prepare the queued inserts in FIFO order while insert slots are free; the
// inserts queued right behind one share its slot while they fit its staging
// (one launch, each request still its own epoch).  Lock held; released
// around the launches.
void prepare_ahead(slash_server* srv, std::unique_lock<std::mutex>& lk) {
  std::vector<const Request*> rs;
  size_t i = srv->prep_scan;
  while (i < srv->pending.size()) {
    if (srv->pending[i].kind != 1 || srv->pending[i].prep >= 0) {
      ++i;
      continue;
    }
    int32_t slot = -1;
    for (size_t o = 0; o < srv->ins.size(); ++o)
      if (!srv->ins[o].busy) {
        slot = (int32_t)o;
        break;
      }
    if (slot < 0) break;
    Slot& s = srv->ins[slot];
    size_t j = i;
    uint32_t rows = 0;
    uint64_t nnz = 0;
    rs.clear();
    while (j < srv->pending.size() && srv->pending[j].kind == 1) {
      Request& r = srv->pending[j];
      if (j > i && (rows + r.n_rows > s.cap_q || nnz + r.idx.size() > s.cap_nnz)) break;
      rows += r.n_rows;
      nnz += r.idx.size();
      r.prep = slot;
      rs.push_back(&r);
      ++j;
    }
    s.reqs.clear();
    s.kind = 1;
    s.busy = true;
    s.prep_failed = false;
    srv->stats.batches++;
    i = j;
    srv->prep_scan = i;
    lk.unlock();
    const double t0 = now_s();
    pack_inserts(s, rs);
    const double t1 = now_s();
    const hipError_t e = prepare_insert(srv, s);
    srv->stats.pack_s += t1 - t0;
    srv->stats.launch_s += now_s() - t1;
    lk.lock();
    if (e != hipSuccess) {
      srv->dev_err = e;
      s.prep_failed = true;
    }
    i = srv->prep_scan;
  }
  srv->prep_scan = i;
}

// Whether the queries at the head of the FIFO fill one batch, or an insert
// ends their run (then waiting cannot make the batch larger).
bool head_run_full(const slash_server* srv, uint32_t max_batch) {
  const uint32_t cap = std::min(max_batch, srv->cap_q);
  uint64_t nnz = 0;
  uint32_t c = 0;
  for (const Request& r : srv->pending) {
    if (r.kind != 0 || c >= cap || nnz + r.idx.size() > srv->cap_nnz) return true;
    nnz += r.idx.size();
    ++c;
  }
  return c >= cap;
}

// Add a batch slot while the budget and the device's free memory allow
// (lock not held).  Returns the new slot or nullptr.
Slot* grow_slots(slash_server* srv) {
  if (srv->slots.size() >= srv->cfg.max_inflight) return nullptr;
  if (srv->hbm_used + srv->per_slot > srv->cfg.hbm_budget_bytes) return nullptr;
  if (now_s() < srv->grow_retry_at) return nullptr;
  size_t free_b = 0, total_b = 0;
  Slot s;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || free_b < srv->per_slot + kFreeReserve ||
      !alloc_slot(s, srv->cap_q, srv->cap_nnz, srv->info.params.k_max, true, 0, 0, srv->slot_ids_bytes)) {
    free_slot(s);
    (void)hipGetLastError();
    srv->grow_retry_at = now_s() + 0.01;
    return nullptr;
  }
  srv->hbm_used += srv->per_slot;
  srv->stats.peak_hbm_bytes = std::max(srv->stats.peak_hbm_bytes, srv->hbm_used);
  // the vector's elements move: only the scheduler thread holds Slot
  // references, and none across this call
  srv->slots.push_back(s);
  return &srv->slots.back();
}

// Launch one step (lock held; released around the launch) and track it:
// the slots it finishes retire with its event; a batch gathered here
// becomes the one waiting to be ranked.  On failure every slot involved is
// failed at once.
void run_step(slash_server* srv, std::unique_lock<std::mutex>& lk, Slot* agg, Slot* cur, bool gather_only,
              Slot* ins) {
  auto id_of = [srv](Slot* x) {
    return x >= srv->ins.data() && x < srv->ins.data() + srv->ins.size()
               ? std::make_pair(true, (uint32_t)(x - srv->ins.data()))
               : std::make_pair(false, (uint32_t)(x - srv->slots.data()));
  };
  Launch ln;
  Slot* done_with[3] = {ins, gather_only ? nullptr : cur, agg};
  for (Slot* x : done_with)
    if (x) ln.slot[ln.n++] = id_of(x);
  Slot& ev_slot = ins ? *ins : (!gather_only && cur) ? *cur : *agg;
  if (agg) srv->gathered = -1;
  lk.unlock();
  const double t0 = now_s(), p0 = srv->stats.pack_s;
  bool fused = false;
  const hipError_t e = launch_step(srv, agg, cur, gather_only, ins, ev_slot, &fused);
  srv->stats.launch_s += (now_s() - t0) - (srv->stats.pack_s - p0);
  lk.lock();
  if (fused) srv->stats.fused_commits++;
  if (e != hipSuccess) {
    // nothing of this launch can be trusted: fail its requests now
    srv->dev_err = e;
    for (Slot* x : {agg, cur, ins})
      if (x) finish_slot(srv, *x, SLASH_E_DEVICE);
    srv->cv.notify_all();
    return;
  }
  srv->inflight.push_back(ln);
  if (gather_only) {
    srv->gathered = id_of(cur).second;
    srv->stats.split_batches++;
  }
}

void scheduler(slash_server* srv) {
  (void)hipSetDevice(srv->device);
  const uint32_t max_batch = srv->cfg.max_batch;
  const double max_wait = srv->cfg.max_wait_us * 1e-6;
  std::vector<std::pair<Slot*, hipError_t>> finished;
  auto slot_of = [srv](const std::pair<bool, uint32_t>& f) -> Slot& {
    return f.first ? srv->ins[f.second] : srv->slots[f.second];
  };
  double busy_since = -1.0;
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    // 1. retire finished work.  Slots and events belong to this thread, so
    //    the events are queried without the lock.
    lk.unlock();
    finished.clear();
    while (!srv->inflight.empty()) {
      const Launch& ln = srv->inflight.front();
      const hipError_t q = hipEventQuery(slot_of(ln.slot[0]).done);
      if (q == hipErrorNotReady) break;
      for (uint32_t i = 0; i < ln.n; ++i) finished.emplace_back(&slot_of(ln.slot[i]), q);
      srv->inflight.pop_front();
    }
    lk.lock();
    // a launch whose table writers stopped waiting may have let queries see
    // part of an insert: every result from then on is reported failed
    const bool gave_up = *(const volatile uint32_t*)srv->fuse.gave_up != 0;
    if (gave_up && srv->dev_err == hipSuccess) srv->dev_err = hipErrorLaunchTimeOut;
    for (auto& [s, q] : finished) {
      if (q != hipSuccess) srv->dev_err = q;
      finish_slot(srv, *s, q == hipSuccess && !gave_up ? SLASH_OK : SLASH_E_DEVICE);
    }
    if (!finished.empty()) srv->cv.notify_all();
    // 2. prepare queued inserts, admit the head of the FIFO.  A batch whose
    //    insert follows it is only gathered in the launch that writes the
    //    insert and ranked in the next launch (or on its own, below, when
    //    none follows soon), so the next epoch need not wait for its ranking.
    double wake_at = 0.0;
    bool slot_wait = false;     // stopped for want of a batch slot
    bool prep_blocked = false;  // stopped at an insert still being prepared
    for (;;) {
      prepare_ahead(srv, lk);
      if (srv->pending.empty()) break;
      Request& head = srv->pending.front();
      Slot* agg = srv->gathered >= 0 ? &srv->slots[srv->gathered] : nullptr;
      if (head.kind == 1) {
        if (head.prep < 0) break;  // waits for an insert slot
        Slot& is = srv->ins[head.prep];
        if (!is.prep_failed && !is_prepared(is)) {
          // its preparation is still running: poll it on the next rounds
          // (finished work keeps being retired meanwhile); one that takes
          // longer than kPrepTimeout is failed
          const double t = now_s();
          if (srv->prep_wait_since < 0) srv->prep_wait_since = t;
          if (t - srv->prep_wait_since <= kPrepTimeout) {
            prep_blocked = true;
            break;
          }
          is.prep_failed = true;
        }
        if (srv->prep_wait_since >= 0) {
          srv->stats.wait_s += now_s() - srv->prep_wait_since;
          srv->prep_wait_since = -1.0;
        }
        Slot& s = take_insert(srv);
        run_step(srv, lk, agg, nullptr, false, &s);
        continue;
      }
      Slot* free_s = nullptr;
      for (Slot& s : srv->slots)
        if (!s.busy) {
          free_s = &s;
          break;
        }
      if (!free_s) {
        lk.unlock();
        free_s = grow_slots(srv);
        lk.lock();
        if (!free_s) {
          slot_wait = true;
          break;
        }
      }
      Slot& s = *free_s;
      if (max_wait > 0 && !srv->stopping) {
        const double due = srv->pending.front().t_submit + max_wait;
        if (!head_run_full(srv, max_batch) && now_s() < due) {
          wake_at = due;  // hold the partial batch back
          break;
        }
      }
      s.reqs.clear();
      uint64_t nnz = 0;
      while (!srv->pending.empty() && s.reqs.size() < std::min(max_batch, s.cap_q)) {
        Request& r = srv->pending.front();
        if (r.kind != 0 || nnz + r.idx.size() > s.cap_nnz) break;
        nnz += r.idx.size();
        s.reqs.push_back(std::move(r));
        pop_head(srv);
      }
      s.kind = 0;
      s.busy = true;
      s.epoch = srv->epoch;
      srv->stats.batches++;
      const bool small = srv->slot_ids_bytes && serve_step_ok(srv->ix, s.reqs.size());
      // the insert queued right behind the batch goes into the same launch
      // when its preparation is done (or always, waiting for it, with
      // insert_fusion 2)
      Slot* ins = nullptr;
      if (small && srv->cfg.insert_fusion != 1 && !srv->pending.empty() && srv->pending.front().kind == 1 &&
          srv->pending.front().prep >= 0) {
        Slot& is = srv->ins[srv->pending.front().prep];
        if (!is.prep_failed && (srv->cfg.insert_fusion == 2 || is_prepared(is))) ins = &take_insert(srv);
      }
      if (agg && !small) {
        run_step(srv, lk, agg, nullptr, false, nullptr);  // rank the gathered batch first
        agg = nullptr;
      }
      // split the batch (gather now, rank in the next launch) only when more
      // requests wait behind the insert, so that a launch will carry the
      // ranking: else it would need a launch of its own
      run_step(srv, lk, agg, &s, ins != nullptr && !srv->pending.empty(), ins);
      uint64_t inflight = 0;
      for (Slot& o : srv->slots) inflight += o.busy;
      srv->stats.peak_inflight = std::max(srv->stats.peak_inflight, inflight);
    }
    // a gathered batch is ranked on its own when no launch will carry it
    // soon: nothing queued, the head held back or waiting for an insert
    // slot, or no batch slot free and none but the gathered one busy (so
    // none will free up)
    if (srv->gathered >= 0) {
      uint32_t others = 0;
      for (const Slot& o : srv->slots) others += o.busy;
      if (srv->pending.empty() || wake_at > 0 || (!slot_wait && !prep_blocked) || others <= 1)
        run_step(srv, lk, &srv->slots[srv->gathered], nullptr, false, nullptr);
    }
    bool busy = false;
    for (Slot& s : srv->ins) busy |= s.busy;
    for (Slot& s : srv->slots) busy |= s.busy;
    // host time with device work in flight
    const double t = now_s();
    if (busy && busy_since < 0) busy_since = t;
    if (!busy && busy_since >= 0) {
      srv->stats.busy_s += t - busy_since;
      busy_since = -1.0;
    }
    if (srv->stopping && srv->pending.empty() && !busy) break;
    if (busy) {
      // device work in flight: poll its events again at once (a sleep would
      // add the timer slack, tens of microseconds, to every completion)
      lk.unlock();
      std::this_thread::yield();
      lk.lock();
    } else if (wake_at > 0) {
      srv->cv.wait_for(lk, std::chrono::duration<double>(std::max(0.0, wake_at - t)));
    } else {
      srv->cv.wait_for(lk, std::chrono::milliseconds(1), [&] { return srv->stopping || !srv->pending.empty(); });
    }
  }
}

void free_server(slash_server* srv) {
  for (Slot& o : srv->slots) free_slot(o);
  for (Slot& o : srv->ins) free_slot(o);
  for (hipStream_t st : {srv->stream, srv->prep})
    if (st) {
      (void)hipStreamSynchronize(st);
      (void)hipStreamDestroy(st);
    }
  (void)hipFree(srv->fuse.dev);
  (void)hipHostFree(srv->fuse.gave_up);
  delete srv;
}

}  // namespace

extern "C" slash_status slash_serve_start(slash_index* ix, const slash_serve_config* cfg, slash_server** out) {
  if (!ix || !cfg || !out) return fail(SLASH_E_INVAL, "NULL argument");
  if (cfg->max_batch == 0 || cfg->max_inflight == 0 || cfg->queue_capacity == 0 || cfg->max_query_nnz == 0)
    return fail(SLASH_E_INVAL, "max_batch, max_inflight, queue_capacity and max_query_nnz must be >= 1");
  if (cfg->insert_fusion > 2) return fail(SLASH_E_INVAL, "insert_fusion must be 0, 1 or 2");
  slash_server* srv = new slash_server();
  srv->ix = ix;
  srv->cfg = *cfg;
  slash_index_info_get(ix, &srv->info);
  srv->next_id = srv->info.n_items;
  (void)hipGetDevice(&srv->device);
  const uint32_t km = srv->info.params.k_max;
  // a batch holds max_batch queries of 64 indices on average, and at least
  // one query of max_query_nnz
  srv->cap_q = cfg->max_batch;
  srv->cap_nnz = std::max<uint64_t>((uint64_t)srv->cap_q * 64, cfg->max_query_nnz);
  srv->per_slot = slot_bytes(srv->cap_q, srv->cap_nnz);
  // a batch small enough for the serving-step kernel can be split: gathered
  // in the launch that writes the insert behind it, ranked in the next one;
  // its slot ids wait in device memory
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, srv->device) != hipSuccess || n_cu < 1) {
    delete srv;
    return fail(SLASH_E_DEVICE, "device attributes");
  }
  if (serve_step_ok(ix, 1)) {
    const uint64_t split_q = std::min<uint64_t>(srv->cap_q, (uint64_t)n_cu / 2);
    srv->slot_ids_bytes = split_q * srv->info.params.L * srv->info.params.R * 4;
    srv->per_slot += srv->slot_ids_bytes;
  }
  // insert staging: 4096 rows of max_insert_nnz indices in total (default
  // the larger of 64 per row and 8 * max_query_nnz)
  const uint32_t ins_rows = 4096;
  const uint64_t ins_nnz = cfg->max_insert_nnz ? cfg->max_insert_nnz
                                               : std::max<uint64_t>((uint64_t)ins_rows * 64, 8ull * cfg->max_query_nnz);
  size_t keys_b = 0, runs_b = 0;
  if (!insert_scratch_bytes(ix, ins_rows, &keys_b, &runs_b))
    return fail(SLASH_E_UNSUPPORTED, "inserts of %u rows cannot be prepared ahead for this index", ins_rows);
  const uint64_t ins_bytes = in_layout(ins_rows, ins_nnz, false).bytes + keys_b + runs_b;
  if (ins_bytes + srv->per_slot > cfg->hbm_budget_bytes) {
    delete srv;
    return fail(SLASH_E_NOMEM, "HBM budget %llu below one batch slot (%llu bytes)",
                (unsigned long long)cfg->hbm_budget_bytes, (unsigned long long)(ins_bytes + srv->per_slot));
  }
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || free_b < ins_bytes + srv->per_slot) {
    delete srv;
    return fail(SLASH_E_NOMEM, "free device memory below one batch slot and the insert staging");
  }
  if (hipStreamCreateWithFlags(&srv->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&srv->prep, hipStreamNonBlocking) != hipSuccess) {
    free_server(srv);
    return fail(SLASH_E_DEVICE, "stream creation failed");
  }
  if (hipMalloc(&srv->fuse.dev, 256) != hipSuccess || hipMemset(srv->fuse.dev, 0, 256) != hipSuccess ||
      hipHostMalloc(&srv->fuse.gave_up, 64, hipHostMallocCoherent) != hipSuccess) {
    free_server(srv);
    return fail(SLASH_E_NOMEM, "fused-launch counters");
  }
  *(volatile uint32_t*)srv->fuse.gave_up = 0;
  srv->ins.emplace_back();
  if (!alloc_slot(srv->ins[0], ins_rows, ins_nnz, km, false, keys_b, runs_b)) {
    free_server(srv);
    return fail(SLASH_E_NOMEM, "insert staging allocation failed");
  }
  srv->hbm_used = ins_bytes;
  // more insert slots (up to kInsertSlots) while the budget still leaves room for a
  // batch slot
  while (srv->ins.size() < kInsertSlots && srv->hbm_used + ins_bytes + srv->per_slot <= cfg->hbm_budget_bytes) {
    srv->ins.emplace_back();
    if (!alloc_slot(srv->ins.back(), ins_rows, ins_nnz, km, false, keys_b, runs_b)) {
      free_slot(srv->ins.back());
      srv->ins.pop_back();
      break;
    }
    srv->hbm_used += ins_bytes;
  }
  // one batch slot now; more are added while work waits for them
  srv->slots.reserve(cfg->max_inflight);
  srv->slots.emplace_back();
  if (!alloc_slot(srv->slots[0], srv->cap_q, srv->cap_nnz, km, true, 0, 0, srv->slot_ids_bytes)) {
    free_server(srv);
    return fail(SLASH_E_NOMEM, "no batch slot fits the HBM budget");
  }
  srv->hbm_used += srv->per_slot;
  srv->stats.peak_hbm_bytes = srv->hbm_used;
  bool warm = true;
  for (Slot& o : srv->ins) warm = warm && warm_slot(srv->prep, o, false);
  warm = warm && warm_slot(srv->stream, srv->slots[0], true);
  // the other batch slots now, as far as the budget and the free memory
  // allow: a slot added while serving stalls the scheduler thread in the
  // allocators for up to a millisecond
  while (warm && srv->slots.size() < cfg->max_inflight) {
    Slot* s = grow_slots(srv);
    if (!s) break;
    warm = warm_slot(srv->stream, *s, true);
  }
  if (warm) {
    // one single-index query loads the query kernels
    Slot& q = srv->slots[0];
    const int64_t ip[2] = {0, 1};
    const int32_t zero = 0;
    const InLayout l = in_layout(1, 1, false);
    warm = hipMemcpy(q.d_in, ip, sizeof ip, hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(q.d_in + l.idx, &zero, 4, hipMemcpyHostToDevice) == hipSuccess &&
           slash_query(ix, slash_csr{(const int64_t*)q.d_in, (const int32_t*)(q.d_in + l.idx), 1}, nullptr, 1,
                       SLASH_FLAG_TRUSTED, q.h_out, q.h_out + km, srv->stream) == SLASH_OK &&
           hipStreamSynchronize(srv->stream) == hipSuccess;
  }
  if (!warm) {
    free_server(srv);
    return fail(SLASH_E_DEVICE, "server warm-up failed");
  }
  srv->th = std::thread(scheduler, srv);
  *out = srv;
  return SLASH_OK;
}

static slash_status enqueue(slash_server* srv, Request&& r, uint64_t* ticket) {
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->closed) return fail(SLASH_E_CLOSED, "server stopped");
  if (srv->pending.size() >= srv->cfg.queue_capacity) {
    srv->stats.rejected_busy++;
    return fail(SLASH_E_BUSY, "queue full");
  }
  r.ticket = srv->next_ticket++;
  r.t_submit = now_s();
  if (ticket) *ticket = r.ticket;
  srv->pending.push_back(std::move(r));
  srv->cv.notify_all();
  return SLASH_OK;
}

extern "C" slash_status slash_serve_submit_query(slash_server* srv, const int32_t* idx, uint32_t nnz, uint32_t k,
                                                 uint64_t* ticket) {
  if (!srv || (!idx && nnz)) return fail(SLASH_E_INVAL, "NULL argument");
  if (nnz == 0 || nnz > srv->cfg.max_query_nnz) return fail(SLASH_E_INVAL, "query nnz %u outside [1, %u]", nnz, srv->cfg.max_query_nnz);
  if (k > srv->info.params.k_max || k > SLASH_SERVE_MAX_K) return fail(SLASH_E_INVAL, "k %u too large", k);
  const uint32_t dim = srv->info.params.dim;
  for (uint32_t i = 0; i < nnz; ++i)
    if (idx[i] < 0 || (uint32_t)idx[i] >= dim) return fail(SLASH_E_INVAL, "index outside [0, dim)");
  Request r;
  r.kind = 0;
  r.k = k;
  r.n_rows = 1;
  r.idx.assign(idx, idx + nnz);
  return enqueue(srv, std::move(r), ticket);
}

extern "C" slash_status slash_serve_submit_insert(slash_server* srv, const int64_t* indptr, const int32_t* idx,
                                                  uint32_t n_rows, uint64_t* ticket) {
  if (!srv || !indptr || (!idx && n_rows)) return fail(SLASH_E_INVAL, "NULL argument");
  if (n_rows == 0 || n_rows > srv->ins[0].cap_q) return fail(SLASH_E_INVAL, "insert of %u rows outside [1, %u]", n_rows, srv->ins[0].cap_q);
  if (indptr[0] != 0) return fail(SLASH_E_INVAL, "indptr[0] must be 0");
  const uint32_t dim = srv->info.params.dim;
  for (uint32_t r = 0; r < n_rows; ++r)
    if (indptr[r + 1] <= indptr[r]) return fail(SLASH_E_INVAL, "empty row in insert");
  const uint64_t nnz = (uint64_t)indptr[n_rows];
  if (nnz > srv->ins[0].cap_nnz) {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stats.rejected_nomem++;
    return fail(SLASH_E_NOMEM, "insert of %llu indices exceeds the staging budget", (unsigned long long)nnz);
  }
  for (uint64_t i = 0; i < nnz; ++i)
    if (idx[i] < 0 || (uint32_t)idx[i] >= dim) return fail(SLASH_E_INVAL, "index outside [0, dim)");
  Request r;
  r.kind = 1;
  r.n_rows = n_rows;
  r.indptr.assign(indptr, indptr + n_rows + 1);
  r.idx.assign(idx, idx + nnz);
  return enqueue(srv, std::move(r), ticket);
}

extern "C" slash_status slash_serve_poll(slash_server* srv, slash_completion* out, uint32_t max, uint32_t* n) {
  if (!srv || !n || (!out && max)) return fail(SLASH_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  uint32_t c = 0;
  while (c < max && !srv->done.empty()) {
    out[c++] = srv->done.front();
    srv->done.pop_front();
  }
  *n = c;
  if (srv->dev_err != hipSuccess) return fail(SLASH_E_DEVICE, "serve: %s", hipGetErrorString(srv->dev_err));
  return SLASH_OK;
}

extern "C" slash_status slash_serve_stop(slash_server* srv, slash_serve_stats* stats) {
  if (!srv) return fail(SLASH_E_INVAL, "NULL server");
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
    srv->closed = true;
    srv->cv.notify_all();
  }
  if (srv->th.joinable()) srv->th.join();
  hipError_t err = srv->dev_err;
  if (stats) *stats = srv->stats;
  free_server(srv);
  if (err != hipSuccess) return fail(SLASH_E_DEVICE, "serve: %s", hipGetErrorString(err));
  return SLASH_OK;
}

extern "C" slash_status slash_serve_replay(slash_server* srv, uint64_t n, const double* t_arr, const uint8_t* is_ins,
                                           const uint32_t* ins_rows, const int64_t* q_indptr, const int32_t* q_idx,
                                           const uint32_t* q_k, const int64_t* ins_indptr, const int32_t* ins_idx,
                                           double* lat, uint32_t* out_ids, uint32_t out_stride) {
  if (!srv || !t_arr || !is_ins || !lat) return fail(SLASH_E_INVAL, "NULL argument");
  std::vector<uint64_t> tickets(n, ~0ull);
  std::vector<int64_t> by_ticket;
  std::atomic<uint64_t> submitted{0};
  std::atomic<int> client_err{0};
  const double t0 = now_s() + 0.002;
  std::thread client([&] {
    uint64_t qi = 0, ii = 0;  // next query row, next insert row
    for (uint64_t i = 0; i < n; ++i) {
      const double due = t0 + t_arr[i];
      while (now_s() < due) {
      }
      slash_status st;
      for (;;) {
        if (is_ins[i]) {
          uint32_t m = ins_rows[i];
          std::vector<int64_t> ip(m + 1);
          for (uint32_t r = 0; r <= m; ++r) ip[r] = ins_indptr[ii + r] - ins_indptr[ii];
          st = slash_serve_submit_insert(srv, ip.data(), ins_idx + ins_indptr[ii], m, &tickets[i]);
        } else {
          st = slash_serve_submit_query(srv, q_idx + q_indptr[qi], (uint32_t)(q_indptr[qi + 1] - q_indptr[qi]),
                                        q_k ? q_k[qi] : 10, &tickets[i]);
        }
        if (st != SLASH_E_BUSY) break;
        std::this_thread::yield();
      }
      if (st != SLASH_OK) {
        client_err = st;
        tickets[i] = ~0ull;
      }
      if (is_ins[i])
        ii += ins_rows[i];
      else
        ++qi;
      submitted.store(i + 1, std::memory_order_release);
    }
  });
  // poll completions; tickets are mapped to requests at the end.  Each
  // completion is kept as a compact record (and its ids only when asked
  // for), in storage sized up front: growing a vector of whole completions
  // (1 KB each) reallocated hundreds of MB while serving, and the page
  // faults and unmapping stalled the scheduler thread for milliseconds.
  struct Done {
    uint64_t ticket;
    double t_done_s;
    uint32_t k, kind;
  };
  std::vector<slash_completion> buf(256);
  uint64_t got = 0;
  std::vector<Done> store;
  store.reserve(n);
  std::vector<uint32_t> id_store;
  if (out_ids) id_store.resize(n * (uint64_t)out_stride);
  slash_status rs = SLASH_OK;
  uint64_t expected = n;
  while (got < expected) {
    uint32_t m = 0;
    rs = slash_serve_poll(srv, buf.data(), (uint32_t)buf.size(), &m);
    if (rs != SLASH_OK) break;
    for (uint32_t j = 0; j < m && store.size() < n; ++j) {
      const slash_completion& c = buf[j];
      if (out_ids && c.kind == 0)
        memcpy(id_store.data() + store.size() * (uint64_t)out_stride, c.ids,
               std::min<uint32_t>(c.k, out_stride) * sizeof(uint32_t));
      store.push_back(Done{c.ticket, c.t_done_s, c.k, c.kind});
    }
    got += m;
    if (client_err.load() && submitted.load() == n) {
      uint64_t ok = 0;
      for (uint64_t i = 0; i < n; ++i) ok += tickets[i] != ~0ull;
      expected = ok;
    }
    if (m == 0) std::this_thread::sleep_for(std::chrono::microseconds(2));
  }
  client.join();
  if (rs != SLASH_OK) return rs;
  uint64_t base = ~0ull;
  for (uint64_t i = 0; i < n; ++i) base = std::min(base, tickets[i]);
  std::vector<int64_t> req_of(n + 1, -1);
  for (uint64_t i = 0; i < n; ++i)
    if (tickets[i] != ~0ull && tickets[i] - base < n) req_of[tickets[i] - base] = (int64_t)i;
  for (size_t x = 0; x < store.size(); ++x) {
    const Done& c = store[x];
    if (c.ticket - base >= n) continue;
    int64_t i = req_of[c.ticket - base];
    if (i < 0) continue;
    lat[i] = c.t_done_s - (t0 + t_arr[i]);
    if (out_ids && c.kind == 0)
      memcpy(out_ids + (uint64_t)i * out_stride, id_store.data() + x * (uint64_t)out_stride,
             std::min<uint32_t>(c.k, out_stride) * sizeof(uint32_t));
  }
  for (uint64_t i = 0; i < n; ++i)
    if (tickets[i] == ~0ull) lat[i] = -1.0;
  if (client_err.load()) return fail((slash_status)client_err.load(), "some requests were rejected");
  return SLASH_OK;
}
