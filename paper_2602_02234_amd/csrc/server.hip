// Continuous-batching evaluation server (host code).
//
// Independent energy/force/virial requests (the paper's MD engine hands the model
// one system per step; a serving loop sees many such systems at once) are queued on
// submit and run as work items on up to max_inflight lanes, each with its own stream:
//
//  * requests of at most CHUNK atoms are packed, in arrival order, into batched steps
//    of at most CHUNK atoms (all atoms of the batch go through each kernel in one
//    launch: concatenated atom arrays, one cell grid per system);
//  * a larger request is split into (request, centre chunk) items of CHUNK centre
//    atoms, evaluated in order on a workspace of its own (lists, E_i and pair
//    gradients of earlier chunks stay there; the last chunk gathers the forces).  After
//    each chunk the request goes to the back of the queue, so the requests that arrived
//    meanwhile run before its next chunk and a small request is never held behind a
//    whole large one.
//
// While one lane's item runs, the worker packs, uploads and launches items on the
// others, so requests that arrive while the GPU is busy are admitted as lanes free up
// and their work overlaps on the device.  Admission is by device-memory footprint: the
// lanes' batch workspaces plus the workspaces of the large requests in progress stay
// within the byte budget.  A request's result does not depend on the other requests of
// its batch nor on chunking: every per-atom kernel computes each atom from that atom's
// data only, and the per-system reductions run in the same fixed order at any offset.
#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/dp.h"
#include "dp_internal.h"

using namespace dp;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int MAX_LANES = 8;
constexpr int64_t CHUNK = 8192;  // atoms per batch, and centre atoms per chunk of a large request
constexpr int MAX_BATCH_SYSTEMS = 256;
// device bytes per atom outside the workspace: coordinates, types, forces
constexpr size_t IO_BYTES_PER_ATOM = 3 * sizeof(double) + sizeof(int) + 3 * sizeof(double);

template <typename T> int grow(T **p, int64_t &cap, int64_t need, bool pinned) {
  if (need <= cap) return DP_OK;
  const int64_t c = std::max<int64_t>(need, cap + cap / 2);
  if (*p) (void)(pinned ? hipHostFree(*p) : hipFree(*p));
  *p = nullptr;
  cap = 0;
  const hipError_t e = pinned ? hipHostMalloc((void **)p, c * sizeof(T), hipHostMallocDefault)
                              : hipMalloc((void **)p, c * sizeof(T));
  if (e != hipSuccess) {
    set_error("dp_server: device or pinned allocation failed");
    return DP_ERR_OOM;
  }
  cap = c;
  return DP_OK;
}

// Device state of one large request while its chunks run: its own workspace and
// input/output arrays.  Kept in a pool and reused.
struct BigSlot {
  bool used = false;
  Workspace ws;
  double *dX = nullptr, *dF = nullptr, *dE = nullptr, *dV = nullptr;
  int *dT = nullptr;
  int64_t cX = 0, cF = 0, cE = 0, cV = 0, cT = 0;
};

struct Request {
  uint64_t id = 0;
  int64_t n = 0;
  std::vector<double> X;
  std::vector<int32_t> T;
  double box[9] = {};
  bool solo = false;  // run alone (after its batch failed)
  // a large request: progress of its chunks and its device state
  bool chunked = false;
  int64_t next_c0 = 0;
  BigSlot *slot = nullptr;
  // results
  int status = DP_OK;
  bool done = false;
  double E = 0.0, V[9] = {};
  std::vector<double> F;
  Clock::time_point t_submit, t_done;
};

struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t done_ev = nullptr;
  Workspace ws;
  double *dX = nullptr, *dF = nullptr, *dE = nullptr, *dV = nullptr;
  int *dT = nullptr;
  double *hX = nullptr, *hF = nullptr, *hE = nullptr, *hV = nullptr;
  int *hT = nullptr;
  unsigned *hflags = nullptr;  // status words of a chunk item
  int64_t cX = 0, cF = 0, cE = 0, cV = 0, cT = 0, chX = 0, chF = 0, chE = 0, chV = 0, chT = 0, chflags = 0;
  std::vector<Request *> batch;  // a batch of small requests, or the one large request of a chunk item
  bool chunk_item = false;
  bool last_chunk = false;
  int64_t atoms = 0;
  bool busy = false;
  int launch_status = DP_OK;
};

}  // namespace

struct dp_server {
  dp_model *m = nullptr;
  size_t budget = 0;
  int nlanes = 2;
  size_t big_bytes = 0;       // budget left by the lanes for the workspaces of large requests
  int64_t max_big_atoms = 0;  // largest request that budget admits
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<uint64_t, Request *> reqs;
  uint64_t next_id = 1;
  Lane lanes[MAX_LANES];
  std::vector<BigSlot> big;
  std::thread worker;
  bool stop = false;
  // statistics
  std::vector<double> lat;
  int64_t atoms_done = 0, completed = 0, batches = 0, max_batch_atoms = 0;
  bool have_first = false;
  Clock::time_point t_first, t_last;
};

namespace {

size_t bytes_per_atom(const dp_model *m) { return ws_bytes_per_atom(m->prec) + IO_BYTES_PER_ATOM; }

#define SRV_TRY(expr)                                \
  do {                                               \
    if ((expr) != hipSuccess) {                      \
      set_error(std::string("dp_server: ") + #expr); \
      return DP_ERR_HIP;                             \
    }                                                \
  } while (0)

// A batch of small requests: one batched step on the lane's own workspace.
int launch_batch(dp_server *s, Lane &L) {
  dp_model *m = s->m;
  const int nsys = (int)L.batch.size();
  int64_t tot = 0;
  for (Request *r : L.batch) tot += r->n;
  int st = ensure_ws(L.ws, m->prec, tot, nsys, false);
  if (st == DP_OK) st = grow(&L.dX, L.cX, 3 * tot, false);
  if (st == DP_OK) st = grow(&L.dF, L.cF, 3 * tot, false);
  if (st == DP_OK) st = grow(&L.dT, L.cT, tot, false);
  if (st == DP_OK) st = grow(&L.dE, L.cE, nsys, false);
  if (st == DP_OK) st = grow(&L.dV, L.cV, 9 * nsys, false);
  if (st == DP_OK) st = grow(&L.hX, L.chX, 3 * tot, true);
  if (st == DP_OK) st = grow(&L.hF, L.chF, 3 * tot, true);
  if (st == DP_OK) st = grow(&L.hT, L.chT, tot, true);
  if (st == DP_OK) st = grow(&L.hE, L.chE, nsys, true);
  if (st == DP_OK) st = grow(&L.hV, L.chV, 9 * nsys, true);
  if (st != DP_OK) return st;
  int64_t off = 0;
  int cells = 0;
  L.ws.off_host[0] = 0;
  for (int k = 0; k < nsys; ++k) {
    Request *r = L.batch[k];
    std::memcpy(L.hX + 3 * off, r->X.data(), 3 * r->n * sizeof(double));
    std::memcpy(L.hT + off, r->T.data(), r->n * sizeof(int));
    Grid g;
    st = make_grid(m->rc, m->rc, r->box, g);
    if (st != DP_OK) return st;
    g.cell_base = cells;
    cells += g.ncells;
    L.ws.grids_host[k] = g;
    off += r->n;
    L.ws.off_host[k + 1] = (int)off;
  }
  if (cells > MAX_CELLS) {
    set_error("dp_server: too many cells in one batch");
    return DP_ERR_TOO_LARGE;
  }
  SRV_TRY(hipMemcpyAsync(L.dX, L.hX, 3 * tot * sizeof(double), hipMemcpyHostToDevice, L.st));
  SRV_TRY(hipMemcpyAsync(L.dT, L.hT, tot * sizeof(int), hipMemcpyHostToDevice, L.st));
  StepArgs a;
  a.n = tot;
  a.nsys = nsys;
  a.X = L.dX;
  a.types = L.dT;
  a.energy = L.dE;
  a.forces = L.dF;
  a.virial = L.dV;
  a.ncells = cells;
  a.lists = LISTS_FRESH;
  st = enqueue_step(m, L.ws, a, L.st, false);
  if (st != DP_OK) return st;
  SRV_TRY(hipMemcpyAsync(L.hF, L.dF, 3 * tot * sizeof(double), hipMemcpyDeviceToHost, L.st));
  SRV_TRY(hipMemcpyAsync(L.hE, L.dE, nsys * sizeof(double), hipMemcpyDeviceToHost, L.st));
  SRV_TRY(hipMemcpyAsync(L.hV, L.dV, 9 * nsys * sizeof(double), hipMemcpyDeviceToHost, L.st));
  SRV_TRY(hipMemcpyAsync(L.ws.flags_host, L.ws.flags, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, L.st));
  SRV_TRY(hipEventRecord(L.done_ev, L.st));
  L.atoms = tot;
  return DP_OK;
}

// The next chunk of a large request, on the request's own workspace; the lane supplies
// its stream and pinned staging.
int launch_chunk(dp_server *s, Lane &L, Request *r, int64_t c0, int64_t c1) {
  dp_model *m = s->m;
  BigSlot &b = *r->slot;
  const int64_t n = r->n;
  const bool first = c0 == 0, last = c1 == n;
  int st = DP_OK;
  if (first) {
    st = ensure_ws(b.ws, m->prec, n, 1, false);
    if (st == DP_OK) st = grow(&b.dX, b.cX, 3 * n, false);
    if (st == DP_OK) st = grow(&b.dF, b.cF, 3 * n, false);
    if (st == DP_OK) st = grow(&b.dT, b.cT, n, false);
    if (st == DP_OK) st = grow(&b.dE, b.cE, 1, false);
    if (st == DP_OK) st = grow(&b.dV, b.cV, 9, false);
    if (st == DP_OK) st = grow(&L.hX, L.chX, 3 * n, true);
    if (st == DP_OK) st = grow(&L.hT, L.chT, n, true);
    if (st != DP_OK) return st;
    Grid g;
    st = make_grid(m->rc, m->rc, r->box, g);
    if (st != DP_OK) return st;
    b.ws.grids_host[0] = g;
    b.ws.off_host[0] = 0;
    b.ws.off_host[1] = (int)n;
    std::memcpy(L.hX, r->X.data(), 3 * n * sizeof(double));
    std::memcpy(L.hT, r->T.data(), n * sizeof(int));
    SRV_TRY(hipMemcpyAsync(b.dX, L.hX, 3 * n * sizeof(double), hipMemcpyHostToDevice, L.st));
    SRV_TRY(hipMemcpyAsync(b.dT, L.hT, n * sizeof(int), hipMemcpyHostToDevice, L.st));
  }
  if (last) {
    st = grow(&L.hF, L.chF, 3 * n, true);
    if (st == DP_OK) st = grow(&L.hE, L.chE, 1, true);
    if (st == DP_OK) st = grow(&L.hV, L.chV, 9, true);
    if (st != DP_OK) return st;
  }
  if ((st = grow(&L.hflags, L.chflags, 4, true)) != DP_OK) return st;
  StepArgs a;
  a.n = n;
  a.nsys = 1;
  a.X = b.dX;
  a.types = b.dT;
  a.energy = b.dE;
  a.forces = b.dF;
  a.virial = b.dV;
  a.ncells = b.ws.grids_host[0].ncells;
  a.lists = LISTS_FRESH;
  a.c0 = c0;
  a.c1 = c1;
  a.first_chunk = first;
  a.last_chunk = last;
  st = enqueue_step(m, b.ws, a, L.st, false);
  if (st != DP_OK) return st;
  if (last) {
    SRV_TRY(hipMemcpyAsync(L.hF, b.dF, 3 * n * sizeof(double), hipMemcpyDeviceToHost, L.st));
    SRV_TRY(hipMemcpyAsync(L.hE, b.dE, sizeof(double), hipMemcpyDeviceToHost, L.st));
    SRV_TRY(hipMemcpyAsync(L.hV, b.dV, 9 * sizeof(double), hipMemcpyDeviceToHost, L.st));
  }
  SRV_TRY(hipMemcpyAsync(L.hflags, b.ws.flags, 4 * sizeof(unsigned), hipMemcpyDeviceToHost, L.st));
  SRV_TRY(hipEventRecord(L.done_ev, L.st));
  L.atoms = c1 - c0;
  return DP_OK;
}
#undef SRV_TRY

void finish_request(dp_server *s, Request *r, int status, Clock::time_point now) {
  r->status = status;
  r->t_done = now;
  r->done = true;
  if (r->slot) {
    r->slot->used = false;
    r->slot = nullptr;
  }
  if (status >= 0) {
    s->lat.push_back(std::chrono::duration<double>(r->t_done - r->t_submit).count());
    s->atoms_done += r->n;
    s->completed += 1;
    s->t_last = now;
  }
}

// Status of a finished step from copied-back flag words (as step_status reads them).
int flags_to_status(const unsigned *f) {
  Workspace tmp;
  tmp.flags_host = const_cast<unsigned *>(f);
  const int st = step_status(tmp);
  return st == DP_RETRY ? DP_ERR_HIP : st;
}

// Called with the lock held once the lane's event has completed.
void lane_complete(dp_server *s, Lane &L) {
  const auto now = Clock::now();
  int st = L.launch_status;
  if (L.chunk_item) {
    Request *r = L.batch[0];
    if (st == DP_OK) st = flags_to_status(L.hflags);
    if (st < 0) {
      finish_request(s, r, st, now);
    } else if (L.last_chunk) {
      r->E = L.hE[0];
      std::memcpy(r->V, L.hV, 9 * sizeof(double));
      r->F.assign(L.hF, L.hF + 3 * r->n);
      finish_request(s, r, st, now);
    } else {
      s->queue.push_back(r);  // its next chunk after the requests that arrived meanwhile
    }
  } else {
    if (st == DP_OK) st = step_status(L.ws);
    if (st < 0 && L.batch.size() > 1) {
      // one request made the batch fail: run each alone to find out which
      for (auto it = L.batch.rbegin(); it != L.batch.rend(); ++it) {
        (*it)->solo = true;
        s->queue.push_front(*it);
      }
    } else {
      int64_t off = 0;
      for (size_t k = 0; k < L.batch.size(); ++k) {
        Request *r = L.batch[k];
        if (st >= 0) {
          r->E = L.hE[k];
          std::memcpy(r->V, L.hV + 9 * k, 9 * sizeof(double));
          r->F.assign(L.hF + 3 * off, L.hF + 3 * (off + r->n));
        }
        off += r->n;
        finish_request(s, r, st, now);
      }
    }
  }
  L.batch.clear();
  L.atoms = 0;
  L.busy = false;
  s->cv_done.notify_all();
  s->cv_work.notify_all();
}

void free_slot_memory(BigSlot &b) {
  free_ws(b.ws);
  void *d[] = {b.dX, b.dF, b.dE, b.dV, b.dT};
  for (void *p : d)
    if (p) (void)hipFree(p);
  b = BigSlot{};
}

// A workspace for the large request r among the pool's unused ones, such that the pool's
// device memory (grow-only workspaces) stays within the part of the budget the lanes
// leave; unused workspaces are released when that makes room.  nullptr: r must wait.
BigSlot *reserve_slot(dp_server *s, const Request *r) {
  const size_t bpa = bytes_per_atom(s->m);
  auto held = [&]() {
    size_t t = 0;
    for (const BigSlot &b : s->big) t += (size_t)b.ws.cap * bpa;
    return t;
  };
  for (int pass = 0; pass < 2; ++pass) {
    for (BigSlot &b : s->big) {
      if (b.used) continue;
      const size_t cap = (size_t)b.ws.cap * bpa;
      const size_t need = (size_t)std::max<int64_t>(b.ws.cap, r->n) * bpa;
      if (held() - cap + need <= s->big_bytes) return &b;
    }
    // release the memory of the unused workspaces, then try once more
    bool freed = false;
    for (BigSlot &b : s->big)
      if (!b.used && b.ws.cap > 0) {
        free_slot_memory(b);
        freed = true;
      }
    if (!freed) break;
  }
  return nullptr;
}

// Takes the next work item for a free lane from the queue (lock held): the chunk of the
// first large request that can run, or a batch of the small requests at the front.
// Returns false when nothing can run now.
bool take_item(dp_server *s, Lane &L, int64_t &c0, int64_t &c1) {
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
    Request *r = *it;
    if (r->chunked) {
      if (!r->slot) {
        BigSlot *b = reserve_slot(s, r);
        if (!b) continue;  // no room for its workspace yet: serve what is behind it
        b->used = true;
        r->slot = b;
      }
      s->queue.erase(it);
      c0 = r->next_c0;
      c1 = std::min<int64_t>(r->n, c0 + CHUNK);
      r->next_c0 = c1;
      L.batch.push_back(r);
      L.chunk_item = true;
      L.last_chunk = c1 == r->n;
      return true;
    }
    // small requests in arrival order from here while they fit one batch
    int64_t atoms = 0;
    auto jt = it;
    while (jt != s->queue.end() && (int)L.batch.size() < MAX_BATCH_SYSTEMS) {
      Request *q = *jt;
      if (q->chunked) break;
      if (!L.batch.empty() && (q->solo || L.batch.front()->solo)) break;
      if (!L.batch.empty() && atoms + q->n > CHUNK) break;
      L.batch.push_back(q);
      atoms += q->n;
      jt = s->queue.erase(jt);
    }
    L.chunk_item = false;
    return true;
  }
  return false;
}

void worker_loop(dp_server *s) {
  (void)hipSetDevice(s->m->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool any_busy = false;
    for (int k = 0; k < s->nlanes; ++k) {
      Lane &L = s->lanes[k];
      if (L.busy && hipEventQuery(L.done_ev) == hipSuccess) lane_complete(s, L);
      any_busy |= L.busy;
    }
    Lane *free_lane = nullptr;
    for (int k = 0; k < s->nlanes; ++k)
      if (!s->lanes[k].busy) {
        free_lane = &s->lanes[k];
        break;
      }
    int64_t c0 = 0, c1 = 0;
    if (free_lane && !s->queue.empty() && take_item(s, *free_lane, c0, c1)) {
      Lane &L = *free_lane;
      L.busy = true;
      s->batches += 1;
      const int64_t atoms = L.chunk_item ? c1 - c0 : [&] {
        int64_t t = 0;
        for (Request *r : L.batch) t += r->n;
        return t;
      }();
      s->max_batch_atoms = std::max(s->max_batch_atoms, atoms);
      lk.unlock();
      L.launch_status = L.chunk_item ? launch_chunk(s, L, L.batch[0], c0, c1) : launch_batch(s, L);
      if (L.launch_status != DP_OK) (void)hipStreamSynchronize(L.st);
      lk.lock();
      if (L.launch_status != DP_OK) lane_complete(s, L);
      continue;
    }
    if (s->stop && s->queue.empty() && !any_busy) break;
    if (any_busy) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      s->cv_work.wait(lk, [&] { return s->stop || !s->queue.empty(); });
    }
  }
}


}  // namespace

extern "C" {

size_t dp_server_footprint(const dp_model *m, int64_t natoms) {
  if (!m || natoms < 1) return 0;
  return (size_t)natoms * bytes_per_atom(m);
}

int dp_server_create(dp_model *m, size_t hbm_budget_bytes, int max_inflight, dp_server **out) {
  if (!m || !out || hbm_budget_bytes == 0 || max_inflight < 1 || max_inflight > MAX_LANES) {
    set_error("dp_server_create: bad argument (max_inflight in 1..8)");
    return DP_ERR_ARG;
  }
  const size_t lane_bytes = (size_t)CHUNK * bytes_per_atom(m);
  if (hbm_budget_bytes < (size_t)max_inflight * lane_bytes) {
    set_error("dp_server_create: the budget does not cover max_inflight batches of " + std::to_string(CHUNK) +
              " atoms");
    return DP_ERR_ARG;
  }
  if (hipSetDevice(m->device) != hipSuccess) {
    set_error("dp_server_create: hipSetDevice failed");
    return DP_ERR_HIP;
  }
  dp_server *s = new dp_server();
  s->m = m;
  s->budget = hbm_budget_bytes;
  s->nlanes = max_inflight;
  // what the lanes leave of the budget holds the workspaces of the large requests in
  // progress (at most max_inflight of them)
  s->big_bytes = hbm_budget_bytes - (size_t)max_inflight * lane_bytes;
  s->max_big_atoms = (int64_t)(s->big_bytes / bytes_per_atom(m));
  s->big.resize(max_inflight);
  for (int k = 0; k < s->nlanes; ++k) {
    Lane &L = s->lanes[k];
    if (hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&L.done_ev, hipEventDisableTiming) != hipSuccess) {
      set_error("dp_server_create: stream or event creation failed");
      dp_server_free(s);
      return DP_ERR_HIP;
    }
  }
  s->worker = std::thread(worker_loop, s);
  *out = s;
  return DP_OK;
}

int dp_submit(dp_server *s, int64_t natoms, const double *coords, const int32_t *types, const double *box,
              uint64_t *request_id) {
  if (!s || natoms < 1 || !coords || !types || !box || !request_id) {
    set_error("dp_submit: bad argument (a periodic box is required)");
    return DP_ERR_ARG;
  }
  if (natoms > CHUNK && natoms > s->max_big_atoms) {
    set_error("dp_submit: the system needs more device memory than the server budget leaves for one request");
    return DP_ERR_TOO_LARGE;
  }
  Grid g;
  int st = make_grid(s->m->rc, s->m->rc, box, g);
  if (st != DP_OK) return st;
  for (int64_t k = 0; k < 3 * natoms; ++k)
    if (!std::isfinite(coords[k])) {
      set_error("dp_submit: non-finite coordinate");
      return DP_ERR_NONFINITE;
    }
  for (int64_t k = 0; k < natoms; ++k)
    if (types[k] < 0 || types[k] >= s->m->ntypes) {
      set_error("dp_submit: atom type outside [0, ntypes)");
      return DP_ERR_TYPE;
    }
  Request *r = new Request();
  r->n = natoms;
  r->chunked = natoms > CHUNK;
  r->X.assign(coords, coords + 3 * natoms);
  r->T.assign(types, types + natoms);
  std::memcpy(r->box, box, 9 * sizeof(double));
  r->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
      delete r;
      set_error("dp_submit: server is shutting down");
      return DP_ERR_ARG;
    }
    r->id = s->next_id++;
    if (!s->have_first) {
      s->have_first = true;
      s->t_first = r->t_submit;
    }
    s->reqs[r->id] = r;
    s->queue.push_back(r);
    *request_id = r->id;
  }
  s->cv_work.notify_all();
  return DP_OK;
}

int dp_wait(dp_server *s, uint64_t id, double timeout_s, double *energy, double *forces, double *virial,
            double *latency_s) {
  if (!s) return DP_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) {
    set_error("dp_wait: unknown request id");
    return DP_ERR_ARG;
  }
  Request *r = it->second;
  const auto pred = [&] { return r->done; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, pred);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    set_error("dp_wait: timed out");
    return DP_ERR_TIMEOUT;
  }
  const int st = r->status;
  if (st >= 0) {
    if (energy) *energy = r->E;
    if (forces) std::memcpy(forces, r->F.data(), 3 * r->n * sizeof(double));
    if (virial) std::memcpy(virial, r->V, 9 * sizeof(double));
  }
  if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
  s->reqs.erase(it);
  delete r;
  return st;
}

int dp_server_stats(dp_server *s, double *p50_s, double *p99_s, double *atom_evals_per_s, int64_t *completed,
                    int64_t *batches, int64_t *max_batch_atoms) {
  if (!s) return DP_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  std::vector<double> v = s->lat;
  std::sort(v.begin(), v.end());
  auto rank = [&](double p) {  // nearest rank
    if (v.empty()) return 0.0;
    size_t k = (size_t)std::ceil(p * v.size());
    k = std::min(std::max<size_t>(k, 1), v.size());
    return v[k - 1];
  };
  if (p50_s) *p50_s = rank(0.50);
  if (p99_s) *p99_s = rank(0.99);
  if (atom_evals_per_s) {
    const double span = s->completed ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0.0;
    *atom_evals_per_s = span > 0 ? s->atoms_done / span : 0.0;
  }
  if (completed) *completed = s->completed;
  if (batches) *batches = s->batches;
  if (max_batch_atoms) *max_batch_atoms = s->max_batch_atoms;
  return DP_OK;
}

void dp_server_free(dp_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->m->device);
  for (int k = 0; k < s->nlanes; ++k) {
    Lane &L = s->lanes[k];
    if (L.st) (void)hipStreamSynchronize(L.st);
    free_ws(L.ws);
    void *d[] = {L.dX, L.dF, L.dE, L.dV, L.dT};
    for (void *p : d)
      if (p) (void)hipFree(p);
    void *h[] = {L.hX, L.hF, L.hE, L.hV, L.hT, L.hflags};
    for (void *p : h)
      if (p) (void)hipHostFree(p);
    if (L.done_ev) (void)hipEventDestroy(L.done_ev);
    if (L.st) (void)hipStreamDestroy(L.st);
  }
  for (BigSlot &b : s->big) free_slot_memory(b);
  for (auto &kv : s->reqs) delete kv.second;
  delete s;
}

}  // extern "C"
