// lk_server.hip -- continuous-batching verification server (include/lk.h).
//
// Requests (one timestep of a session's geometry each) wait in a FIFO queue.
// Every slot owns an lk_ctx, a HIP stream and a host thread; a free slot takes
// the queue head as soon as the device-memory budget has room for it, so
// requests that arrive while others run are admitted as slots and memory free
// up, and their kernels share the device concurrently.  A request runs
//   potential link search -> direct sum -> verify against the session's
//   resident expected matrix,
// with its device buffers from the stream-ordered allocator (no device-wide
// synchronisation when they come and go).  Large requests cap their
// persistent grid at three quarters of the resident waves and small ones at a
// quarter, so a large job never blocks the device for the small ones behind it.
//
// Memory admission: a request is charged its own buffers for a first guess of
// its pair count, and its slot the workspace its context would grow to
// (pair search, direct sum, verification, and the Barnes-Hut trees or
// crossing-count boxes of the mode); sessions are charged their resident
// arrays.  Once the request's pairs are counted the charge is corrected,
// waiting for memory if it grew, and after the request the slot's real
// workspace replaces the estimate.  The workspace reserved when the server is
// created lies outside the budget.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/lk.h"
#include "lk_internal.h"

namespace {

constexpr double kBigTerms = 1.0e9;  // requests above this many terms count as large
// A large request's direct sum runs as consecutive calls over runs of its
// pair list of at most this many terms (about 11 ms of the device each):
// between two of them the other slots' kernels get the compute units,
// so a small request never waits for a whole large one.  A pair's value does
// not depend on the run it is in (its lane layout depends only on its own
// sizes and the run's pair count, which depends only on the request).
constexpr double kRunTerms = 1.0e10;

struct Session {
  int32_t n_loops = 0;
  int64_t n_vert = 0;
  std::vector<int64_t> off;  // host copy of the offsets (work estimates)
  int64_t* d_off = nullptr;
  int32_t* d_exp_pairs = nullptr;
  int32_t* d_exp_lk = nullptr;
  int64_t n_exp = 0;
  int64_t bytes = 0;
  int64_t refs = 0;     // queued or running requests
  bool closing = false;
};

struct Request {
  int64_t id = 0;
  int64_t session = 0;
  const void* xyz = nullptr;
  int dtype = LK_F32;
  int where = LK_MEM_HOST;
  int64_t bytes = 0;  // budget charge
  lk_result res{};
  std::vector<int32_t> pairs, lk, mism;
  std::vector<double> real;
  bool done = false;
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct lk_server {
  int device = 0;
  int mode = LK_MIXED;
  int64_t budget = 0;
  // bytes charged against the budget: sessions, admitted requests, and the
  // slots' workspace growth beyond what the server reserved at creation
  int64_t in_use = 0;
  int running = 0;  // admitted requests not yet finished
  int waiting = 0;  // of those, waiting for memory after their pair count came in
  int32_t max_loops = 0;
  int64_t max_pairs = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> pending;
  std::unordered_map<int64_t, std::shared_ptr<Request>> requests;
  std::unordered_map<int64_t, Session> sessions;
  int64_t next_id = 1, next_session = 1;
  bool stopping = false;
  std::string err;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  struct Slot {
    lk_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    std::thread th;
    int64_t ws_base = 0;     // workspace reserved at creation (outside the budget)
    int64_t ws_charged = 0;  // growth beyond ws_base, charged to in_use
    int64_t last_session = 0;
  };
  std::vector<Slot> slots;

  lk_status fail(lk_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return st;
  }
};

namespace {

size_t dtype_size(int dtype) { return dtype == LK_F64 ? 8 : 4; }

// First guess of a request's candidate pairs (corrected once they are counted).
int64_t guess_pairs(const lk_server* srv, const Session& S) {
  int64_t pairs = 16 * (int64_t)S.n_loops;
  return pairs > srv->max_pairs ? srv->max_pairs : pairs;
}

// Device bytes of a request's own buffers for `pairs` candidate pairs: the
// geometry copy (host input), pairs, values, integers, flags and mismatch
// records (as run_request allocates them).
int64_t request_bytes(const Session& S, int dtype, int where, int64_t pairs) {
  int64_t b = 0;
  if (where == LK_MEM_HOST) b += S.n_vert * 3 * (int64_t)dtype_size(dtype);
  return b + pairs * (8 + 8 + 4 + 4) + 16 * (pairs + S.n_exp) + 64;
}

// Workspace growth a slot's context may need for a request with `pairs`
// pairs beyond what it already holds (charged when the request is admitted).
int64_t workspace_extra(const lk_server* srv, const lk_server::Slot& slot, const Session& S,
                        int64_t pairs) {
  const int64_t need =
      lk::ctx_workspace_need(srv->mode, S.n_loops, pairs, S.n_vert, pairs + S.n_exp);
  const int64_t have = slot.ws_base + slot.ws_charged;
  return need > have ? need - have : 0;
}

// Charge `delta` more bytes (negative: release).  A request whose real size
// came out larger than its charge waits until the others have freed enough,
// unless every other running request is waiting too (then it goes over the
// budget rather than deadlock).  Called with the lock held.
void recharge(lk_server* srv, std::unique_lock<std::mutex>& lock, int64_t delta) {
  if (delta > 0 && srv->in_use + delta > srv->budget) {
    ++srv->waiting;
    srv->cv_done.notify_all();  // other waiters re-check whether everyone waits
    srv->cv_done.wait(lock, [&] {
      return srv->in_use + delta <= srv->budget || srv->running - srv->waiting <= 0;
    });
    --srv->waiting;
  }
  srv->in_use += delta;
}

// Run one request on a slot (called without the server lock held).
void run_request(lk_server* srv, lk_server::Slot& slot, Request& R, const Session& S) {
  lk_ctx* ctx = slot.ctx;
  hipStream_t st = slot.stream;
  lk_result& res = R.res;
  auto failed = [&](int status) {
    res.status = status;
    return;
  };
  (void)hipSetDevice(srv->device);
  if (slot.last_session != R.session) {
    // another session's offsets may sit at a freed session's address: the
    // context must not reuse the vertex count it cached for that address
    lk::ctx_forget_offsets(ctx);
    slot.last_session = R.session;
  }
  void* xyz = const_cast<void*>(R.xyz);
  void* xyz_copy = nullptr;
  const size_t xyz_bytes = (size_t)S.n_vert * 3 * dtype_size(R.dtype);
  if (R.where == LK_MEM_HOST) {
    if (hipMallocAsync(&xyz_copy, xyz_bytes ? xyz_bytes : 8, st) != hipSuccess)
      return failed(LK_ENOMEM);
    if (hipMemcpyAsync(xyz_copy, R.xyz, xyz_bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
      hipFreeAsync(xyz_copy, st);
      return failed(LK_EDEVICE);
    }
    xyz = xyz_copy;
  }
  int64_t n = 0;
  lk_status s = lk_build_pairs(ctx, xyz, R.dtype, S.d_off, S.n_loops, nullptr, 0, &n, st);
  if (s != LK_OK && s != LK_ECAPACITY) {
    if (xyz_copy) hipFreeAsync(xyz_copy, st);
    return failed(s);
  }
  if (n > srv->max_pairs) {
    if (xyz_copy) hipFreeAsync(xyz_copy, st);
    return failed(LK_ECAPACITY);
  }
  {
    // the charge made on admission guessed the pair count: correct it, for
    // the request's buffers and for the workspace its context grows to
    std::unique_lock<std::mutex> lock(srv->mu);
    const int64_t real = request_bytes(S, R.dtype, R.where, n);
    const int64_t ws = workspace_extra(srv, slot, S, n);
    recharge(srv, lock, (real - R.bytes) + ws);
    R.bytes = real;
    slot.ws_charged += ws;
  }
  const int64_t cap_m = n + S.n_exp;
  char* buf = nullptr;
  const size_t bytes = (size_t)n * (8 + 8 + 4 + 4) + (size_t)cap_m * 16 + 64;
  if (hipMallocAsync((void**)&buf, bytes, st) != hipSuccess) {
    if (xyz_copy) hipFreeAsync(xyz_copy, st);
    return failed(LK_ENOMEM);
  }
  int32_t* d_pairs = (int32_t*)buf;
  double* d_real = (double*)(buf + 8 * (size_t)n);
  int32_t* d_lk = (int32_t*)(buf + 16 * (size_t)n);
  uint32_t* d_flags = (uint32_t*)(buf + 20 * (size_t)n);
  int32_t* d_mism = (int32_t*)(buf + 24 * (size_t)n);
  int64_t n2 = 0, n_mis = 0;
  R.pairs.resize((size_t)n * 2);
  R.lk.resize((size_t)n);
  R.real.resize((size_t)n);
  std::vector<uint32_t> flags((size_t)n);
  s = lk_build_pairs(ctx, xyz, R.dtype, S.d_off, S.n_loops, d_pairs, n, &n2, st);
  if (s == LK_OK && n > 0) {
    // work estimate on the host: terms = sum of N_a N_b over the pairs
    if (hipMemcpyAsync(R.pairs.data(), d_pairs, 8 * (size_t)n, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      s = LK_EDEVICE;
    double terms = 0.0;
    for (int64_t q = 0; q < n; ++q) {
      const int32_t i = R.pairs[2 * q], j = R.pairs[2 * q + 1];
      terms += (double)(S.off[i + 1] - S.off[i]) * (double)(S.off[j + 1] - S.off[j]);
    }
    res.terms = terms;
    if (s == LK_OK) s = lk_set_option(ctx, LK_OPT_WAVES_PER_CU, terms >= kBigTerms ? 12 : 4);
    // runs of at most kRunTerms terms (a single larger pair is a run alone)
    int64_t q0 = 0;
    while (s == LK_OK && q0 < n) {
      int64_t q1 = q0;
      double run = 0.0;
      while (q1 < n) {
        const int32_t i = R.pairs[2 * q1], j = R.pairs[2 * q1 + 1];
        const double t = (double)(S.off[i + 1] - S.off[i]) * (double)(S.off[j + 1] - S.off[j]);
        if (q1 > q0 && run + t > kRunTerms) break;
        run += t;
        ++q1;
      }
      s = lk_direct_sum(ctx, xyz, R.dtype, S.d_off, S.n_loops, d_pairs + 2 * q0, q1 - q0,
                        srv->mode, d_real + q0, d_lk + q0, d_flags + q0, st);
      q0 = q1;
    }
  }
  if (s == LK_OK)
    s = lk_verify(ctx, d_pairs, d_lk, n, S.d_exp_pairs, S.d_exp_lk, S.n_exp, 0, &n_mis, d_mism,
                  cap_m, st);
  if (s == LK_OK && n > 0) {
    if (hipMemcpyAsync(R.lk.data(), d_lk, 4 * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(R.real.data(), d_real, 8 * (size_t)n, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(flags.data(), d_flags, 4 * (size_t)n, hipMemcpyDeviceToHost, st) !=
            hipSuccess)
      s = LK_EDEVICE;
  }
  const int64_t n_rec = n_mis < cap_m ? n_mis : cap_m;
  R.mism.resize((size_t)n_rec * 4);
  if (s == LK_OK && n_rec > 0 &&
      hipMemcpyAsync(R.mism.data(), d_mism, 16 * (size_t)n_rec, hipMemcpyDeviceToHost, st) !=
          hipSuccess)
    s = LK_EDEVICE;
  if (hipStreamSynchronize(st) != hipSuccess && s == LK_OK) s = LK_EDEVICE;
  hipFreeAsync(buf, st);
  if (xyz_copy) hipFreeAsync(xyz_copy, st);
  int64_t flagged = 0, refits = 0;
  for (uint32_t f : flags) {
    if (f & (LK_FLAG_NONFINITE | LK_FLAG_BADPAIR | LK_FLAG_BADLOOP | LK_FLAG_AMBIGUOUS)) ++flagged;
    if (f & LK_FLAG_REFIT) ++refits;
  }
  res.refits = refits;
  res.n_pairs = n;
  res.n_mismatch = n_mis;
  res.n_flagged = flagged;
  res.status = s;
}

void slot_loop(lk_server* srv, int index) {
  lk_server::Slot& slot = srv->slots[index];
  hipSetDevice(srv->device);
  for (;;) {
    std::shared_ptr<Request> R;
    Session S;
    {
      std::unique_lock<std::mutex> lock(srv->mu);
      int64_t extra = 0;
      srv->cv_work.wait(lock, [&] {
        if (srv->pending.empty()) return srv->stopping;
        const auto& head = srv->pending.front();
        const Session& hs = srv->sessions[head->session];
        extra = workspace_extra(srv, slot, hs, guess_pairs(srv, hs));
        return srv->in_use + head->bytes + extra <= srv->budget || srv->running == 0;
      });
      if (srv->pending.empty()) return;  // stopping and drained
      R = srv->pending.front();
      srv->pending.pop_front();
      srv->in_use += R->bytes + extra;
      slot.ws_charged += extra;
      ++srv->running;
      R->res.t_admit = now_s(srv->t0);
      R->res.slot = index;
      S = srv->sessions[R->session];  // copy of the descriptor (device pointers stay valid)
    }
    run_request(srv, slot, *R, S);
    // the workspace the context really holds now (it only grows)
    const int64_t grown = lk::ctx_workspace_bytes(slot.ctx) - slot.ws_base;
    {
      std::lock_guard<std::mutex> lock(srv->mu);
      srv->in_use += grown - slot.ws_charged;
      slot.ws_charged = grown;
      --srv->running;
      srv->in_use -= R->bytes;
      R->res.bytes = R->bytes;
      R->res.t_done = now_s(srv->t0);
      R->done = true;
      Session& live = srv->sessions[R->session];
      if (--live.refs == 0 && live.closing) {
        hipFree(live.d_off);
        hipFree(live.d_exp_pairs);
        hipFree(live.d_exp_lk);
        srv->in_use -= live.bytes;
        srv->sessions.erase(R->session);
      }
    }
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

lk_status lk_server_create(lk_server** out, int device, int32_t slots, int64_t mem_budget,
                           int mode, int32_t max_loops, int64_t max_pairs) {
  if (!out || slots < 1 || slots > 8 || mem_budget < 0 || max_loops < 1 || max_pairs < 1 ||
      (mode != LK_MIXED && mode != LK_PLAIN_F64 && mode != LK_CROSSINGS && mode != LK_BARNES_HUT))
    return LK_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return LK_EDEVICE;
  auto* srv = new (std::nothrow) lk_server();
  if (!srv) return LK_ENOMEM;
  srv->device = device;
  srv->mode = mode;
  srv->max_loops = max_loops;
  srv->max_pairs = max_pairs;
  if (mem_budget == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete srv;
      return LK_EDEVICE;
    }
    mem_budget = (int64_t)(0.8 * (double)fr);
  }
  srv->budget = mem_budget;
  srv->slots.resize((size_t)slots);
  for (auto& sl : srv->slots) {
    lk_status st = lk_create(&sl.ctx, device);
    if (st == LK_OK) st = lk_set_option(sl.ctx, LK_OPT_GRAPH, 0);
    if (st == LK_OK) st = lk_reserve(sl.ctx, max_loops, max_pairs, 2 * max_pairs + max_loops);
    if (st == LK_OK && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
      st = LK_EDEVICE;
    if (st == LK_OK) sl.ws_base = lk::ctx_workspace_bytes(sl.ctx);
    if (st != LK_OK) {
      for (auto& s2 : srv->slots) {
        if (s2.ctx) lk_destroy(s2.ctx);
        if (s2.stream) hipStreamDestroy(s2.stream);
      }
      delete srv;
      return st;
    }
  }
  for (int k = 0; k < slots; ++k) srv->slots[k].th = std::thread(slot_loop, srv, k);
  *out = srv;
  return LK_OK;
}

void lk_server_destroy(lk_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    srv->stopping = true;
  }
  srv->cv_work.notify_all();
  for (auto& sl : srv->slots)
    if (sl.th.joinable()) sl.th.join();
  hipSetDevice(srv->device);
  for (auto& sl : srv->slots) {
    if (sl.stream) hipStreamSynchronize(sl.stream);
    if (sl.ctx) lk_destroy(sl.ctx);
    if (sl.stream) hipStreamDestroy(sl.stream);
  }
  for (auto& kv : srv->sessions) {
    hipFree(kv.second.d_off);
    hipFree(kv.second.d_exp_pairs);
    hipFree(kv.second.d_exp_lk);
  }
  delete srv;
}

const char* lk_server_last_error(const lk_server* srv) {
  return srv ? srv->err.c_str() : "null server";
}

lk_status lk_server_open_session(lk_server* srv, const int64_t* off, int32_t n_loops,
                                 const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp,
                                 int64_t* session) {
  if (!srv) return LK_EINVAL;
  if (!off || !session || n_loops < 1 || n_exp < 0 || (n_exp > 0 && (!exp_pairs || !exp_lk)))
    return srv->fail(LK_EINVAL, "bad session arguments");
  if (n_loops > srv->max_loops)
    return srv->fail(LK_ECAPACITY, "%d loops exceed the server's %d", n_loops, srv->max_loops);
  Session S;
  S.n_loops = n_loops;
  S.off.assign(off, off + n_loops + 1);
  S.n_vert = off[n_loops] - off[0];
  S.n_exp = n_exp;
  S.bytes = 8 * (int64_t)(n_loops + 1) + 12 * n_exp + 16;
  hipSetDevice(srv->device);
  if (hipMalloc(&S.d_off, 8 * (size_t)(n_loops + 1)) != hipSuccess ||
      hipMalloc(&S.d_exp_pairs, 8 * (size_t)(n_exp > 0 ? n_exp : 1)) != hipSuccess ||
      hipMalloc(&S.d_exp_lk, 4 * (size_t)(n_exp > 0 ? n_exp : 1)) != hipSuccess) {
    hipFree(S.d_off);
    hipFree(S.d_exp_pairs);
    hipFree(S.d_exp_lk);
    return srv->fail(LK_ENOMEM, "session allocation failed");
  }
  if (hipMemcpy(S.d_off, off, 8 * (size_t)(n_loops + 1), hipMemcpyHostToDevice) != hipSuccess ||
      (n_exp > 0 &&
       (hipMemcpy(S.d_exp_pairs, exp_pairs, 8 * (size_t)n_exp, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(S.d_exp_lk, exp_lk, 4 * (size_t)n_exp, hipMemcpyHostToDevice) != hipSuccess))) {
    hipFree(S.d_off);
    hipFree(S.d_exp_pairs);
    hipFree(S.d_exp_lk);
    return srv->fail(LK_EDEVICE, "session upload failed");
  }
  std::lock_guard<std::mutex> lock(srv->mu);
  const int64_t id = srv->next_session++;
  srv->in_use += S.bytes;
  srv->sessions[id] = std::move(S);
  *session = id;
  return LK_OK;
}

lk_status lk_server_close_session(lk_server* srv, int64_t session) {
  if (!srv) return LK_EINVAL;
  std::lock_guard<std::mutex> lock(srv->mu);
  auto it = srv->sessions.find(session);
  if (it == srv->sessions.end() || it->second.closing)
    return srv->fail(LK_ENOTFOUND, "no session %lld", (long long)session);
  it->second.closing = true;
  if (it->second.refs == 0) {
    hipSetDevice(srv->device);
    hipFree(it->second.d_off);
    hipFree(it->second.d_exp_pairs);
    hipFree(it->second.d_exp_lk);
    srv->in_use -= it->second.bytes;
    srv->sessions.erase(it);
  }
  return LK_OK;
}

lk_status lk_server_submit(lk_server* srv, int64_t session, const void* xyz, int dtype, int where,
                           int64_t* request_id) {
  if (!srv) return LK_EINVAL;
  if (!xyz || !request_id || (dtype != LK_F32 && dtype != LK_F64) ||
      (where != LK_MEM_HOST && where != LK_MEM_DEVICE))
    return srv->fail(LK_EINVAL, "bad submit arguments");
  auto R = std::make_shared<Request>();
  {
    std::lock_guard<std::mutex> lock(srv->mu);
    if (srv->stopping) return srv->fail(LK_EBUSY, "server is stopping");
    auto it = srv->sessions.find(session);
    if (it == srv->sessions.end() || it->second.closing)
      return srv->fail(LK_ENOTFOUND, "no session %lld", (long long)session);
    R->id = srv->next_id++;
    R->session = session;
    R->xyz = xyz;
    R->dtype = dtype;
    R->where = where;
    R->bytes = request_bytes(it->second, dtype, where, guess_pairs(srv, it->second));
    if (R->bytes > srv->budget)
      return srv->fail(LK_ECAPACITY, "request needs %lld bytes, budget %lld",
                       (long long)R->bytes, (long long)srv->budget);
    R->res.id = R->id;
    R->res.t_submit = now_s(srv->t0);
    it->second.refs++;
    srv->requests[R->id] = R;
    srv->pending.push_back(R);
    *request_id = R->id;
  }
  srv->cv_work.notify_all();
  return LK_OK;
}

lk_status lk_server_wait(lk_server* srv, int64_t id, int32_t timeout_ms, lk_result* res,
                         int32_t* pairs_out, int32_t* lk_out, double* real_out,
                         int32_t* mism_out, int64_t cap) {
  if (!srv) return LK_EINVAL;
  std::unique_lock<std::mutex> lock(srv->mu);
  auto it = srv->requests.find(id);
  if (it == srv->requests.end()) return srv->fail(LK_ENOTFOUND, "no request %lld", (long long)id);
  std::shared_ptr<Request> R = it->second;
  auto ready = [&] { return R->done; };
  if (timeout_ms < 0)
    srv->cv_done.wait(lock, ready);
  else if (!srv->cv_done.wait_for(lock, std::chrono::milliseconds(timeout_ms), ready))
    return LK_EBUSY;
  if (res) *res = R->res;
  const int64_t n = (int64_t)R->lk.size();
  const int64_t k = cap < n ? cap : n;
  if (pairs_out && k > 0) memcpy(pairs_out, R->pairs.data(), 8 * (size_t)k);
  if (lk_out && k > 0) memcpy(lk_out, R->lk.data(), 4 * (size_t)k);
  if (real_out && k > 0) memcpy(real_out, R->real.data(), 8 * (size_t)k);
  const int64_t nm = (int64_t)R->mism.size() / 4;
  const int64_t km = cap < nm ? cap : nm;
  if (mism_out && km > 0) memcpy(mism_out, R->mism.data(), 16 * (size_t)km);
  srv->requests.erase(it);
  return LK_OK;
}

}  // extern "C"
