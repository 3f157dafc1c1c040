// Serving loop support: admission under a device-memory budget and a fixed
// number of concurrent slots, so that requests arriving while others execute
// are admitted as soon as a slot and budget free up and their work overlaps
// on the device (continuous batching). A request runs either as its own
// launch on its slot's stream, or, once the server has started its device
// request ring, as an entry of that ring served by one resident launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hiccl_impl.hpp"

using namespace hiccl;

struct hiccl_server_s {
  struct Req {
    int slot = -1;
    size_t footprint = 0;
    bool launched = false, done = false;
    hipEvent_t start = nullptr, stop = nullptr;
    double device_us = 0;
    hiccl_comm_t comm = nullptr;        // the launched communicator
    int status = HICCL_SUCCESS;         // its run's outcome once done
    uint32_t ring_pos = 0;              // device ring: the request's position
  };
  size_t budget = 0, used = 0;
  std::vector<hipStream_t> streams;
  std::vector<int64_t> slot_owner;     // ticket or -1
  std::unordered_map<uint64_t, Req> reqs;
  uint64_t next = 1;
  int share_grid = 0;                  // workgroups of a request that runs beside others
  DeviceRing* ring = nullptr;          // set: requests go to the device request ring
};

#define HIP_OK(expr, what)                                                         \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) return fail(HICCL_ERR_HIP, std::string(what) + ": " + hipGetErrorString(_e)); \
  } while (0)

static void release(hiccl_server_s* s, uint64_t ticket, hiccl_server_s::Req& r) {
  if (r.slot >= 0 && s->slot_owner[r.slot] == int64_t(ticket)) s->slot_owner[r.slot] = -1;
  s->used -= r.footprint;
  r.footprint = 0;
  r.slot = -1;
}

extern "C" {

int hiccl_server_create(size_t hbm_budget, int slots, hiccl_server_t* out) {
  if (!out || slots < 1 || hbm_budget == 0) return fail(HICCL_ERR_INVALID_ARG, "bad server parameters");
  auto* s = new hiccl_server_s;
  s->budget = hbm_budget;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    cus = 1;
  // concurrent requests share the device: about three workgroups per compute unit in total
  s->share_grid = std::max(1, 3 * cus / slots);
  for (int i = 0; i < slots; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      hiccl_server_destroy(s);
      return fail(HICCL_ERR_HIP, "stream creation failed");
    }
    s->streams.push_back(st);
    s->slot_owner.push_back(-1);
  }
  *out = s;
  return HICCL_SUCCESS;
}

int hiccl_server_admit(hiccl_server_t s, size_t footprint, uint64_t* ticket) {
  if (!s || !ticket) return fail(HICCL_ERR_INVALID_ARG, "NULL argument");
  if (footprint > s->budget) return fail(HICCL_ERR_INVALID_ARG, "request footprint exceeds the whole budget");
  if (s->used + footprint > s->budget) return fail(HICCL_ERR_BUSY, "not enough budget free");
  int slot = -1;
  for (size_t i = 0; i < s->slot_owner.size(); ++i)
    if (s->slot_owner[i] < 0) {
      slot = int(i);
      break;
    }
  if (slot < 0) return fail(HICCL_ERR_BUSY, "no slot free");
  uint64_t t = s->next++;
  hiccl_server_s::Req r;
  r.slot = slot;
  r.footprint = footprint;
  s->slot_owner[slot] = int64_t(t);
  s->used += footprint;
  s->reqs[t] = r;
  *ticket = t;
  return HICCL_SUCCESS;
}

int hiccl_server_stream(hiccl_server_t s, uint64_t ticket, void** stream) {
  if (!s || !stream) return fail(HICCL_ERR_INVALID_ARG, "NULL argument");
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second.slot < 0) return fail(HICCL_ERR_INVALID_ARG, "unknown or finished ticket");
  *stream = s->streams[it->second.slot];
  return HICCL_SUCCESS;
}

int hiccl_server_launch(hiccl_server_t s, uint64_t ticket, hiccl_comm_t comm) {
  if (!s || !comm) return fail(HICCL_ERR_INVALID_ARG, "NULL argument");
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || it->second.slot < 0 || it->second.launched)
    return fail(HICCL_ERR_STATE, "ticket is not admitted or already launched");
  auto& r = it->second;
  hipStream_t st = s->streams[r.slot];
  // a request that starts while others run gets a share of the device; one
  // that starts alone gets the executor's full default grid
  if (int rc = hiccl_server_progress(s)) return rc;
  int running = 0;
  for (const auto& kv : s->reqs) running += kv.second.launched && !kv.second.done;
  if (int rc = hiccl_set_grid(comm, running ? s->share_grid : 0)) return rc;
  // a launch that fails releases its ticket (slot and budget), so the caller can admit again
  auto give_up = [&](int rc) {
    if (r.start) (void)hipEventDestroy(r.start);
    if (r.stop) (void)hipEventDestroy(r.stop);
    r.start = r.stop = nullptr;
    release(s, ticket, r);
    s->reqs.erase(it);
    return rc;
  };
  if (s->ring) {
    if (int rc = ring_push(s->ring, comm->c, &r.ring_pos)) return give_up(rc);
    r.launched = true;
    r.comm = comm;
    return HICCL_SUCCESS;
  }
  if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess ||
      hipEventRecord(r.start, st) != hipSuccess)
    return give_up(fail(HICCL_ERR_HIP, "request events"));
  // with several slots any request may come to share the device with others while it runs, so the
  // persistent executor claims from one tile queue: progress then holds however many of its
  // workgroups are resident (the communicator's own claim setting is left as it was)
  const int rc = s->streams.size() > 1 ? run_one_queue(comm, st) : hiccl_run(comm, st);
  if (rc) return give_up(rc);
  if (hipEventRecord(r.stop, st) != hipSuccess) return give_up(fail(HICCL_ERR_HIP, "request event record"));
  r.launched = true;
  r.comm = comm;
  return HICCL_SUCCESS;
}

int hiccl_server_submit(hiccl_server_t s, hiccl_comm_t comm, uint64_t* ticket) {
  if (!s || !comm || !ticket) return fail(HICCL_ERR_INVALID_ARG, "NULL argument");
  if (!comm->c.planned) return fail(HICCL_ERR_STATE, "call hiccl_init before submitting");
  uint64_t t = 0;
  if (int rc = hiccl_server_admit(s, size_t(comm_footprint(comm->c)), &t)) return rc;
  if (int rc = hiccl_server_launch(s, t, comm)) return rc;   // a failed launch releases the ticket
  *ticket = t;
  return HICCL_SUCCESS;
}

int hiccl_server_progress(hiccl_server_t s) {
  if (!s) return fail(HICCL_ERR_INVALID_ARG, "NULL server");
  for (auto& kv : s->reqs) {
    auto& r = kv.second;
    if (!r.launched || r.done) continue;
    if (s->ring) {
      int done = 0, aborted = 0;
      if (int rc = ring_check(s->ring, r.ring_pos, &done, &aborted)) return rc;
      if (!done) continue;
      r.status = aborted ? HICCL_ERR_TIMEOUT : HICCL_SUCCESS;
      r.done = true;
      release(s, kv.first, r);
      continue;
    }
    hipError_t q = hipEventQuery(r.stop);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return fail(HICCL_ERR_HIP, std::string("request failed: ") + hipGetErrorString(q));
    float ms = 0;
    if (hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) r.device_us = ms * 1e3;
    r.status = hiccl_wait(r.comm);      // finished: reads the run's status (TIMEOUT if a wait expired)
    r.done = true;
    release(s, kv.first, r);
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
    r.start = r.stop = nullptr;
  }
  return HICCL_SUCCESS;
}

int hiccl_server_poll(hiccl_server_t s, uint64_t ticket, int* done, double* device_us) {
  if (!s) return fail(HICCL_ERR_INVALID_ARG, "NULL server");
  if (int rc = hiccl_server_progress(s)) return rc;
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(HICCL_ERR_INVALID_ARG, "unknown ticket");
  if (done) *done = it->second.done ? 1 : 0;
  if (device_us) *device_us = it->second.device_us;
  int rc = HICCL_SUCCESS;
  if (it->second.done) {
    rc = it->second.status;
    s->reqs.erase(it);
    if (rc) return fail(rc, "the request's executor gave up a dependency wait (spin limit reached)");
  }
  return rc;
}

int hiccl_server_drain(hiccl_server_t s) {
  if (!s) return fail(HICCL_ERR_INVALID_ARG, "NULL server");
  for (hipStream_t st : s->streams) HIP_OK(hipStreamSynchronize(st), "stream sync");
  if (!s->ring) return hiccl_server_progress(s);
  // ring requests: poll their completion words (a dependency wait is bounded, so they finish)
  for (int i = 0;; ++i) {
    if (int rc = hiccl_server_progress(s)) return rc;
    bool pending = false;
    for (const auto& kv : s->reqs) pending |= kv.second.launched && !kv.second.done;
    if (!pending) return HICCL_SUCCESS;
    if (i >= 600000) return fail(HICCL_ERR_TIMEOUT, "ring requests did not complete within 60 s");
    std::this_thread::sleep_for(std::chrono::microseconds(100));
  }
}

int hiccl_server_start_ring(hiccl_server_t s, int grid, int idle_ms) {
  if (!s) return fail(HICCL_ERR_INVALID_ARG, "NULL server");
  if (grid < 0 || grid == 1 || idle_ms < 1 || idle_ms > 60000)
    return fail(HICCL_ERR_INVALID_ARG, "ring grid must be 0 or >= 2, idle time 1..60000 ms");
  if (s->ring) return fail(HICCL_ERR_STATE, "the device ring is already started");
  for (const auto& kv : s->reqs)
    if (kv.second.launched && !kv.second.done) return fail(HICCL_ERR_STATE, "requests are in flight");
  return ring_create(grid, uint32_t(idle_ms), 4096, &s->ring);
}

int hiccl_server_usage(hiccl_server_t s, size_t* used_bytes, int* running) {
  if (!s) return fail(HICCL_ERR_INVALID_ARG, "NULL server");
  if (used_bytes) *used_bytes = s->used;
  if (running) {
    int n = 0;
    for (int64_t o : s->slot_owner) n += o >= 0;
    *running = n;
  }
  return HICCL_SUCCESS;
}

int hiccl_server_destroy(hiccl_server_t s) {
  if (!s) return HICCL_SUCCESS;
  if (s->ring) {
    if (int rc = ring_destroy(s->ring)) return rc;   // the resident kernel did not stop: keep everything
    s->ring = nullptr;
  }
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (auto& kv : s->reqs) {
    if (kv.second.start) (void)hipEventDestroy(kv.second.start);
    if (kv.second.stop) (void)hipEventDestroy(kv.second.stop);
  }
  delete s;
  return HICCL_SUCCESS;
}

}  // extern "C"
