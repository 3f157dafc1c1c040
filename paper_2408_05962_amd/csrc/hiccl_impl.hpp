// Internal data structures of the hierarchical collective executor.
//
// Host side (plan.cpp): registration, race checking, factorization,
// channel split, dependency DAG, ordering, tiling, byte accounting, and a
// host-memory schedule checker. Device side (device.hip): the task-table
// upload and the copy / fused-reduce / persistent executor kernels.
#pragma once

#include <cstdint>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hiccl.h"

namespace hiccl {

constexpr int kCopy = 0;
constexpr int kReduce = 1;
constexpr int kFp8Block = 256;

// Element size in bytes of a payload type.
inline size_t elem_size(int dt) {
  switch (dt) {
    case HICCL_INT32:
    case HICCL_FLOAT32: return 4;
    case HICCL_BFLOAT16: return 2;
    case HICCL_FP8_E4M3: return 1;
  }
  return 0;
}

// Granularity (elements) of stripe / channel / tile boundaries: whole
// 16-byte vectors, and whole scale blocks for fp8.
inline size_t align_elems(int dt) {
  return dt == HICCL_FP8_E4M3 ? size_t(kFp8Block) : 16 / elem_size(dt);
}

// A location: element 0 of an operand range. Space 0 = caller memory
// (absolute byte address), space 1 = library workspace (byte offset).
struct Loc {
  int space = 0;
  uint64_t addr = 0;     // data byte address / offset of element 0
  uint64_t scales = 0;   // fp8: address / offset of element 0's block scale
  Loc at(uint64_t elems, int dt) const {
    Loc l = *this;
    l.addr += elems * elem_size(dt);
    if (dt == HICCL_FP8_E4M3) l.scales += (elems / kFp8Block) * sizeof(float);
    return l;
  }
};

struct Prim {
  int kind = 0;                  // 0 multicast, 1 reduction
  int root = 0;
  std::vector<int> leaves;
  std::vector<hiccl_buf_t> send, recv;   // nranks entries
  size_t count = 0;
  int op = HICCL_SUM;
  int step = 0;
};

// One factorized transfer or reduction node of one branch (stripe), before
// the channel split.
struct Op {
  int kind = kCopy;
  std::vector<Loc> src;
  std::vector<int> src_rank;
  Loc dst;
  int dst_rank = 0;
  bool dst_ws = false;
  uint64_t count = 0;            // elements of the branch
  uint64_t offset = 0;           // element offset of the branch in the primitive
  int stripe = 0;
  int ring_step = 0;
  bool whole = false;            // spans the primitive (local root copy), split on its own
};

struct Task {
  int kind = kCopy;
  int op = HICCL_SUM;
  int dtype = HICCL_FLOAT32;
  std::vector<Loc> src;
  std::vector<int> src_rank;
  Loc dst;
  int dst_rank = 0;
  bool dst_ws = false;
  uint64_t count = 0;
  uint64_t offset = 0;
  int prim = 0, step = 0, stripe = 0, channel = 0, ring_step = 0;
  int comm = 0;                  // index of the communicator inside a merged batch
  std::vector<int> preds, succs;
  int stage = 0;
  uint64_t tile_elems = 0;
  uint32_t first_tile = 0, ntiles = 0;
};

struct Plan {
  std::vector<Task> tasks;       // claim order
  std::vector<uint32_t> tile_task;
  std::vector<uint32_t> stage_tile_begin;   // per stage, first tile (stage order only), plus an end entry
  uint64_t ws_bytes = 0;
  uint64_t nedges = 0;
  int nstages = 0;
  uint64_t hbm_read = 0, hbm_written = 0;
};

struct ExecCfg {
  int mode = HICCL_EXEC_PERSISTENT;
  size_t tile_bytes = 64 * 1024;
  int grid = 0;
  int order = HICCL_ORDER_STAGE;
  uint32_t spin_limit = 1u << 22;
  int queues = 8;
  int batch = 4;
  bool trace = false;            // persistent executor: stamp each task's start and end (hiccl_set_trace)
};

struct DeviceState;              // device.hip
void device_state_free(DeviceState*);
void device_state_set_spin_limit(DeviceState*, uint32_t polls);   // takes effect on the next run
struct StaticState;              // device.hip: host image of the tables for hiccl_run_static
void static_state_free(StaticState*);

struct Comm {
  int P = 1;
  int dtype = HICCL_FLOAT32;
  std::vector<Prim> prims;
  int step = 0;
  std::vector<int> hier;
  int stripe = 1, ring = 1, pipe = 1;
  int share = -1;                // plan only this rank's tasks (-1: all)
  ExecCfg exec;
  bool planned = false;
  Plan plan;
  void* user_ws = nullptr;
  size_t user_ws_bytes = 0;
  DeviceState* dev = nullptr;
  StaticState* stat = nullptr;
  bool last_static = false;      // the latest run was hiccl_run_static (hiccl_wait follows it)
  ~Comm() {
    if (dev) device_state_free(dev);
    if (stat) static_state_free(stat);
  }
};

// ------------------------------------------------------------ error helpers
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

// Device request ring of the serving form (device.hip). A resident launch
// serves appended requests in order; positions count appended requests.
struct DeviceRing;
int ring_create(int grid, uint32_t idle_ms, uint32_t cap, DeviceRing** out);
int ring_push(DeviceRing* r, Comm& c, uint32_t* pos);
int ring_check(DeviceRing* r, uint32_t pos, int* done, int* aborted);
int ring_destroy(DeviceRing* r);

// plan.cpp
int build_plan(Comm& c);
void order_and_tile(Plan& p, int order, size_t tile_bytes);
uint64_t tile_elems_for(size_t tile_bytes, int dtype);
int hier_depth(int a, int b, const std::vector<int>& h);
uint64_t comm_footprint(const Comm& c);
int run_one_queue(hiccl_comm_t comm, void* stream);   // device.hip
int batch_members_disjoint(const std::vector<const Comm*>& comms);

}  // namespace hiccl

struct hiccl_comm_s {
  hiccl::Comm c;
};
