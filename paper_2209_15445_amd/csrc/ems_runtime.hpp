// ems_runtime.hpp -- host runtime internals shared by the C ABI and the
// offload server (not part of the public interface).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/ems.h"
#include "ems_device.hpp"
#include "ems_geometry.hpp"

namespace ems {

hipError_t launch_visit(const KArgs& a, bool photons, uint32_t blocks, hipStream_t s);
hipError_t launch_inject(const KArgs& a, const InjRec* rec, uint32_t n, hipStream_t s);
hipError_t launch_census(const KArgs& a, hipStream_t s);
hipError_t launch_atomic_probe(double* cells, uint64_t n_cells, uint64_t n_ops, hipStream_t s);
hipError_t launch_reset_rows(const KArgs& a, const uint32_t* rows, uint32_t n, hipStream_t s);
hipError_t launch_gather_rows(const KArgs& a, const uint32_t* rows, uint32_t n, char* out, hipStream_t s);
hipError_t visit_occupancy(const KArgs& a, int* per_cu_g, int* per_cu_l, int* per_cu_s);
hipError_t launch_short(const KArgs& a, uint32_t blocks, hipStream_t s);
// primaries in device memory: check pass (chk: first invalid, species
// counts) and stage pass (injection records with ids) of k of them
hipError_t launch_check_primaries(const KArgs& a, const void* p, uint64_t n, unsigned long long* chk, hipStream_t s);
hipError_t launch_stage_primaries(const KArgs& a, const void* p, uint32_t k, const uint32_t* keys,
                                  unsigned long long* row_next, InjRec* out, hipStream_t s);
// zero bytes at p (8-byte aligned) with a kernel on stream s
hipError_t launch_fill_zero(void* p, uint64_t bytes, hipStream_t s);

// a primary as the public header lays it out (64 bytes)
struct PrimRec {
  uint32_t event, species;
  double E, pos[3], dir[3];
};

// workspace regions (byte offsets) and the queue capacity
struct Layout {
  uint64_t ctl, tab, zp, smat, bvh, bleaf, bbox, brec, nbr_off, nbr, mat, elem, edep, ledger, live, rows, gather, exits, profile, log, inj, queues, total;
  uint64_t dkey, drow, dchk;  // device enqueue: event keys, ids per row, check words
  uint64_t squeues;           // short-electron buffers (two of cap_s, spill of cap_p)
  uint64_t cap_s, cap_p;
  uint64_t cap;
  uint32_t inj_chunk;  // primaries staged per injection launch
};

// bytes of one queued track in the configured form
uint64_t queue_track_bytes(const ems_config* c);
// deposit columns of a geometry (slabs, or boxes + world) and the bits of
// the packed queue word that hold the volume
uint32_t n_cols(const ems_geometry* g);
uint32_t vol_bits(const ems_geometry* g);
// entries of the per-face neighbour lists of a box geometry
uint64_t nbr_entries(const ems_geometry* g);
// host view of a box hierarchy
BoxNav host_nav(const ems_geometry* g, const BvhHost& h);

// sets the calling thread's error text and returns code
ems_status fail(ems_status code, const std::string& msg);

}  // namespace ems

struct ems_ctx {
  using TableSet = ems::TableSet;
  using Layout = ems::Layout;
  using KArgs = ems::KArgs;
  using InjRec = ems::InjRec;
  using Ctl = ems::Ctl;
  int device = 0;
  ems_config cfg;
  std::vector<double> z;
  std::vector<uint32_t> smat;   // material per volume
  std::vector<double> blo, bhi;  // box geometry bounds
  ems::BvhHost bvh;
  ems::BoxNav nav{};             // host view of bvh
  uint32_t ncols = 0;            // deposit columns
  std::vector<ems_material> mats;
  ems_geometry geo;
  TableSet ts;
  Layout L;
  char* ws = nullptr;
  hipStream_t stream = nullptr;
  KArgs args{};
  uint32_t blocks_g = 0, blocks_l = 0, blocks_s = 0;
  std::vector<uint64_t> row_count;
  std::vector<uint32_t> keys;  // RNG event key per row (host; travels with each injected track)
  // where the batch's primaries came from since the last reset (0: none,
  // 1: host memory, 2: device memory): the two paths count ids per row in
  // different places (row_count here, the workspace's row counters there)
  uint32_t source = 0;
  bool keys_dirty = true;  // keys changed since their last upload (device enqueues read them there)
  unsigned long long chk_host[4] = {0, 0, 0, 0};
  uint64_t pending[3] = {0, 0, 0};
  InjRec* pin_inj = nullptr;
  Ctl* pin_ctl = nullptr;
  uint32_t* pin_rows = nullptr;  // row lists (server)
  char* pin_gather = nullptr;    // gathered result rows (server)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<hipEvent_t> evk;  // per-launch events (EMS_F_KERNEL_TIMING)
  hipGraphExec_t graph = nullptr;  // captured chunk of graph_k iterations
  uint32_t graph_k = 0;
  bool graph_off = false;  // capture failed once: direct launches
  bool failed = false;
  // created by ems_create_static: the workspace is the library's static
  // device array, host staging is ordinary memory, no events, no graphs
  bool no_alloc = false;
  std::vector<InjRec> host_inj;
  Ctl host_ctl{};
  ems_run_stats stats{};
};

#define HIPCHK(ctx, call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      (ctx)->failed = true;                                                                    \
      return fail(EMS_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));            \
    }                                                                                          \
  } while (0)

namespace ems {
// workspace bytes of (cfg, geo); no_alloc: the layout of a context without
// allocations (smaller injection staging)
ems_status rt_workspace_bytes(const ems_config* cfg, const ems_geometry* geo, bool no_alloc, uint64_t* bytes);
// ems_create, with or without allocations of its own (pinned staging,
// events, graphs); no_alloc refuses EMS_F_KERNEL_TIMING and EMS_F_EVENT_LIVE
ems_status rt_create(const ems_config* cfg, const ems_geometry* geo, void* d_ws, uint64_t bytes, void* stream,
                     bool no_alloc, ems_ctx** out);
// One context at a time may hold a device's static workspace (the
// library's device array behind ems_create_static): rt_hold_static returns
// false while another context holds it; ems_destroy releases it.
constexpr int kMaxStaticDevices = 64;
bool rt_hold_static(int dev);
void rt_release_static(int dev);
// size of the static workspace (one copy per GPU) and the device address of
// device dev's copy, taken once per device with that device current
constexpr uint64_t kStaticWorkspaceBytes = EMS_STATIC_WORKSPACE_BYTES;
hipError_t static_workspace(int dev, void** p);
// validate, prepare and append n primaries to the current queues (all or
// nothing); rows listed in fresh_rows restart their track ids at 0
ems_status rt_enqueue(ems_ctx* c, const ems_primary* p, uint64_t n);
ems_status rt_enqueue_device(ems_ctx* c, const ems_primary* d_primaries, uint64_t n);
// K iterations (after a census of the injected tracks); the status block is
// left in c->pin_ctl; queue errors are returned as status codes
ems_status rt_chunk(ems_ctx* c, uint32_t K);
// zero the deposits, ledgers and live counters of the listed rows and
// restart their track ids (server; needs EMS_F_EVENT_LIVE)
ems_status rt_reset_rows(ems_ctx* c, const uint32_t* rows, uint32_t n);
// copy the deposits and ledgers of the listed rows to the host:
// edep[n][n_slabs], ledger[n] (server; needs EMS_F_EVENT_LIVE)
ems_status rt_gather_rows(ems_ctx* c, const uint32_t* rows, uint32_t n, double* edep, ems_ledger* ledger);
// copy the live-track counters of all rows to host
ems_status rt_read_live(ems_ctx* c, int32_t* host);
// move the outgoing-track records gathered since the last call to the host
// (after a chunk; *total counts all, including those beyond exit_capacity)
// and restart the device list
ems_status rt_take_exits(ems_ctx* c, std::vector<ems_primary>& out, uint64_t* total);
}  // namespace ems
