// ems_api.cpp -- host runtime and C ABI of the transport library.
//
// Host side of the paper's stepping workflow (section 3) and of its
// hybrid-integration contract (section 4): tracks come in, the population is
// stepped on the GPU until it is empty, per-event deposits go back out.  The
// device memory and the stream are the caller's (PyTorch provides them); the
// library only carves the workspace and enqueues work on that stream.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "ems_runtime.hpp"

using namespace ems;

static_assert(sizeof(ems_primary) == 64, "primary record is 64 bytes");
static_assert(sizeof(LedgerDev) == sizeof(ems_ledger), "ledger layouts agree");
static_assert(sizeof(StepRec) == sizeof(ems_step_record), "step record layouts agree");
static_assert(sizeof(ExitRec) == sizeof(ems_primary), "exit records are primary records");

namespace ems {
namespace {
thread_local std::string g_err;
}
ems_status fail(ems_status code, const std::string& msg) {
  g_err = msg;
  return code;
}
}  // namespace ems

namespace ems {
uint32_t n_cols(const ems_geometry* g) { return g->n_boxes ? g->n_boxes + 1 : g->n_slabs; }
uint32_t vol_bits(const ems_geometry* g) {
  uint32_t b = kSlabBits;
  while (((1ull << b) - 1) <= n_cols(g)) ++b;  // the all-ones field is never a volume
  return b;
}
// entries of the per-face neighbour lists of a box geometry (the workspace
// plan needs the count, so the lists are built here for it)
uint64_t nbr_entries(const ems_geometry* g) {
  BvhHost h;
  std::string err;
  build_bvh(g->box_lo, g->box_hi, g->n_boxes, h, err);
  return h.nbr.size();
}
BoxNav host_nav(const ems_geometry* g, const BvhHost& h) {
  BoxNav n{};
  n.node = h.node.data();
  n.leaf = h.leaf.data();
  n.box = h.box.data();
  n.rec = h.rec.data();
  n.nbr_off = h.nbr_off.data();
  n.nbr = h.nbr.data();
  for (int k = 0; k < 3; ++k) {
    n.wlo[k] = g->world_lo[k];
    n.whi[k] = g->world_hi[k];
  }
  n.n_boxes = g->n_boxes;
  return n;
}
}  // namespace ems

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint32_t kInjectChunk = 1u << 18;
constexpr uint32_t kInjectChunkNoAlloc = 1u << 14;  // static workspace: smaller staging

uint64_t align_up(uint64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }


// box geometry: finite boxes inside the world, known materials, no two
// boxes sharing interior points (sweep over x), step counts that fit beside
// the volume index
ems_status check_boxes(const ems_config* c, const ems_geometry* g) {
  if (g->n_slabs != 0) return fail(EMS_E_INVALID, "a box geometry has no slabs (n_slabs = 0)");
  if (g->n_boxes > kMaxBoxes || !g->box_lo || !g->box_hi || !g->box_material)
    return fail(EMS_E_INVALID, "box geometry needs 1..2^24 boxes with bounds and materials");
  if (g->world_material >= g->n_materials) return fail(EMS_E_INVALID, "world material index out of range");
  for (int k = 0; k < 3; ++k)
    if (!(g->world_lo[k] < g->world_hi[k]) || !isfinite(g->world_lo[k]) || !isfinite(g->world_hi[k]))
      return fail(EMS_E_INVALID, "world box must be finite with lo < hi");
  const double *lo = g->box_lo, *hi = g->box_hi;
  for (uint32_t i = 0; i < g->n_boxes; ++i) {
    if (g->box_material[i] >= g->n_materials) return fail(EMS_E_INVALID, "box material index out of range");
    for (int k = 0; k < 3; ++k)
      if (!(lo[3 * i + k] < hi[3 * i + k]) || !(lo[3 * i + k] >= g->world_lo[k]) || !(hi[3 * i + k] <= g->world_hi[k]))
        return fail(EMS_E_INVALID, "box " + std::to_string(i) + " is empty or outside the world");
  }
  std::vector<uint32_t> order(g->n_boxes);
  for (uint32_t i = 0; i < g->n_boxes; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return lo[3 * a] < lo[3 * b]; });
  for (uint32_t x = 0; x < g->n_boxes; ++x) {
    const uint32_t i = order[x];
    for (uint32_t y = x + 1; y < g->n_boxes && lo[3 * order[y]] < hi[3 * i]; ++y) {
      const uint32_t j = order[y];
      if (lo[3 * j + 1] < hi[3 * i + 1] && lo[3 * i + 1] < hi[3 * j + 1] && lo[3 * j + 2] < hi[3 * i + 2] &&
          lo[3 * i + 2] < hi[3 * j + 2])
        return fail(EMS_E_INVALID, "boxes " + std::to_string(i) + " and " + std::to_string(j) + " overlap");
    }
  }
  if ((uint64_t)c->max_steps_per_track >= (1ull << (32 - vol_bits(g))))
    return fail(EMS_E_INVALID, "max_steps_per_track too large for this many boxes");
  return EMS_OK;
}

ems_status check_inputs(const ems_config* c, const ems_geometry* g) {
  if (!c || !g) return fail(EMS_E_INVALID, "null config or geometry");
  if (c->abi_version != EMS_ABI_VERSION) return fail(EMS_E_VERSION, "abi_version mismatch");
  if (c->precision != EMS_FP64 && c->precision != EMS_MIXED) return fail(EMS_E_INVALID, "precision must be EMS_FP64 or EMS_MIXED");
  if (g->n_materials < 1 || g->n_materials > 4 || !g->materials)
    return fail(EMS_E_INVALID, "geometry needs 1..4 materials");
  if (g->n_boxes) {
    ems_status bs = check_boxes(c, g);
    if (bs) return bs;
  } else {
    if (g->n_slabs < 1 || g->n_slabs > kMaxSlabs || !g->z_mm || !g->material)
      return fail(EMS_E_INVALID, "geometry needs 1..4095 slabs with planes and materials");
    if (!(g->half_xy_mm > 0.0) || !isfinite(g->half_xy_mm)) return fail(EMS_E_INVALID, "half_xy_mm must be > 0");
    for (uint32_t i = 0; i < g->n_slabs; ++i) {
      if (!(g->z_mm[i + 1] > g->z_mm[i]) || !isfinite(g->z_mm[i + 1]) || !isfinite(g->z_mm[i]))
        return fail(EMS_E_INVALID, "z planes must be finite and strictly increasing");
      if (g->material[i] >= g->n_materials) return fail(EMS_E_INVALID, "slab material index out of range");
    }
  }
  for (uint32_t i = 0; i < g->n_materials; ++i) {
    const ems_material& m = g->materials[i];
    if (!(m.density_g_cm3 > 0.0) || !(m.I_eV > 0.0) || !isfinite(m.density_g_cm3) || !isfinite(m.I_eV))
      return fail(EMS_E_INVALID, "material density and I must be positive");
    if (m.n_elements > (uint32_t)kMaxElements) return fail(EMS_E_INVALID, "a compound has 1..4 elements");
    if (m.n_elements == 0 && (!(m.Z >= 1.0) || !(m.A_g_mol > 0.0) || !isfinite(m.Z) || !isfinite(m.A_g_mol)))
      return fail(EMS_E_INVALID, "element Z >= 1 and A > 0 required");
    for (uint32_t k = 0; k < m.n_elements; ++k)
      if (!(m.el_Z[k] >= 1.0) || !(m.el_A[k] > 0.0) || !(m.el_atoms[k] > 0.0) || !isfinite(m.el_Z[k]) ||
          !isfinite(m.el_A[k]) || !isfinite(m.el_atoms[k]))
        return fail(EMS_E_INVALID, "compound elements need Z >= 1, A > 0 and atoms > 0");
  }
  if (c->n_bins < 2 || c->n_bins > 2000 || !(c->emin_MeV > 0.0) || !(c->emax_MeV > c->emin_MeV))
    return fail(EMS_E_INVALID, "bad energy grid");
  if (!(c->gamma_cut_MeV > c->emin_MeV) || !(c->electron_cut_MeV > c->emin_MeV))
    return fail(EMS_E_INVALID, "production cuts must exceed emin");
  if (!(c->dr_over_range > 0.0 && c->dr_over_range <= 1.0) || !(c->final_range_mm > 0.0) ||
      !(c->lin_loss_limit > 0.0 && c->lin_loss_limit < 1.0))
    return fail(EMS_E_INVALID, "bad step-function parameters");
  if (!isfinite(c->bz_tesla)) return fail(EMS_E_INVALID, "bz must be finite");
  if (c->process_mask & ~kPAllBits) return fail(EMS_E_INVALID, "unknown process_mask bits");
  if (c->max_steps_per_track < 1 || c->max_steps_per_track > kMaxStepsPerTrack || c->max_events < 1)
    return fail(EMS_E_INVALID, "max_steps_per_track in [1, 2^20 - 1] and max_events >= 1");
  if (c->steps_per_visit < 1 || c->steps_per_visit > 1024) return fail(EMS_E_INVALID, "steps_per_visit in [1, 1024]");
  if (c->refill_below > 63) return fail(EMS_E_INVALID, "refill_below in [0, 63]");
  if (c->interact_min > 64) return fail(EMS_E_INVALID, "interact_min in [0, 64]");
  if (c->photon_steps_per_visit < 1 || c->photon_steps_per_visit > 1024)
    return fail(EMS_E_INVALID, "photon_steps_per_visit in [1, 1024]");
  if (c->photon_refill_below > 63) return fail(EMS_E_INVALID, "photon_refill_below in [0, 63]");
  if (c->exit_capacity > (1ull << 32)) return fail(EMS_E_INVALID, "exit_capacity above 2^32");
  if (!(c->short_electron_MeV >= 0.0) || !isfinite(c->short_electron_MeV))
    return fail(EMS_E_INVALID, "short_electron_MeV must be finite and >= 0");
  if (c->track_capacity < 64 || c->track_capacity > (1ull << 28))
    return fail(EMS_E_INVALID, "track_capacity must be in [64, 2^28]");
  return EMS_OK;
}

// bytes of one table value and of one queued track in the chosen form
uint64_t real_bytes(const ems_config* c) { return c->precision == EMS_MIXED ? 4 : 8; }

// element block: screening constants [mat][4][2] (double), then the partial
// pair / brems totals [mat][4][2][nodes] in the arithmetic type
uint64_t elem_const_bytes(const ems_geometry* g) { return (uint64_t)g->n_materials * kMaxElements * 2 * 8; }
uint64_t elem_bytes(const ems_config* c, const ems_geometry* g) {
  return elem_const_bytes(g) + (uint64_t)g->n_materials * kMaxElements * 2 * (c->n_bins + 1) * real_bytes(c);
}

}  // namespace

namespace ems {
uint64_t queue_track_bytes(const ems_config* c) {
  return c->precision == EMS_MIXED ? track_bytes<float>() : track_bytes<double>();
}
}  // namespace ems

namespace {

Layout plan(const ems_config* c, const ems_geometry* g, uint32_t inj_chunk = kInjectChunk) {
  Layout L{};
  L.inj_chunk = inj_chunk;
  const uint64_t nodes = c->n_bins + 1;
  L.cap = (c->track_capacity + 63) / 64 * 64;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    const uint64_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.ctl = take(sizeof(Ctl));
  // photon block, then lepton block (8-byte aligned between them)
  L.tab = take((g->n_materials * kGammaTables * nodes * real_bytes(c) + 7) / 8 * 8 +
               g->n_materials * kLeptonTables * nodes * real_bytes(c));
  L.zp = take(g->n_boxes ? 0 : (g->n_slabs + 1) * 8ull);
  L.smat = take(n_cols(g) * 4ull);  // material per volume
  // box hierarchy: at most 2 n - 1 nodes, leaf ids, bounds by box
  L.bvh = take(g->n_boxes ? (2ull * g->n_boxes) * sizeof(BvhNode) : 0);
  L.bleaf = take(g->n_boxes * 4ull);
  L.bbox = take(g->n_boxes * 48ull);
  L.brec = take(g->n_boxes * sizeof(BoxRec));
  L.nbr_off = take(g->n_boxes ? (6ull * g->n_boxes + 1) * 4 : 0);
  L.nbr = take(g->n_boxes ? nbr_entries(g) * 4 : 0);
  L.mat = take(g->n_materials * sizeof(MatRT));
  L.elem = take(elem_bytes(c, g));
  L.edep = take((uint64_t)c->max_events * n_cols(g) * 8);
  L.ledger = take((uint64_t)c->max_events * sizeof(LedgerDev));
  L.live = take((uint64_t)c->max_events * 4);
  const bool server = (c->flags & EMS_F_EVENT_LIVE) != 0;
  L.rows = take(server ? (uint64_t)c->max_events * 4 : 0);
  L.gather = take(server ? (uint64_t)c->max_events * (n_cols(g) * 8ull + sizeof(LedgerDev)) : 0);
  L.exits = take(c->exit_capacity * sizeof(ExitRec));
  L.profile = take((c->flags & EMS_F_PROFILE) ? (uint64_t)c->profile_capacity * 3 * 4 : 0);
  L.log = take((c->flags & EMS_F_STEPLOG) ? c->steplog_capacity * sizeof(StepRec) : 0);
  L.inj = take((uint64_t)inj_chunk * sizeof(InjRec));
  L.dkey = take((uint64_t)c->max_events * 4);
  L.drow = take((uint64_t)c->max_events * 8);
  L.dchk = take(4 * 8);
  L.queues = take(6 * L.cap * queue_track_bytes(c));
  // short electrons: two buffers of half the queue capacity and a spill
  // buffer a quarter larger (room for the unused ends of append chunks)
  L.cap_s = c->short_electron_MeV > 0.0 ? (L.cap / 2 + 63) / 64 * 64 : 0;
  L.cap_p = L.cap_s + L.cap_s / 4;
  L.squeues = take((2 * L.cap_s + L.cap_p) * queue_track_bytes(c));
  L.total = o;
  return L;
}

TableSet tables_for(const ems_config* c, const ems_geometry* g) {
  TableParams p;
  p.n_bins = c->n_bins;
  p.emin = c->emin_MeV;
  p.emax = c->emax_MeV;
  p.gamma_cut = c->gamma_cut_MeV;
  p.electron_cut = c->electron_cut_MeV;
  p.process_mask = c->process_mask;
  std::vector<MaterialIn> mats;
  for (uint32_t i = 0; i < g->n_materials; ++i) {
    const ems_material& m = g->materials[i];
    MaterialIn in{m.Z, m.A_g_mol, m.density_g_cm3, m.I_eV, m.n_elements, {}, {}, {}};
    for (uint32_t k = 0; k < m.n_elements; ++k) {
      in.el_Z[k] = m.el_Z[k];
      in.el_A[k] = m.el_A[k];
      in.el_atoms[k] = m.el_atoms[k];
    }
    mats.push_back(in);
  }
  return build_tables(p, mats);
}

StepEnv<double> env_for(const ems_config* c, const ems_geometry* g, const TableSet& ts) {
  StepEnv<double> e{};
  e.nodes = ts.nodes;
  e.n_slabs = n_cols(g);  // deposit columns (slabs, or boxes + world)
  e.lnemin = ts.lnemin;
  e.dlog = ts.dlog;
  e.inv_dlog = 1.0 / ts.dlog;
  e.half_xy = g->half_xy_mm;
  e.bz = c->bz_tesla;
  e.ecut = c->emin_MeV;
  e.tcut = c->electron_cut_MeV;
  e.kcut = c->gamma_cut_MeV;
  e.alpha = c->dr_over_range;
  e.rho = c->final_range_mm;
  e.lin = c->lin_loss_limit;
  e.mask = c->process_mask;
  e.seed = c->seed;
  e.max_steps = c->max_steps_per_track;
  return e;
}

// true if [p, p + bytes) lies inside one device allocation
bool device_range(const void* p, uint64_t bytes) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (at.type != hipMemoryTypeDevice) return false;
  void* base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  const uintptr_t b = reinterpret_cast<uintptr_t>(base), q = reinterpret_cast<uintptr_t>(p);
  return q >= b && bytes <= size - (q - b);
}

// slab of a point; a point on a plane belongs to the slab it moves into
int32_t locate(const double* z, uint32_t n, double zz, double uz) {
  uint32_t lo = 0, hi = n;  // z[lo] <= zz < z[hi]
  if (zz >= z[n]) return (int32_t)n - 1;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (z[mid] <= zz) lo = mid;
    else hi = mid;
  }
  if (lo > 0 && zz == z[lo] && uz < 0.0) lo -= 1;
  return (int32_t)lo;
}

// validate and convert primaries; ids are running indices per row, keys
// the rows' event keys
ems_status prepare(const ems_geometry& g, const BoxNav* nav, uint32_t max_events, const ems_primary* p, uint64_t n,
                   std::vector<uint64_t>& row_count, const std::vector<uint32_t>& keys, std::vector<InjRec>& out) {
  for (uint64_t i = 0; i < n; ++i) {
    const ems_primary& q = p[i];
    const double d2 = q.dir[0] * q.dir[0] + q.dir[1] * q.dir[1] + q.dir[2] * q.dir[2];
    bool ok = q.event < max_events && q.species <= EMS_POSITRON && q.ekin_MeV > 0.0 && isfinite(q.ekin_MeV) &&
              d2 > 0.0 && isfinite(d2);
    if (ok && g.n_boxes)
      ok = isfinite(q.pos_mm[0]) && isfinite(q.pos_mm[1]) && isfinite(q.pos_mm[2]) &&
           bvh_locate(*nav, q.pos_mm, q.dir) >= 0;
    else if (ok)
      ok = q.pos_mm[2] >= g.z_mm[0] && q.pos_mm[2] <= g.z_mm[g.n_slabs] && fabs(q.pos_mm[0]) <= g.half_xy_mm &&
           fabs(q.pos_mm[1]) <= g.half_xy_mm;
    if (!ok) return fail(EMS_E_INVALID, "invalid primary #" + std::to_string(i));
  }
  out.resize(n);
  for (uint64_t i = 0; i < n; ++i) {
    const ems_primary& q = p[i];
    const double nrm = sqrt(q.dir[0] * q.dir[0] + q.dir[1] * q.dir[1] + q.dir[2] * q.dir[2]);
    InjRec& r = out[i];
    r.x = q.pos_mm[0];
    r.y = q.pos_mm[1];
    r.z = q.pos_mm[2];
    r.ux = q.dir[0] / nrm;
    r.uy = q.dir[1] / nrm;
    r.uz = q.dir[2] / nrm;
    r.E = q.ekin_MeV;
    r.ev = q.event;
    r.sp = q.species;
    if (g.n_boxes) {
      const double pp[3] = {r.x, r.y, r.z}, uu[3] = {r.ux, r.uy, r.uz};
      r.slab = bvh_locate(*nav, pp, uu);
    } else {
      r.slab = locate(g.z_mm, g.n_slabs, r.z, r.uz);
    }
    r.id = row_count[q.event]++;
    r.key = keys[q.event];
  }
  return EMS_OK;
}

// The mixed form compares FP32 interpolated totals against bounds; bounds
// are raised by 2^-20 (relative) so FP32 rounding of the interpolation (a few
// 1e-7) never exceeds them.  A larger bound only adds null collisions.
constexpr double kBoundInflation = 1.0 + 0x1p-20;

void inflate_bounds(MatRT& m) {
  for (int i = 0; i < 2; ++i) {
    m.up_em[i] *= kBoundInflation;
    m.up_ep[i] *= kBoundInflation;
  }
}

// table blocks as laid out on the device, values of type R; the photon block
// is padded to 8 bytes
template <class R>
void pack_tables(const TableSet& ts, uint32_t n_mat, std::vector<char>& out) {
  std::vector<R> g, l;
  const bool mixed = sizeof(R) == 4;
  for (uint32_t m = 0; m < n_mat; ++m)
    for (int t = 0; t < kGammaTables; ++t)
      for (uint32_t j = 0; j < ts.nodes; ++j) g.push_back((R)ts.at(m, t, j));
  for (uint32_t m = 0; m < n_mat; ++m) {
    for (int t = kGammaTables; t < kNumTables; ++t)
      for (uint32_t j = 0; j < ts.nodes; ++j) {
        const bool bound = t == tPMem || t == tPMep;
        l.push_back((R)(mixed && bound ? ts.at(m, t, j) * kBoundInflation : ts.at(m, t, j)));
      }
    // node totals of the discrete processes, as the step code would sum
    // the packed values (e-: Moller, brems; e+: Bhabha, brems, annihilation)
    for (uint32_t j = 0; j < ts.nodes; ++j) {
      R s = R(0);
      s += (R)ts.at(m, tMoller, j);
      s += (R)ts.at(m, tBrem, j);
      l.push_back(s);
    }
    for (uint32_t j = 0; j < ts.nodes; ++j) {
      R s = R(0);
      s += (R)ts.at(m, tBhabha, j);
      s += (R)ts.at(m, tBrem, j);
      s += (R)ts.at(m, tAnnih, j);
      l.push_back(s);
    }
  }
  const size_t gb = (g.size() * sizeof(R) + 7) / 8 * 8;
  out.assign(gb + l.size() * sizeof(R), 0);
  memcpy(out.data(), g.data(), g.size() * sizeof(R));
  memcpy(out.data() + gb, l.data(), l.size() * sizeof(R));
}

// element block as laid out on the device: constants (double), then the
// partial totals in type R
template <class R>
void pack_elements(const TableSet& ts, std::vector<char>& out) {
  const size_t cb = ts.elc.size() * sizeof(double);
  out.assign(cb + ts.el.size() * sizeof(R), 0);
  memcpy(out.data(), ts.elc.data(), cb);
  R* t = reinterpret_cast<R*>(out.data() + cb);
  for (size_t i = 0; i < ts.el.size(); ++i) t[i] = (R)ts.el[i];
}

template <class R, int GEO>
ems_status host_transport(const ems_config& c2, const ems_geometry* geo, const ems_primary* prim, uint64_t n,
                          uint32_t n_events, const uint32_t* keys, double* edep, ems_ledger* ledger,
                          ems_step_record* log, uint64_t log_cap, uint64_t* log_n);

}  // namespace


extern "C" {

uint32_t ems_abi_version(void) { return EMS_ABI_VERSION; }

ems_status ems_probe_atomics(void* d_cells, uint64_t n_cells, uint64_t n_ops, void* stream, double* ms) {
  if (!d_cells || !n_cells || !n_ops || !ms) return fail(EMS_E_INVALID, "null pointer or zero size");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(EMS_E_DEVICE, "event creation failed");
  }
  float t = 0.0f;
  const bool ok = hipMemsetAsync(d_cells, 0, n_cells * 8, s) == hipSuccess && hipEventRecord(e0, s) == hipSuccess &&
                  launch_atomic_probe(static_cast<double*>(d_cells), n_cells, n_ops, s) == hipSuccess &&
                  hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                  hipEventElapsedTime(&t, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!ok) return fail(EMS_E_DEVICE, "atomic probe failed");
  *ms = t;
  return EMS_OK;
}

const char* ems_last_error(void) { return g_err.c_str(); }

ems_status ems_workspace_bytes(const ems_config* cfg, const ems_geometry* geo, uint64_t* bytes) {
  return rt_workspace_bytes(cfg, geo, false, bytes);
}

ems_status ems_host_tables(const ems_config* cfg, const ems_geometry* geo, double* out, uint64_t n) {
  ems_status st = check_inputs(cfg, geo);
  if (st) return st;
  const uint64_t nodes = cfg->n_bins + 1;
  const uint64_t need = (uint64_t)geo->n_materials * kNumExport * nodes;
  if (!out || n < need) return fail(EMS_E_INVALID, "output buffer too small");
  TableSet ts = tables_for(cfg, geo);
  for (uint32_t m = 0; m < geo->n_materials; ++m)
    for (int t = 0; t < kNumExport; ++t)
      for (uint64_t j = 0; j < nodes; ++j) out[((uint64_t)m * kNumExport + t) * nodes + j] = ts.at(m, t, (uint32_t)j);
  return EMS_OK;
}

ems_status ems_export_tables(ems_ctx* c, double* out, uint64_t n) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  const uint64_t nodes = c->ts.nodes, nm = c->geo.n_materials;
  const uint64_t need = nm * kNumExport * nodes;
  if (!out || n < need) return fail(EMS_E_INVALID, "output buffer too small");
  // the device copy as uploaded: photon block [mat][3][nodes] (padded to 8
  // bytes), then the lepton block [mat][12][nodes], in the form's type
  const uint64_t rb = real_bytes(&c->cfg);
  const uint64_t gbytes = (nm * kGammaTables * nodes * rb + 7) / 8 * 8;
  const uint64_t lbytes = nm * kLeptonTables * nodes * rb;
  std::vector<char> dev(gbytes + lbytes);
  HIPCHK(c, hipMemcpyAsync(dev.data(), c->ws + c->L.tab, dev.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  auto value = [&](uint64_t byte_off, uint64_t i) {
    if (rb == 4) {
      float f;
      memcpy(&f, dev.data() + byte_off + i * 4, 4);
      return (double)f;
    }
    double d;
    memcpy(&d, dev.data() + byte_off + i * 8, 8);
    return d;
  };
  for (uint64_t m = 0; m < nm; ++m)
    for (int t = 0; t < kNumExport; ++t)
      for (uint64_t j = 0; j < nodes; ++j)
        out[(m * kNumExport + t) * nodes + j] =
            t < kGammaTables ? value(0, (m * kGammaTables + t) * nodes + j)
                             : value(gbytes, (m * kLeptonTables + (t - kGammaTables)) * nodes + j);
  return EMS_OK;
}

ems_status ems_create(const ems_config* cfg, const ems_geometry* geo, void* d_ws, uint64_t bytes, void* stream,
                      ems_ctx** out) {
  return rt_create(cfg, geo, d_ws, bytes, stream, false, out);
}

ems_status ems_create_static(const ems_config* cfg, const ems_geometry* geo, void* stream, ems_ctx** out) {
  uint64_t need = 0;
  ems_status st = rt_workspace_bytes(cfg, geo, true, &need);
  if (st) return st;
  if (!out) return fail(EMS_E_INVALID, "null output");
  if (need > kStaticWorkspaceBytes)
    return fail(EMS_E_CAPACITY, "the configuration needs " + std::to_string(need) +
                                    " workspace bytes; the static workspace holds " +
                                    std::to_string(kStaticWorkspaceBytes));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(EMS_E_DEVICE, "no HIP device");
  if (dev < 0 || dev >= kMaxStaticDevices) return fail(EMS_E_INVALID, "device index beyond the static workspaces");
  if (!rt_hold_static(dev)) return fail(EMS_E_BUSY, "another context holds this device's static workspace");
  void* ws = nullptr;
  const hipError_t e = static_workspace(dev, &ws);
  if (e != hipSuccess) {
    rt_release_static(dev);
    return fail(EMS_E_DEVICE, std::string("static workspace address: ") + hipGetErrorString(e));
  }
  st = rt_create(cfg, geo, ws, kStaticWorkspaceBytes, stream, true, out);
  if (st) rt_release_static(dev);
  return st;
}

}  // extern "C"

namespace ems {

namespace {
std::mutex g_static_mu;
bool g_static_held[kMaxStaticDevices];
}  // namespace

bool rt_hold_static(int dev) {
  if (dev < 0 || dev >= kMaxStaticDevices) return false;
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (g_static_held[dev]) return false;
  g_static_held[dev] = true;
  return true;
}

void rt_release_static(int dev) {
  if (dev < 0 || dev >= kMaxStaticDevices) return;
  std::lock_guard<std::mutex> lk(g_static_mu);
  g_static_held[dev] = false;
}

ems_status rt_workspace_bytes(const ems_config* cfg, const ems_geometry* geo, bool no_alloc, uint64_t* bytes) {
  ems_status st = check_inputs(cfg, geo);
  if (st) return st;
  if (!bytes) return fail(EMS_E_INVALID, "null output");
  *bytes = plan(cfg, geo, no_alloc ? kInjectChunkNoAlloc : kInjectChunk).total;
  return EMS_OK;
}

ems_status rt_create(const ems_config* cfg, const ems_geometry* geo, void* d_ws, uint64_t bytes, void* stream,
                     bool no_alloc, ems_ctx** out) {
  ems_status st = check_inputs(cfg, geo);
  if (st) return st;
  if (!out || !d_ws) return fail(EMS_E_INVALID, "null workspace or output");
  if (((uintptr_t)d_ws) % kAlign) return fail(EMS_E_INVALID, "workspace must be 256-byte aligned");
  if (no_alloc && (cfg->flags & (EMS_F_KERNEL_TIMING | EMS_F_EVENT_LIVE)))
    return fail(EMS_E_INVALID, "a context without allocations takes neither EMS_F_KERNEL_TIMING nor EMS_F_EVENT_LIVE");
  Layout L = plan(cfg, geo, no_alloc ? kInjectChunkNoAlloc : kInjectChunk);
  if (bytes < L.total) return fail(EMS_E_CAPACITY, "workspace smaller than ems_workspace_bytes");
  ems_ctx* c = new ems_ctx();
  c->no_alloc = no_alloc;
  c->cfg = *cfg;
  c->mats.assign(geo->materials, geo->materials + geo->n_materials);
  c->geo = *geo;
  if (geo->n_boxes) {
    c->blo.assign(geo->box_lo, geo->box_lo + 3ull * geo->n_boxes);
    c->bhi.assign(geo->box_hi, geo->box_hi + 3ull * geo->n_boxes);
    c->smat.assign(geo->box_material, geo->box_material + geo->n_boxes);
    c->smat.push_back(geo->world_material);  // material per volume, the world last
    c->geo.box_lo = c->blo.data();
    c->geo.box_hi = c->bhi.data();
    c->geo.box_material = c->smat.data();
    c->geo.z_mm = nullptr;
    c->geo.material = nullptr;
    std::string err;
    if (!build_bvh(c->blo.data(), c->bhi.data(), geo->n_boxes, c->bvh, err)) {
      delete c;
      return fail(EMS_E_INVALID, err);
    }
    c->nav = host_nav(&c->geo, c->bvh);
  } else {
    c->z.assign(geo->z_mm, geo->z_mm + geo->n_slabs + 1);
    c->smat.assign(geo->material, geo->material + geo->n_slabs);
    c->geo.z_mm = c->z.data();
    c->geo.material = c->smat.data();
  }
  c->geo.materials = c->mats.data();
  c->ncols = n_cols(geo);
  c->ts = tables_for(cfg, geo);
  c->L = L;
  c->ws = static_cast<char*>(d_ws);
  c->stream = static_cast<hipStream_t>(stream);
  c->row_count.assign(cfg->max_events, 0);
  auto bad = [&](ems_status s) {
    delete c;
    return s;
  };
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return bad(fail(EMS_E_DEVICE, "no HIP device"));
  c->device = dev;
  const uint64_t nodes = cfg->n_bins + 1;
  const uint32_t staged = geo->n_boxes ? 0u : geo->n_slabs;  // box geometries keep planes and materials global
  const uint32_t common = (uint32_t)((geo->n_boxes ? 0u : staged + 1) * 8 + geo->n_materials * sizeof(MatRT) + staged * 4 + 64);
  const uint64_t rb = real_bytes(cfg);
  const uint64_t gbytes = (geo->n_materials * kGammaTables * nodes * rb + 7) / 8 * 8;
  const uint64_t lbytes = (geo->n_materials * kLeptonTables * nodes * rb + 7) / 8 * 8;
  const uint32_t lds_g = (uint32_t)gbytes + common;
  const uint32_t lds_l = (uint32_t)lbytes + common;
  if (lds_l > 160u * 1024u) return bad(fail(EMS_E_INVALID, "tables exceed LDS"));

  KArgs& a = c->args;
  a.qbase = c->ws + L.queues;
  a.sbase = c->ws + L.squeues;
  a.cap_s = L.cap_s;
  a.cap_p = L.cap_p;
  a.short_E = cfg->short_electron_MeV;
  a.ctl = reinterpret_cast<Ctl*>(c->ws + L.ctl);
  a.edep = reinterpret_cast<double*>(c->ws + L.edep);
  a.ledger = reinterpret_cast<LedgerDev*>(c->ws + L.ledger);
  a.tab_g = c->ws + L.tab;
  a.tab_l = c->ws + L.tab + gbytes;
  a.zplane = reinterpret_cast<const double*>(c->ws + L.zp);
  a.slab_mat = reinterpret_cast<const uint32_t*>(c->ws + L.smat);
  a.mat = reinterpret_cast<const MatRT*>(c->ws + L.mat);
  a.el_c = reinterpret_cast<const double*>(c->ws + L.elem);
  a.el_tab = c->ws + L.elem + elem_const_bytes(geo);
  a.log = reinterpret_cast<StepRec*>(c->ws + L.log);
  a.profile = reinterpret_cast<uint32_t*>(c->ws + L.profile);
  a.live_ev = reinterpret_cast<int32_t*>(c->ws + L.live);
  a.exits = reinterpret_cast<ExitRec*>(c->ws + L.exits);
  a.exit_cap = cfg->exit_capacity;
  a.cap = L.cap;
  a.max_events = cfg->max_events;
  a.log_cap = (cfg->flags & EMS_F_STEPLOG) ? cfg->steplog_capacity : 0;
  a.profile_cap = (cfg->flags & EMS_F_PROFILE) ? cfg->profile_capacity : 0;
  a.flags = cfg->flags;
  a.n_mat = geo->n_materials;
  a.lds_g = lds_g;
  a.lds_l = lds_l;
  a.steps_per_visit = cfg->steps_per_visit;
  a.refill_below = cfg->refill_below;
  a.interact_min = cfg->interact_min;
  a.photon_steps_per_visit = cfg->photon_steps_per_visit;
  a.photon_refill_below = cfg->photon_refill_below;
  a.precision = cfg->precision == EMS_MIXED ? 1u : 0u;
  a.env = env_for(cfg, geo, c->ts);
  a.geo = geo->n_boxes ? 1u : 0u;
  a.vol_bits = vol_bits(geo);
  // the smallest kernel variants that cover the configuration's optional
  // parts (the others are compiled out of them)
  bool compound = false;
  for (const MatRT& m : c->ts.rt) compound = compound || m.n_el > 1;
  const bool record = (cfg->flags & (EMS_F_STEPLOG | EMS_F_FULL_LEDGER | EMS_F_EVENT_LIVE)) || cfg->exit_capacity;
  const uint32_t need_l = (cfg->bz_tesla != 0.0 ? kFField : 0) |
                          (cfg->process_mask & EMS_P_MSC ? kFMsc : 0) | (cfg->process_mask & EMS_P_FLUCT ? kFFluct : 0) |
                          (compound ? kFCompound : 0) | (record ? kFRecord : 0);
  const uint32_t need_g = (compound ? kFCompound : 0) | (record ? kFRecord : 0);
  constexpr uint32_t kAllParts = kFAll & ~kFShort;
  a.feat_l = need_l == 0 ? 0u
             : (geo->n_boxes == 0 && (need_l & ~(uint32_t)(kFField | kFRecord)) == 0) ? (uint32_t)(kFField | kFRecord)
                                                                                      : kAllParts;
  a.feat_g = need_g == 0 ? 0u : kAllParts;
  // the short-electron routing is compiled into variants of its own
  if (L.cap_s) {
    a.feat_g |= kFShort;
    a.feat_l |= kFShort;
  }
  if (cfg->flags & EMS_F_FULL_KERNELS) a.feat_g = a.feat_l = kFAll;
  if (geo->n_boxes) {
    // device view of the hierarchy (same layout as the host one)
    a.env.nav = c->nav;
    a.env.nav.node = reinterpret_cast<const BvhNode*>(c->ws + L.bvh);
    a.env.nav.leaf = reinterpret_cast<const uint32_t*>(c->ws + L.bleaf);
    a.env.nav.box = reinterpret_cast<const double*>(c->ws + L.bbox);
    a.env.nav.rec = reinterpret_cast<const BoxRec*>(c->ws + L.brec);
    a.env.nav.nbr_off = reinterpret_cast<const uint32_t*>(c->ws + L.nbr_off);
    a.env.nav.nbr = reinterpret_cast<const uint32_t*>(c->ws + L.nbr);
  }
  int per_g = 0, per_l = 0, per_s = 0;
  if (visit_occupancy(a, &per_g, &per_l, &per_s) != hipSuccess || per_g < 1 || per_l < 1 || per_s < 1)
    return bad(fail(EMS_E_DEVICE, "cannot configure the visit kernels"));
  // one resident wave of blocks per launch; blocks grid-stride over the queue
  const uint32_t cus = (uint32_t)prop.multiProcessorCount;
  c->blocks_g = cfg->launch_blocks ? cfg->launch_blocks : cus * (uint32_t)per_g;
  c->blocks_l = cfg->launch_blocks ? cfg->launch_blocks : cus * (uint32_t)per_l;
  c->blocks_s = cfg->launch_blocks ? cfg->launch_blocks : cus * (uint32_t)per_s;
  a.waves_g = c->blocks_g * 4;  // 256-thread blocks of 64-lane waves
  a.waves_l = c->blocks_l * 4;
  a.waves_s = c->blocks_s * 4;

  if (no_alloc) {
    // ordinary host memory for the staging and the status block; no events,
    // chunks launched directly (no graph)
    c->host_inj.resize(L.inj_chunk);
    c->pin_inj = c->host_inj.data();
    c->pin_ctl = &c->host_ctl;
    c->graph_off = true;
  } else if (hipHostMalloc(reinterpret_cast<void**>(&c->pin_inj), (uint64_t)L.inj_chunk * sizeof(InjRec)) !=
                 hipSuccess ||
             hipHostMalloc(reinterpret_cast<void**>(&c->pin_ctl), sizeof(Ctl)) != hipSuccess ||
             hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
    return bad(fail(EMS_E_DEVICE, "pinned host allocation or event creation failed"));
  }
  // device table layout: photon block [mat][3][nodes], then lepton block
  // [mat][10][nodes], in the arithmetic type of the chosen form
  std::vector<char> packed, elem;
  std::vector<MatRT> rt = c->ts.rt;
  if (cfg->precision == EMS_MIXED) {
    pack_tables<float>(c->ts, geo->n_materials, packed);
    pack_elements<float>(c->ts, elem);
    for (MatRT& m : rt) inflate_bounds(m);
  } else {
    pack_tables<double>(c->ts, geo->n_materials, packed);
    pack_elements<double>(c->ts, elem);
  }
  c->keys.resize(cfg->max_events);
  for (uint32_t i = 0; i < cfg->max_events; ++i) c->keys[i] = i;
  if (cfg->flags & EMS_F_EVENT_LIVE) {
    const uint64_t gb = (uint64_t)cfg->max_events * (n_cols(geo) * 8ull + sizeof(LedgerDev));
    if (hipHostMalloc(reinterpret_cast<void**>(&c->pin_rows), cfg->max_events * 4ull) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&c->pin_gather), gb) != hipSuccess)
      return bad(fail(EMS_E_DEVICE, "pinned host allocation failed"));
  }
  hipStream_t s = c->stream;
  bool ok = launch_fill_zero(c->ws + L.ctl, sizeof(Ctl), s) == hipSuccess &&
            hipMemcpyAsync(c->ws + L.tab, packed.data(), packed.size(), hipMemcpyHostToDevice, s) == hipSuccess &&
            (c->z.empty() ||
             hipMemcpyAsync(c->ws + L.zp, c->z.data(), c->z.size() * 8, hipMemcpyHostToDevice, s) == hipSuccess) &&
            (c->bvh.node.empty() ||
             (hipMemcpyAsync(c->ws + L.bvh, c->bvh.node.data(), c->bvh.node.size() * sizeof(BvhNode),
                             hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync(c->ws + L.bleaf, c->bvh.leaf.data(), c->bvh.leaf.size() * 4, hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemcpyAsync(c->ws + L.bbox, c->bvh.box.data(), c->bvh.box.size() * 8, hipMemcpyHostToDevice, s) ==
                  hipSuccess &&
              hipMemcpyAsync(c->ws + L.nbr_off, c->bvh.nbr_off.data(), c->bvh.nbr_off.size() * 4,
                             hipMemcpyHostToDevice, s) == hipSuccess &&
              hipMemcpyAsync(c->ws + L.brec, c->bvh.rec.data(), c->bvh.rec.size() * sizeof(BoxRec),
                             hipMemcpyHostToDevice, s) == hipSuccess &&
              (c->bvh.nbr.empty() || hipMemcpyAsync(c->ws + L.nbr, c->bvh.nbr.data(), c->bvh.nbr.size() * 4,
                                                    hipMemcpyHostToDevice, s) == hipSuccess))) &&
            hipMemcpyAsync(c->ws + L.smat, c->smat.data(), c->smat.size() * 4, hipMemcpyHostToDevice, s) == hipSuccess &&
            hipMemcpyAsync(c->ws + L.mat, rt.data(), rt.size() * sizeof(MatRT), hipMemcpyHostToDevice, s) ==
                hipSuccess &&
            hipMemcpyAsync(c->ws + L.elem, elem.data(), elem.size(), hipMemcpyHostToDevice, s) == hipSuccess &&
            launch_fill_zero(c->ws + L.edep, (L.live - L.edep) + (uint64_t)cfg->max_events * 4, s) == hipSuccess &&
            launch_fill_zero(c->ws + L.queues, 6 * L.cap * queue_track_bytes(cfg), s) == hipSuccess &&
            launch_fill_zero(c->ws + L.squeues, (2 * L.cap_s + L.cap_p) * queue_track_bytes(cfg), s) == hipSuccess &&
            launch_fill_zero(c->ws + L.drow, (uint64_t)cfg->max_events * 8, s) == hipSuccess &&
            hipStreamSynchronize(s) == hipSuccess;
  if (!ok) {
    if (!no_alloc) {
      (void)hipHostFree(c->pin_inj);
      (void)hipHostFree(c->pin_ctl);
      if (c->pin_rows) (void)hipHostFree(c->pin_rows);
      if (c->pin_gather) (void)hipHostFree(c->pin_gather);
      (void)hipEventDestroy(c->ev0);
      (void)hipEventDestroy(c->ev1);
    }
    return bad(fail(EMS_E_DEVICE, "workspace initialisation failed"));
  }
  *out = c;
  return EMS_OK;
}

}  // namespace ems

extern "C" {

ems_status ems_destroy(ems_ctx* c) {
  if (!c) return EMS_OK;
  (void)hipStreamSynchronize(c->stream);
  if (c->no_alloc) {
    rt_release_static(c->device);
    delete c;
    return EMS_OK;
  }
  if (c->pin_inj) (void)hipHostFree(c->pin_inj);
  if (c->pin_ctl) (void)hipHostFree(c->pin_ctl);
  if (c->pin_rows) (void)hipHostFree(c->pin_rows);
  if (c->pin_gather) (void)hipHostFree(c->pin_gather);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  for (hipEvent_t e : c->evk) (void)hipEventDestroy(e);
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  delete c;
  return EMS_OK;
}

ems_status ems_set_event_keys(ems_ctx* c, uint32_t first, uint32_t n, const uint32_t* keys) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  if (!keys || (uint64_t)first + n > c->cfg.max_events) return fail(EMS_E_INVALID, "rows out of range");
  std::copy(keys, keys + n, c->keys.begin() + first);  // applied to tracks enqueued from now on
  c->keys_dirty = true;
  return EMS_OK;
}

ems_status ems_enqueue(ems_ctx* c, const ems_primary* p, uint64_t n) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  return rt_enqueue(c, p, n);
}

ems_status ems_enqueue_device(ems_ctx* c, const ems_primary* p, uint64_t n) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  return rt_enqueue_device(c, p, n);
}

ems_status ems_run(ems_ctx* c) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  const auto t0 = std::chrono::steady_clock::now();
  const uint32_t K = c->cfg.steps_per_launch ? c->cfg.steps_per_launch : 16;
  for (;;) {
    const ems_status st = rt_chunk(c, K);
    if (st) return st;
    const Ctl& s = *c->pin_ctl;
    if (s.live == 0) break;
    // a track lives at most max_steps iterations; generations are few
    if ((uint64_t)s.iteration > 64ull * c->cfg.max_steps_per_track + 4096) {
      c->failed = true;
      return fail(EMS_E_STATE, "iteration guard reached");
    }
  }
  c->stats.run_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  for (int i = 0; i < 3; ++i) c->pending[i] = 0;
  return EMS_OK;
}

ems_status ems_read_edep_device(ems_ctx* c, uint32_t first, uint32_t n, double* out) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  if ((uint64_t)first + n > c->cfg.max_events) return fail(EMS_E_INVALID, "rows out of range");
  if (n == 0) return EMS_OK;
  const uint64_t row = (uint64_t)c->ncols * 8;
  if (!out || !device_range(out, n * row)) return fail(EMS_E_INVALID, "output is not n rows in one device allocation");
  HIPCHK(c, hipMemcpyAsync(out, c->ws + c->L.edep + first * row, n * row, hipMemcpyDeviceToDevice, c->stream));
  return EMS_OK;
}

ems_status ems_read_edep(ems_ctx* c, uint32_t first, uint32_t n, double* out) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  if (!out || (uint64_t)first + n > c->cfg.max_events) return fail(EMS_E_INVALID, "rows out of range");
  const uint64_t row = c->ncols * 8ull;
  HIPCHK(c, hipMemcpyAsync(out, c->ws + c->L.edep + first * row, n * row, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EMS_OK;
}

ems_status ems_read_ledger(ems_ctx* c, uint32_t first, uint32_t n, ems_ledger* out) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  if (!out || (uint64_t)first + n > c->cfg.max_events) return fail(EMS_E_INVALID, "rows out of range");
  HIPCHK(c, hipMemcpyAsync(out, c->ws + c->L.ledger + first * sizeof(LedgerDev), n * sizeof(LedgerDev),
                           hipMemcpyDeviceToHost, c->stream));
  std::vector<double> ed((size_t)n * c->ncols);
  const uint64_t row = c->ncols * 8ull;
  HIPCHK(c, hipMemcpyAsync(ed.data(), c->ws + c->L.edep + first * row, n * row, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (uint32_t i = 0; i < n; ++i) {
    double s = 0.0;
    for (uint32_t k = 0; k < c->ncols; ++k) s += ed[(size_t)i * c->ncols + k];
    out[i].edep = s;
  }
  return EMS_OK;
}

ems_status ems_reset_tallies(ems_ctx* c) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  const Layout& L = c->L;
  HIPCHK(c, launch_fill_zero(c->ws + L.edep, (uint64_t)c->cfg.max_events * c->ncols * 8, c->stream));
  HIPCHK(c, launch_fill_zero(c->ws + L.ledger, (uint64_t)c->cfg.max_events * sizeof(LedgerDev), c->stream));
  HIPCHK(c, launch_fill_zero(c->ws + L.live, (uint64_t)c->cfg.max_events * 4, c->stream));
  if (c->args.profile_cap)
    HIPCHK(c, launch_fill_zero(c->ws + L.profile, (uint64_t)c->args.profile_cap * 12, c->stream));
  // keep the queues (empty after a run) but restart counters and statistics
  HIPCHK(c, hipMemcpyAsync(c->pin_ctl, c->ws + L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  Ctl fresh{};
  fresh.cur = c->pin_ctl->cur;
  for (int s = 0; s < 3; ++s) {
    fresh.n_home[s] = c->pin_ctl->n_home[s];
    fresh.n_sec[s] = c->pin_ctl->n_sec[s];
    fresh.n_real[s] = c->pin_ctl->n_real[s];
  }
  fresh.n_short = c->pin_ctl->n_short;
  fresh.n_short_real = c->pin_ctl->n_short_real;
  *c->pin_ctl = fresh;
  HIPCHK(c, hipMemcpyAsync(c->ws + L.ctl, c->pin_ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->source == 2) {
    HIPCHK(c, launch_fill_zero(c->ws + L.drow, (uint64_t)c->cfg.max_events * 8, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->source = 0;
  std::fill(c->row_count.begin(), c->row_count.end(), 0);
  c->stats = ems_run_stats{};
  return EMS_OK;
}

ems_status ems_read_steplog(ems_ctx* c, ems_step_record* out, uint64_t cap, uint64_t* n) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  if (!n) return fail(EMS_E_INVALID, "null count");
  HIPCHK(c, hipMemcpyAsync(c->pin_ctl, c->ws + c->L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const uint64_t total = c->pin_ctl->log_n;
  *n = total;
  const uint64_t k = std::min<uint64_t>(std::min<uint64_t>(total, c->args.log_cap), out ? cap : 0);
  if (k) {
    HIPCHK(c, hipMemcpyAsync(out, c->ws + c->L.log, k * sizeof(StepRec), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return EMS_OK;
}

ems_status ems_read_exits(ems_ctx* c, ems_primary* out, uint64_t cap, uint64_t* n) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  if (!n) return fail(EMS_E_INVALID, "null count");
  HIPCHK(c, hipMemcpyAsync(c->pin_ctl, c->ws + c->L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  const uint64_t total = c->pin_ctl->exit_n;
  *n = total;
  const uint64_t k = std::min<uint64_t>(std::min<uint64_t>(total, c->cfg.exit_capacity), out ? cap : 0);
  if (k) {
    HIPCHK(c, hipMemcpyAsync(out, c->ws + c->L.exits, k * sizeof(ExitRec), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return EMS_OK;
}

ems_status ems_read_profile(ems_ctx* c, uint32_t* out, uint32_t cap, uint32_t* n) {
  if (!c) return fail(EMS_E_INVALID, "null context");
  if (c->failed) return fail(EMS_E_STATE, "context failed earlier");
  if (!n) return fail(EMS_E_INVALID, "null count");
  HIPCHK(c, hipMemcpyAsync(c->pin_ctl, c->ws + c->L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  *n = c->pin_ctl->iteration;
  const uint32_t k = std::min<uint32_t>(std::min<uint32_t>(*n, c->args.profile_cap), out ? cap : 0);
  if (k) {
    HIPCHK(c, hipMemcpyAsync(out, c->ws + c->L.profile, k * 12ull, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return EMS_OK;
}

ems_status ems_stats(ems_ctx* c, ems_run_stats* out) {
  if (!c || !out) return fail(EMS_E_INVALID, "null argument");
  *out = c->stats;
  return EMS_OK;
}

ems_status ems_debug_host_transport(const ems_config* cfg, const ems_geometry* geo, const ems_primary* prim,
                                   uint64_t n, uint32_t n_events, const uint32_t* keys, double* edep,
                                   ems_ledger* ledger, ems_step_record* log, uint64_t log_cap, uint64_t* log_n) {
  ems_config c2 = *cfg;
  c2.max_events = n_events ? n_events : 1;
  ems_status st = check_inputs(&c2, geo);
  if (st) return st;
  if (!edep || !ledger || (n && !prim)) return fail(EMS_E_INVALID, "null buffers");
  if (geo->n_boxes) {
    if (c2.precision == EMS_MIXED)
      return host_transport<float, 1>(c2, geo, prim, n, n_events, keys, edep, ledger, log, log_cap, log_n);
    return host_transport<double, 1>(c2, geo, prim, n, n_events, keys, edep, ledger, log, log_cap, log_n);
  }
  if (c2.precision == EMS_MIXED)
    return host_transport<float, 0>(c2, geo, prim, n, n_events, keys, edep, ledger, log, log_cap, log_n);
  return host_transport<double, 0>(c2, geo, prim, n, n_events, keys, edep, ledger, log, log_cap, log_n);
}

}  // extern "C"

namespace {

// Breadth-first host loop over the same step code as the kernels (test hook).
template <class R, int GEO>
ems_status host_transport(const ems_config& c2, const ems_geometry* geo, const ems_primary* prim, uint64_t n,
                          uint32_t n_events, const uint32_t* keys, double* edep, ems_ledger* ledger,
                          ems_step_record* log, uint64_t log_cap, uint64_t* log_n) {
  TableSet ts = tables_for(&c2, geo);
  StepEnv<R> env = retype<R>(env_for(&c2, geo, ts));
  std::vector<char> packed;
  pack_tables<R>(ts, geo->n_materials, packed);
  std::vector<MatRT> rt = ts.rt;
  if (sizeof(R) == 4)
    for (MatRT& m : rt) inflate_bounds(m);
  const size_t gb = (geo->n_materials * kGammaTables * ts.nodes * sizeof(R) + 7) / 8 * 8;
  env.tg = reinterpret_cast<const R*>(packed.data());
  env.tl = reinterpret_cast<const R*>(packed.data() + gb);
  std::vector<uint32_t> vmat;
  BvhHost bvh;
  if (geo->n_boxes) {
    std::string err;
    if (!build_bvh(geo->box_lo, geo->box_hi, geo->n_boxes, bvh, err)) return fail(EMS_E_INVALID, err);
    env.nav = host_nav(geo, bvh);
    vmat.assign(geo->box_material, geo->box_material + geo->n_boxes);
    vmat.push_back(geo->world_material);
    env.zplane = nullptr;
    env.slab_mat = vmat.data();
  } else {
    env.zplane = geo->z_mm;
    env.slab_mat = geo->material;
  }
  env.mat = rt.data();
  std::vector<char> elem;
  pack_elements<R>(ts, elem);
  env.elc = reinterpret_cast<const double*>(elem.data());
  env.elt = reinterpret_cast<const R*>(elem.data() + ts.elc.size() * sizeof(double));
  std::vector<uint64_t> rows(n_events, 0);
  std::vector<uint32_t> row_keys(n_events);
  for (uint32_t e = 0; e < n_events; ++e) row_keys[e] = keys ? keys[e] : e;
  std::vector<InjRec> recs;
  ems_status st = prepare(*geo, &env.nav, n_events, prim, n, rows, row_keys, recs);
  if (st) return st;
  const uint32_t nc = n_cols(geo);
  memset(edep, 0, sizeof(double) * n_events * nc);
  memset(ledger, 0, sizeof(ems_ledger) * n_events);
  std::vector<Trk<R>> cur[3], nxt[3];
  for (const InjRec& r : recs) {
    Trk<R> t{r.x, r.y, r.z, (R)r.ux, (R)r.uy, (R)r.uz, r.E, r.id, r.ev, r.key, 0, r.slab};
    cur[r.sp].push_back(t);
  }
  struct HostSink {
    const ems_geometry* geo;
    double* edep;
    ems_ledger* ledger;
    ems_step_record* log;
    uint64_t log_cap, nlog;
    void apply(int sp, const Trk<R>& t, const StepOut<R>& o, double e0) {
      ems_ledger& L = ledger[t.ev];
      edep[(size_t)t.ev * n_cols(geo) + o.slab] += o.dep;
      L.escaped[sp] += o.escaped;
      L.killed += o.killed;
      L.charged_len += o.clen;
      L.n_steps += 1;
      L.n_null += o.null;
      L.n_pair += o.pair;
      L.n_annih += o.annih;
      for (int k = 0; k < o.nsec; ++k) L.n_created[o.sec[k].sp] += 1;
      if (log && nlog < log_cap) {
        ems_step_record& r = log[nlog];
        r.event = t.ev;
        r.species = (uint32_t)sp;
        r.id = t.id;
        r.step = t.n - 1;
        r.slab_after = t.slab;
        r.limiter = o.limiter;
        r.process = o.process;
        r.e_before = e0;
        r.e_after = t.E;
        r.pos_after[0] = t.x;
        r.pos_after[1] = t.y;
        r.pos_after[2] = t.z;
        r.step_len = o.step_len;
        r.edep = o.dep;
      }
      ++nlog;
    }
  } sink{geo, edep, ledger, log, log_cap, 0};
  const int max_visit = (int)c2.steps_per_visit;
  for (;;) {
    if (cur[0].empty() && cur[1].empty() && cur[2].empty()) break;
    for (int sp = 0; sp < 3; ++sp) {
      for (Trk<R> t : cur[sp]) {
        VisitState<R> vs;
        StepOut<R> o;
        visit_begin<2>(env, sp, t, vs);
        for (;;) {
          const double e0 = t.E;
          const bool end = visit_step<2, R, GEO>(env, sp, vs, t, o, max_visit);
          if (o.pending) interact<2>(env, t, o);
          sink.apply(sp, t, o, e0);
          if (end) break;
        }
        if (o.nsec > 0) {
          for (int k = 0; k < o.nsec; ++k) {
            const Sec<R>& s = o.sec[k];
            nxt[s.sp].push_back(Trk<R>{t.x, t.y, t.z, s.ux, s.uy, s.uz, s.E, s.id, t.ev, t.key, 0, o.slab});
          }
        }
        if (t.slab >= 0) nxt[sp].push_back(t);
      }
      cur[sp].clear();
    }
    for (int sp = 0; sp < 3; ++sp) cur[sp].swap(nxt[sp]);
  }
  const uint64_t nlog = sink.nlog;
  for (uint32_t e = 0; e < n_events; ++e) {
    double s = 0.0;
    for (uint32_t k = 0; k < nc; ++k) s += edep[(size_t)e * nc + k];
    ledger[e].edep = s;
  }
  if (log_n) *log_n = nlog;
  return EMS_OK;
}

}  // namespace

namespace ems {

ems_status rt_enqueue(ems_ctx* c, const ems_primary* p, uint64_t n) {
  if (n == 0) return EMS_OK;
  if (!p) return fail(EMS_E_INVALID, "null primaries");
  if (c->source == 2)
    return fail(EMS_E_STATE, "primaries of this batch came from device memory: reset the tallies before enqueueing from "
                             "host memory");
  uint64_t add[3] = {0, 0, 0};
  for (uint64_t i = 0; i < n; ++i)
    if (p[i].species <= EMS_POSITRON) add[p[i].species] += 1;
  for (int s = 0; s < 3; ++s)
    if (c->pending[s] + add[s] > c->L.cap) return fail(EMS_E_CAPACITY, "queue capacity exceeded by primaries");
  std::vector<uint64_t> rows = c->row_count;
  std::vector<InjRec> recs;
  ems_status st = prepare(c->geo, &c->nav, c->cfg.max_events, p, n, rows, c->keys, recs);
  if (st) return st;
  for (uint64_t done = 0; done < n; done += c->L.inj_chunk) {
    const uint32_t k = (uint32_t)std::min<uint64_t>(c->L.inj_chunk, n - done);
    HIPCHK(c, hipStreamSynchronize(c->stream));  // pinned staging is free again
    memcpy(c->pin_inj, recs.data() + done, k * sizeof(InjRec));
    InjRec* d = reinterpret_cast<InjRec*>(c->ws + c->L.inj);
    HIPCHK(c, hipMemcpyAsync(d, c->pin_inj, k * sizeof(InjRec), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_inject(c->args, d, k, c->stream));
  }
  c->row_count.swap(rows);
  for (int s = 0; s < 3; ++s) c->pending[s] += add[s];
  c->source = 1;
  return EMS_OK;
}

ems_status rt_enqueue_device(ems_ctx* c, const ems_primary* p, uint64_t n) {
  static_assert(sizeof(ems_primary) == sizeof(PrimRec) && offsetof(ems_primary, ekin_MeV) == offsetof(PrimRec, E) &&
                    offsetof(ems_primary, dir) == offsetof(PrimRec, dir),
                "primary layout");
  if (n == 0) return EMS_OK;
  if (!p) return fail(EMS_E_INVALID, "null primaries");
  if (c->source == 1)
    return fail(EMS_E_STATE, "primaries of this batch came from host memory: reset the tallies before enqueueing from "
                             "device memory");
  if (n > (1ull << 40) || !device_range(p, n * sizeof(ems_primary)))
    return fail(EMS_E_INVALID, "primaries are not n records in one device allocation");
  const Layout& L = c->L;
  uint32_t* keys = reinterpret_cast<uint32_t*>(c->ws + L.dkey);
  if (c->keys_dirty) {
    HIPCHK(c, hipMemcpyAsync(keys, c->keys.data(), c->keys.size() * 4, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->keys_dirty = false;
  }
  unsigned long long* chk = reinterpret_cast<unsigned long long*>(c->ws + L.dchk);
  HIPCHK(c, launch_fill_zero(chk, sizeof(c->chk_host), c->stream));
  HIPCHK(c, launch_check_primaries(c->args, p, n, chk, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->chk_host, chk, sizeof(c->chk_host), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->chk_host[0]) return fail(EMS_E_INVALID, "invalid primary #" + std::to_string(n - c->chk_host[0]));
  for (int s = 0; s < 3; ++s)
    if (c->pending[s] + c->chk_host[1 + s] > c->L.cap) return fail(EMS_E_CAPACITY, "queue capacity exceeded by primaries");
  InjRec* d = reinterpret_cast<InjRec*>(c->ws + L.inj);
  unsigned long long* rows = reinterpret_cast<unsigned long long*>(c->ws + L.drow);
  for (uint64_t done = 0; done < n; done += L.inj_chunk) {
    const uint32_t k = (uint32_t)std::min<uint64_t>(L.inj_chunk, n - done);
    HIPCHK(c, launch_stage_primaries(c->args, p + done, k, keys, rows, d, c->stream));
    HIPCHK(c, launch_inject(c->args, d, k, c->stream));
  }
  for (int s = 0; s < 3; ++s) c->pending[s] += c->chk_host[1 + s];
  c->source = 2;
  return EMS_OK;
}

// The kernels of one chunk: census, then K iterations (photon launch, e-/e+
// launch), with a HIP event after every launch when timing (direct
// launches only: events recorded inside a graph are not timeable here).
// Returns the first error.
static hipError_t enqueue_chunk(ems_ctx* c, uint32_t K, bool timing) {
  hipError_t e = launch_census(c->args, c->stream);
  if (e == hipSuccess && timing) e = hipEventRecord(c->evk[0], c->stream);
  for (uint32_t k = 0; k < K && e == hipSuccess; ++k) {
    if (c->args.cap_s) e = launch_short(c->args, c->blocks_s, c->stream);
    if (e == hipSuccess && timing) e = hipEventRecord(c->evk[3 * k + 1], c->stream);
    if (e == hipSuccess) e = launch_visit(c->args, true, c->blocks_g, c->stream);
    if (e == hipSuccess && timing) e = hipEventRecord(c->evk[3 * k + 2], c->stream);
    if (e == hipSuccess) e = launch_visit(c->args, false, c->blocks_l, c->stream);
    if (e == hipSuccess && timing) e = hipEventRecord(c->evk[3 * k + 3], c->stream);
  }
  return e;
}

// Capture one chunk of K iterations as a graph.  The kernels read every
// changing quantity from the device control block, so one graph serves all
// chunks; it holds kernel nodes only (no memset or event nodes).
static hipError_t capture_chunk(ems_ctx* c, uint32_t K) {
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return e;
  const hipError_t el = enqueue_chunk(c, K, false);
  e = hipStreamEndCapture(c->stream, &g);
  if (el != hipSuccess) e = el;
  if (e == hipSuccess) e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  if (e == hipSuccess) c->graph_k = K;
  else c->graph = nullptr;
  return e;
}

ems_status rt_chunk(ems_ctx* c, uint32_t K) {
  const bool timing = (c->cfg.flags & EMS_F_KERNEL_TIMING) != 0;
  while (timing && c->evk.size() < 3 * (size_t)K + 1) {
    hipEvent_t e = nullptr;
    HIPCHK(c, hipEventCreate(&e));
    c->evk.push_back(e);
  }
  bool graph = !timing && !(c->cfg.flags & EMS_F_NO_GRAPH) && c->stream != nullptr && !c->graph_off;
  if (graph && c->graph && c->graph_k != K) {
    HIPCHK(c, hipGraphExecDestroy(c->graph));
    c->graph = nullptr;
  }
  if (graph && !c->graph && capture_chunk(c, K) != hipSuccess) {
    // capture not available here: launch directly from now on
    (void)hipGetLastError();
    c->graph_off = true;
    graph = false;
  }
  const bool span = c->ev0 != nullptr;  // contexts without allocations keep no events
  if (span) HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  if (graph) {
    HIPCHK(c, hipGraphLaunch(c->graph, c->stream));
    c->stats.graph_launches += 1;
  } else {
    HIPCHK(c, enqueue_chunk(c, K, timing));
  }
  if (span) HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->pin_ctl, c->ws + c->L.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  float ms = 0.0f;
  if (span) HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  const Ctl& s = *c->pin_ctl;
  ems_run_stats& st = c->stats;
  st.step_kernel_ms += ms;
  for (uint32_t k = 0; timing && k < K; ++k) {
    float a = 0.0f, b = 0.0f, d = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&d, c->evk[3 * k], c->evk[3 * k + 1]));
    HIPCHK(c, hipEventElapsedTime(&a, c->evk[3 * k + 1], c->evk[3 * k + 2]));
    HIPCHK(c, hipEventElapsedTime(&b, c->evk[3 * k + 2], c->evk[3 * k + 3]));
    st.kernel_ms[0] += a;
    st.kernel_ms[1] += b;
    st.kernel_ms[2] += d;
  }
  st.made_by[0] = s.made_by[0];
  st.made_by[1] = s.made_by[1];
  st.launches += K;
  st.iterations = s.iteration;
  for (int i = 0; i < 3; ++i) {
    st.steps[i] = s.steps[i];
    st.visits[i] = s.visits[i];
    st.created[i] = s.created[i];
    st.peak_live[i] = s.peak[i];
  }
  st.deferred = s.deferred;
  st.short_steps = s.steps_s;
  st.steplog_overflow = (c->args.log_cap && s.log_n > c->args.log_cap) ? 1u : 0u;
  if (s.error & kErrOverflow) {
    c->failed = true;
    return fail(EMS_E_CAPACITY, "track queue overflow");
  }
  if (s.error & kErrStall) {
    c->failed = true;
    return fail(EMS_E_CAPACITY, "track queues too small to make progress");
  }
  if (s.error & kErrCorrupt) {
    c->failed = true;
    return fail(EMS_E_STATE, "a queue record indexed outside the tallies or the slab stack");
  }
  return EMS_OK;
}

ems_status rt_reset_rows(ems_ctx* c, const uint32_t* rows, uint32_t n) {
  if (!c->pin_rows) return fail(EMS_E_STATE, "row lists need EMS_F_EVENT_LIVE");
  if (n == 0) return EMS_OK;
  for (uint32_t i = 0; i < n; ++i)
    if (rows[i] >= c->cfg.max_events) return fail(EMS_E_INVALID, "row out of range");
  HIPCHK(c, hipStreamSynchronize(c->stream));  // pinned row list is free again
  memcpy(c->pin_rows, rows, n * 4ull);
  uint32_t* d = reinterpret_cast<uint32_t*>(c->ws + c->L.rows);
  HIPCHK(c, hipMemcpyAsync(d, c->pin_rows, n * 4ull, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_reset_rows(c->args, d, n, c->stream));
  for (uint32_t i = 0; i < n; ++i) c->row_count[rows[i]] = 0;
  return EMS_OK;
}

ems_status rt_gather_rows(ems_ctx* c, const uint32_t* rows, uint32_t n, double* edep, ems_ledger* ledger) {
  if (!c->pin_rows) return fail(EMS_E_STATE, "row lists need EMS_F_EVENT_LIVE");
  if (n == 0) return EMS_OK;
  for (uint32_t i = 0; i < n; ++i)
    if (rows[i] >= c->cfg.max_events) return fail(EMS_E_INVALID, "row out of range");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  memcpy(c->pin_rows, rows, n * 4ull);
  uint32_t* d = reinterpret_cast<uint32_t*>(c->ws + c->L.rows);
  const size_t stride = c->ncols * 8ull + sizeof(LedgerDev);
  HIPCHK(c, hipMemcpyAsync(d, c->pin_rows, n * 4ull, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, launch_gather_rows(c->args, d, n, c->ws + c->L.gather, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->pin_gather, c->ws + c->L.gather, n * stride, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (uint32_t i = 0; i < n; ++i) {
    const char* src = c->pin_gather + i * stride;
    double* e = edep + (size_t)i * c->ncols;
    memcpy(e, src, c->ncols * 8ull);
    memcpy(&ledger[i], src + c->ncols * 8ull, sizeof(LedgerDev));
    double sum = 0.0;
    for (uint32_t k = 0; k < c->ncols; ++k) sum += e[k];
    ledger[i].edep = sum;
  }
  return EMS_OK;
}

ems_status rt_take_exits(ems_ctx* c, std::vector<ems_primary>& out, uint64_t* total) {
  out.clear();
  *total = c->pin_ctl->exit_n;  // as of the last chunk's status read
  const uint64_t k = std::min<uint64_t>(*total, c->cfg.exit_capacity);
  if (*total == 0) return EMS_OK;
  out.resize(k);
  if (k) HIPCHK(c, hipMemcpyAsync(out.data(), c->ws + c->L.exits, k * sizeof(ExitRec), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, launch_fill_zero(c->ws + c->L.ctl + offsetof(Ctl, exit_n), sizeof(unsigned long long), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->pin_ctl->exit_n = 0;
  return EMS_OK;
}

ems_status rt_read_live(ems_ctx* c, int32_t* host) {
  HIPCHK(c, hipMemcpyAsync(host, c->ws + c->L.live, c->cfg.max_events * 4ull, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return EMS_OK;
}

}  // namespace ems
