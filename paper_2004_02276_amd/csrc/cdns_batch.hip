// cdns_batch.hip -- batched runner over many resident instances.
//
// A batch holds up to kMaxSlots solver contexts.  Their descriptors are
// mirrored into a device array and a work table (active instances and the
// prefix sums of their work items per phase kind).  One RK step of the
// whole batch is a fixed sequence of persistent kernels -- one launch per
// phase for all instances -- captured once as a HIP graph; attaching or
// detaching an instance rewrites the descriptor array and the table only.
#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "../../include/cdns.h"
#include "cdns_internal.h"

namespace cdns {
const Desc& ctx_desc(const cdns_ctx* c);
int& ctx_batch_refs(cdns_ctx* c);
}  // namespace cdns

using cdns::BatchTable;
using cdns::Desc;

struct cdns_batch {
  int max_slots = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  Desc* descs_dev = nullptr;
  BatchTable* tab_dev = nullptr;
  std::vector<cdns_ctx*> slot;
  std::vector<double> cfl, dtf;
  std::vector<Desc> descs_h;
  BatchTable tab_h{};
  bool dirty = true;
  hipGraphExec_t gexec = nullptr;
  int tile_x = 0, tile_y = 0, precision = -1;
  int64_t steps = 0;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

void drop_graph(cdns_batch* b) {
  if (b->gexec) {
    (void)hipGraphExecDestroy(b->gexec);
    b->gexec = nullptr;
  }
}

hipError_t enqueue_batch_step(cdns_batch* b, hipStream_t st) {
  using namespace cdns;
  hipError_t e;
  auto ph = [&](int p, int stage) {
    return launch_batch_phase(p, b->descs_dev, b->tab_dev, stage, b->tile_x, b->tile_y,
                              b->precision, st);
  };
  if ((e = ph(BPH_DT_PART, 0)) != hipSuccess) return e;
  if ((e = ph(BPH_DT_FINAL, 0)) != hipSuccess) return e;
  for (int stage = 0; stage < 3; ++stage) {
    const int seq[] = {BPH_BEGIN, BPH_GHOST_X, BPH_GHOST_Y, BPH_SENSOR, BPH_IFLAGS,
                       BPH_WENO,  BPH_RHS,     BPH_FORCE, BPH_RK};
    for (int p : seq)
      if ((e = ph(p, stage)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Rebuild the host table and upload descriptors + table (synchronously, so
// the host copies may change right after).
hipError_t upload(cdns_batch* b) {
  BatchTable& T = b->tab_h;
  std::memset(&T, 0, sizeof(T));
  int n = 0;
  for (int s = 0; s < b->max_slots; ++s) {
    if (!b->slot[s]) continue;
    Desc D = cdns::ctx_desc(b->slot[s]);
    D.cfl = b->cfl[s];
    D.dt_fixed = b->dtf[s] > 0.0 ? b->dtf[s] : 0.0;
    b->descs_h[s] = D;
    T.inst[n++] = s;
  }
  T.ninst = n;
  for (int k = 0; k < cdns::WK_COUNT; ++k) {
    T.pre[k][0] = 0;
    for (int a = 0; a < n; ++a)
      T.pre[k][a + 1] = T.pre[k][a] + cdns::batch_items(b->descs_h[T.inst[a]], k);
  }
  hipError_t e = hipMemcpyAsync(b->descs_dev, b->descs_h.data(), b->max_slots * sizeof(Desc),
                                hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->tab_dev, &T, sizeof(T), hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e == hipSuccess) b->dirty = false;
  return e;
}

}  // namespace

extern "C" {

size_t cdns_batch_workspace_bytes(int32_t max_slots) {
  if (max_slots < 1 || max_slots > cdns::kMaxSlots) return 0;
  return align_up((size_t)max_slots * sizeof(Desc)) + align_up(sizeof(BatchTable));
}

cdns_status cdns_batch_create(int32_t max_slots, void* workspace_dev, size_t workspace_bytes,
                              void* hip_stream, cdns_batch** out) {
  if (!out) return CDNS_EINVAL;
  *out = nullptr;
  if (max_slots < 1 || max_slots > cdns::kMaxSlots || !workspace_dev) return CDNS_EINVAL;
  if (((uintptr_t)workspace_dev) % kAlign != 0) return CDNS_EINVAL;
  if (workspace_bytes < cdns_batch_workspace_bytes(max_slots)) return CDNS_ENOMEM;
  cdns_batch* b = new cdns_batch();
  b->max_slots = max_slots;
  b->stream = (hipStream_t)hip_stream;
  b->descs_dev = (Desc*)workspace_dev;
  b->tab_dev = (BatchTable*)((char*)workspace_dev + align_up((size_t)max_slots * sizeof(Desc)));
  b->slot.assign(max_slots, nullptr);
  b->cfl.assign(max_slots, 0.8);
  b->dtf.assign(max_slots, 0.0);
  b->descs_h.resize(max_slots);
  std::memset(b->descs_h.data(), 0, max_slots * sizeof(Desc));
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return CDNS_EHIP;
  }
  if (upload(b) != hipSuccess) {
    (void)hipStreamDestroy(b->cap);
    delete b;
    return CDNS_EHIP;
  }
  *out = b;
  return CDNS_OK;
}

cdns_status cdns_batch_attach(cdns_batch* b, cdns_ctx* ctx, int32_t* slot) {
  if (!b || !ctx || !slot) return CDNS_EINVAL;
  const Desc& D = cdns::ctx_desc(ctx);
  if (D.bc[0] == cdns::BC_DF_INFLOW) return CDNS_EUNSUP;  // per-step inflow state not batched
  if (D.cl != 2 || D.wr != 3) return CDNS_EUNSUP;           // batched kernels: default orders
  for (int s = 0; s < b->max_slots; ++s)
    if (b->slot[s] == ctx) return CDNS_EBUSY;
  bool any = false;
  for (int s = 0; s < b->max_slots; ++s) any |= b->slot[s] != nullptr;
  if (any && (D.tile_x != b->tile_x || D.tile_y != b->tile_y || D.precision != b->precision))
    return CDNS_EINVAL;  // one tile shape and precision per batch
  for (int s = 0; s < b->max_slots; ++s) {
    if (b->slot[s]) continue;
    if (!any) {
      if (D.tile_x != b->tile_x || D.tile_y != b->tile_y || D.precision != b->precision)
        drop_graph(b);
      b->tile_x = D.tile_x;
      b->tile_y = D.tile_y;
      b->precision = D.precision;
    }
    b->slot[s] = ctx;
    b->cfl[s] = D.cfl > 0.0 ? D.cfl : 0.8;
    b->dtf[s] = 0.0;
    cdns::ctx_batch_refs(ctx) += 1;
    b->dirty = true;
    *slot = s;
    return CDNS_OK;
  }
  return CDNS_EBUSY;
}

cdns_status cdns_batch_detach(cdns_batch* b, int32_t s) {
  if (!b || s < 0 || s >= b->max_slots || !b->slot[s]) return CDNS_EINVAL;
  cdns::ctx_batch_refs(b->slot[s]) -= 1;
  b->slot[s] = nullptr;
  b->dirty = true;
  return CDNS_OK;
}

cdns_status cdns_batch_set_step(cdns_batch* b, int32_t s, double cfl, double dt_fixed) {
  if (!b || s < 0 || s >= b->max_slots || !b->slot[s]) return CDNS_EINVAL;
  if (!(dt_fixed > 0.0) && !(cfl > 0.0)) return CDNS_EINVAL;
  b->cfl[s] = cfl;
  b->dtf[s] = dt_fixed;
  b->dirty = true;
  return CDNS_OK;
}

cdns_status cdns_batch_step(cdns_batch* b, int32_t nsteps) {
  if (!b || nsteps < 0) return CDNS_EINVAL;
  hipError_t e;
  if (b->dirty && (e = upload(b)) != hipSuccess) return CDNS_EHIP;
  if (b->tab_h.ninst == 0 || nsteps == 0) return CDNS_OK;
  if (!b->gexec) {
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return CDNS_EHIP;
    hipError_t le = enqueue_batch_step(b, b->cap);
    e = hipStreamEndCapture(b->cap, &g);
    if (le != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return CDNS_EHIP;
    }
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->gexec = nullptr;
      return CDNS_EHIP;
    }
  }
  for (int i = 0; i < nsteps; ++i)
    if ((e = hipGraphLaunch(b->gexec, b->stream)) != hipSuccess) return CDNS_EHIP;
  b->steps += nsteps;
  return CDNS_OK;
}

cdns_status cdns_batch_destroy(cdns_batch* b) {
  if (!b) return CDNS_EINVAL;
  for (int s = 0; s < b->max_slots; ++s)
    if (b->slot[s]) cdns::ctx_batch_refs(b->slot[s]) -= 1;
  drop_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return CDNS_OK;
}

}  // extern "C"
