// Batched form of the solve: many independent problems in one call.
//
// Problems are grouped by solver handle and right-hand-side count.  The
// batch fixes a packed layout in which every group is one contiguous slab,
// so a group is solved by the batched passes of its solver in one launch per
// pass (its problems and right-hand sides are just more lines of the same
// launch).  The whole batch can be captured once into a HIP graph whose
// groups hang off forked streams, so independent groups overlap on the GPU
// and a replay costs one graph launch.

#include <hip/hip_runtime.h>

#include <new>
#include <vector>

#include "hofem.h"
#include "kernels.h"

namespace {

constexpr int kSideStreams = 4;

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Group {
  hofem_solver solver;
  int nrhs_each;
  int nprob = 0;
  size_t per_rhs = 0;
  size_t offset = 0;      // values
  size_t ws_offset[4] = {0, 0, 0, 0};   // bytes, per mode
  size_t ws_bytes[4] = {0, 0, 0, 0};
};

}  // namespace

struct hofem_batch_s {
  int count = 0;
  std::vector<Group> groups;
  std::vector<size_t> offsets;   // count + 1 values
  size_t ws_total[4] = {0, 0, 0, 0};
  // graph cache: one instantiated graph for the last (mode, buffers, iterations)
  hipGraphExec_t exec = nullptr;
  int g_mode = -1, g_iter = -1;
  const void* g_f = nullptr;
  void* g_u = nullptr;
  void* g_ws = nullptr;
  hipStream_t side[kSideStreams] = {};
  std::vector<hipEvent_t> events;
  bool warm[4] = {false, false, false, false};
};

namespace {

int run_groups(hofem_batch_s* B, int mode, const void* f_dev, void* u_dev, void* ws_dev,
               int max_iter, hipStream_t origin, bool forked) {
  const size_t es = mode == HOFEM_MODE_FP32 ? sizeof(float) : sizeof(double);
  hipError_t e;
  if (forked) {
    e = hipEventRecord(B->events[0], origin);
    if (e != hipSuccess) return hofem::record_hip_error(e);
  }
  for (size_t g = 0; g < B->groups.size(); ++g) {
    const Group& G = B->groups[g];
    hipStream_t st = origin;
    if (forked) {
      st = B->side[g % kSideStreams];
      e = hipStreamWaitEvent(st, B->events[0], 0);
      if (e != hipSuccess) return hofem::record_hip_error(e);
    }
    const unsigned char* f = static_cast<const unsigned char*>(f_dev) + G.offset * es;
    unsigned char* u = static_cast<unsigned char*>(u_dev) + G.offset * es;
    void* ws = G.ws_bytes[mode] ? static_cast<unsigned char*>(ws_dev) + G.ws_offset[mode] : nullptr;
    const int rc = hofem_solve(G.solver, mode, f, u, G.nprob * G.nrhs_each, ws, G.ws_bytes[mode],
                               max_iter, 0.0, st, nullptr);
    if (rc != HOFEM_OK) return rc;
    if (forked) {
      e = hipEventRecord(B->events[1 + g], st);
      if (e == hipSuccess) e = hipStreamWaitEvent(origin, B->events[1 + g], 0);
      if (e != hipSuccess) return hofem::record_hip_error(e);
    }
  }
  return HOFEM_OK;
}

void drop_graph(hofem_batch_s* B) {
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  B->exec = nullptr;
  B->g_mode = -1;
}

}  // namespace

extern "C" {

int hofem_batch_create(const hofem_batch_problem* probs, int count, hofem_batch* out) {
  if (!probs || count < 1 || !out) return HOFEM_EINVAL;
  hofem_batch B = new (std::nothrow) hofem_batch_s;
  if (!B) return HOFEM_ENOMEM;
  B->count = count;
  std::vector<int> gid(count);
  for (int p = 0; p < count; ++p) {
    if (!probs[p].solver || probs[p].nrhs < 1) {
      delete B;
      return HOFEM_EINVAL;
    }
    int g = -1;
    for (size_t i = 0; i < B->groups.size(); ++i)
      if (B->groups[i].solver == probs[p].solver && B->groups[i].nrhs_each == probs[p].nrhs) {
        g = (int)i;
        break;
      }
    if (g < 0) {
      Group G{};
      G.solver = probs[p].solver;
      G.nrhs_each = probs[p].nrhs;
      if (hofem_solver_size(G.solver, &G.per_rhs) != HOFEM_OK) {
        delete B;
        return HOFEM_EINVAL;
      }
      B->groups.push_back(G);
      g = (int)B->groups.size() - 1;
    }
    gid[p] = g;
    B->groups[g].nprob++;
  }
  // packed layout: groups in order of first appearance, problems in input order
  size_t off = 0;
  for (Group& G : B->groups) {
    G.offset = off;
    off += (size_t)G.nprob * G.nrhs_each * G.per_rhs;
  }
  B->offsets.assign(count + 1, 0);
  std::vector<size_t> next(B->groups.size());
  for (size_t g = 0; g < B->groups.size(); ++g) next[g] = B->groups[g].offset;
  for (int p = 0; p < count; ++p) {
    Group& G = B->groups[gid[p]];
    B->offsets[p] = next[gid[p]];
    next[gid[p]] += (size_t)G.nrhs_each * G.per_rhs;
  }
  B->offsets[count] = off;
  // workspace per mode: one region per group (groups may run concurrently)
  for (int mode = 0; mode < 3; ++mode) {
    size_t w = 0;
    for (Group& G : B->groups) {
      size_t b = 0;
      if (hofem_solver_workspace_bytes(G.solver, mode, G.nprob * G.nrhs_each, &b) != HOFEM_OK) {
        delete B;
        return HOFEM_EINVAL;
      }
      G.ws_offset[mode] = w;
      G.ws_bytes[mode] = b;
      w += align256(b);
    }
    B->ws_total[mode] = w;
  }
  for (int i = 0; i < kSideStreams; ++i) {
    if (hipStreamCreateWithFlags(&B->side[i], hipStreamNonBlocking) != hipSuccess) {
      hofem_batch_destroy(B);
      return HOFEM_EHIP;
    }
  }
  B->events.assign(B->groups.size() + 1, nullptr);
  for (hipEvent_t& ev : B->events) {
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      hofem_batch_destroy(B);
      return HOFEM_EHIP;
    }
  }
  *out = B;
  return HOFEM_OK;
}

void hofem_batch_destroy(hofem_batch B) {
  if (!B) return;
  drop_graph(B);
  for (hipEvent_t ev : B->events)
    if (ev) (void)hipEventDestroy(ev);
  for (hipStream_t s : B->side)
    if (s) (void)hipStreamDestroy(s);
  delete B;
}

int hofem_batch_offsets(hofem_batch B, size_t* out_host, size_t len) {
  if (!B || !out_host || len != (size_t)B->count + 1) return HOFEM_EINVAL;
  for (size_t i = 0; i < len; ++i) out_host[i] = B->offsets[i];
  return HOFEM_OK;
}

int hofem_batch_groups(hofem_batch B, int* groups) {
  if (!B || !groups) return HOFEM_EINVAL;
  *groups = (int)B->groups.size();
  return HOFEM_OK;
}

int hofem_batch_workspace_bytes(hofem_batch B, int mode, size_t* bytes) {
  if (!B || !bytes || mode < 0 || mode > 2) return HOFEM_EINVAL;
  *bytes = B->ws_total[mode];
  return HOFEM_OK;
}

int hofem_batch_solve(hofem_batch B, int mode, const void* f_dev, void* u_dev, void* ws_dev,
                      size_t ws_bytes, int max_iter, int use_graph, void* stream) {
  if (!B || !f_dev || !u_dev || mode < 0 || mode > 2 || max_iter < 0) return HOFEM_EINVAL;
  if (mode == HOFEM_MODE_FP32_IR && f_dev == u_dev) return HOFEM_EINVAL;
  if (ws_bytes < B->ws_total[mode] || (B->ws_total[mode] && !ws_dev)) return HOFEM_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!use_graph || !B->warm[mode] || st == nullptr) {
    // eager: every group on the caller's stream (this also performs the
    // one-time kernel set-up that must not happen inside a capture; the
    // legacy default stream cannot be captured)
    const int rc = run_groups(B, mode, f_dev, u_dev, ws_dev, max_iter, st, false);
    if (rc == HOFEM_OK) B->warm[mode] = true;
    return rc;
  }
  if (!(B->exec && B->g_mode == mode && B->g_f == f_dev && B->g_u == u_dev &&
        B->g_ws == ws_dev && B->g_iter == max_iter)) {
    drop_graph(B);
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hofem::record_hip_error(e);
    const int rc = run_groups(B, mode, f_dev, u_dev, ws_dev, max_iter, st, true);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(st, &graph);
    if (rc != HOFEM_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hofem::record_hip_error(e);
    e = hipGraphInstantiate(&B->exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      B->exec = nullptr;
      return hofem::record_hip_error(e);
    }
    B->g_mode = mode;
    B->g_f = f_dev;
    B->g_u = u_dev;
    B->g_ws = ws_dev;
    B->g_iter = max_iter;
  }
  hipError_t e = hipGraphLaunch(B->exec, st);
  if (e != hipSuccess) return hofem::record_hip_error(e);
  return HOFEM_OK;
}

}  // extern "C"
