// gconn_api.hip -- the extern "C" entry points declared in include/gconn.h:
// host-side argument checks, workspace sizing, and the incremental handle.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>

#include "gconn_internal.hpp"

namespace gconn {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

gconn_status fail(gconn_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

gconn_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return GCONN_EDEVICE;
}

bool is_union_find(int link) {
  return link == GCONN_LINK_ASYNC || link == GCONN_LINK_HOOKS || link == GCONN_LINK_EARLY ||
         link == GCONN_LINK_REM_CAS || link == GCONN_LINK_ECL || link == GCONN_LINK_AFFOREST ||
         link == GCONN_LINK_REM_LOCK || link == GCONN_LINK_JTB;
}

gconn_status check_options(const gconn_options& o) {
  if (o.sample < GCONN_SAMPLE_NONE || o.sample > GCONN_SAMPLE_BFS)
    return fail(GCONN_EINVAL, "options.sample out of range");
  if (o.link < GCONN_LINK_ASYNC || o.link > GCONN_LINK_JTB)
    return fail(GCONN_EINVAL, "options.link out of range");
  if (o.find < GCONN_FIND_NAIVE || o.find > GCONN_FIND_TWO_TRY_SPLIT)
    return fail(GCONN_EINVAL, "options.find out of range");
  if (o.link == GCONN_LINK_JTB) {
    if (o.find != GCONN_FIND_NAIVE && o.find != GCONN_FIND_TWO_TRY_SPLIT)
      return fail(GCONN_EUNSUPPORTED, "Union-JTB finds are FindSimple (NAIVE) or TwoTrySplit");
    if (o.sample != GCONN_SAMPLE_NONE && o.sample != GCONN_SAMPLE_KOUT)
      return fail(GCONN_EUNSUPPORTED, "Union-JTB samples with k-out or not at all");
  } else if (o.find == GCONN_FIND_TWO_TRY_SPLIT) {
    return fail(GCONN_EUNSUPPORTED, "FIND_TWO_TRY_SPLIT belongs to Union-JTB");
  }
  if (o.splice < GCONN_SPLICE_SPLIT_ONE || o.splice > GCONN_SPLICE_ATOMIC)
    return fail(GCONN_EINVAL, "options.splice out of range");
  if (o.lt_variant < 0 || o.lt_variant >= GCONN_LT_COUNT)
    return fail(GCONN_EINVAL, "options.lt_variant out of range");
  if ((o.link == GCONN_LINK_REM_CAS || o.link == GCONN_LINK_REM_LOCK) &&
      o.find == GCONN_FIND_COMPRESS)
    return fail(GCONN_EUNSUPPORTED,
                "Union-Rem-CAS / Rem-Lock combine with FindNaive, FindSplit or FindHalve only");
  if (o.k < 1 || o.k > 64) return fail(GCONN_EINVAL, "options.k must be in [1, 64]");
  if (o.hb_n < 1 || o.hb_n > 1024) return fail(GCONN_EINVAL, "options.hb_n must be in [1, 1024]");
  if (o.lmax_samples < 1 || o.lmax_samples > kMaxLmaxSamples)
    return fail(GCONN_EINVAL, "options.lmax_samples must be in [1, 4096]");
  if (o.schedule < 0 || o.schedule > 6) return fail(GCONN_EINVAL, "options.schedule out of range");
  if (o.atomic_compress != 0 && o.atomic_compress != 1)
    return fail(GCONN_EINVAL, "options.atomic_compress must be 0 or 1");
  if (o.kout_prelink != 0 && o.kout_prelink != 1)
    return fail(GCONN_EINVAL, "options.kout_prelink must be 0 or 1");
  if (o.kout_local != 0 && o.kout_local != 1)
    return fail(GCONN_EINVAL, "options.kout_local must be 0 or 1");
  if (o.block < 64 || o.block > 1024 || (o.block % 64) != 0)
    return fail(GCONN_EINVAL, "options.block must be a multiple of 64 in [64, 1024]");
  return GCONN_OK;
}

gconn_status check_device_ptr(const void* p, const char* name) {
  if (!p) return fail(GCONN_EINVAL, std::string(name) + " is NULL");
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();  // do not leave the query's error for a later launch check
    return fail(GCONN_EINVAL, std::string(name) + " is not device-accessible memory");
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged &&
      attr.type != hipMemoryTypeHost && attr.type != hipMemoryTypeUnified)
    return fail(GCONN_EINVAL, std::string(name) + " is not device-accessible memory");
  return GCONN_OK;
}

gconn_status check_device_ready() {
  static std::mutex mu;
  static int checked[64] = {0};  // 0 unknown, 1 ok, -1 not gfx950
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(GCONN_ENODEV, "no HIP device");
  }
  if (dev < 0 || dev >= 64) return fail(GCONN_ENODEV, "unexpected device index");
  std::lock_guard<std::mutex> lock(mu);
  if (checked[dev] == 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
      (void)hipGetLastError();
      return fail(GCONN_ENODEV, "hipGetDeviceProperties failed");
    }
    checked[dev] = (std::strncmp(prop.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
  }
  if (checked[dev] < 0) return fail(GCONN_ENODEV, "current device is not gfx950");
  return GCONN_OK;
}

gconn_status check_graph(const gconn_graph* g) {
  if (!g) return fail(GCONN_EINVAL, "graph is NULL");
  if (g->format != GCONN_CSR && g->format != GCONN_COO)
    return fail(GCONN_EINVAL, "graph.format must be GCONN_CSR or GCONN_COO");
  if (g->n > 0xFFFFFFFEu) return fail(GCONN_EINVAL, "graph.n must be <= 0xFFFFFFFE");
  if (g->format == GCONN_CSR) {
    if (!g->offsets_64 && g->m > 0xFFFFFFFFull)
      return fail(GCONN_EINVAL, "m exceeds uint32 offsets; pass uint64 offsets");
    if (g->n > 0 || g->m > 0) GCONN_TRY(check_device_ptr(g->offsets, "graph.offsets"));
    if (g->m > 0) GCONN_TRY(check_device_ptr(g->nbrs, "graph.nbrs"));
  } else {
    if (g->m > 0) {
      GCONN_TRY(check_device_ptr(g->nbrs, "graph.nbrs (COO src)"));
      GCONN_TRY(check_device_ptr(g->dst, "graph.dst"));
    }
  }
  return GCONN_OK;
}

static gconn_status resolve_options(const gconn_options* opt, gconn_options* out) {
  if (opt) *out = *opt;
  else gconn_options_default(out);
  return check_options(*out);
}

static gconn_status check_workspace(void* ws, size_t have, size_t need) {
  if (have < need)
    return fail(GCONN_ENOMEM, "workspace has " + std::to_string(have) + " bytes, needs " +
                                  std::to_string(need));
  GCONN_TRY(check_device_ptr(ws, "workspace"));
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(GCONN_EINVAL, "workspace must be 256-byte aligned");
  return GCONN_OK;
}

}  // namespace gconn

using namespace gconn;

// Scratch memory of gconn_cc_noalloc: a file-scope device array, so that the
// call needs no allocation.  Each device the library runs on holds its own
// copy (GCONN_NOALLOC_SCRATCH_BYTES) until the process ends.  In host code the
// array's name is only a host-side stand-in: its device address is taken once
// per device with hipGetSymbolAddress and only that address reaches kernels.
static __device__ __align__(256) uint8_t scratch[GCONN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_dev[kMaxScratchDevices] = {};

// Device address of the current device's scratch array (looked up on the
// first call made with that device current).
gconn_status scratch_on_current_device(uint8_t** out) {
  int dev = -1;
  GCONN_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(GCONN_ENODEV, "device index " + std::to_string(dev) + " out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    GCONN_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0)
      return fail(GCONN_EDEVICE, "scratch array has no 256-byte aligned device address");
    g_scratch_dev[dev] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch_dev[dev];
  return GCONN_OK;
}

}  // namespace

struct gconn_inc {
  uint32_t n_max;
  uint32_t* P;
  uint32_t* H;
  uint64_t* W;  // Union-JTB words (in the workspace), else NULL
  uint8_t* ws;
  size_t ws_bytes;
  gconn_options opt;
};

struct gconn_exec {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// Record body(stream) on a private non-blocking stream into a HIP graph and
// instantiate it.  Argument checks happen before; nothing runs on the device.
template <class Body>
gconn_status capture_exec(Body&& body, gconn_exec** out) {
  if (gconn::profiling())
    return gconn::fail(GCONN_EUNSUPPORTED, "phase profiling is on: its events cannot be captured");
  hipStream_t cs = nullptr;
  GCONN_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return gconn::hip_fail(e, "hipStreamBeginCapture");
  }
  const gconn_status st = body(cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (st != GCONN_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return gconn::hip_fail(e, "hipStreamEndCapture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return gconn::hip_fail(e, "hipGraphInstantiate");
  }
  gconn_exec* h = new (std::nothrow) gconn_exec;
  if (!h) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return gconn::fail(GCONN_EINVAL, "host allocation of the handle failed");
  }
  h->graph = graph;
  h->exec = exec;
  *out = h;
  return GCONN_OK;
}

}  // namespace

extern "C" {

void gconn_options_default(gconn_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->sample = GCONN_SAMPLE_KOUT;
  o->link = GCONN_LINK_ASYNC;
  o->find = GCONN_FIND_SPLIT;
  o->splice = GCONN_SPLICE_SPLIT_ONE;
  o->lt_variant = GCONN_LT_PRF;
  o->k = 2;
  o->hb_n = 4;
  o->lmax_samples = 1024;
  o->seed = 1;
  o->kout_random = 0;
  o->validate = 0;
  o->block = 256;
  o->schedule = 0;
  o->atomic_compress = 1;
  o->kout_prelink = 0;
  o->kout_local = 0;
}

gconn_status gconn_workspace_size(const gconn_graph* g, const gconn_options* opt, int want_forest,
                                  int want_labels, size_t* bytes) {
  clear_error();
  if (!g || !bytes) return fail(GCONN_EINVAL, "graph or bytes is NULL");
  gconn_options o;
  GCONN_TRY(resolve_options(opt, &o));
  if (g->format != GCONN_CSR && g->format != GCONN_COO)
    return fail(GCONN_EINVAL, "graph.format must be GCONN_CSR or GCONN_COO");
  *bytes = plan_workspace(*g, o, want_forest != 0, want_labels != 0).total;
  return GCONN_OK;
}

gconn_status gconn_cc(const gconn_graph* g, uint32_t* labels_out, void* workspace,
                      size_t workspace_bytes, const gconn_options* opt, gconn_stats* stats,
                      void* stream) {
  clear_error();
  gconn_options o;
  GCONN_TRY(resolve_options(opt, &o));
  GCONN_TRY(check_device_ready());
  GCONN_TRY(check_graph(g));
  if (g->format == GCONN_COO) o.sample = GCONN_SAMPLE_NONE;
  if (g->n > 0) GCONN_TRY(check_device_ptr(labels_out, "labels_out"));
  const WsLayout L = plan_workspace(*g, o, false, true);
  GCONN_TRY(check_workspace(workspace, workspace_bytes, L.total));
  return run_static(*g, labels_out, nullptr, nullptr, true, static_cast<uint8_t*>(workspace), L, o,
                    stats, static_cast<hipStream_t>(stream));
}

gconn_status gconn_cc_noalloc(const gconn_graph* g, uint32_t* labels_out,
                              const gconn_options* opt, gconn_stats* stats, void* stream) {
  clear_error();
  gconn_options o;
  GCONN_TRY(resolve_options(opt, &o));
  // Phase profiling creates HIP events on first use; this entry point makes
  // no such call.
  if (gconn::profiling())
    return fail(GCONN_EUNSUPPORTED, "phase profiling is on: gconn_cc_noalloc does not time phases");
  GCONN_TRY(check_device_ready());
  GCONN_TRY(check_graph(g));
  if (g->format == GCONN_COO) o.sample = GCONN_SAMPLE_NONE;
  if (g->n > 0) GCONN_TRY(check_device_ptr(labels_out, "labels_out"));
  const WsLayout L = plan_workspace(*g, o, false, true);
  if (L.total > GCONN_NOALLOC_SCRATCH_BYTES)
    return fail(GCONN_ENOMEM, "graph and options need " + std::to_string(L.total) +
                                  " bytes of scratch; gconn_cc_noalloc has " +
                                  std::to_string((size_t)GCONN_NOALLOC_SCRATCH_BYTES) +
                                  " (use gconn_cc with a workspace)");
  uint8_t* ws = nullptr;
  GCONN_TRY(scratch_on_current_device(&ws));
  return run_static(*g, labels_out, nullptr, nullptr, true, ws, L, o, stats,
                    static_cast<hipStream_t>(stream));
}

gconn_status gconn_spanning_forest(const gconn_graph* g, uint32_t* fu, uint32_t* fv,
                                   uint32_t* labels_out, void* workspace, size_t workspace_bytes,
                                   const gconn_options* opt, gconn_stats* stats, void* stream) {
  clear_error();
  gconn_options o;
  GCONN_TRY(resolve_options(opt, &o));
  if (o.link == GCONN_LINK_LT || o.link == GCONN_LINK_LP)
    return fail(GCONN_EUNSUPPORTED,
                "spanning forest needs a root-based finish: a union-find rule or SV");
  if ((o.link == GCONN_LINK_REM_CAS || o.link == GCONN_LINK_REM_LOCK) &&
      o.splice == GCONN_SPLICE_ATOMIC)
    return fail(GCONN_EUNSUPPORTED,
                "spanning forests need root-based links; Rem's splice re-hangs non-roots "
                "without an edge to record");
  GCONN_TRY(check_device_ready());
  GCONN_TRY(check_graph(g));
  if (g->format == GCONN_COO) o.sample = GCONN_SAMPLE_NONE;
  if (g->n > 0) {
    GCONN_TRY(check_device_ptr(fu, "fu"));
    GCONN_TRY(check_device_ptr(fv, "fv"));
    if (labels_out) GCONN_TRY(check_device_ptr(labels_out, "labels_out"));
  }
  const bool labels = labels_out != nullptr;
  const WsLayout L = plan_workspace(*g, o, true, labels);
  GCONN_TRY(check_workspace(workspace, workspace_bytes, L.total));
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  uint32_t* P = labels ? labels_out : reinterpret_cast<uint32_t*>(ws + L.P);
  return run_static(*g, P, fu, fv, labels, ws, L, o, stats, static_cast<hipStream_t>(stream));
}

gconn_status gconn_inc_workspace_size(uint32_t n_max, const gconn_graph* initial,
                                      const gconn_options* opt, size_t* bytes) {
  clear_error();
  if (!bytes) return fail(GCONN_EINVAL, "bytes is NULL");
  gconn_options o;
  GCONN_TRY(resolve_options(opt, &o));
  size_t total = align_up(sizeof(Ctrl), 256);
  if (needs_claims(o.link)) total += align_up(4ull * n_max + 1, 256);
  if (o.link == GCONN_LINK_JTB) total += align_up(8ull * n_max + 1, 256);
  if (initial) total += plan_workspace(*initial, o, false, true).total;
  *bytes = total;
  return GCONN_OK;
}

gconn_status gconn_inc_create(uint32_t n_max, uint32_t* parent_buf, const gconn_graph* initial,
                              void* workspace, size_t workspace_bytes, const gconn_options* opt,
                              void* stream, gconn_inc** out) {
  clear_error();
  if (!out) return fail(GCONN_EINVAL, "out is NULL");
  *out = nullptr;
  gconn_options o;
  GCONN_TRY(resolve_options(opt, &o));
  if (!is_union_find(o.link))
    return fail(GCONN_EUNSUPPORTED, "incremental batches use a union-find rule");
  if (n_max > 0xFFFFFFFEu) return fail(GCONN_EINVAL, "n_max must be <= 0xFFFFFFFE");
  GCONN_TRY(check_device_ready());
  if (n_max > 0) GCONN_TRY(check_device_ptr(parent_buf, "parent_buf"));
  if (initial) {
    GCONN_TRY(check_graph(initial));
    if (initial->n > n_max) return fail(GCONN_EINVAL, "initial graph has more than n_max vertices");
  }
  size_t need = 0;
  GCONN_TRY(gconn_inc_workspace_size(n_max, initial, &o, &need));
  GCONN_TRY(check_workspace(workspace, workspace_bytes, need));
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint8_t* ws = static_cast<uint8_t*>(workspace);
  size_t at = align_up(sizeof(Ctrl), 256);
  uint32_t* H = nullptr;
  uint64_t* W = nullptr;
  if (needs_claims(o.link)) {
    H = reinterpret_cast<uint32_t*>(ws + at);
    at += align_up(4ull * n_max + 1, 256);
  }
  if (o.link == GCONN_LINK_JTB) {
    W = reinterpret_cast<uint64_t*>(ws + at);
    at += align_up(8ull * n_max + 1, 256);
    GCONN_TRY(launch_jtb_init(W, n_max, s));
  } else {
    GCONN_TRY(launch_iota(parent_buf, n_max, s));
  }
  if (H) GCONN_TRY(launch_fill(H, 0xFFFFFFFFu, n_max, s));
  if (initial && initial->n > 0) {
    gconn_options io = o;
    if (initial->format == GCONN_COO) io.sample = GCONN_SAMPLE_NONE;
    const WsLayout L = plan_workspace(*initial, io, false, true);
    if (W)
      GCONN_TRY(run_static_jtb(*initial, nullptr, nullptr, nullptr, false, ws + at, L, io, nullptr,
                               s, W));
    else
      GCONN_TRY(
          run_static(*initial, parent_buf, nullptr, nullptr, true, ws + at, L, io, nullptr, s));
  }
  gconn_inc* h = new (std::nothrow) gconn_inc;
  if (!h) return fail(GCONN_EINVAL, "host allocation of the handle failed");
  h->n_max = n_max;
  h->P = parent_buf;
  h->H = H;
  h->W = W;
  h->ws = ws;
  h->ws_bytes = workspace_bytes;
  h->opt = o;
  *out = h;
  return GCONN_OK;
}

static gconn_status validate_ids(gconn_inc* h, const uint32_t* a, const uint32_t* b, uint64_t k,
                                 hipStream_t s);

gconn_status gconn_inc_insert_batch(gconn_inc* h, const uint32_t* src, const uint32_t* dst,
                                    uint64_t k, void* stream) {
  clear_error();
  if (!h) return fail(GCONN_EINVAL, "handle is NULL");
  if (k == 0) return GCONN_OK;
  GCONN_TRY(check_device_ptr(src, "src"));
  GCONN_TRY(check_device_ptr(dst, "dst"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->opt.validate) GCONN_TRY(validate_ids(h, src, dst, k, s));
  if (h->W) return launch_jtb_insert(h->opt, h->W, src, dst, k, s);
  return launch_insert(h->opt, h->P, h->H, src, dst, k, s);
}

gconn_status gconn_inc_query_batch(gconn_inc* h, const uint32_t* a, const uint32_t* b, uint64_t q,
                                   uint8_t* out, void* stream) {
  clear_error();
  if (!h) return fail(GCONN_EINVAL, "handle is NULL");
  if (q == 0) return GCONN_OK;
  GCONN_TRY(check_device_ptr(a, "a"));
  GCONN_TRY(check_device_ptr(b, "b"));
  GCONN_TRY(check_device_ptr(out, "out"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->opt.validate) GCONN_TRY(validate_ids(h, a, b, q, s));
  if (h->W) return launch_jtb_query(h->opt, h->W, nullptr, a, b, q, out, s);
  return launch_query(h->opt, h->P, a, b, q, out, s);
}

gconn_status gconn_inc_mixed_batch(gconn_inc* h, const uint8_t* kind, const uint32_t* a,
                                   const uint32_t* b, uint64_t count, uint8_t* out, void* stream) {
  clear_error();
  if (!h) return fail(GCONN_EINVAL, "handle is NULL");
  if (count == 0) return GCONN_OK;
  GCONN_TRY(check_device_ptr(kind, "kind"));
  GCONN_TRY(check_device_ptr(a, "a"));
  GCONN_TRY(check_device_ptr(b, "b"));
  GCONN_TRY(check_device_ptr(out, "out"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->opt.validate) {
    GCONN_TRY(validate_ids(h, a, b, count, s));
    GCONN_TRY(validate_kinds(kind, count, reinterpret_cast<Ctrl*>(h->ws), s));
  }
  if (h->W) return launch_jtb_mixed(h->opt, h->W, kind, a, b, count, out, s);
  return launch_mixed(h->opt, h->P, h->H, kind, a, b, count, out, s);
}

gconn_status gconn_inc_labels(gconn_inc* h, uint32_t* labels_out, void* stream) {
  clear_error();
  if (!h) return fail(GCONN_EINVAL, "handle is NULL");
  if (h->n_max == 0) return GCONN_OK;
  GCONN_TRY(check_device_ptr(labels_out, "labels_out"));
  if (h->W)
    return launch_jtb_labels(h->W, h->n_max, labels_out, h->P, static_cast<hipStream_t>(stream));
  return launch_finalize(h->P, h->n_max, labels_out, static_cast<hipStream_t>(stream));
}

gconn_status gconn_inc_destroy(gconn_inc* h) {
  clear_error();
  delete h;
  return GCONN_OK;
}

gconn_status gconn_cc_batch_workspace_size(const gconn_batch* b, size_t* bytes) {
  clear_error();
  return batch_workspace_size(b, bytes);
}

gconn_status gconn_cc_batch(const gconn_batch* b, uint32_t* labels_out, void* workspace,
                            size_t workspace_bytes, const gconn_class_options* classes,
                            uint32_t num_classes, uint32_t lmax_samples, uint64_t seed,
                            gconn_stats* stats, void* stream) {
  clear_error();
  return run_batch(b, labels_out, workspace, workspace_bytes, classes, num_classes, lmax_samples,
                   seed, stats, static_cast<hipStream_t>(stream));
}

gconn_status gconn_autotune(const gconn_graph* graphs, uint32_t num_graphs,
                            const gconn_options* candidates, uint32_t num_candidates,
                            uint32_t reps, uint32_t* labels_scratch, void* workspace,
                            size_t workspace_bytes, void* stream, uint32_t* best,
                            double* times_ms) {
  clear_error();
  return autotune(graphs, num_graphs, candidates, num_candidates, reps, labels_scratch, workspace,
                  workspace_bytes, static_cast<hipStream_t>(stream), best, times_ms);
}

gconn_status gconn_cc_capture(const gconn_graph* g, uint32_t* labels_out, void* workspace,
                              size_t workspace_bytes, const gconn_options* opt, gconn_exec** out) {
  clear_error();
  if (!out) return fail(GCONN_EINVAL, "out is NULL");
  *out = nullptr;
  gconn_options o;
  GCONN_TRY(resolve_options(opt, &o));
  if (!is_union_find(o.link))
    return fail(GCONN_EUNSUPPORTED, "SV, LT and LP check their rounds on the host: not capturable");
  if (o.sample == GCONN_SAMPLE_BFS)
    return fail(GCONN_EUNSUPPORTED, "BFS sampling checks its frontier on the host: not capturable");
  if (o.validate) return fail(GCONN_EUNSUPPORTED, "validation synchronises: not capturable");
  GCONN_TRY(check_device_ready());
  GCONN_TRY(check_graph(g));
  if (g->format == GCONN_COO) o.sample = GCONN_SAMPLE_NONE;
  if (g->n > 0) GCONN_TRY(check_device_ptr(labels_out, "labels_out"));
  const WsLayout L = plan_workspace(*g, o, false, true);
  GCONN_TRY(check_workspace(workspace, workspace_bytes, L.total));
  const gconn_graph gc = *g;
  return capture_exec(
      [&](hipStream_t cs) {
        return run_static(gc, labels_out, nullptr, nullptr, true, static_cast<uint8_t*>(workspace),
                          L, o, nullptr, cs);
      },
      out);
}

gconn_status gconn_cc_batch_capture(const gconn_batch* b, uint32_t* labels_out, void* workspace,
                                    size_t workspace_bytes, const gconn_class_options* classes,
                                    uint32_t num_classes, uint32_t lmax_samples, uint64_t seed,
                                    gconn_exec** out) {
  clear_error();
  if (!out) return fail(GCONN_EINVAL, "out is NULL");
  *out = nullptr;
  if (!b) return fail(GCONN_EINVAL, "batch is NULL");
  const gconn_batch bc = *b;
  return capture_exec(
      [&](hipStream_t cs) {
        return run_batch(&bc, labels_out, workspace, workspace_bytes, classes, num_classes,
                         lmax_samples, seed, nullptr, cs);
      },
      out);
}

gconn_status gconn_exec_launch(gconn_exec* e, void* stream) {
  clear_error();
  if (!e) return fail(GCONN_EINVAL, "handle is NULL");
  GCONN_HIP(hipGraphLaunch(e->exec, static_cast<hipStream_t>(stream)));
  return GCONN_OK;
}

gconn_status gconn_exec_destroy(gconn_exec* e) {
  clear_error();
  if (!e) return GCONN_OK;
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->graph) (void)hipGraphDestroy(e->graph);
  delete e;
  return GCONN_OK;
}

gconn_status gconn_profile_enable(int on) { return profile_enable(on); }

gconn_status gconn_profile_read(gconn_phase_times* out, int reset) {
  clear_error();
  return profile_read(out, reset);
}

const char* gconn_status_string(gconn_status s) {
  switch (s) {
    case GCONN_OK: return "GCONN_OK";
    case GCONN_EINVAL: return "GCONN_EINVAL: invalid argument";
    case GCONN_ENOMEM: return "GCONN_ENOMEM: workspace too small";
    case GCONN_EDEVICE: return "GCONN_EDEVICE: HIP error";
    case GCONN_ENODEV: return "GCONN_ENODEV: no gfx950 device";
    case GCONN_EBUSY: return "GCONN_EBUSY: admission refused";
    case GCONN_ETIMEOUT: return "GCONN_ETIMEOUT: bounded wait expired";
    case GCONN_EUNSUPPORTED: return "GCONN_EUNSUPPORTED: unsupported option combination";
  }
  return "unknown gconn_status";
}

const char* gconn_last_error(void) { return g_last_error.c_str(); }

const char* gconn_version(void) { return "gconn-gfx950 0.1.0"; }

}  // extern "C"

static gconn_status validate_ids(gconn_inc* h, const uint32_t* a, const uint32_t* b, uint64_t k,
                                 hipStream_t s) {
  return validate_pairs(a, b, k, h->n_max, reinterpret_cast<Ctrl*>(h->ws), s);
}
