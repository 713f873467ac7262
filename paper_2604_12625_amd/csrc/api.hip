// C ABI entry points: argument validation, context lifecycle, graph capture.
#include <climits>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "internal.hpp"

namespace ndgi {

// Scratch of ndgi_decode_binned_noalloc: a file-scope device array, one copy on every GPU
// the library runs on, held until the process ends.  In host code the array's name is not
// a device address: its address on a device comes from hipGetSymbolAddress, taken once per
// device (with that device current) by ndgi_create and kept per device here and in the
// context.
static __device__ __align__(256) unsigned char scratch[NDGI_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current device.
static int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(NDGI_ERR_UNSUPPORTED, "create: device %d >= %d", device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(NDGI_ERR_HIP, "create: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return NDGI_OK;
}

static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

void clear_error() { g_last_error.clear(); }

int resident_wgs(const ndgi_ctx* ctx, const void* kernel) {
  auto& occ = const_cast<ndgi_ctx*>(ctx)->occupancy;
  auto it = occ.find(kernel);
  int per_cu;
  if (it == occ.end()) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kernel, 256, 0) != hipSuccess || b < 1) b = 1;
    occ[kernel] = b;
    per_cu = b;
  } else {
    per_cu = it->second;
  }
  const int cap = ctx->waves_per_cu / 4 > 0 ? ctx->waves_per_cu / 4 : 1;
  return ctx->n_cu * (per_cu < cap ? per_cu : cap);
}

int check_model(const ndgi_model* m, const char* who) {
  if (!m) return fail(NDGI_ERR_INVALID_ARG, "%s: model is NULL", who);
  if (m->W < 4 || m->H < 4 || m->W > 16384 || m->H > 16384 || (m->W & 3) || (m->H & 3))
    return fail(NDGI_ERR_INVALID_ARG, "%s: W, H must be multiples of 4 in [4, 16384] (got %d x %d)", who, m->W, m->H);
  if (m->Gw < 1 || m->Gh < 1 || m->Gw > 16384 || m->Gh > 16384)
    return fail(NDGI_ERR_INVALID_ARG, "%s: grid size %d x %d out of range", who, m->Gw, m->Gh);
  if (m->T < 1 || m->T > 1024) return fail(NDGI_ERR_INVALID_ARG, "%s: T=%d out of range", who, m->T);
  if ((m->grid_dtype != NDGI_DTYPE_F32 && m->grid_dtype != NDGI_DTYPE_F16) ||
      (m->mlp_dtype != NDGI_DTYPE_F32 && m->mlp_dtype != NDGI_DTYPE_F16))
    return fail(NDGI_ERR_INVALID_ARG, "%s: unknown dtype", who);
  if (m->reserved0 != 0) return fail(NDGI_ERR_INVALID_ARG, "%s: reserved0 must be 0", who);
  if (!m->bc4 || !m->grid || !m->mlp) return fail(NDGI_ERR_INVALID_ARG, "%s: NULL model buffer", who);
  const uint64_t grid_bytes = (uint64_t)m->T * m->Gh * m->Gw * 8 * (m->grid_dtype == NDGI_DTYPE_F16 ? 2 : 4);
  if (grid_bytes >= (1ull << 32) || (uint64_t)m->W * m->H * 4 >= (1ull << 32))
    return fail(NDGI_ERR_UNSUPPORTED, "%s: map or grid of 4 GiB or more", who);
  return NDGI_OK;
}

static int check_pages(ndgi_ctx* ctx, const ndgi_model* models, int32_t n_models, const ndgi_page_req* reqs,
                       const int32_t* n_reqs, int32_t max_reqs, int32_t page, void* dst, int64_t pitch, int32_t prec) {
  if (!ctx) return fail(NDGI_ERR_INVALID_ARG, "decode_pages: ctx is NULL");
  if (prec != NDGI_PREC_F32 && prec != NDGI_PREC_F16) return fail(NDGI_ERR_INVALID_ARG, "decode_pages: bad prec %d", prec);
  if (n_models < 0 || max_reqs < 0) return fail(NDGI_ERR_INVALID_ARG, "decode_pages: negative count");
  if (page < 16 || page > 4096 || (page & 15))
    return fail(NDGI_ERR_INVALID_ARG, "decode_pages: page=%d must be a multiple of 16 in [16, 4096]", page);
  if (page % (16 * ctx->tile_w) || page % (4 * ctx->tile_h))
    return fail(NDGI_ERR_INVALID_ARG, "decode_pages: page=%d is not a multiple of the sub-tile %dx%d", page,
                16 * ctx->tile_w, 4 * ctx->tile_h);
  if (pitch < page) return fail(NDGI_ERR_INVALID_ARG, "decode_pages: dst_pitch=%lld < page", (long long)pitch);
  if (!n_reqs || !dst || (n_models > 0 && !models) || (max_reqs > 0 && !reqs))
    return fail(NDGI_ERR_INVALID_ARG, "decode_pages: NULL pointer");
  return NDGI_OK;
}

// Replay the graph captured for `key`, capturing it on first use: `launch(stream)` issues
// the work on the context's capture stream.
template <typename Launch>
static int launch_graph(ndgi_ctx* c, const GraphKey& key, Launch launch) {
  auto it = c->graphs.find(key);
  hipStream_t s = std::get<10>(key);
  if (it == c->graphs.end()) {
    hipGraph_t graph = nullptr;
    NDGI_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    const int rc = launch(c->capture_stream);
    hipError_t e = hipStreamEndCapture(c->capture_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);   // the launch's own error is the one reported
      return rc;
    }
    if (e != hipSuccess) return fail(NDGI_ERR_HIP, "pages graph: capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);   // the executable graph does not need it
    if (e != hipSuccess) return fail(NDGI_ERR_HIP, "pages graph: instantiate failed: %s", hipGetErrorString(e));
    it = c->graphs.emplace(key, exec).first;
  }
  NDGI_HIP(hipGraphLaunch(it->second, s));
  return NDGI_OK;
}

}  // namespace ndgi

using namespace ndgi;

extern "C" {

const char* ndgi_last_error(void) { return g_last_error.c_str(); }

int ndgi_create(ndgi_ctx** out, int32_t device) {
  clear_error();
  if (!out) return fail(NDGI_ERR_INVALID_ARG, "create: out is NULL");
  *out = nullptr;
  int n = 0;
  NDGI_HIP(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(NDGI_ERR_INVALID_ARG, "create: device %d of %d", device, n);
  NDGI_HIP(hipSetDevice(device));
  ndgi_ctx* c = new ndgi_ctx();
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return fail(NDGI_ERR_HIP, "create: hipGetDeviceProperties failed");
  }
  c->n_cu = prop.multiProcessorCount;
  c->train_waves = c->n_cu * 8;
  if (const int rc = scratch_address(device, &c->scratch_dev)) {
    delete c;
    return rc;
  }
  bool ok = hipMalloc(&c->flags_dev, 256) == hipSuccess &&
            hipMalloc(&c->partials_dev, sizeof(float) * (size_t)c->train_waves * kPartialStride) == hipSuccess &&
            hipMalloc(&c->loss_part_dev, sizeof(double) * (size_t)c->train_waves) == hipSuccess &&
            hipMalloc(&c->stage_dev, sizeof(float) * (size_t)(c->train_waves / 64 + 1) * kPartialStride) ==
                hipSuccess &&
            hipMemset(c->flags_dev, 0, 256) == hipSuccess &&
            hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    ndgi_destroy(c);
    return fail(NDGI_ERR_OUT_OF_MEMORY, "create: workspace allocation failed");
  }
  *out = c;
  return NDGI_OK;
}

int ndgi_destroy(ndgi_ctx* c) {
  clear_error();
  if (!c) return NDGI_OK;
  // best-effort teardown: every release is attempted, the first failure is reported
  hipError_t first = hipSetDevice(c->device);
  auto keep = [&](hipError_t e) {
    if (first == hipSuccess) first = e;
  };
  for (auto& kv : c->graphs) keep(hipGraphExecDestroy(kv.second));
  if (c->capture_stream) keep(hipStreamDestroy(c->capture_stream));
  keep(hipFree(c->flags_dev));
  keep(hipFree(c->partials_dev));
  keep(hipFree(c->loss_part_dev));
  keep(hipFree(c->stage_dev));
  keep(hipFree(c->dec_ws));
  delete c;
  if (first != hipSuccess) return fail(NDGI_ERR_HIP, "destroy: %s", hipGetErrorString(first));
  return NDGI_OK;
}

int ndgi_get_error_flags(ndgi_ctx* c, hipStream_t s, uint32_t* flags_out) {
  clear_error();
  if (!c || !flags_out) return fail(NDGI_ERR_INVALID_ARG, "get_error_flags: NULL argument");
  NDGI_HIP(hipStreamSynchronize(s));
  uint32_t f = 0;
  NDGI_HIP(hipMemcpy(&f, c->flags_dev, sizeof(f), hipMemcpyDeviceToHost));
  NDGI_HIP(hipMemset(c->flags_dev, 0, sizeof(uint32_t)));
  *flags_out = f;
  return NDGI_OK;
}

int ndgi_bc4_decode_blocks(const uint8_t* blocks, int64_t n, uint8_t* out16, hipStream_t s) {
  clear_error();
  if (n < 0) return fail(NDGI_ERR_INVALID_ARG, "bc4_decode_blocks: n < 0");
  if (n == 0) return NDGI_OK;
  if (!blocks || !out16) return fail(NDGI_ERR_INVALID_ARG, "bc4_decode_blocks: NULL pointer");
  return launch_bc4_blocks(blocks, n, out16, 0, s);
}

int ndgi_bc4_decode_blocks_impl(const uint8_t* blocks, int64_t n, uint8_t* out16, int32_t impl, hipStream_t s) {
  clear_error();
  if (n < 0) return fail(NDGI_ERR_INVALID_ARG, "bc4_decode_blocks_impl: n < 0");
  if (impl < 0 || impl > 2) return fail(NDGI_ERR_INVALID_ARG, "bc4_decode_blocks_impl: impl %d", impl);
  if (n == 0) return NDGI_OK;
  if (!blocks || !out16) return fail(NDGI_ERR_INVALID_ARG, "bc4_decode_blocks_impl: NULL pointer");
  return launch_bc4_blocks(blocks, n, out16, impl, s);
}

int ndgi_bc7_decode_blocks(const uint8_t* blocks, int64_t n, uint8_t* out64, hipStream_t s) {
  clear_error();
  if (n < 0) return fail(NDGI_ERR_INVALID_ARG, "bc7_decode_blocks: n < 0");
  if (n == 0) return NDGI_OK;
  if (!blocks || !out64) return fail(NDGI_ERR_INVALID_ARG, "bc7_decode_blocks: NULL pointer");
  if (((uintptr_t)blocks | (uintptr_t)out64) & 15)
    return fail(NDGI_ERR_INVALID_ARG, "bc7_decode_blocks: blocks and out64 must be 16-byte aligned");
  return launch_bc7_blocks(blocks, n, out64, s);
}

int ndgi_decode(ndgi_ctx* c, const ndgi_model* m, const float* uvt, int64_t n, void* out, int32_t prec,
                hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "decode: ctx is NULL");
  if (n < 0) return fail(NDGI_ERR_INVALID_ARG, "decode: n < 0");
  if (prec != NDGI_PREC_F32 && prec != NDGI_PREC_F16) return fail(NDGI_ERR_INVALID_ARG, "decode: bad prec %d", prec);
  int rc = check_model(m, "decode");
  if (rc) return rc;
  if (n == 0) return NDGI_OK;
  if (!uvt || !out) return fail(NDGI_ERR_INVALID_ARG, "decode: NULL query/output pointer");
  if (c->dec_ws && binned_route(*m, n, c->dec_ws_bytes))
    return launch_decode_binned(c, *m, uvt, n, out, prec, c->dec_ws, c->dec_ws_bytes, s);
  return launch_decode(c, *m, uvt, n, out, prec, s);
}

int ndgi_reserve_decode(ndgi_ctx* c, const ndgi_model* m, int64_t max_queries) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "reserve_decode: ctx is NULL");
  if (max_queries < 0 || max_queries > INT32_MAX)
    return fail(NDGI_ERR_INVALID_ARG, "reserve_decode: max_queries out of [0, 2^31)");
  if (max_queries == 0) {
    if (c->dec_ws) {
      NDGI_HIP(hipSetDevice(c->device));
      NDGI_HIP(hipDeviceSynchronize());   // no decode of this context may still use it
      NDGI_HIP(hipFree(c->dec_ws));
    }
    c->dec_ws = nullptr;
    c->dec_ws_bytes = 0;
    return NDGI_OK;
  }
  int rc = check_model(m, "reserve_decode");
  if (rc) return rc;
  int64_t need = 0;
  rc = binned_workspace(*m, max_queries, &need);
  if (rc) return rc;
  if (need <= c->dec_ws_bytes) return NDGI_OK;   // the current reservation already holds it
  NDGI_HIP(hipSetDevice(c->device));
  void* p = nullptr;
  if (hipMalloc(&p, (size_t)need) != hipSuccess)
    return fail(NDGI_ERR_OUT_OF_MEMORY, "reserve_decode: %lld bytes", (long long)need);
  if (c->dec_ws) {
    NDGI_HIP(hipDeviceSynchronize());
    NDGI_HIP(hipFree(c->dec_ws));
  }
  c->dec_ws = p;
  c->dec_ws_bytes = need;
  return NDGI_OK;
}

int ndgi_decode_binned_workspace(const ndgi_model* m, int64_t n, int64_t* bytes_out) {
  clear_error();
  if (!bytes_out) return fail(NDGI_ERR_INVALID_ARG, "decode_binned_workspace: bytes_out is NULL");
  *bytes_out = 0;
  if (n < 0 || n > INT32_MAX) return fail(NDGI_ERR_INVALID_ARG, "decode_binned_workspace: n out of [0, 2^31)");
  int rc = check_model(m, "decode_binned_workspace");
  if (rc) return rc;
  return binned_workspace(*m, n, bytes_out);
}

int ndgi_decode_binned(ndgi_ctx* c, const ndgi_model* m, const float* uvt, int64_t n, void* out, int32_t prec,
                       void* workspace, int64_t workspace_bytes, hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "decode_binned: ctx is NULL");
  if (n < 0 || n > INT32_MAX) return fail(NDGI_ERR_INVALID_ARG, "decode_binned: n out of [0, 2^31)");
  if (prec != NDGI_PREC_F32 && prec != NDGI_PREC_F16)
    return fail(NDGI_ERR_INVALID_ARG, "decode_binned: bad prec %d", prec);
  int rc = check_model(m, "decode_binned");
  if (rc) return rc;
  if (n == 0) return NDGI_OK;
  if (!uvt || !out || !workspace) return fail(NDGI_ERR_INVALID_ARG, "decode_binned: NULL query/output/workspace");
  return launch_decode_binned(c, *m, uvt, n, out, prec, workspace, workspace_bytes, s);
}

int ndgi_decode_binned_noalloc(ndgi_ctx* c, const ndgi_model* m, const float* uvt, int64_t n, void* out,
                               int32_t prec, hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "decode_binned_noalloc: ctx is NULL");
  if (n < 0 || n > INT32_MAX) return fail(NDGI_ERR_INVALID_ARG, "decode_binned_noalloc: n out of [0, 2^31)");
  if (prec != NDGI_PREC_F32 && prec != NDGI_PREC_F16)
    return fail(NDGI_ERR_INVALID_ARG, "decode_binned_noalloc: bad prec %d", prec);
  int rc = check_model(m, "decode_binned_noalloc");
  if (rc) return rc;
  int64_t need = 0;
  rc = binned_workspace(*m, n, &need);
  if (rc) return rc;
  if (need > NDGI_NOALLOC_SCRATCH_BYTES)
    return fail(NDGI_ERR_INVALID_ARG,
                "decode_binned_noalloc: %lld queries on a %dx%d map need %lld bytes of scratch, above the static "
                "%lld bytes; decode in smaller batches or call ndgi_decode_binned with a workspace",
                (long long)n, m->W, m->H, (long long)need, (long long)NDGI_NOALLOC_SCRATCH_BYTES);
  if (n == 0) return NDGI_OK;
  if (!uvt || !out) return fail(NDGI_ERR_INVALID_ARG, "decode_binned_noalloc: NULL query/output");
  return launch_decode_binned(c, *m, uvt, n, out, prec, c->scratch_dev, NDGI_NOALLOC_SCRATCH_BYTES, s);
}

int ndgi_decode_pages(ndgi_ctx* c, const ndgi_model* models, int32_t n_models, const ndgi_page_req* reqs,
                      const int32_t* n_reqs, int32_t max_reqs, int32_t page, void* dst, int64_t pitch,
                      int32_t prec, hipStream_t s) {
  clear_error();
  int rc = check_pages(c, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, prec);
  if (rc) return rc;
  return launch_pages(c, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, prec, s);
}

int ndgi_decode_pages_graph(ndgi_ctx* c, const ndgi_model* models, int32_t n_models, const ndgi_page_req* reqs,
                            const int32_t* n_reqs, int32_t max_reqs, int32_t page, void* dst, int64_t pitch,
                            int32_t prec, hipStream_t s) {
  clear_error();
  int rc = check_pages(c, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, prec);
  if (rc) return rc;
  return launch_graph(c, GraphKey{0, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, prec, s},
                      [&](hipStream_t cs) {
                        return launch_pages(c, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, prec, cs);
                      });
}

int32_t ndgi_hybrid_mlp_size(int32_t hidden) {
  if (hidden != 16 && hidden != 64) return -1;
  return hidden * NDGI_HYBRID_IN + hidden + hidden * hidden + hidden + 3 * hidden + 3;
}

int ndgi_hybrid_decode(ndgi_ctx* c, const ndgi_hybrid_model* m, const float* uvt, int64_t n, void* out,
                       int32_t prec, hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode: ctx is NULL");
  if (n < 0) return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode: n < 0");
  if (prec != NDGI_PREC_F32 && prec != NDGI_PREC_F16)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode: bad prec %d", prec);
  int rc = check_hybrid(m, "hybrid_decode");
  if (rc) return rc;
  if (n == 0) return NDGI_OK;
  if (!uvt || !out) return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode: NULL query/output pointer");
  return launch_hybrid_query(c, *m, uvt, n, out, prec, s);
}

static int check_hybrid_pages(ndgi_ctx* c, const ndgi_hybrid_model* models, int32_t n_models,
                              const ndgi_page_req* reqs, const int32_t* n_reqs, int32_t max_reqs, int32_t page,
                              void* dst, int64_t pitch, int32_t prec, int32_t widths, int32_t border) {
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode_pages: ctx is NULL");
  if (widths < 0 || widths > 3) return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode_pages: widths=%d not in 0..3", widths);
  if (border < 0 || border > 32 || border > page)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode_pages: border=%d not in 0..min(32, page)", border);
  if (prec != NDGI_PREC_F32 && prec != NDGI_PREC_F16)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode_pages: bad prec %d", prec);
  if (n_models < 0 || max_reqs < 0) return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode_pages: negative count");
  if (page < 1 || page > 4096)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode_pages: page=%d not in [1, 4096]", page);
  if (pitch < page + 2 * border)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode_pages: dst_pitch=%lld < page + 2 border", (long long)pitch);
  if (!n_reqs || !dst || (n_models > 0 && !models) || (max_reqs > 0 && !reqs))
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_decode_pages: NULL pointer");
  return NDGI_OK;
}

int ndgi_hybrid_decode_pages(ndgi_ctx* c, const ndgi_hybrid_model* models, int32_t n_models,
                             const ndgi_page_req* reqs, const int32_t* n_reqs, int32_t max_reqs, int32_t page,
                             void* dst, int64_t pitch, int32_t prec, int32_t widths, int32_t border,
                             hipStream_t s) {
  clear_error();
  int rc = check_hybrid_pages(c, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, prec, widths, border);
  if (rc) return rc;
  return launch_hybrid_pages(c, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, prec, widths, border, s);
}

int ndgi_hybrid_decode_pages_graph(ndgi_ctx* c, const ndgi_hybrid_model* models, int32_t n_models,
                                   const ndgi_page_req* reqs, const int32_t* n_reqs, int32_t max_reqs,
                                   int32_t page, void* dst, int64_t pitch, int32_t prec, int32_t widths,
                                   int32_t border, hipStream_t s) {
  clear_error();
  int rc = check_hybrid_pages(c, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, prec, widths, border);
  if (rc) return rc;
  return launch_graph(c, GraphKey{1 + widths + 4 * border, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch,
                                  prec, s},
                      [&](hipStream_t cs) {
                        return launch_hybrid_pages(c, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch,
                                                   prec, widths, border, cs);
                      });
}

int ndgi_set_launch(ndgi_ctx* c, int32_t tile_w, int32_t tile_h, int32_t waves_per_cu) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "set_launch: ctx is NULL");
  if (tile_w < 1 || tile_w > 32 || tile_h < 1 || tile_h > 32 || waves_per_cu < 1 || waves_per_cu > 32)
    return fail(NDGI_ERR_INVALID_ARG, "set_launch: tile_w, tile_h, waves_per_cu must be in [1, 32]");
  NDGI_HIP(hipSetDevice(c->device));
  for (auto& kv : c->graphs) NDGI_HIP(hipGraphExecDestroy(kv.second));
  c->graphs.clear();
  c->tile_w = tile_w;
  c->tile_h = tile_h;
  c->waves_per_cu = waves_per_cu;
  return NDGI_OK;
}

}  // extern "C"
