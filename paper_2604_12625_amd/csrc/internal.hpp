// Host-side internals shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <map>
#include <string>
#include <tuple>

#include "ndgi.h"

namespace ndgi {

// thread-local message of the last failed call
int fail(int code, const char* fmt, ...);
void clear_error();

#define NDGI_HIP(expr)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) return ::ndgi::fail(NDGI_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// (layout kind: 0 ndgi_model, 1 + widths + 4 border hybrid; models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, prec, stream)
using GraphKey = std::tuple<int, const void*, int32_t, const void*, const void*, int32_t, int32_t,
                            void*, int64_t, int32_t, hipStream_t>;

// Workgroups of 256 threads that one launch may keep resident: CUs x the kernel's
// occupancy (so a persistent or grid-stride grid runs in one round), capped by the
// launch shape's waves per CU.
int resident_wgs(const ndgi_ctx* ctx, const void* kernel);

// per-wave gradient partial slots reserved for the decoder weights
constexpr int kPartialStride = 1712;   // >= NDGI_MLP_SIZE, multiple of 16

}  // namespace ndgi

struct ndgi_ctx {
  int device = 0;
  int n_cu = 0;
  int tile_w = 1, tile_h = 4, waves_per_cu = 32;  // page decode launch shape
  hipStream_t capture_stream = nullptr;
  uint32_t* flags_dev = nullptr;
  void* scratch_dev = nullptr;   // this device's copy of the static scratch of decode_binned_noalloc
  void* dec_ws = nullptr;        // workspace reserved by ndgi_reserve_decode (binned route of ndgi_decode)
  int64_t dec_ws_bytes = 0;
  // training workspace
  int train_waves = 0;          // persistent waves of the training kernel
  float* partials_dev = nullptr;  // [train_waves][kPartialStride]
  double* loss_part_dev = nullptr;  // [train_waves]
  float* stage_dev = nullptr;     // [train_waves / 64 + 1][kPartialStride]: first reduction stage
  std::map<ndgi::GraphKey, hipGraphExec_t> graphs;
  std::map<const void*, int> occupancy;   // kernel -> resident 256-thread workgroups per CU
};

namespace ndgi {
// Where the block encoders read 8-bit texels: texels in memory (u8 != NULL: [blocks][16][C],
// texel s = 4 row + col), or a block-parameterised map of a hybrid training state
// (endpoints [..][H/4][W/4][4][2], weights [..][H][W][4] or, codec 1, [..][H][W]) reconstructed
// as kind (kSrcLerp, kSrcRounded, kSrcDirect) says; a footprint of the map is one block of 4
// channels.
struct TexSrc {
  const uint8_t* u8;
  int C;
  const float* ep;
  const float* w;
  int W, H, codec, kind;
};
// n blocks (BC7: footprints; BC4: footprint * 4 + channel for a map source) into out.
int launch_encode(const TexSrc& S, int codec, int64_t n, uint8_t* out, int n_cu, hipStream_t s);
int check_model(const ndgi_model* m, const char* who);
int launch_decode(ndgi_ctx* ctx, const ndgi_model& m, const float* uvt, int64_t n, void* out, int prec,
                  hipStream_t s);
int launch_pages(ndgi_ctx* ctx, const ndgi_model* models, int32_t n_models, const ndgi_page_req* reqs,
                 const int32_t* n_reqs, int32_t max_reqs, int32_t page, void* dst, int64_t pitch, int prec,
                 hipStream_t s);
int launch_bc4_blocks(const uint8_t* blocks, int64_t n, uint8_t* out, int impl, hipStream_t s);
int launch_bc7_blocks(const uint8_t* blocks, int64_t n, uint8_t* out, hipStream_t s);
int launch_import_map(const uint8_t* blocks, int codec, int W, int H, int S, float* w, int n_cu, hipStream_t s);
int binned_workspace(const ndgi_model& m, int64_t n, int64_t* bytes);
// Whether ndgi_decode takes the binned kernels for n queries on m with a reserved workspace
// of ws_bytes: the map bins, there are at least kRouteQueriesPerTile queries per tile on
// average, and the workspace holds the layout.
constexpr int64_t kRouteQueriesPerTile = 100;
bool binned_route(const ndgi_model& m, int64_t n, int64_t ws_bytes);
int launch_decode_binned(ndgi_ctx* ctx, const ndgi_model& m, const float* uvt, int64_t n, void* out, int prec,
                         void* ws, int64_t ws_bytes, hipStream_t s);
int check_hybrid(const ndgi_hybrid_model* m, const char* who);
int launch_adam(ndgi_ctx* c, float* p, float* g, float* m, float* v, int64_t n, int64_t clamp_end, int64_t off_mlp,
                float lr_feat, float lr_mlp, float beta1, float beta2, float eps, int64_t step, hipStream_t s);
int launch_fill_zero(ndgi_ctx* c, float* p, int64_t n, hipStream_t s);
int launch_convert(ndgi_ctx* c, const float* src, void* dst, int dt, int64_t n, hipStream_t s);
int launch_hybrid_query(ndgi_ctx* ctx, const ndgi_hybrid_model& m, const float* uvt, int64_t n, void* out, int prec,
                        hipStream_t s);
int launch_hybrid_pages(ndgi_ctx* ctx, const ndgi_hybrid_model* models, int32_t n_models, const ndgi_page_req* reqs,
                        const int32_t* n_reqs, int32_t max_reqs, int32_t page, void* dst, int64_t pitch, int prec,
                        int32_t widths, int32_t border, hipStream_t s);
}  // namespace ndgi
