/*
 * ndgi.h -- C ABI of the MI355X (gfx950) Neural Dynamic GI decode and training library.
 *
 * The method (arXiv 2604.12625) represents a set of time-varying lightmaps by feature
 * maps plus a small MLP: the lighting at (u, v, t) is I = H_Theta(u, v, t) (Sec. 3.1,
 * Eq. 3).  This library implements the data-parallel hot path of that representation
 * for two layouts: the paper's hybrid feature maps (section "hybrid layout" below) and
 * this one:
 *
 *   spatial map  W x H texels, 8 channels, each channel BC4 block-compressed
 *                (two 8-bit endpoints and sixteen 3-bit selectors per 4x4 block;
 *                Sec. 3.4, Eq. 6-7 and supplementary Sec. B)
 *   grid         Gw x Gh nodes x T time keys, 8 channels, FP32 or FP16, sampled
 *                bilinearly in space and linearly in time (the spatio-temporal feature
 *                map of Sec. 3.3)
 *   decoder      16 -> 32 -> 32 -> 3 MLP, ReLU hidden layers, exponential output
 *                (HDR RGB); inputs are [S_0..S_7, G_0..G_7]
 *
 * Conventions shared by every entry point
 *   - Every pointer named *_dev or documented as "device" is device memory of the GPU
 *     the context was created on; "host" pointers are ordinary host memory.
 *   - The caller owns every buffer it passes.  The library never frees caller memory
 *     and never allocates per call; a context owns only its own workspace.
 *   - Calls are asynchronous on the given stream (0 = the null stream).  Arguments are
 *     validated before anything is launched, so an argument error writes nothing.
 *     Faults inside kernels surface at the caller's next synchronisation.
 *   - Return value: NDGI_OK (0) or a negative NDGI_ERR_* code; ndgi_last_error()
 *     returns a message for the calling thread's last failure.  No C++ exception
 *     crosses this interface.
 *   - A context may be used by one host thread at a time.
 */
#ifndef NDGI_H
#define NDGI_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define NDGI_OK                0
#define NDGI_ERR_INVALID_ARG  (-1)
#define NDGI_ERR_UNSUPPORTED  (-2)
#define NDGI_ERR_HIP          (-3)
#define NDGI_ERR_OUT_OF_MEMORY (-4)

/* storage dtypes */
#define NDGI_DTYPE_F32 0
#define NDGI_DTYPE_F16 1

/* compute precision of the decode path
 *   NDGI_PREC_F32: FP32 feature math, FP32 matrix cores (MFMA), FP32 output [n][3]
 *   NDGI_PREC_F16: FP32 feature math rounded once to FP16, FP16 MFMA with FP32
 *                  accumulation, FP32 exp, FP16 output [n][3] */
#define NDGI_PREC_F32 0
#define NDGI_PREC_F16 1

/* device error flags (ndgi_get_error_flags) */
#define NDGI_FLAG_BAD_PAGE_REQUEST 1u
#define NDGI_FLAG_BAD_SAMPLE       2u  /* ndgi_train_step: a sample outside the state's map */

/* number of packed decoder parameters: [W1 32x16 | b1 32 | W2 32x32 | b2 32 | W3 3x32 | b3 3],
 * row-major W[out][in], layer y = W x + b */
#define NDGI_MLP_SIZE 1699

/* A compressed model Theta (Eq. 5) in the layout above.  64 bytes, the same layout on
 * host and device (ndgi_decode_pages reads an array of these from device memory). */
typedef struct ndgi_model {
    int32_t W, H;        /* spatial map size in texels; multiples of 4, 4..16384        */
    int32_t Gw, Gh;      /* grid nodes per row / column, >= 1                          */
    int32_t T;           /* time keys at t_k = k/T on a periodic day, 1..1024           */
    int32_t grid_dtype;  /* NDGI_DTYPE_F32 or NDGI_DTYPE_F16                            */
    int32_t mlp_dtype;   /* NDGI_DTYPE_F32 or NDGI_DTYPE_F16                            */
    int32_t reserved0;   /* must be 0                                                   */
    const uint8_t* bc4;  /* device [H/4][W/4][8 channels][8 bytes]; the 8 single-channel
                            blocks of one 4x4 footprint are contiguous (64 bytes)          */
    const void* grid;    /* device [T][Gh][Gw][8] in grid_dtype                          */
    const void* mlp;     /* device [NDGI_MLP_SIZE] in mlp_dtype                          */
    const void* reserved1;
} ndgi_model;

/* One virtual-texturing page request (supplementary Sec. C: a tile of a lightmap decoded
 * into the physical texture).  24 bytes. */
typedef struct ndgi_page_req {
    int32_t model;       /* index into the models array                                 */
    int32_t page_x;      /* page column: texels x = page*page_x .. page*page_x+page-1   */
    int32_t page_y;      /* page row                                                    */
    float t;             /* time of day; wrapped into [0, 1)                            */
    int64_t dst_offset;  /* texel index in dst of the page's texel (0, 0)               */
} ndgi_page_req;

typedef struct ndgi_ctx ndgi_ctx;

/* ---------------------------------------------------------------- context, errors */

/* Create a context on HIP device `device` (it becomes current for the calling thread).
 * Allocates the context workspace (error flags, per-wave gradient partials, loss and
 * statistics scratch).  *out receives the context.  Errors: INVALID_ARG (bad device or
 * out == NULL), HIP, OUT_OF_MEMORY. */
int ndgi_create(ndgi_ctx** out, int32_t device);

/* Release the context, its workspace and any captured graphs.  NULL is a no-op.  Every
 * release is attempted and the context is freed in any case; Errors: HIP (the first release
 * that failed). */
int ndgi_destroy(ndgi_ctx* ctx);

/* Message describing the calling thread's most recent failed call ("" if none).
 * The pointer stays valid until the thread's next library call. */
const char* ndgi_last_error(void);

/* Synchronise `stream`, then read and clear the context's device error flags
 * (NDGI_FLAG_* bits) into *flags_out (host). */
int ndgi_get_error_flags(ndgi_ctx* ctx, hipStream_t stream, uint32_t* flags_out);

/* ---------------------------------------------------------------- block decoder */

/* Decode n BC4 blocks (supplementary Sec. B: texel = interpolation of two endpoints;
 * Eq. 7), bit-exactly.  blocks: device [n][8] bytes (e0, e1, 48-bit little-endian
 * selector field; texel s = 4*row + col uses bits 3s..3s+2).  out16: device [n][16]
 * bytes, texel s at out16[16*i + s].  e0 > e1 selects the 8-value palette
 * round((7-j)/7 e0 + j/7 e1), j = 1..6; otherwise the 6-value palette
 * round((5-j)/5 e0 + j/5 e1), j = 1..4, plus 0 and 255; selector 0 = e0, 1 = e1.
 * n = 0 is a no-op.  Errors: INVALID_ARG (n < 0, NULL pointers when n > 0). */
int ndgi_bc4_decode_blocks(const uint8_t* blocks, int64_t n, uint8_t* out16, hipStream_t stream);

/* The same decode through one of the texel decoders inside the decode kernels, for checking
 * them exhaustively: impl 0 = the integer decoder above, 1 = the float decoder of the query,
 * page and hybrid kernels (floor(e0 + 0.5 + j (e1 - e0) / D) as one FMA), 2 = the row decoder
 * of the frame and binned kernels (palette built once per block in FP16 packs, four texels
 * per byte permute).  Same layouts and errors as ndgi_bc4_decode_blocks (also impl out of
 * 0..2). */
int ndgi_bc4_decode_blocks_impl(const uint8_t* blocks, int64_t n, uint8_t* out16, int32_t impl,
                                hipStream_t stream);

/* Decode n BC7 blocks of modes 4, 5 and 6, the single-subset modes with four channels (the
 * block format of the hybrid layout's F_uv and F_uvt, NDGI_CODEC_BC7; Sec. 3.4 compresses
 * with several modes), bit-exactly, as the hybrid decode reads them.  blocks: device [n][16]
 * bytes, 16-byte aligned, each a 128-bit little-endian value; the mode is the position of
 * the lowest set bit of byte 0:
 *  - mode 6: 7-bit endpoint values R0 R1 G0 G1 B0 B1 A0 A1 at bits 7..62, p-bits at 63 and
 *    64, texel 0's 3-bit index at 65..67, texel s's 4-bit index at 64 + 4 s; E = (v << 1) | p;
 *  - mode 5: rotation at bits 6..7, 7-bit colour values R0 R1 G0 G1 B0 B1 from bit 8, 8-bit
 *    alpha values at 50 and 58, 2-bit colour indices from bit 66, 2-bit alpha indices from 97;
 *  - mode 4: rotation at bits 5..6, index selection at 7, 5-bit colour values from bit 8,
 *    6-bit alpha values at 38 and 44, a 2-bit index set from bit 50 and a 3-bit set from 81
 *    (colour takes the 2-bit set when the selection is 0, the 3-bit set when it is 1);
 * in an index set texel 0's index has one bit less (its top bit is 0); an n-bit value v
 * expands to E = (v << (8 - n)) | (v >> (2n - 8)).  out64: device [n][16][4] bytes, 16-byte
 * aligned: channel c of texel s = 4*row + col at out64[64*i + 4*s + c] =
 * ((64 - w) E0 + w E1 + 32) >> 6 with w the b-bit weight of the texel's index (b = 2: 0 21
 * 43 64; b = 3: 0 9 18 27 37 46 55 64; b = 4: 0 4 9 13 17 21 26 30 34 38 43 47 51 55 60 64),
 * colour with the colour index, alpha with the alpha index; then a rotation r > 0 exchanges
 * channel r - 1 and channel 3.  A block of any other mode (or none) decodes to 0.
 * n = 0 is a no-op.  Errors: INVALID_ARG (n < 0, NULL or misaligned pointers when n > 0). */
int ndgi_bc7_decode_blocks(const uint8_t* blocks, int64_t n, uint8_t* out64, hipStream_t stream);

/* ---------------------------------------------------------------- block encoders */
/* The paper block-compresses its trained feature maps after quantising them to 8 bits
 * (Sec. 3.4, last paragraph of Feature Map Compression) and names no encoder.  These encode
 * 8-bit texel values; ndgi_hybrid_encode applies them to a training state. */

/* BC4: for each block of 16 texels (texels: device [n][16] bytes, texel s = 4*row + col) the
 * block of least summed squared error over all 65536 endpoint pairs of both palette modes
 * (ndgi_bc4_decode_blocks' palettes), each texel at its nearest palette entry: the exact
 * optimum.  Ties: the lowest e0 * 256 + e1, then per texel the lowest selector.  out: device
 * [n][8], 8-byte aligned.  n = 0 is a no-op.  Errors: INVALID_ARG (n < 0, NULL or misaligned
 * pointers). */
int ndgi_bc4_encode_blocks(const uint8_t* texels, int64_t n, uint8_t* out, hipStream_t stream);

/* BC7 with modes 6, 5 and 4: for each block of 16 RGBA texels (texels: device [n][16][4]
 * bytes) the candidate of least summed squared error among a mode-6 block, a mode-5 block
 * under each of the 4 rotations and a mode-4 block under each rotation and both index
 * selections (ties: mode 6, then mode 5 by rotation, then mode 4 by rotation, then selection),
 * each found by a fixed integer search (the optimum is out of reach: 2^58 endpoint settings
 * in mode 6).  Mode 6: (1) endpoints at the corners of the texels' bounding box along its
 * principal diagonal (reference channel = largest spread; a channel runs min -> max when its
 * covariance with the reference is >= 0, else max -> min); (2) both endpoints quantised for
 * each of the four p-bit pairs, v = clamp(floor((x - p + 1) / 2), 0, 127); (3) twice, the
 * least-squares endpoints of the current indices (2x2 normal equations per channel, exact
 * integers, rounded half up, clamped to 0..255), quantised as in (2); (4) best-improvement
 * local search at steps 8, 4, 2, 1 (at most 64 rounds each) over 22 moves in a fixed order:
 * each 7-bit value of endpoint 0 then endpoint 1 by -s, +s; all four values of endpoint 0 then
 * endpoint 1 by -s, +s; the p-bit of endpoint 0, then of endpoint 1, flipped (moves leaving
 * 0..127 are not taken), the first strictly best move taken while it improves; a candidate
 * replaces the current block only when strictly better, and every candidate's indices are
 * refitted (each texel its least-error index, the lowest on ties); (5) when texel 0's index
 * is >= 8 the endpoints swap and each index J becomes 15 - J.  Modes 5 and 4 (the rotated
 * texels: channel r - 1 and channel 3 exchanged) fit the colour endpoints (3 channels) and
 * the alpha endpoints (1 channel) apart, each by the same steps at its value width n and
 * index width b: (1) as above (one channel: min -> max), each 8-bit target quantised to the
 * n-bit value whose expansion is nearest (ties to the lower); (2) twice, least squares as
 * above, quantised likewise; (3) local search at steps 2^(n-4) .. 1 over each value of
 * endpoint 0 then endpoint 1 by -s, +s, then (colour) all values of one endpoint by -s, +s;
 * (4) when texel 0's index has its top bit set, the endpoints swap and J becomes
 * 2^b - 1 - J.  out: device [n][16], 16-byte aligned, in ndgi_bc7_decode_blocks' layout.
 * Reproduces exactly any texels that a mode-6 block using indices 0 and 15 decodes to.
 * n = 0 is a no-op.  Errors: INVALID_ARG. */
int ndgi_bc7_encode_blocks(const uint8_t* texels, int64_t n, uint8_t* out, hipStream_t stream);

/* ---------------------------------------------------------------- decode */

/* Random-access decode of n queries (Sec. 3.1 Eq. 3; Sec. 3.3 "random access"):
 *   uvt: device float [n][3] = (u, v, t).  u, v in [0, 1) address texel centres
 *        ((u*W - 0.5), (v*H - 0.5) in texel units); outside [0, 1) they clamp to the
 *        edge.  t is wrapped into [0, 1); keys are periodic (key T-1 blends into key 0).
 *        A query with a non-finite coordinate decodes to NaN.
 *   out: device [n][3]; float if prec == NDGI_PREC_F32, _Float16 if NDGI_PREC_F16.
 *   model: host pointer to a descriptor whose buffers are device memory.
 * With a workspace reserved by ndgi_reserve_decode that holds the binned layout for (model,
 * n), and at least 100 queries per 32 x 32-texel tile on average, the call runs the binned
 * kernels of ndgi_decode_binned (the same result bit for bit); otherwise one pass in query
 * order.
 * n = 0 is a no-op.  Errors: INVALID_ARG (bad descriptor, sizes, prec, NULL buffers). */
int ndgi_decode(ndgi_ctx* ctx, const ndgi_model* model, const float* uvt, int64_t n,
                void* out, int32_t prec, hipStream_t stream);

/* Reserve (allocate, once) the context's decode workspace for up to max_queries queries on
 * maps of model's sizes, so that later ndgi_decode calls with many queries per tile take the
 * binned kernels (Sec. 3.3 "random access" at batch scale) without allocating.  A
 * reservation that already holds the layout is kept; a larger one replaces it (the device
 * is synchronised before the old one is freed); max_queries = 0 releases it (model may then
 * be NULL).  Call it when no decode of this context is in flight.
 * Errors: INVALID_ARG (ctx NULL, bad descriptor, max_queries out of [0, 2^31)), UNSUPPORTED
 * (maps the binned kernels do not take), OUT_OF_MEMORY, HIP. */
int ndgi_reserve_decode(ndgi_ctx* ctx, const ndgi_model* model, int64_t max_queries);

/* Binned random-access decode: the same result as ndgi_decode, bit for bit, for the same
 * queries (Sec. 3.1 Eq. 3; Sec. 3.3 "random access"), reached by first counting-sorting the
 * queries by the 32x32 (64x64 on maps above 4096x4096 texels) tile of their bilinear
 * footprint so that each tile's BC4 blocks are decoded once into LDS and its grid window
 * is reused from cache.  Pays off when there are on the order of a hundred queries or
 * more per tile; for sparse queries use ndgi_decode.
 *   uvt, out, prec, model: as for ndgi_decode; n < 2^31.
 *   workspace: caller-owned device memory, 256-byte aligned, of at least the size that
 *              ndgi_decode_binned_workspace reports for (model, n); its contents on entry
 *              are ignored and on return are unspecified.  Calls that share a workspace
 *              must be ordered on one stream.
 * Nothing is allocated; the call is safe to capture in a HIP graph.
 * Errors: INVALID_ARG (as ndgi_decode; workspace NULL, misaligned or too small);
 * UNSUPPORTED (maps of more than 16384 tiles of 64x64 texels, i.e. above 8192x8192). */
int ndgi_decode_binned_workspace(const ndgi_model* model, int64_t n, int64_t* bytes_out);
int ndgi_decode_binned(ndgi_ctx* ctx, const ndgi_model* model, const float* uvt, int64_t n,
                       void* out, int32_t prec, void* workspace, int64_t workspace_bytes,
                       hipStream_t stream);

/* Binned decode that allocates nothing and takes no workspace: for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same kernels and the same result, bit for bit, as
 * ndgi_decode_binned; the sort's scratch is a static device array of
 * NDGI_NOALLOC_SCRATCH_BYTES bytes that the library holds on each GPU it runs on until the
 * process ends (its address is taken once per device by ndgi_create).
 *   uvt, out, prec, model, n: as for ndgi_decode_binned.
 * The call fails with INVALID_ARG when ndgi_decode_binned_workspace reports more than
 * NDGI_NOALLOC_SCRATCH_BYTES for (model, n) (above 2,084,320 queries on a 4096x4096 map with a
 * 1024x1024 grid, 4,061,680 on a 1024x1024 map with a 256x256 grid), before any launch.
 * No hipMalloc, hipFree or allocating library call is made.  Every call on one GPU shares
 * that GPU's scratch, whose contents carry over from the last call (nothing in it needs to
 * start at zero): calls that overlap on one GPU, from any context, stream or thread, race
 * and give undefined results; order them on one stream.
 * Errors: as ndgi_decode_binned. */
#define NDGI_NOALLOC_SCRATCH_BYTES (64ll << 20)
int ndgi_decode_binned_noalloc(ndgi_ctx* ctx, const ndgi_model* model, const float* uvt, int64_t n,
                               void* out, int32_t prec, hipStream_t stream);

/* Batched virtual-texturing page decode (Sec. 3.5; supplementary Sec. C): every valid
 * request decodes the page x page texel centres of its page of models_dev[model] at its
 * time t and writes texel (i, j) of the page to dst[dst_offset + j*dst_pitch + i]
 * ([..][3] elements of float or _Float16 by prec).  One persistent launch covers all
 * requests; each map may have its own size and decoder weights.
 *   models_dev: device array of n_models descriptors.
 *   reqs_dev:   device array of at least max_reqs requests.
 *   n_reqs_dev: device int32 holding the number of requests to serve (read by the
 *               kernel, clamped to [0, max_reqs]) so that a captured graph can be
 *               replayed with new requests.
 *   page:       page side in texels, a multiple of 16, 16..4096.
 * A request whose model index is outside [0, n_models) or whose page does not lie
 * inside its map is skipped and sets NDGI_FLAG_BAD_PAGE_REQUEST.  The caller guarantees
 * that dst holds every texel addressed by a valid request.
 * Errors: INVALID_ARG (sizes, prec, NULL pointers). */
int ndgi_decode_pages(ndgi_ctx* ctx, const ndgi_model* models_dev, int32_t n_models,
                      const ndgi_page_req* reqs_dev, const int32_t* n_reqs_dev,
                      int32_t max_reqs, int32_t page, void* dst, int64_t dst_pitch,
                      int32_t prec, hipStream_t stream);

/* Same work as ndgi_decode_pages, launched as a HIP graph: the first call for a given
 * argument set captures the persistent launch into a graph owned by the context, later
 * calls with the same arguments replay it (new requests and counts are picked up from
 * device memory).  Errors: as ndgi_decode_pages, plus HIP. */
int ndgi_decode_pages_graph(ndgi_ctx* ctx, const ndgi_model* models_dev, int32_t n_models,
                            const ndgi_page_req* reqs_dev, const int32_t* n_reqs_dev,
                            int32_t max_reqs, int32_t page, void* dst, int64_t dst_pitch,
                            int32_t prec, hipStream_t stream);

/* Launch shape of the page decoder, chosen by an autotuner: each work item is a
 * (16*tile_w) x (4*tile_h) texel sub-tile of one page; waves_per_cu persistent waves per
 * compute unit.  tile_w, tile_h in 1..32 (page must be a multiple of both sub-tile sides,
 * checked per call); waves_per_cu in 1..32.  Also sets the launch size of ndgi_decode.
 * Drops captured graphs.  Errors: INVALID_ARG, HIP (releasing a captured graph). */
int ndgi_set_launch(ndgi_ctx* ctx, int32_t tile_w, int32_t tile_h, int32_t waves_per_cu);

/* ---------------------------------------------------------------- training */

/* Trainable state of one model under BC simulation (Sec. 3.4, Eq. 6-7).  All arrays are
 * float32 device memory with one flat layout shared by params, grads, adam_m, adam_v:
 *   [ endpoints [H/4][W/4][8][2]  (e1, e2 of each block and channel, in [0, 1])
 *   | weights   [H][W][8]         (per-texel interpolation weight, in [0, 1])
 *   | grid      [T][Gh][Gw][8]
 *   | mlp       [NDGI_MLP_SIZE] ]
 * ndgi_train_param_count() gives the total length. */
typedef struct ndgi_train_state {
    int32_t W, H, Gw, Gh, T;  /* W, H multiples of 4, <= 4096; T <= 256 */
    int32_t reserved0;
    float* params;
    float* grads;
    float* adam_m;
    float* adam_v;
    int64_t step;             /* Adam steps taken so far; ADAM and FUSED increment it */
    float lr_feat;            /* Adam learning rate of endpoints, weights and grid      */
    float lr_mlp;             /* Adam learning rate of the decoder                      */
    float beta1, beta2, eps;
    float reserved1;
} ndgi_train_state;

/* One batch of training samples.  A sample is texel (x, y) of key k, i.e. t = k/T. */
typedef struct ndgi_batch {
    const uint32_t* samples;  /* device [n]: x | y << 12 | k << 24                       */
    int64_t n;                /* number of samples, >= 1                                 */
    const uint16_t* target;   /* device FP16 bits [T][H][W][3] (LOSS_GRAD, FUSED)         */
    float* pred;              /* device [n][3] (written by FORWARD; optional otherwise)   */
    const float* grad_pred;   /* device [n][3] dLoss/dpred (BACKWARD)                     */
} ndgi_batch;

#define NDGI_TRAIN_FORWARD   0  /* pred = H_Theta(samples) under BC simulation               */
#define NDGI_TRAIN_BACKWARD  1  /* grads += d(sum grad_pred . pred)/dparams (features recomputed) */
#define NDGI_TRAIN_LOSS_GRAD 2  /* *loss_dev = L2 loss (FP64); grads += dL/dparams           */
#define NDGI_TRAIN_FUSED     3  /* LOSS_GRAD, then ADAM                                      */
#define NDGI_TRAIN_ADAM      4  /* Adam step on all params (PyTorch semantics, dense), clamp
                                   endpoints and weights to [0, 1], zero grads, step += 1    */
#define NDGI_TRAIN_ZERO_GRAD 5  /* grads = 0                                                 */

/* Total number of float parameters of a state with the given sizes. */
int64_t ndgi_train_param_count(int32_t W, int32_t H, int32_t Gw, int32_t Gh, int32_t T);

/* Run one training operation (modes above) on `state` (host struct of device pointers;
 * its `step` is updated on the host by ADAM and FUSED).  loss_dev: device double, written
 * by LOSS_GRAD and FUSED (mean over samples and channels of (pred - target)^2; the sum is
 * accumulated in FP64).  The quantisation is E = rint(fl32(255 e)), J = rint(fl32(7 w)),
 * texel value floor(((7-J) E1 + J E2 + 3)/7) / 255; gradients reach e1, e2, w through the
 * straight-through derivative of Eq. 7 at (E/255, J/7).  A sample with x >= W, y >= H or
 * k >= T is skipped (it adds nothing to the loss or the gradients but still counts in n)
 * and sets NDGI_FLAG_BAD_SAMPLE.
 * Errors: INVALID_ARG (sizes, mode, NULL pointers needed by the mode). */
int ndgi_train_step(ndgi_ctx* ctx, ndgi_train_state* state, const ndgi_batch* batch,
                    int32_t mode, double* loss_dev, hipStream_t stream);

/* Export the trained state as a decodable model (Sec. 3.4, last paragraph): BC4 blocks
 * whose decode equals the BC-simulated texels bit for bit (E1 > E2: (e0, e1) = (E1, E2);
 * E1 < E2: swapped with J -> 7 - J; E1 = E2: 6-value block of selector 0), the grid and
 * the decoder converted to grid_dtype / mlp_dtype (round to nearest even).
 *   bc4_out: device [H/4][W/4][8][8]; grid_out: device [T][Gh][Gw][8]; mlp_out: device
 *   [NDGI_MLP_SIZE].  Errors: INVALID_ARG. */
int ndgi_export(ndgi_ctx* ctx, const ndgi_train_state* state, uint8_t* bc4_out,
                void* grid_out, int32_t grid_dtype, void* mlp_out, int32_t mlp_dtype,
                hipStream_t stream);

/* ---------------------------------------------------------------- hybrid layout */

/* The paper's own feature layout (Sec. 3.3, Eq. 4-5; Table 1; Table 3), decoded by its
 * GELU decoder (Sec. 4).  Four feature maps per model:
 *   F_uv   W x H texels, 4 channels, block-compressed per 4x4 footprint (codec below:
 *          [H/4][W/4][4][8 bytes] BC4 or [H/4][W/4][16 bytes] BC7)
 *   F_uvt  Gu x Gv texels x S time slices, 4 channels, each slice block-compressed on its
 *          own (Sec. 3.4): [S][Gv/4][Gu/4] footprints as for F_uv
 *   F_ut   U x Tt texels, 2 channels, 8-bit: [Tt][U][2] bytes
 *   F_vt   V x Tt texels, 2 channels, 8-bit: [Tt][V][2] bytes
 * and a decoder 16 -> hidden -> hidden -> 3 (hidden 16 or 64; GELU x*Phi(x) on the hidden
 * layers, no output activation), packed row-major as [W1 hidden x 16 | b1 | W2 hidden x
 * hidden | b2 | W3 3 x hidden | b3] (ndgi_hybrid_mlp_size values).
 * Sampling at (u, v, t):
 *   - a stored byte q is the feature value q / 255;
 *   - every spatial axis (W, H; Gu, Gv; U; V) is sampled at texel centres, bilinearly, with
 *     clamp to the edge (as for ndgi_model);
 *   - t is clamped to [0, 1].  With a key table (n_keys times k_0 < ... < k_{n-1} of the
 *     baked lightmaps, Sec. 3.1) t maps piecewise linearly to tau, k_i -> i / (n - 1),
 *     and tau clamps to [0, 1]; without one tau = t.  The time axes of F_uvt (S slices),
 *     F_ut and F_vt (Tt rows) hold sample k at tau = k / (N - 1) and interpolate linearly;
 *   - the decoder input is [V_uvt (4), V_uv (4), V_ut (2), V_vt (2), gamma(t) (4)] with
 *     gamma(t) = [sin(pi t), cos(pi t), sin(2 pi t), cos(2 pi t)] of the clamped t (Eq. 4).
 * 96 bytes, the same layout on host and device. */
#define NDGI_HYBRID_IN 16
#define NDGI_HYBRID_MAX_KEYS 256
/* Block formats of F_uv and F_uvt:
 *   NDGI_CODEC_BC4  one BC4 block per channel (8 bytes per 4x4 footprint and channel: a weight
 *                   per texel and channel), 16 bits per texel for the 4 channels;
 *   NDGI_CODEC_BC7  one BC7 block per footprint of mode 4, 5 or 6 (ndgi_bc7_decode_blocks;
 *                   16 bytes; mode 6: 7-bit RGBA endpoints with a p-bit each, one 4-bit index
 *                   per texel shared by the 4 channels, as Eq. 6 writes the simulation), 8
 *                   bits per texel - the rate of the paper's Table 3. */
#define NDGI_CODEC_BC4 0
#define NDGI_CODEC_BC7 1

typedef struct ndgi_hybrid_model {
    int32_t W, H;         /* F_uv size; multiples of 4, 4..16384                          */
    int32_t Gu, Gv;       /* F_uvt size; multiples of 4, 4 <= Gu <= W, 4 <= Gv <= H       */
    int32_t S;            /* F_uvt time slices, 1..1024                                   */
    int32_t U, V;         /* F_ut / F_vt spatial size, 1 <= U <= W, 1 <= V <= H           */
    int32_t Tt;           /* F_ut / F_vt time rows, 1..1024                               */
    int32_t hidden;       /* decoder width: 16 or 64                                      */
    int32_t mlp_dtype;    /* NDGI_DTYPE_F32 or NDGI_DTYPE_F16                             */
    int32_t n_keys;       /* 0, or 2..NDGI_HYBRID_MAX_KEYS key times                      */
    int32_t codec;        /* NDGI_CODEC_BC4 or NDGI_CODEC_BC7 (block format of F_uv, F_uvt) */
    const uint8_t* fuv;   /* device [H/4][W/4][4][8] (BC4) or [H/4][W/4][16] (BC7)        */
    const uint8_t* fuvt;  /* device [S][Gv/4][Gu/4][4][8] (BC4) or [S][Gv/4][Gu/4][16]   */
    const uint8_t* fut;   /* device [Tt][U][2]                                            */
    const uint8_t* fvt;   /* device [Tt][V][2]                                            */
    const float* keys;    /* device [n_keys], strictly increasing in [0, 1] (the caller
                             guarantees the order; it is not checked)                     */
    const void* mlp;      /* device [ndgi_hybrid_mlp_size(hidden)] in mlp_dtype            */
} ndgi_hybrid_model;

/* Number of packed decoder values for a hidden width (16 or 64); -1 otherwise. */
int32_t ndgi_hybrid_mlp_size(int32_t hidden);

/* Random-access decode of n queries of a hybrid model (Sec. 3.1 Eq. 3, Sec. 3.3 Eq. 4):
 *   uvt: device float [n][3]; out: device [n][3] of float (NDGI_PREC_F32: FP32 features,
 *   FP32 MFMA) or _Float16 (NDGI_PREC_F16: FP32 features, FP16 MFMA with FP32
 *   accumulation, FP16 out).  A query with a non-finite coordinate decodes to NaN.
 *   model: host pointer to a descriptor whose buffers are device memory.
 * n = 0 is a no-op.  Errors: INVALID_ARG (descriptor out of the ranges above, n < 0, prec,
 * NULL buffers). */
int ndgi_hybrid_decode(ndgi_ctx* ctx, const ndgi_hybrid_model* model, const float* uvt, int64_t n,
                       void* out, int32_t prec, hipStream_t stream);

/* Virtual-texturing page decode of hybrid models (Sec. 3.5; supplementary Sec. C): the
 * same request convention as ndgi_decode_pages (request count read from device memory),
 * with t clamped to [0, 1] and page 1..4096 texels (the paper's tiles are 128).  Each map
 * (one per-tile model in the paper's production setting) has its own descriptor and
 * decoder.
 *   widths: decoder widths among the requests' models, bit 0 = hidden 16, bit 1 = hidden
 *           64, 0 = either.  One persistent launch runs per width named; naming only the
 *           width in use saves the launch of the other.
 *   border: 0..min(32, page) texels of border around each page (supplementary Virtual
 *           Texturing section: tiles are stored with a border for hardware filtering, padded
 *           by mirroring).  A request then writes a
 *           (page + 2 border)^2 region at dst_offset with dst_pitch >= page + 2 border;
 *           region texel (i, j) is the decode at map texel (mirror(page * page_x - border
 *           + i, W), mirror(page * page_y - border + j, H)), mirror(i, n) = -1 - i below 0,
 *           2n - 1 - i from n (the map reflected about its edges).  Inside the map the
 *           border repeats the neighbouring texels; for a per-tile model it mirrors the tile.
 * A request whose model index or page is out of range, whose descriptor breaks the ranges
 * above, or whose decoder width is not in `widths`, is skipped and sets
 * NDGI_FLAG_BAD_PAGE_REQUEST.  Errors: INVALID_ARG (sizes, prec, widths, border, pitch,
 * NULL pointers). */
int ndgi_hybrid_decode_pages(ndgi_ctx* ctx, const ndgi_hybrid_model* models_dev, int32_t n_models,
                             const ndgi_page_req* reqs_dev, const int32_t* n_reqs_dev, int32_t max_reqs,
                             int32_t page, void* dst, int64_t dst_pitch, int32_t prec, int32_t widths,
                             int32_t border, hipStream_t stream);

/* Same work launched as a HIP graph owned by the context (captured on the first call for
 * an argument set, replayed afterwards), as ndgi_decode_pages_graph. */
int ndgi_hybrid_decode_pages_graph(ndgi_ctx* ctx, const ndgi_hybrid_model* models_dev, int32_t n_models,
                                   const ndgi_page_req* reqs_dev, const int32_t* n_reqs_dev,
                                   int32_t max_reqs, int32_t page, void* dst, int64_t dst_pitch,
                                   int32_t prec, int32_t widths, int32_t border, hipStream_t stream);

/* Trainable state of n_models hybrid models of equal sizes (Sec. 3.4, Eq. 6-7; Sec. 4; the
 * paper trains one model per virtual-texture tile).  Per model the feature block is
 *   [ F_uv endpoints [H/4][W/4][4][2] | F_uv weights [H][W][4]
 *   | F_uvt endpoints [S][Gv/4][Gu/4][4][2] | F_uvt weights [S][Gv][Gu][4]
 *   | F_ut [Tt][U][2] | F_vt [Tt][V][2] ]
 * (weights [H][W] and [S][Gv][Gu] with codec NDGI_CODEC_BC7) and the decoder block
 * [ndgi_hybrid_mlp_size(hidden)]; params, grads, adam_m and adam_v
 * hold all feature blocks, model after model, then all decoder blocks:
 * n_models * ndgi_hybrid_train_param_count values (with several models Tt * (U + V) must be
 * even, so that every feature block is 16-byte aligned).  Sizes as ndgi_hybrid_model, with
 * W, H <= 4096.  A training sample is texel (x, y) of baked frame f: t = keys[f] (keys given) or
 * f / (frames - 1), and tau = f / (frames - 1); model m's samples are batch entries
 * [m * per_model, (m + 1) * per_model) and its target is target[m]. */
typedef struct ndgi_hybrid_train_state {
    int32_t W, H, Gu, Gv, S, U, V, Tt, hidden;
    int32_t frames;           /* baked frames of the target, 1..256                       */
    int32_t n_models;         /* models trained together (one per tile), >= 1             */
    int32_t per_model;        /* samples per model in a batch; with n_models > 1 a multiple
                                 of 64 and n = n_models * per_model (ignored for 1 model)  */
    int32_t codec;            /* NDGI_CODEC_BC4: a weight per texel and channel;
                                 NDGI_CODEC_BC7: one weight per texel (Eq. 6)             */
    int32_t reserved0;        /* must be 0                                                */
    const float* keys;        /* device [frames] frame times, or NULL (uniform)           */
    float* params;
    float* grads;
    float* adam_m;
    float* adam_v;
    int64_t step;             /* Adam steps taken; ADAM and FUSED increment it            */
    float lr_feat, lr_mlp;    /* Adam learning rates of the feature maps / the decoder    */
    float beta1, beta2, eps;
    uint32_t seed;            /* seed of the noise draws                                  */
} ndgi_hybrid_train_state;

typedef struct ndgi_hybrid_batch {
    const uint32_t* samples;  /* device [n]: x | y << 12 | f << 24; x, y and f above the
                                 map's last texel or frame are clamped to it               */
    int64_t n;                /* 1 .. 2^31 - 1                                            */
    const float* target;      /* device [n_models][frames][H][W][3] preprocessed target
                                 (LOSS_GRAD, FUSED; see ndgi_hybrid_normalize_target)     */
    float* pred;              /* device [n][3] (FORWARD)                                  */
} ndgi_hybrid_batch;

/* Feature flags of a hybrid training step.  With no flag F_uv and every F_uvt slice are the
 * continuous Eq. 7 lerp of their block endpoints and per-texel weights (Eq. 6): this is the
 * paper's BC simulation (Sec. 3.4; the supplementary ablation's "w/ BC simulation" arm).
 *   NOISE   U(-1/2, 1/2) / 256 added to each of the 12 sampled map values (Sec. 3.4's noise
 *           equation names V_ut and V_vt with alpha = 1/256; the same section adds noise to
 *           the sampled V_uvt and V_uv); draw c of sample s in a step is the SplitMix64
 *           output of seed * 0x9E3779B97F4A7C15 + step * 2^32 + 16 s + c, top 24 bits / 2^24
 *           - 1/2.
 *   DIRECT  F_uv / F_uvt are per-texel values, the state's weights themselves (the state
 *           must have codec NDGI_CODEC_BC4: one value per texel and channel; endpoints are
 *           unused and get no gradient).  The supplementary ablation's "w/o BC simulation"
 *           arm (a directly optimised map, block-compressed after training), and the layout
 *           ndgi_hybrid_import writes.  Excludes BCSIM.
 *   BCSIM   rounding to the block format's grid during training, a variant the paper does
 *           not describe: E = rint(fl32(255 e)), J = rint(fl32(7 w)), value
 *           floor(((7-J) E1 + J E2 + 3)/7) / 255, straight-through gradient of Eq. 7 at
 *           (E/255, J/7).  With codec NDGI_CODEC_BC7 each endpoint takes the mode-6 7-bit
 *           values and p-bit E = 2 v + p nearest to fl32(255 e) in summed squared error
 *           (v = rint((x - p)/2) clamped to 0..127, ties p = 0), J = rint(fl32(15 w)),
 *           weight wt = (64 J + 7)/15, value ((64 - wt) E1 + wt E2 + 32) >> 6 / 255,
 *           gradient at (E/255, wt/64).  The forward then equals the decode of
 *           ndgi_hybrid_export's blocks.
 *   QPLANES F_ut and F_vt rounded to 8 bits as a decode sees them (decoder fine-tune on
 *           frozen features: lr_feat = 0). */
#define NDGI_HTRAIN_BCSIM   1
#define NDGI_HTRAIN_NOISE   2
#define NDGI_HTRAIN_QPLANES 4
#define NDGI_HTRAIN_DIRECT  8

/* Float parameters of one model of a hybrid state; -1 for sizes out of range. */
int64_t ndgi_hybrid_train_param_count(int32_t W, int32_t H, int32_t Gu, int32_t Gv, int32_t S, int32_t U,
                                      int32_t V, int32_t Tt, int32_t hidden, int32_t codec);

/* One hybrid training operation: mode NDGI_TRAIN_FORWARD (pred), NDGI_TRAIN_LOSS_GRAD
 * (grads += the gradient of each model's loss, the mean over that model's own samples and
 * channels of (pred - target)^2, so a model trains as it would alone (Sec. 4 trains one model
 * per tile); *loss_dev = the mean of the models' losses, FP64), FUSED
 * (LOSS_GRAD then ADAM), ADAM (dense Adam, PyTorch semantics, feature maps projected to
 * [0, 1], grads zeroed, step += 1), ZERO_GRAD.  flags: NDGI_HTRAIN_*.  Errors: INVALID_ARG
 * (also DIRECT with BCSIM or with a BC7-layout state). */
int ndgi_hybrid_train_step(ndgi_ctx* ctx, ndgi_hybrid_train_state* state, const ndgi_hybrid_batch* batch,
                           int32_t mode, int32_t flags, double* loss_dev, hipStream_t stream);

/* Export model `model` of a trained state as a decodable hybrid model (Sec. 3.4 last
 * paragraph): blocks of F_uv and of every F_uvt slice in the state's codec (BC4:
 * [H/4][W/4][4][8] and [S][Gv/4][Gu/4][4][8] in the encoding of ndgi_export; BC7 mode 6:
 * [H/4][W/4][16] and [S][Gv/4][Gu/4][16], endpoints and indices of the simulation, the
 * endpoints swapped and every index J replaced by 15 - J when texel 0's would be >= 8),
 * planes rounded to 8 bits (rint of fl32(255 v)), decoder converted to mlp_dtype.  The decode of the export at a training sample equals the FORWARD with
 * BCSIM | QPLANES.  Errors: INVALID_ARG. */
int ndgi_hybrid_export(ndgi_ctx* ctx, const ndgi_hybrid_train_state* state, int32_t model,
                       uint8_t* fuv_out, uint8_t* fuvt_out, uint8_t* fut_out, uint8_t* fvt_out,
                       void* mlp_out, int32_t mlp_dtype, hipStream_t stream);

/* The paper's export (Sec. 3.4, last paragraph of Feature Map Compression) of model `model`
 * of a trained state: F_uv and every F_uvt slice reconstructed as a training step with
 * `flags` reads them (no flag: the FP32 Eq. 7 lerp fl32(fl32(fl32(1 - w) e1) + fl32(w e2));
 * DIRECT: the weights; BCSIM: the rounded simulation's texel), quantised to 8 bits as
 * clamp(rint(fl32(255 v)), 0, 255) (BCSIM: its byte), and block-encoded in `codec` by
 * ndgi_bc4_encode_blocks (one block per channel, [H/4][W/4][4][8], [S][Gv/4][Gu/4][4][8]) or
 * ndgi_bc7_encode_blocks ([H/4][W/4][16], [S][Gv/4][Gu/4][16]); planes rounded to 8 bits
 * (rint of fl32(255 v)); the decoder converted to mlp_dtype.  Any output may be NULL to skip
 * it (e.g. only the decoder and planes of a fine-tuned imported state).  Outputs are device
 * memory, block outputs aligned to their block size.  Errors: INVALID_ARG (also DIRECT with
 * BCSIM or with a BC7-layout state). */
int ndgi_hybrid_encode(ndgi_ctx* ctx, const ndgi_hybrid_train_state* state, int32_t model, int32_t flags,
                       int32_t codec, uint8_t* fuv_out, uint8_t* fuvt_out, uint8_t* fut_out, uint8_t* fvt_out,
                       void* mlp_out, int32_t mlp_dtype, hipStream_t stream);

/* Import of a block-compressed hybrid model into model `model` of a state with the BC4 layout
 * (one value per texel and channel) and the model's sizes, for the final training stage
 * (Sec. 4: the decoder fine-tuned on frozen features under quantisation and BC compression):
 * F_uv / F_uvt weights = the decoded byte / 255 (FP32 division) in [H][W][4] and
 * [S][Gv][Gu][4], their endpoints (0, 1), planes = byte / 255, the decoder as float.  A step
 * with DIRECT | QPLANES (lr_feat = 0) then reads exactly what a decode of the model reads.
 * model: host descriptor of device buffers.  Errors: INVALID_ARG (sizes differ, BC7-layout
 * state, model index). */
int ndgi_hybrid_import(ndgi_ctx* ctx, const ndgi_hybrid_model* model, ndgi_hybrid_train_state* state,
                       int32_t model_index, hipStream_t stream);

/* Target preprocessing of Sec. 4: y^(1/gamma) per texel and channel, divided per frame and
 * channel by its mean.  target: device FP16 bits [frames][H][W][3]; out: device float, same
 * shape; means: device double [frames][3] (the means, for ndgi_hybrid_restore).
 * Errors: INVALID_ARG. */
int ndgi_hybrid_normalize_target(ndgi_ctx* ctx, const uint16_t* target, int32_t frames, int32_t W,
                                 int32_t H, float gamma, float* out, double* means, hipStream_t stream);

/* Inverse for one decoded frame: out = max(pred * mean, 0)^gamma, pred [texels][3] of
 * pred_dtype, mean3 device double [3], out device float [texels][3]. */
int ndgi_hybrid_restore(ndgi_ctx* ctx, const void* pred, int32_t pred_dtype, int64_t texels,
                        const double* mean3, float gamma, float* out, hipStream_t stream);

/* ---------------------------------------------------------------- evaluation */

/* Per-tile statistics for the tiled PSNR of supplementary Sec. D.2, in FP64.
 *   pred:   device [H][W][3] of pred_dtype (one decoded map)
 *   target: device FP16 bits [H][W][3]
 *   stats:  device double [ceil(H/tile)][ceil(W/tile)][3] = (max of target, min of
 *           target, sum of squared error over the tile's texels and channels).
 * tile in 1..4096.  Errors: INVALID_ARG. */
int ndgi_tile_stats(ndgi_ctx* ctx, const void* pred, int32_t pred_dtype,
                    const uint16_t* target, int32_t W, int32_t H, int32_t tile,
                    double* stats, hipStream_t stream);

/* Tiled PSNR of supplementary Sec. D.2 from ndgi_tile_stats outputs, in FP64:
 *   stats:   device double [n_maps][ceil(H/tile)][ceil(W/tile)][3] (n_maps maps of W x H)
 *   tile_db: device double [n_maps][ceil(H/tile)][ceil(W/tile)] or NULL: each tile's
 *            10 log10(range^2 / MSE), range = max - min of the target over the tile and its
 *            channels, MSE over its texels and channels; NaN for a tile of zero range
 *            (skipped), 100 dB for MSE 0
 *   summary: device double [5] = (mean of tile_db over scored tiles, global PSNR over every
 *            texel with the range of all tiles, least tile PSNR, scored tiles, tiles).
 * Errors: INVALID_ARG. */
int ndgi_psnr(ndgi_ctx* ctx, const double* stats, int32_t n_maps, int32_t W, int32_t H, int32_t tile,
              double* tile_db, double* summary, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* NDGI_H */
