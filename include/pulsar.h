/*
 * pulsar.h - C ABI of the MI355X (gfx950) sphere renderer.
 *
 * The renderer implements the differentiable sphere-based projection step of
 * Pulsar (Lassner and Zollhoefer): a scene of spheres (position p_i, payload
 * f_i of C channels, radius r_i, opacity o_i; paper Sec. 3.1) is rendered by a
 * pinhole camera (R, t and the intrinsics focal length and sensor width;
 * Sec. 3.2) into a C-channel feature image F whose pixels blend every
 * intersected sphere with the weights of Eq. 1 (Sec. 3.2). The backward pass
 * returns the gradients of a scalar loss with respect to position, radius,
 * opacity, payload and background, given dLoss/dF; gradients flow through the
 * K nearest hits of each pixel (App. B, Step 2 and "Preparing for the backward
 * pass"; Sec. 2 on blending all spheres but differentiating the first few).
 *
 * Conventions shared by every entry point:
 *   - Camera frame: x right, y down, z forward; x_cam = R x_world + t.
 *     Pixel (row i, column j) looks through the sensor point
 *     ((j + 1/2) s/W - s/2, (i + 1/2) s/W - (s H/W)/2, f): square pixels of
 *     pitch s/W, principal point at the sensor centre.
 *   - The depth of a hit is the distance along the unit pixel ray to the
 *     front intersection, t in [znear, zfar]; z = (zfar - t)/(zfar - znear) is
 *     the [0, 1] depth of Eq. 1 with 0 at the far plane (Sec. 3.2).
 *   - The normalised distance d_i of Eq. 1 enters as 1 - q/R, q the distance
 *     of the sphere centre from the ray: 1 on the central ray, 0 at the
 *     silhouette.
 *   - A sphere takes part iff its inputs are finite, r > 0 and its camera-space
 *     depth satisfies c_z - R >= znear. A hit needs q < R and t <= zfar.
 *   - The background is blended with weight exp(eps/gamma) (Sec. 3.2).
 *   - Array pointers are DEVICE pointers to row-major, densely packed float32
 *     data owned by the caller. The library never allocates device memory and
 *     never synchronises the stream, except pulsar_query_status.
 *   - All work is enqueued on `stream` (a hipStream_t, NULL = null stream).
 *     Inputs must stay valid and unmodified until the work has finished.
 *   - Every return value is PULSAR_OK (0) or a negative PULSAR_ERR_* code. All
 *     argument checks run on the host before anything is enqueued.
 */
#ifndef PULSAR_H_
#define PULSAR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PULSAR_OK 0
/* a required pointer is NULL, a size or parameter is out of range */
#define PULSAR_ERR_INVALID_ARGUMENT (-1)
/* ws_bytes is smaller than pulsar_workspace_size() */
#define PULSAR_ERR_WORKSPACE (-2)
/* a flag or size this build does not implement */
#define PULSAR_ERR_UNSUPPORTED (-3)
/* a HIP launch or runtime call failed */
#define PULSAR_ERR_HIP (-4)
/* reported by pulsar_query_status only: the (tile, sphere) pairs of the last
 * forward did not fit into max_pairs; its outputs are invalid */
#define PULSAR_ERR_CAPACITY (-5)
/* pulsar_fwd_noalloc only: the call needs more workspace than its static
 * scratch buffer holds (PULSAR_NOALLOC_SCRATCH_BYTES) */
#define PULSAR_ERR_SCRATCH (-6)

/* Pinhole camera (Sec. 3.2, Lst. 1: focal length f and sensor width s share
 * one unit). Host struct, passed by pointer. */
typedef struct pulsar_camera {
  float R[9];          /* row-major world-to-camera rotation */
  float t[3];          /* translation: x_cam = R x_world + t */
  float focal;         /* f > 0 */
  float sensor_width;  /* s > 0; pitch = s / width */
  float znear;         /* > 0; spheres must lie beyond it (c_z - R >= znear) */
  float zfar;          /* > znear; hits beyond it are ignored */
  int32_t width;       /* W in [1, 65535] */
  int32_t height;      /* H in [1, 65535] */
} pulsar_camera_t;

/* Flags of pulsar_params_t.flags.
 *
 * PULSAR_NO_BWD_AUX: the forward keeps no backward state. It still writes the
 *   image and, when aux is not NULL, the log-normaliser, but skips tracking
 *   each pixel's K nearest hits (App. B keeps backward information optional).
 *   A pulsar_bwd on that workspace must then set PULSAR_REBIN; without it
 *   pulsar_bwd returns PULSAR_ERR_INVALID_ARGUMENT for this flag.
 * PULSAR_REBIN: pulsar_bwd rebuilds what it needs from the scene itself
 *   (projection, tile lists and each pixel's K-th nearest hit: App. B, Steps
 *   0-2 without the blend's image output) instead of reading the state a
 *   pulsar_fwd left in the workspace. Any workspace of the right size works,
 *   and other calls may use it between the forward and the backward. image and
 *   aux must still be the forward's outputs for the same inputs. The
 *   gradients are bitwise those of a pulsar_bwd right after pulsar_fwd. In
 *   pulsar_fwd the flag has no effect.
 * PULSAR_GRAD_PAPER_NORM: the paper's gradients for optimisation instead of
 *   exact derivatives (pulsar_bwd only):
 *   every gradient of a sphere (position, radius, opacity, payload) is divided
 *   by the number of pixels it received gradients from (App. B), and spheres
 *   whose projected radius R f / (c_z pitch) is at most 3 pixels get no
 *   position or radius gradient (Sec. 3.2, Sec. 7 limitation 1). The camera
 *   gradients of pulsar_bwd_camera are normalised by each sphere's image area
 *   (App. B): the part that comes from a sphere is scaled by
 *   1e-3 / (pi (R f / (c_z pitch))^2) before the sum over spheres. The
 *   background gradient stays exact.
 * PULSAR_BLEND_TOPK: the other reading of K (Sec. 3.2, App. B Step 2): only
 *   each pixel's K nearest hits in (t, index) order enter Eq. 1, in the image
 *   and in the log-normaliser. The forward then makes one more raster pass
 *   (the K-th nearest hit of every pixel, before blending). pulsar_bwd needs
 *   no flag for it: given that image and aux, its gradients are the exact
 *   derivatives of the top-K blend (away from changes of the K nearest).
 * PULSAR_ORTHO: orthographic instead of pinhole projection (Sec. 3.1 names
 *   both): the ray of pixel (i, j) starts at its centre on the sensor plane
 *   z = 0 of camera space and runs along +z, so t is the distance from that
 *   plane and focal plays no part (it must still be valid). The minimum size
 *   becomes the constant radius min_radius_px * pitch. pulsar_bwd_camera
 *   returns PULSAR_ERR_UNSUPPORTED for it.
 * PULSAR_STORE_HITS: the paper's preparation for the backward pass (App. B):
 *   the forward also stores every pixel's K nearest hits (depth and sphere
 *   index, 8 K bytes per pixel at the end of the workspace; pixels of tiles
 *   that no sphere touches have none) and pulsar_bwd
 *   takes them from there pixel by pixel, recomputing each stored hit's
 *   geometry, instead of re-testing every (tile, sphere) pair against the
 *   pixel's K-th nearest hit. The per-sphere sums are then gathered with
 *   float atomics, so the gradients equal those of the default backward up
 *   to summation order (they are not bitwise reproducible). Forward and
 *   backward must both set it (with PULSAR_REBIN the backward stores them
 *   itself); a backward on a workspace whose forward stored no hits writes
 *   zero gradients and pulsar_query_status reports
 *   PULSAR_ERR_INVALID_ARGUMENT.
 * PULSAR_BWD_TILES: the backward walks the forward's tile lists (a block per
 *   work item, one thread per (tile, sphere) pair, each pair's sums in a slot
 *   of its own, then a pass per sphere over its slots). Without it the
 *   backward walks the spheres in index order (a thread per sphere whose
 *   pixels are shared out over the lanes of its wave, no slots, no second
 *   pass), unless the forward met a sphere touching more than 16 tiles:
 *   that decision is taken on the device and the tile walk runs instead, as
 *   the walk in sphere order would give all of that sphere's pixels to one
 *   wave. Both walks compute the same terms and differ only in summation
 *   order. The stored-hits backward and payloads of more than 32 channels
 *   always use slots. */
#define PULSAR_NO_BWD_AUX 0x1u
#define PULSAR_REBIN 0x2u
#define PULSAR_GRAD_PAPER_NORM 0x4u
#define PULSAR_BLEND_TOPK 0x8u
#define PULSAR_ORTHO 0x10u
#define PULSAR_STORE_HITS 0x20u
#define PULSAR_BWD_TILES 0x40u

/* min_radius_px preset for the paper's rule that every sphere is drawn at
 * least one pixel large, so none falls between the pixel rays (App. B,
 * Step 0): a projected disk of radius sqrt(2)/2 pixel contains a pixel
 * centre wherever it lies. */
#define PULSAR_MIN_RADIUS_PX_PAPER 0.70710678f

/* Render parameters (host struct). */
typedef struct pulsar_params {
  float gamma;          /* blending softness of Eq. 1, in [1e-5, 1] (Sec. 3.2) */
  float eps;            /* background offset of Eq. 1, >= 0, typically 1e-5 */
  float min_radius_px;  /* >= 0. When > 0 a sphere is drawn at least this many
                           pixels wide in radius: R = max(r, min_radius_px * pitch * c_z / f)
                           (App. B, Step 0). 0 = off. */
  int32_t K;            /* nearest hits per pixel that receive gradients, 1..32 */
  uint32_t flags;       /* OR of PULSAR_NO_BWD_AUX, PULSAR_REBIN,
                           PULSAR_GRAD_PAPER_NORM, PULSAR_BLEND_TOPK,
                           PULSAR_ORTHO, PULSAR_STORE_HITS and
                           PULSAR_BWD_TILES; any other bit
                           is reserved (PULSAR_ERR_UNSUPPORTED) */
  int32_t max_pairs;    /* capacity of (screen tile, sphere) pairs; 0 = default
                           (2 n + number of tiles + 65536) */
  int32_t depth_bits;   /* reserved, must be 0 (PULSAR_ERR_UNSUPPORTED
                           otherwise): every tile list holds its spheres in
                           the order of their index */
  int32_t chunk;        /* sphere records per raster work item: 0 = automatic
                           (128), else a multiple of 64 in [64, 1024]. Long tile
                           lists are split into work items of this size and
                           their partial blends merged. Changes only the
                           summation order. */
  int32_t raster_blocks;/* blocks of the persistent raster kernels: 0 = automatic
                           (4096), else in [256, 65536]. Never changes the image;
                           gradients only within float atomic reordering. */
  float stop_share;     /* early ray termination (Sec. 3.2 and App. B, Step 2):
                           0 = off (default; every hit blends). In (0, 1):
                           each pixel takes its hits in ascending order of
                           their sphere's earliest possible hit distance
                           (float32 of |c| - R, c_z - R orthographic; ties by
                           index) and stops before the first hit whose
                           largest possible weight exp(z(that distance) /
                           gamma) is below stop_share / (1 - stop_share) of
                           the running denominator of Eq. 1 (opacity <= 1 is
                           assumed for the bound): no farther sphere can then
                           take that share of the pixel. Only the blended
                           hits enter the image, the log-normaliser and the K
                           nearest that pulsar_bwd differentiates. Every tile
                           is then one work item (chunk is ignored) and its
                           list is sorted by that distance. Combining it with
                           PULSAR_BLEND_TOPK is PULSAR_ERR_UNSUPPORTED;
                           pulsar_bwd must get the forward's value. */
} pulsar_params_t;

/* Bytes of device workspace one pulsar_fwd / pulsar_bwd pair needs for n
 * spheres, a width x height image and C channels. Host-only arithmetic.
 * Returns 0 for invalid arguments. A workspace sized for n works for any
 * smaller sphere count with the same image size and parameters. */
size_t pulsar_workspace_size(int32_t n, int32_t width, int32_t height, int32_t C,
                             const pulsar_params_t* params);

/* Forward pass (Eq. 1 over all hits; App. B, Steps 0-2).
 *   pos [n,3], radius [n]      sphere centres (world) and radii
 *   opacity [n] or NULL        NULL means o = 1 for every sphere; o >= 0 is a
 *                              precondition and is not checked on the device
 *   payload [n,C]              feature vector f_i of every sphere, C >= 1
 *   background [C]             background feature
 *   image [H,W,C]  (out)       F, channels last
 *   aux [H,W]      (out)       per-pixel L = log of the Eq. 1 denominator,
 *                              needed by pulsar_bwd; may be NULL if no backward
 *                              pass follows (then no backward state is kept,
 *                              as with PULSAR_NO_BWD_AUX)
 *   ws, ws_bytes               caller-owned device workspace; after the call it
 *                              holds the sorted tile lists that pulsar_bwd reuses
 * n = 0 is valid and renders the background. Outputs must not alias inputs. */
int pulsar_fwd(const float* pos, const float* radius, const float* opacity,
               const float* payload, int32_t n, int32_t C, const float* background,
               const pulsar_camera_t* cam, const pulsar_params_t* params, float* image,
               float* aux, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * pulsar_fwd with no workspace argument. Every other argument, result and
 * error is that of pulsar_fwd. The workspace is a static device array of
 * PULSAR_NOALLOC_SCRATCH_BYTES that every GPU the library runs this call on
 * holds until the process ends; the call allocates no device memory. A call
 * whose pulsar_workspace_size exceeds it returns PULSAR_ERR_SCRATCH before
 * anything is enqueued. All calls on one GPU share that GPU's array, which
 * keeps the last call's contents (nothing in it needs clearing): calls whose
 * work overlaps on one GPU (other streams, other threads) race and must be
 * serialised by the caller, and a pulsar_bwd cannot reuse the state (use a
 * workspace and PULSAR_REBIN for gradients). The device status of the call
 * lives in that array and cannot be queried: a call whose (tile, sphere)
 * pairs exceed params.max_pairs leaves invalid outputs, so size max_pairs
 * for the scene (the default, 2 n + tiles + 65536, holds any scene whose
 * spheres touch two tiles each on average). */
#define PULSAR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int pulsar_fwd_noalloc(const float* pos, const float* radius, const float* opacity,
                       const float* payload, int32_t n, int32_t C, const float* background,
                       const pulsar_camera_t* cam, const pulsar_params_t* params, float* image,
                       float* aux, void* stream);

/* Backward pass (App. B, "The Backward Pass"): given grad_image = dLoss/dF
 * [H,W,C], writes (overwrites, never accumulates)
 *   grad_pos [n,3], grad_radius [n], grad_opacity [n], grad_payload [n,C],
 *   grad_background [C].
 * Any output may be NULL when that gradient is not needed (Sec. App. B: only
 * required gradients are computed); grad_opacity must be NULL when opacity is.
 * Scene, camera, params, image and aux must be exactly those of the preceding
 * pulsar_fwd on the same workspace, with no other call on that workspace in
 * between, unless params.flags has PULSAR_REBIN (then only image and aux must
 * come from a forward of the same inputs). The flags that act on the
 * backward alone (PULSAR_REBIN, PULSAR_GRAD_PAPER_NORM) may differ from the
 * forward's, PULSAR_BLEND_TOPK is ignored here (image and aux carry it),
 * PULSAR_NO_BWD_AUX needs PULSAR_REBIN (below) and PULSAR_ORTHO must match. The per-pixel hits are recomputed
 * from the sorted tile lists; nothing per pixel beyond image and aux is
 * stored. PULSAR_NO_BWD_AUX without PULSAR_REBIN, or aux NULL, is
 * PULSAR_ERR_INVALID_ARGUMENT. */
int pulsar_bwd(const float* pos, const float* radius, const float* opacity,
               const float* payload, int32_t n, int32_t C, const float* background,
               const pulsar_camera_t* cam, const pulsar_params_t* params, const float* image,
               const float* aux, const float* grad_image, float* grad_pos, float* grad_radius,
               float* grad_opacity, float* grad_payload, float* grad_background, void* ws,
               size_t ws_bytes, void* stream);

/* pulsar_bwd plus the camera gradients (Sec. 3.1: the render map is
 * differentiable in the camera as well as in the scene), for
 * grad_camera [14] (out, not NULL): dLoss/dR as a row-major 3x3 (R taken as a
 * free matrix: the caller chains through its own rotation parameters),
 * dLoss/dt [3], dLoss/dfocal and dLoss/dsensor_width. Every other argument,
 * state requirement and error is that of pulsar_bwd; NULL grad_camera is
 * PULSAR_ERR_INVALID_ARGUMENT.
 * The camera acts through the camera-space centres c = R p + t of every
 * sphere and, via the ratio focal / sensor_width, through every pixel ray and
 * the minimum-size radius (App. B, Step 0), so focal dL/dfocal + sensor_width
 * dL/dsensor_width = 0. Like the scene gradients these are the derivatives
 * of the truncated backward: a pixel passes gradients to its K nearest hits
 * only. Sums are taken in FP64 over per-sphere FP32 terms, in a fixed order. */
int pulsar_bwd_camera(const float* pos, const float* radius, const float* opacity,
                      const float* payload, int32_t n, int32_t C, const float* background,
                      const pulsar_camera_t* cam, const pulsar_params_t* params,
                      const float* image, const float* aux, const float* grad_image,
                      float* grad_pos, float* grad_radius, float* grad_opacity,
                      float* grad_payload, float* grad_background, float* grad_camera, void* ws,
                      size_t ws_bytes, void* stream);

/* ---- Batched rendering: several independent scenes in one call.
 *
 * Each scene is the problem of Sec. 3.1-3.2 on its own: a sphere set, a
 * camera and an image size. A batched call renders all of them with one
 * launch per pipeline stage (all scenes' tiles share the persistent raster
 * grid), which is what a loop of single-scene calls cannot do for small
 * scenes. The results equal those of pulsar_fwd / pulsar_bwd per scene up to
 * float summation order.
 *
 * Packing (B scenes, N = sum of n_b spheres, P = sum of H_b W_b pixels):
 *   pos [N,3], radius [N], opacity [N] or NULL, payload [N,C]
 *       scene b owns rows n_0 + ... + n_{b-1} onwards, in scene order;
 *   background [B,C]                 one background feature per scene;
 *   image [P,C], aux [P], grad_image [P,C]
 *       scene b owns the H_b x W_b row-major block of pixels that starts after
 *       the pixels of scenes 0 .. b-1;
 *   grad_pos [N,3], grad_radius [N], grad_opacity [N], grad_payload [N,C],
 *   grad_background [B,C]            packed like their inputs.
 * C, K, gamma and every other parameter are shared. The scene array is read
 * on the host during the call only; its cameras are copied into the launch
 * arguments, so a captured graph replays with the cameras of capture time
 * while reading the sphere and image buffers afresh at every replay. */
#define PULSAR_MAX_SCENES 4096

typedef struct pulsar_scene {
  pulsar_camera_t camera;  /* camera and image size of this scene */
  int32_t n;               /* its number of spheres, >= 0 */
  int32_t reserved;        /* must be 0 */
} pulsar_scene_t;

/* Workspace bytes of a batched pair of calls on these B scenes (1 <= B <=
 * PULSAR_MAX_SCENES). Returns 0 for invalid arguments. For B = 1 it equals
 * pulsar_workspace_size of that scene. */
size_t pulsar_batch_workspace_size(const pulsar_scene_t* scenes, int32_t B, int32_t C,
                                   const pulsar_params_t* params);

/* Batched forward: pulsar_fwd for every scene, packed as described above.
 * Totals must satisfy N < 2^31 and fewer than 2^31 8x8 tiles. */
int pulsar_fwd_batched(const pulsar_scene_t* scenes, int32_t B, const float* pos,
                       const float* radius, const float* opacity, const float* payload,
                       int32_t C, const float* background, const pulsar_params_t* params,
                       float* image, float* aux, void* ws, size_t ws_bytes, void* stream);

/* Batched backward: pulsar_bwd for every scene; the same rules on NULL
 * outputs and on pairing with the preceding forward apply. */
/* pulsar_fwd_batched with the cameras read from device memory when the work
 * runs rather than when the call is made: d_cameras [B] pulsar_camera_t in
 * device memory (caller-owned; read by this call's first kernels), while
 * scenes[b].camera only gives the image sizes (and must be valid). A graph
 * captured from this call renders, at each replay, with the cameras
 * d_cameras then holds (image sizes and sphere counts stay those of the
 * capture). The device computes the camera constants as the host does, so
 * the results equal pulsar_fwd_batched with those cameras bitwise. Device
 * cameras cannot be checked on the host: an invalid one (the checks
 * pulsar_fwd makes) makes pulsar_query_status report
 * PULSAR_ERR_INVALID_ARGUMENT, and the outputs are undefined. A
 * pulsar_bwd_batched on the same workspace without PULSAR_REBIN uses the
 * cameras this forward read; with PULSAR_REBIN it would use those of its
 * own scenes argument. */
int pulsar_fwd_batched_devcam(const pulsar_scene_t* scenes, int32_t B,
                              const pulsar_camera_t* d_cameras, const float* pos,
                              const float* radius, const float* opacity, const float* payload,
                              int32_t C, const float* background, const pulsar_params_t* params,
                              float* image, float* aux, void* ws, size_t ws_bytes,
                              void* stream);

int pulsar_bwd_batched(const pulsar_scene_t* scenes, int32_t B, const float* pos,
                       const float* radius, const float* opacity, const float* payload,
                       int32_t C, const float* background, const pulsar_params_t* params,
                       const float* image, const float* aux, const float* grad_image,
                       float* grad_pos, float* grad_radius, float* grad_opacity,
                       float* grad_payload, float* grad_background, void* ws,
                       size_t ws_bytes, void* stream);

/* pulsar_bwd_batched plus the camera gradients of every scene, grad_camera
 * [B,14] (out, not NULL), row b laid out as in pulsar_bwd_camera. */
int pulsar_bwd_camera_batched(const pulsar_scene_t* scenes, int32_t B, const float* pos,
                              const float* radius, const float* opacity, const float* payload,
                              int32_t C, const float* background, const pulsar_params_t* params,
                              const float* image, const float* aux, const float* grad_image,
                              float* grad_pos, float* grad_radius, float* grad_opacity,
                              float* grad_payload, float* grad_background, float* grad_camera,
                              void* ws, size_t ws_bytes, void* stream);

/* Synchronises `stream` and reports the status the device wrote into the
 * workspace during the last pulsar_fwd: PULSAR_OK, PULSAR_ERR_CAPACITY, or
 * PULSAR_ERR_INVALID_ARGUMENT when a camera pulsar_fwd_batched_devcam read
 * from device memory was invalid. If pairs is not NULL it receives the
 * number of (tile, sphere) pairs that forward produced. */
int pulsar_query_status(const void* ws, size_t ws_bytes, void* stream, int64_t* pairs);

/* The status without synchronising: once a forward's work has completed, the
 * first PULSAR_STATUS_BYTES bytes of its workspace hold, little-endian,
 * uint32 status (0: PULSAR_OK, else minus the PULSAR_ERR_* code), uint32
 * pairs stored, uint64 pairs produced. A caller may copy them behind the
 * forward on its stream (into pinned host memory, say) and read them later,
 * which keeps the stream free of host synchronisation (graph capture). */
#define PULSAR_STATUS_BYTES 16

/* Static English description of a status code. Never NULL. */
const char* pulsar_status_string(int code);

/* Message of the last PULSAR_ERR_HIP raised by this thread, or "". */
const char* pulsar_last_hip_error(void);

/* Stage timing, a profiling aid. While enabled (process-wide), every
 * pulsar_fwd / pulsar_bwd records a pair of HIP events on its stream around
 * each stage below; pulsar_timing_read waits for the recorded events and adds
 * their elapsed times per stage into total_ms[PULSAR_NUM_STAGES] and the
 * number of timed launches into counts[PULSAR_NUM_STAGES] (either may be
 * NULL), then forgets them. Enabling costs one event pair per stage and call;
 * it never changes results. pulsar_timing_enable returns the previous state. */
#define PULSAR_STAGE_PROJECT 0    /* K1: projection, culling, sphere records */
#define PULSAR_STAGE_BINNING 1    /* K2-K5: pair scan, emission, radix sort, tile ranges */
#define PULSAR_STAGE_RASTER_FWD 2 /* K6: per-tile forward blend (and empty-tile fill) */
#define PULSAR_STAGE_ZERO 3       /* clearing of the gradient outputs */
#define PULSAR_STAGE_RASTER_BWD 4 /* K7: backward with recomputed hits (sphere walk, or the
                                     tile walk when asked for with PULSAR_BWD_TILES) */
#define PULSAR_STAGE_FINALIZE 5   /* K8: world-space gradients, background sum */
#define PULSAR_STAGE_MERGE 6      /* K6b: merge of split tiles' partial blends */
#define PULSAR_STAGE_RASTER_BWD_TILES 7 /* K7 tile walk beside the default sphere walk
                                           (returns at once unless a sphere is very large) */
#define PULSAR_NUM_STAGES 8
int pulsar_timing_enable(int on);
int pulsar_timing_read(double* total_ms, int64_t* counts);
const char* pulsar_stage_name(int stage);

/* ABI version of this header, currently 3. */
int pulsar_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PULSAR_H_ */
