// Internal declarations shared by the C ABI (capi.cpp) and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "pulsar.h"

namespace pulsar {

// One wave64 renders one 8x8 screen tile: lane l owns pixel (l / 8, l % 8).
constexpr int kTileW = 8;
constexpr int kTileH = 8;
constexpr int kWave = 64;
constexpr int kProjectBlock = 256;           // spheres per projection block
// binning: a stable LSD radix sort of the pairs by tile number, digits of
// at most kMaxDigitBits bits; every counting kernel has at most
// kMaxSortBlocks blocks, so the block x digit count matrices stay small
constexpr int kMaxDigitBits = 8;
constexpr int kMaxSortBlocks = 256;
constexpr int kSortMinBlock = 2048;          // pairs per sorting block, at least
constexpr int kEmitThreads = 1024;
constexpr int kEmitRound = 4 * kEmitThreads;  // spheres per emission round, 4 per thread
constexpr int kMaxK = 32;
constexpr int kFwdChannels = 32;             // channels per forward pass (more: several passes)
constexpr int kBwdChannels = 32;             // channels kept in registers by the backward
constexpr int kChunkDefault = 128;           // sphere records per raster work item
constexpr int kRasterGridDefault = 4096;     // persistent raster grid (one wave per block)
constexpr int kUploadScenes = 12;            // scene descriptors per upload launch
constexpr int kBgBlockPixels = 1024;         // pixels per background-gradient block
constexpr int kCamSpan = 1024;               // spheres per camera-gradient partial sum
constexpr int kRecPayload = 16;              // payload channels kept in the sphere record
// a sphere touching more tiles than this sends the default backward to the
// walk over the tile lists (the walk in sphere order would give all of its
// pixels to one wave)
constexpr uint32_t kBigTiles = 16;
constexpr uint32_t kFirstChunk = 0x80000000u;  // work item flag: first chunk of its tile
constexpr uint32_t kNoSlot = 0xffffffffu;      // work item writes final pixels, no partial state

// Device status block at the start of the workspace.
struct Status {
  uint32_t code;                // PULSAR_OK or PULSAR_ERR_CAPACITY
  uint32_t used;                // pairs stored and sorted: the pair count, or 0 past capacity
  unsigned long long pairs;     // pairs the scene produced
  uint32_t nfull;               // work items with exactly chunk records (front of the list)
  uint32_t nshort;              // shorter work items (back of the list)
  uint32_t npartials;           // partial blend states needed by tiles with several work items
  uint32_t nmerge;              // tiles with several work items
  uint32_t bad_cam;             // a camera read from device memory was invalid
  uint32_t hits_k;              // the forward stored K nearest hits per pixel (0: none)
  uint32_t big_spheres;         // a sphere touches more than kBigTiles tiles
  uint32_t pad[53];
};
static_assert(sizeof(Status) == 256, "status block");
static_assert(offsetof(Status, pairs) + sizeof(unsigned long long) == PULSAR_STATUS_BYTES,
              "the documented status prefix");

// Raster work items: full chunks fill the list from the front, shorter ones
// from the back (full chunks, the costlier items, are taken first).
__host__ __device__ inline uint32_t item_slot(uint32_t i, uint32_t nfull, uint32_t max_items) {
  return i < nfull ? i : max_items - 1u - (i - nfull);
}
// Work items of the call (none after a capacity overflow).
__device__ inline uint32_t item_count(const Status* st) {
  return st->code == 0u ? st->nfull + st->nshort : 0u;
}

// Camera constants in the form the kernels use.
struct CamDev {
  float R[9];
  float t[3];
  float f, s, znear, zfar;
  float pitch;  // s / W
  float sh;     // sensor height s H / W
  int W, H, tiles_x, tiles_y;
  // FP64 camera constants, computed once on the host with the same
  // expressions the kernels would evaluate (so the results are identical)
  double dpitch;      // s / W
  double dinv_pitch;  // W / s
  double dsh;         // s H / W
  double dhalf_sh;    // 0.5 s H / W
  // orthographic projection: rays along +z from the pixel centres on the
  // sensor plane; f is then 1, so the pinhole expressions of the kernels
  // (ray direction (x_s, y_s, f) with x_s = y_s = 0) give those rays
  int ortho;
};

// Blend constants of Eq. 1 in base-2 exponent units.
struct BlendConst {
  float kz;         // log2(e) / (gamma (zfar - znear)): o z / gamma * log2(e) = o (zfar - t) kz
  float eps2;       // eps / gamma * log2(e): exponent of the background weight
  float zfar;
  float inv_gamma;  // 1 / gamma
  float inv_span;   // 1 / (zfar - znear)
};

// One scene of a call: its camera and blend constants and where its spheres,
// tiles, pixels and background-gradient blocks start in the packed arrays.
// A single-scene call is a batch of one.
struct SceneDev {
  CamDev cam;
  BlendConst bc;
  uint32_t sph_off;    // first sphere
  uint32_t n;          // spheres
  uint32_t tile_off;   // first tile in the global tile numbering
  uint32_t bgblk_off;  // first background-gradient block
  unsigned long long pix_off;  // first pixel (index into the packed [P] planes)
};

// Device copy of the scene table plus three ascending start arrays of B + 1
// entries each (spheres, tiles, background blocks) for scene lookup.
constexpr int kStartArrays = 3;
struct SceneTable {
  const SceneDev* scenes;
  const uint32_t* sph_start;
  const uint32_t* tile_start;
  const uint32_t* blk_start;
  int B;
};

// Workspace layout: byte offsets of every buffer, all 256-byte aligned.
struct Plan {
  int64_t n, C, T, npix, cap, nbgblk;
  int B, chunk, raster_grid;
  int nblk_proj;
  // binning: LSD passes over the tile number and the digit width of each;
  // emission blocks of emit_rounds rounds of kEmitRound spheres
  int sort_passes, sort_digit, emit_rounds, nblk_emit;
  int rec4;           // float4 per sphere record: 4 (geometry) or 8 (with the payload row)
  int estop;          // early termination: tiles are sorted by earliest hit distance
  int K, store_hits;  // stored per-pixel K nearest hits (PULSAR_STORE_HITS)
  int bwd_tiles;      // the backward walks the tile lists (PULSAR_BWD_TILES)
  size_t off_hits;    // [npix][K] (t, sphere index), last in the workspace
  size_t off_tmin;    // [n] float32 earliest possible hit distance (early termination)
  size_t off_stop;    // [npix] (distance, pair position) of the first skipped hit
  size_t off_status, off_counts, off_trect, off_rec;
  size_t off_partials, off_boff;
  size_t off_ebase;   // [nblk_emit + 1] first pair of each emission block (u64)
  size_t off_mat;     // block x digit counts of the current pass, digit-major
  size_t off_keys;    // [cap] tile of every pair, sorted (the final pass's output)
  size_t off_vals;    // [cap] sphere index of every pair, tile by tile
  size_t off_keys2, off_vals2;  // the other buffers of the ping-pong
  size_t off_trange;  // [T] first and end pair of each tile (uint2)
  // raster work items: per tile uint4 (first partial-state slot, chunks, 0, 0);
  // the work list uint4 (tile | kFirstChunk, begin, end, slot or kNoSlot);
  // block sums of the chunk scan; the partial blend states; the per-pixel
  // K-th nearest hit (t, sphere id); background-gradient block sums
  size_t off_tinfo, off_desc, off_pstate, off_thr, off_bgsum;  // off_thr: [npix] float4
  size_t off_mlist;  // tiles with several work items (tile, first slot, items), for the merge
  size_t off_scenes, off_starts;  // scene table and its start arrays
  // backward: one sum slot per (tile, sphere) pair at its emission position,
  // bwd_ps4 float4 each (dL/dc, dL/dR | dL/df[cm] | dL/do, dL/d(f/s), pixel
  // count, padding)
  size_t off_pslot;
  // camera gradients: per sphere float4 (dL/dc, dL/d(f/s)); per-scene runs of
  // partial sums, 16 doubles each (scene b's run starts at b + first sphere /
  // kCamSpan)
  size_t off_camg, off_campart;
  int64_t ncampart;
  int bwd_ps4;
  int64_t max_chunks, pcap;
  int fwd_cm, klist_slots, pstride;
  size_t total;
};

// Validates the scenes and fills the host copy of the scene table (offsets in
// scene order). Returns PULSAR_OK or an error code.
int make_scenes(const pulsar_scene_t* scenes, int B, const pulsar_params_t* p,
                std::vector<SceneDev>* out);
// Fills `out` from a validated scene table and returns PULSAR_OK, or returns
// an error code.
// fwd_only: a forward that keeps no backward state (no backward buffers).
int make_plan(const std::vector<SceneDev>& sc, int C, const pulsar_params_t* p, Plan* out,
              bool fwd_only = false);
CamDev make_cam(const pulsar_camera_t* c);
BlendConst make_blend(const pulsar_camera_t* c, const pulsar_params_t* p);

struct FwdArgs {
  const float* pos;
  const float* radius;
  const float* opacity;
  const float* payload;
  const float* bg;
  int n, C, K;
  float* image;
  float* aux;
  float min_radius_px;
  bool track;  // keep each pixel's K nearest hits for a following backward
  bool topk;   // blend only each pixel's K nearest hits
  float stop_share;  // early termination share (0: off)
  // cameras read from device memory when the work runs (null: the host table)
  const pulsar_camera_t* d_cams;
  float gamma, eps;  // for the blend constants of device cameras
  bool ortho;
};

struct BwdArgs {
  const float* pos;
  const float* radius;
  const float* opacity;
  const float* payload;
  int n, C, K;
  const float* image;
  const float* aux;
  const float* grad_image;
  float* grad_pos;
  float* grad_radius;
  float* grad_opacity;
  float* grad_payload;
  float* grad_bg;
  float* grad_cam;  // [B, 14]: dL/dR (3x3), dL/dt, dL/df, dL/ds per scene, or null
  bool paper_norm;  // per-pixel averaging and the 3-pixel position gate
  float min_radius_px;
  float eps2;  // eps / gamma * log2(e), the background exponent (camera independent)
  // the thresholds were rebuilt by the backward (their stored L is that of
  // the full blend, which differs from the caller's under the top-K blend)
  bool rebinned;
};

// Enqueue the forward / backward pipelines. The forward first copies the
// host scene table into the workspace; the backward uses that copy. They
// return the first launch error.
hipError_t launch_forward(const Plan& plan, const std::vector<SceneDev>& scenes,
                          const FwdArgs& a, char* ws, hipStream_t stream);
hipError_t launch_backward(const Plan& plan, const BwdArgs& a, char* ws, hipStream_t stream);
// The forward's backward state without its image: projection, binning and a
// raster pass that only keeps each pixel's K nearest hits (image and aux of
// `a` are not written and may be NULL).
hipError_t launch_rebin(const Plan& plan, const std::vector<SceneDev>& scenes, const FwdArgs& a,
                        char* ws, hipStream_t stream);

// Stage timing hooks (no-ops unless pulsar_timing_enable(1) was called).
void stage_begin(int stage, hipStream_t stream);
void stage_end(int stage, hipStream_t stream);
// While one exists, the calling thread's launches record no timing events.
struct TimingOff {
  TimingOff();
  ~TimingOff();
};
// Records the HIP error for pulsar_last_hip_error; returns PULSAR_ERR_HIP.
int fail_hip(hipError_t e);

// Pointers into the workspace.
template <typename T>
inline T* ws_ptr(char* ws, size_t off) {
  return reinterpret_cast<T*>(ws + off);
}

inline SceneTable scene_table(const Plan& q, char* ws) {
  SceneTable t;
  t.scenes = ws_ptr<SceneDev>(ws, q.off_scenes);
  const uint32_t* st = ws_ptr<uint32_t>(ws, q.off_starts);
  t.sph_start = st;
  t.tile_start = st + (q.B + 1);
  t.blk_start = st + 2 * (q.B + 1);
  t.B = q.B;
  return t;
}

}  // namespace pulsar
