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
// binning: the (bin block, tile) count matrix is built and read in slices of
// kBinSlice tiles; K3 handles 64 tiles per block of kScanThreads threads, each
// wave up to kBinRowsPerWave rows of the matrix (so at most kBinMaxG rows)
constexpr int kBinThreads = 256;
constexpr int kBinSliceBits = 13;
constexpr int kBinSlice = 1 << kBinSliceBits;
constexpr int kScanThreads = 1024;
constexpr int kBinRowsPerWave = 16;
constexpr int kBinMaxG = kBinRowsPerWave * (kScanThreads / 64);
constexpr long long kBinCells = 1LL << 22;  // matrix size the bin-block sizes aim for
constexpr int kMaxK = 32;
constexpr int kFwdChannels = 32;             // channels per forward pass (more: several passes)
constexpr int kBwdChannels = 32;             // channels kept in registers by the backward
constexpr int kChunkDefault = 128;           // sphere records per raster work item
constexpr int kRasterGridDefault = 4096;     // persistent raster grid (one wave per block)
constexpr int kUploadScenes = 12;            // scene descriptors per upload launch
constexpr int kBgBlockPixels = 1024;         // pixels per background-gradient block
constexpr int kCamSpan = 1024;               // spheres per camera-gradient partial sum
constexpr uint32_t kFirstChunk = 0x80000000u;  // work item flag: first chunk of its tile
constexpr uint32_t kNoSlot = 0xffffffffu;      // work item writes final pixels, no partial state

// Device status block at the start of the workspace.
struct Status {
  uint32_t code;                // PULSAR_OK or PULSAR_ERR_CAPACITY
  uint32_t used;                // pairs actually stored: min(pairs, capacity)
  unsigned long long pairs;     // pairs the scene produced
  uint32_t nchunks;             // raster work items (chunks of <= chunk records of one tile)
  uint32_t npartials;           // partial blend states needed by tiles with several chunks
  uint32_t nfull;               // work items with exactly chunk records (listed first)
  uint32_t nmerge;              // tiles with several work items
  uint32_t pad[56];
};

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
  // binning: the scene's spheres in bin_G bin blocks of bin_S (a multiple of
  // kBinThreads) and its tiles in `slices` slices of kBinSlice; its work
  // units (bin block, slice) are unit_off .. unit_off + bin_G slices - 1,
  // bin block g's counts per tile are row row_off + g T_b of the matrix
  uint32_t bin_S, bin_G, slices, unit_off;
  unsigned long long row_off;
};

// Device copy of the scene table plus four ascending start arrays of B + 1
// entries each (spheres, tiles, background blocks, binning units) for scene
// lookup.
constexpr int kStartArrays = 4;
struct SceneTable {
  const SceneDev* scenes;
  const uint32_t* sph_start;
  const uint32_t* tile_start;
  const uint32_t* blk_start;
  const uint32_t* unit_start;
  int B;
};

// Workspace layout: byte offsets of every buffer, all 256-byte aligned.
struct Plan {
  int64_t n, C, T, npix, cap, nbgblk;
  int B, chunk, raster_grid;
  int nblk_proj;
  // binning: work units (bin block, tile slice) of all scenes and the size
  // of the count matrix
  int64_t bin_units, bin_cells;
  size_t off_status, off_counts, off_trect, off_rec;
  size_t off_partials, off_boff;
  size_t off_bmat;    // [G, T] pairs per (bin block, tile), then their offsets inside the tile
  size_t off_tcount;  // [T] pairs per tile
  size_t off_gsum;    // [T / 64] sums over groups of 64 tiles (pairs, work-item counts)
  size_t off_vals;    // [cap] sphere index of every pair, tile by tile
  size_t off_ranges;  // [T + 1] first pair of each tile
  // raster work items: per tile uint4 (first partial-state slot, chunks, 0, 0);
  // the work list uint4 (tile | kFirstChunk, begin, end, slot or kNoSlot);
  // block sums of the chunk scan; the partial blend states; the per-pixel
  // K-th nearest hit (t, sphere id); background-gradient block sums
  size_t off_tinfo, off_desc, off_pstate, off_thr, off_bgsum;
  size_t off_mlist;  // tiles with several work items, for the merge kernel
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
  t.unit_start = st + 3 * (q.B + 1);
  t.B = q.B;
  return t;
}

}  // namespace pulsar
