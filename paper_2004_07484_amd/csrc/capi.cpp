// C ABI of the sphere renderer: host-side validation, workspace planning and
// the entry points declared in include/pulsar.h. Every check runs before any
// work is enqueued, so a failing call leaves the stream untouched.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pulsar_internal.h"

namespace pulsar {
namespace {

thread_local std::string g_last_hip_error;

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool finite_all(const float* v, int k) {
  for (int i = 0; i < k; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

int check_camera(const pulsar_camera_t* c) {
  if (!c) return PULSAR_ERR_INVALID_ARGUMENT;
  if (!finite_all(c->R, 9) || !finite_all(c->t, 3)) return PULSAR_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(c->focal) || !(c->focal > 0.f)) return PULSAR_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(c->sensor_width) || !(c->sensor_width > 0.f))
    return PULSAR_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(c->znear) || !(c->znear > 0.f)) return PULSAR_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(c->zfar) || !(c->zfar > c->znear)) return PULSAR_ERR_INVALID_ARGUMENT;
  if (c->width < 1 || c->width > 65535 || c->height < 1 || c->height > 65535)
    return PULSAR_ERR_INVALID_ARGUMENT;
  return PULSAR_OK;
}

int check_params(const pulsar_params_t* p) {
  if (!p) return PULSAR_ERR_INVALID_ARGUMENT;
  // gamma in [1e-5, 1] (Sec. 3.2); a relative slack of 1e-6 admits float rounding of 1e-5
  if (!std::isfinite(p->gamma) || p->gamma < 1e-5f * (1.f - 1e-6f) || p->gamma > 1.f)
    return PULSAR_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(p->eps) || p->eps < 0.f) return PULSAR_ERR_INVALID_ARGUMENT;
  if (!std::isfinite(p->min_radius_px) || p->min_radius_px < 0.f)
    return PULSAR_ERR_INVALID_ARGUMENT;
  if (p->K < 1 || p->K > kMaxK) return PULSAR_ERR_INVALID_ARGUMENT;
  if (p->max_pairs < 0) return PULSAR_ERR_INVALID_ARGUMENT;
  // the tile lists are in sphere order; a depth key is no longer offered
  if (p->depth_bits != 0) return PULSAR_ERR_UNSUPPORTED;
  if (p->chunk != 0 && (p->chunk < 64 || p->chunk > 1024 || p->chunk % 64 != 0))
    return PULSAR_ERR_INVALID_ARGUMENT;
  if (p->raster_blocks != 0 && (p->raster_blocks < 256 || p->raster_blocks > 65536))
    return PULSAR_ERR_INVALID_ARGUMENT;
  if ((p->flags & ~(PULSAR_NO_BWD_AUX | PULSAR_REBIN | PULSAR_GRAD_PAPER_NORM |
                    PULSAR_BLEND_TOPK | PULSAR_ORTHO | PULSAR_STORE_HITS |
                    PULSAR_BWD_TILES)) != 0u)
    return PULSAR_ERR_UNSUPPORTED;
  if (!std::isfinite(p->stop_share) || p->stop_share < 0.f || p->stop_share >= 1.f)
    return PULSAR_ERR_INVALID_ARGUMENT;
  // the top-K blend with early termination is not built
  if (p->stop_share > 0.f && (p->flags & PULSAR_BLEND_TOPK) != 0u) return PULSAR_ERR_UNSUPPORTED;
  return PULSAR_OK;
}

// ---- stage timing
std::atomic<int> g_timing{0};
thread_local int g_timing_off = 0;  // > 0: this thread's calls record no events
std::mutex g_timing_mu;
struct Mark {
  int stage;
  hipEvent_t begin, end;
};
std::vector<Mark> g_marks;        // completed begin/end pairs awaiting read-out
hipEvent_t g_open[PULSAR_NUM_STAGES] = {};  // begin events without their end yet

}  // namespace

int fail_hip(hipError_t e) {
  g_last_hip_error = hipGetErrorString(e);
  return PULSAR_ERR_HIP;
}

TimingOff::TimingOff() { ++g_timing_off; }
TimingOff::~TimingOff() { --g_timing_off; }

void stage_begin(int stage, hipStream_t stream) {
  if (g_timing_off > 0 || !g_timing.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, stream);
  if (g_open[stage]) (void)hipEventDestroy(g_open[stage]);
  g_open[stage] = e;
}

void stage_end(int stage, hipStream_t stream) {
  if (g_timing_off > 0 || !g_timing.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  if (!g_open[stage]) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, stream);
  g_marks.push_back(Mark{stage, g_open[stage], e});
  g_open[stage] = nullptr;
}

int make_scenes(const pulsar_scene_t* scenes, int B, const pulsar_params_t* p,
                std::vector<SceneDev>* out) {
  if (!scenes || B < 1 || B > PULSAR_MAX_SCENES) return PULSAR_ERR_INVALID_ARGUMENT;
  int rc = check_params(p);
  if (rc != PULSAR_OK) return rc;
  out->clear();
  out->reserve(size_t(B));
  int64_t sph = 0, tiles = 0, blk = 0;
  unsigned long long pix = 0;
  for (int b = 0; b < B; ++b) {
    const pulsar_scene_t& sc = scenes[b];
    rc = check_camera(&sc.camera);
    if (rc != PULSAR_OK) return rc;
    if (sc.n < 0) return PULSAR_ERR_INVALID_ARGUMENT;
    if (sc.reserved != 0) return PULSAR_ERR_UNSUPPORTED;
    SceneDev d;
    std::memset(&d, 0, sizeof(d));
    d.cam = make_cam(&sc.camera);
    if ((p->flags & PULSAR_ORTHO) != 0u) {
      d.cam.ortho = 1;
      d.cam.f = 1.f;  // the kernels' ray direction (0, 0, f) is then the unit +z
    }
    d.bc = make_blend(&sc.camera, p);
    d.sph_off = uint32_t(sph);
    d.n = uint32_t(sc.n);
    d.tile_off = uint32_t(tiles);
    d.bgblk_off = uint32_t(blk);
    d.pix_off = pix;
    const int64_t npix = int64_t(sc.camera.width) * sc.camera.height;
    sph += sc.n;
    tiles += int64_t(d.cam.tiles_x) * d.cam.tiles_y;
    blk += (npix + kBgBlockPixels - 1) / kBgBlockPixels;
    pix += (unsigned long long)npix;
    // sphere indices and tile numbers carry a flag in bit 31
    if (sph > INT32_MAX || tiles > INT32_MAX || blk > INT32_MAX)
      return PULSAR_ERR_INVALID_ARGUMENT;
    out->push_back(d);
  }
  return PULSAR_OK;
}

int make_plan(const std::vector<SceneDev>& sc, int C, const pulsar_params_t* p, Plan* out,
              bool fwd_only) {
  if (sc.empty() || C < 1) return PULSAR_ERR_INVALID_ARGUMENT;
  int rc = check_params(p);
  if (rc != PULSAR_OK) return rc;
  const SceneDev& last = sc.back();
  const int64_t lastpix = int64_t(last.cam.W) * last.cam.H;
  Plan q;
  std::memset(&q, 0, sizeof(q));
  q.B = int(sc.size());
  q.n = int64_t(last.sph_off) + last.n;
  q.C = C;
  q.T = int64_t(last.tile_off) + int64_t(last.cam.tiles_x) * last.cam.tiles_y;
  q.npix = int64_t(last.pix_off) + lastpix;
  q.nbgblk = int64_t(last.bgblk_off) + (lastpix + kBgBlockPixels - 1) / kBgBlockPixels;
  q.chunk = p->chunk > 0 ? p->chunk : kChunkDefault;
  // early termination walks each tile's whole list in order: one work item
  // per tile (no partial states, no merge)
  q.estop = p->stop_share > 0.f ? 1 : 0;
  if (q.estop) q.chunk = 1 << 30;
  q.raster_grid = p->raster_blocks > 0 ? p->raster_blocks : kRasterGridDefault;
  const int64_t n = q.n;
  int64_t cap = p->max_pairs > 0 ? int64_t(p->max_pairs) : 2 * n + q.T + 65536;
  if (cap > (int64_t(1) << 31) - 1) cap = (int64_t(1) << 31) - 1;
  q.cap = cap;
  q.nblk_proj = int((n + kProjectBlock - 1) / kProjectBlock);
  // LSD passes: enough digits of at most kMaxDigitBits bits for the tile
  // numbers 0 .. T - 1 (none for a single tile), all of the same width
  int bits = 0;
  while ((int64_t(1) << bits) < q.T) ++bits;
  q.sort_passes = (bits + kMaxDigitBits - 1) / kMaxDigitBits;
  q.sort_digit = q.sort_passes > 0 ? (bits + q.sort_passes - 1) / q.sort_passes : 0;
  // emission blocks: at most kMaxSortBlocks of them, whole rounds each
  const int64_t per_round = int64_t(kMaxSortBlocks) * kEmitRound;
  q.emit_rounds = int((n + per_round - 1) / per_round);
  if (q.emit_rounds < 1) q.emit_rounds = 1;
  const int64_t spb = int64_t(q.emit_rounds) * kEmitRound;
  q.nblk_emit = int((n + spb - 1) / spb);
  if (q.nblk_emit < 1) q.nblk_emit = 1;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align_up(bytes);
    return at;
  };
  const size_t nn = size_t(n > 0 ? n : 1);
  q.off_status = take(sizeof(Status));
  q.off_scenes = take(size_t(q.B) * sizeof(SceneDev));
  q.off_starts = take(size_t(kStartArrays) * size_t(q.B + 1) * 4);
  q.off_counts = take(nn * 4);
  q.off_trect = take(nn * 8);
  // records: 64 bytes of geometry. (Copying payload rows of up to
  // kRecPayload channels behind them, so that a raster gather touches one
  // 128-byte line, halved the raster kernels' fetched bytes but cost the
  // projection more time than the latency-bound raster kernels saved;
  // rec4 = 8 selects that layout.)
  q.rec4 = 4;
  q.off_rec = take(nn * size_t(q.rec4) * 16);
  q.off_partials = take(size_t(q.nblk_proj + 1) * 8);
  q.off_boff = take(size_t(q.nblk_proj + 1) * 8);
  q.off_ebase = take(size_t(q.nblk_emit + 1) * 8);
  // block x digit counts, with room for the last block's vector reads past the end
  q.off_mat = take((size_t(kMaxSortBlocks) << kMaxDigitBits) * 4 + 4096 * 4);
  q.off_keys = take(size_t(cap) * 4);
  q.off_vals = take(size_t(cap) * 4);
  q.off_keys2 = take(size_t(q.sort_passes > 0 ? cap : 1) * 4);
  q.off_vals2 = take(size_t(q.sort_passes > 0 ? cap : 1) * 4);
  q.off_trange = take(size_t(q.T) * 8);
  // early termination: every sphere's earliest possible hit distance
  q.off_tmin = take(q.estop ? nn * 4 : 0);
  q.max_chunks = (cap + q.chunk - 1) / q.chunk + q.T;
  // partial blend states: a tile of L > chunk pairs needs ceil(L / chunk)
  // < 2 L / chunk of them, so 2 cap / chunk + 1 bounds their sum
  q.pcap = 2 * ((cap + q.chunk - 1) / q.chunk) + 1;
  q.fwd_cm = C < kFwdChannels ? C : kFwdChannels;
  int km = 4;  // register K-list slots: a power of two >= K, at least 4
  while (km < p->K) km *= 2;
  q.klist_slots = km;
  q.pstride = 2 + q.fwd_cm + 2 * km;  // m, D, numerator[cm], K-list (t, id)
  q.off_tinfo = take(size_t(q.T) * 16);
  q.off_desc = take(size_t(q.max_chunks) * 16);
  // a forward that keeps no backward state needs none of the backward's
  // buffers (the top-K blend still needs the per-pixel thresholds)
  const bool bwd = !fwd_only;
  const bool thr = bwd || (p->flags & PULSAR_BLEND_TOPK) != 0u;
  q.off_bgsum = take(bwd ? size_t(q.nbgblk) * size_t(C) * 4 : 0);
  q.off_pstate = take(size_t(q.pcap) * kWave * size_t(q.pstride) * 4);
  q.off_thr = take(thr ? size_t(q.npix) * 16 : 0);
  // early termination: per pixel the first hit it skipped, for the backward
  q.off_stop = take(q.estop ? size_t(q.npix) * 8 : 0);
  q.off_mlist = take(size_t(q.T) * 16);
  // the backward kernel instance keeps cm >= C channels, a power of two up to
  // 32; wider payloads keep only dL/dc, dL/dR | dL/do in the record
  int bcm = 1;
  while (bcm < C && bcm < kBwdChannels) bcm *= 2;
  q.bwd_ps4 = C <= kBwdChannels ? 1 + (bcm + 6) / 4 : 2;
  q.ncampart = int64_t(q.B) + n / kCamSpan + 1;
  q.off_camg = take(bwd ? nn * 16 : 0);
  q.off_campart = take(bwd ? size_t(q.ncampart) * 16 * 8 : 0);
  // per-pair slots for the backward passes that gather through them (the
  // tile walk, which the default backward also takes for scenes with very
  // large spheres, the stored hits, wide payloads). They come after
  // everything the forward writes.
  q.bwd_tiles = (p->flags & PULSAR_BWD_TILES) != 0u ? 1 : 0;
  q.off_pslot = take(bwd ? size_t(cap) * size_t(q.bwd_ps4) * 16 : 0);
  // the stored per-pixel K nearest hits come last, so every other offset is
  // the same with or without them
  q.K = p->K;
  q.store_hits = (p->flags & PULSAR_STORE_HITS) != 0u ? 1 : 0;
  q.off_hits = take(q.store_hits ? size_t(q.npix) * size_t(p->K) * 8 : 0);
  q.total = o;
  *out = q;
  return PULSAR_OK;
}

CamDev make_cam(const pulsar_camera_t* c) {
  CamDev d;
  for (int i = 0; i < 9; ++i) d.R[i] = c->R[i];
  for (int i = 0; i < 3; ++i) d.t[i] = c->t[i];
  d.f = c->focal;
  d.s = c->sensor_width;
  d.znear = c->znear;
  d.zfar = c->zfar;
  d.W = c->width;
  d.H = c->height;
  d.pitch = float(double(c->sensor_width) / double(c->width));
  d.sh = float(double(c->sensor_width) * double(c->height) / double(c->width));
  d.tiles_x = (c->width + kTileW - 1) / kTileW;
  d.tiles_y = (c->height + kTileH - 1) / kTileH;
  d.dpitch = double(c->sensor_width) / double(c->width);
  d.dinv_pitch = double(c->width) / double(c->sensor_width);
  d.dsh = double(c->sensor_width) * double(c->height) / double(c->width);
  d.dhalf_sh = 0.5 * double(c->sensor_width) * double(c->height) / double(c->width);
  d.ortho = 0;
  return d;
}

BlendConst make_blend(const pulsar_camera_t* c, const pulsar_params_t* p) {
  const double log2e = 1.4426950408889634;
  const double span = double(c->zfar) - double(c->znear);
  BlendConst b;
  b.kz = float(log2e / (double(p->gamma) * span));
  b.eps2 = float(double(p->eps) / double(p->gamma) * log2e);
  b.zfar = c->zfar;
  b.inv_gamma = float(1.0 / double(p->gamma));
  b.inv_span = float(1.0 / span);
  return b;
}

}  // namespace pulsar

using namespace pulsar;

extern "C" {

size_t pulsar_batch_workspace_size(const pulsar_scene_t* scenes, int32_t B, int32_t C,
                                   const pulsar_params_t* params) {
  std::vector<SceneDev> sc;
  if (make_scenes(scenes, B, params, &sc) != PULSAR_OK) return 0;
  Plan q;
  if (make_plan(sc, C, params, &q) != PULSAR_OK) return 0;
  return q.total;
}

size_t pulsar_workspace_size(int32_t n, int32_t width, int32_t height, int32_t C,
                             const pulsar_params_t* params) {
  pulsar_scene_t sc;
  std::memset(&sc, 0, sizeof(sc));
  // any valid camera: the workspace depends on the image size only
  sc.camera.R[0] = sc.camera.R[4] = sc.camera.R[8] = 1.f;
  sc.camera.focal = sc.camera.sensor_width = 1.f;
  sc.camera.znear = 1.f;
  sc.camera.zfar = 2.f;
  sc.camera.width = width;
  sc.camera.height = height;
  sc.n = n;
  return pulsar_batch_workspace_size(&sc, 1, C, params);
}

static int fwd_impl(const pulsar_scene_t* scenes, int32_t B, const pulsar_camera_t* d_cams,
                    const float* pos, const float* radius, const float* opacity,
                    const float* payload, int32_t C, const float* background,
                    const pulsar_params_t* params, float* image, float* aux, void* ws,
                    size_t ws_bytes, void* stream) {
  std::vector<SceneDev> sc;
  int rc = make_scenes(scenes, B, params, &sc);
  if (rc != PULSAR_OK) return rc;
  if (C < 1) return PULSAR_ERR_INVALID_ARGUMENT;
  Plan q;
  rc = make_plan(sc, C, params, &q);
  if (rc != PULSAR_OK) return rc;
  if (q.n > 0 && (!pos || !radius || !payload)) return PULSAR_ERR_INVALID_ARGUMENT;
  if (!background || !image || !ws) return PULSAR_ERR_INVALID_ARGUMENT;
  if (ws_bytes < q.total) return PULSAR_ERR_WORKSPACE;
  FwdArgs a;
  a.pos = pos;
  a.radius = radius;
  a.opacity = opacity;
  a.payload = payload;
  a.bg = background;
  a.n = int(q.n);
  a.C = C;
  a.K = params->K;
  a.image = image;
  a.aux = aux;
  a.min_radius_px = params->min_radius_px;
  a.track = aux != nullptr && (params->flags & PULSAR_NO_BWD_AUX) == 0u;
  a.topk = (params->flags & PULSAR_BLEND_TOPK) != 0u;
  a.stop_share = params->stop_share;
  a.d_cams = d_cams;
  a.gamma = params->gamma;
  a.eps = params->eps;
  a.ortho = (params->flags & PULSAR_ORTHO) != 0u;
  hipError_t e = launch_forward(q, sc, a, static_cast<char*>(ws),
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail_hip(e);
  return PULSAR_OK;
}

int pulsar_fwd_batched(const pulsar_scene_t* scenes, int32_t B, const float* pos,
                       const float* radius, const float* opacity, const float* payload,
                       int32_t C, const float* background, const pulsar_params_t* params,
                       float* image, float* aux, void* ws, size_t ws_bytes, void* stream) {
  return fwd_impl(scenes, B, nullptr, pos, radius, opacity, payload, C, background, params,
                  image, aux, ws, ws_bytes, stream);
}

int pulsar_fwd_batched_devcam(const pulsar_scene_t* scenes, int32_t B,
                              const pulsar_camera_t* d_cameras, const float* pos,
                              const float* radius, const float* opacity, const float* payload,
                              int32_t C, const float* background, const pulsar_params_t* params,
                              float* image, float* aux, void* ws, size_t ws_bytes,
                              void* stream) {
  if (!d_cameras) return PULSAR_ERR_INVALID_ARGUMENT;
  return fwd_impl(scenes, B, d_cameras, pos, radius, opacity, payload, C, background, params,
                  image, aux, ws, ws_bytes, stream);
}

static int bwd_impl(const pulsar_scene_t* scenes, int32_t B, const float* pos,
                    const float* radius, const float* opacity, const float* payload, int32_t C,
                    const float* background, const pulsar_params_t* params, const float* image,
                    const float* aux, const float* grad_image, float* grad_pos,
                    float* grad_radius, float* grad_opacity, float* grad_payload,
                    float* grad_background, float* grad_camera, void* ws, size_t ws_bytes,
                    void* stream) {
  std::vector<SceneDev> sc;
  int rc = make_scenes(scenes, B, params, &sc);
  if (rc != PULSAR_OK) return rc;
  if (C < 1) return PULSAR_ERR_INVALID_ARGUMENT;
  Plan q;
  rc = make_plan(sc, C, params, &q);
  if (rc != PULSAR_OK) return rc;
  if (q.n > 0 && (!pos || !radius || !payload)) return PULSAR_ERR_INVALID_ARGUMENT;
  if (!background || !image || !aux || !grad_image || !ws) return PULSAR_ERR_INVALID_ARGUMENT;
  if (grad_opacity && !opacity) return PULSAR_ERR_INVALID_ARGUMENT;
  const bool rebin = (params->flags & PULSAR_REBIN) != 0u;
  const bool paper_norm = (params->flags & PULSAR_GRAD_PAPER_NORM) != 0u;
  // without the forward's thresholds in the workspace only a rebin can help
  if (!rebin && (params->flags & PULSAR_NO_BWD_AUX) != 0u) return PULSAR_ERR_INVALID_ARGUMENT;
  if (ws_bytes < q.total) return PULSAR_ERR_WORKSPACE;
  if (rebin) {
    FwdArgs f;
    f.pos = pos;
    f.radius = radius;
    f.opacity = opacity;
    f.payload = payload;
    f.bg = background;
    f.n = int(q.n);
    f.C = C;
    f.K = params->K;
    f.image = nullptr;
    f.aux = nullptr;
    f.min_radius_px = params->min_radius_px;
    f.track = true;
    f.topk = false;
    f.stop_share = params->stop_share;
    f.d_cams = nullptr;
    f.gamma = params->gamma;
    f.eps = params->eps;
    f.ortho = (params->flags & PULSAR_ORTHO) != 0u;
    hipError_t e = launch_rebin(q, sc, f, static_cast<char*>(ws),
                                static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail_hip(e);
  }
  BwdArgs a;
  a.pos = pos;
  a.radius = radius;
  a.opacity = opacity;
  a.payload = payload;
  a.n = int(q.n);
  a.C = C;
  a.K = params->K;
  a.image = image;
  a.aux = aux;
  a.grad_image = grad_image;
  a.grad_pos = grad_pos;
  a.grad_radius = grad_radius;
  a.grad_opacity = grad_opacity;
  a.grad_payload = grad_payload;
  a.grad_bg = grad_background;
  a.grad_cam = grad_camera;
  a.paper_norm = paper_norm;
  a.min_radius_px = params->min_radius_px;
  a.eps2 = sc[0].bc.eps2;
  a.rebinned = rebin;
  hipError_t e = launch_backward(q, a, static_cast<char*>(ws), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail_hip(e);
  return PULSAR_OK;
}

int pulsar_bwd_batched(const pulsar_scene_t* scenes, int32_t B, const float* pos,
                       const float* radius, const float* opacity, const float* payload,
                       int32_t C, const float* background, const pulsar_params_t* params,
                       const float* image, const float* aux, const float* grad_image,
                       float* grad_pos, float* grad_radius, float* grad_opacity,
                       float* grad_payload, float* grad_background, void* ws,
                       size_t ws_bytes, void* stream) {
  return bwd_impl(scenes, B, pos, radius, opacity, payload, C, background, params, image, aux,
                  grad_image, grad_pos, grad_radius, grad_opacity, grad_payload, grad_background,
                  nullptr, ws, ws_bytes, stream);
}

int pulsar_bwd_camera_batched(const pulsar_scene_t* scenes, int32_t B, const float* pos,
                              const float* radius, const float* opacity, const float* payload,
                              int32_t C, const float* background, const pulsar_params_t* params,
                              const float* image, const float* aux, const float* grad_image,
                              float* grad_pos, float* grad_radius, float* grad_opacity,
                              float* grad_payload, float* grad_background, float* grad_camera,
                              void* ws, size_t ws_bytes, void* stream) {
  if (!grad_camera) return PULSAR_ERR_INVALID_ARGUMENT;
  // the focal and sensor-width terms follow the pinhole rays
  if (params && (params->flags & PULSAR_ORTHO) != 0u) return PULSAR_ERR_UNSUPPORTED;
  return bwd_impl(scenes, B, pos, radius, opacity, payload, C, background, params, image, aux,
                  grad_image, grad_pos, grad_radius, grad_opacity, grad_payload, grad_background,
                  grad_camera, ws, ws_bytes, stream);
}

static pulsar_scene_t single_scene(const pulsar_camera_t* cam, int32_t n) {
  pulsar_scene_t sc;
  std::memset(&sc, 0, sizeof(sc));
  sc.camera = *cam;
  sc.n = n;
  return sc;
}

int pulsar_fwd(const float* pos, const float* radius, const float* opacity,
               const float* payload, int32_t n, int32_t C, const float* background,
               const pulsar_camera_t* cam, const pulsar_params_t* params, float* image,
               float* aux, void* ws, size_t ws_bytes, void* stream) {
  if (!cam) return PULSAR_ERR_INVALID_ARGUMENT;
  const pulsar_scene_t sc = single_scene(cam, n);
  return pulsar_fwd_batched(&sc, 1, pos, radius, opacity, payload, C, background, params,
                            image, aux, ws, ws_bytes, stream);
}

int pulsar_bwd(const float* pos, const float* radius, const float* opacity,
               const float* payload, int32_t n, int32_t C, const float* background,
               const pulsar_camera_t* cam, const pulsar_params_t* params, const float* image,
               const float* aux, const float* grad_image, float* grad_pos, float* grad_radius,
               float* grad_opacity, float* grad_payload, float* grad_background, void* ws,
               size_t ws_bytes, void* stream) {
  if (!cam) return PULSAR_ERR_INVALID_ARGUMENT;
  const pulsar_scene_t sc = single_scene(cam, n);
  return pulsar_bwd_batched(&sc, 1, pos, radius, opacity, payload, C, background, params,
                            image, aux, grad_image, grad_pos, grad_radius, grad_opacity,
                            grad_payload, grad_background, ws, ws_bytes, stream);
}

int pulsar_bwd_camera(const float* pos, const float* radius, const float* opacity,
                      const float* payload, int32_t n, int32_t C, const float* background,
                      const pulsar_camera_t* cam, const pulsar_params_t* params,
                      const float* image, const float* aux, const float* grad_image,
                      float* grad_pos, float* grad_radius, float* grad_opacity,
                      float* grad_payload, float* grad_background, float* grad_camera, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!cam) return PULSAR_ERR_INVALID_ARGUMENT;
  const pulsar_scene_t sc = single_scene(cam, n);
  return pulsar_bwd_camera_batched(&sc, 1, pos, radius, opacity, payload, C, background, params,
                                   image, aux, grad_image, grad_pos, grad_radius, grad_opacity,
                                   grad_payload, grad_background, grad_camera, ws, ws_bytes,
                                   stream);
}

int pulsar_query_status(const void* ws, size_t ws_bytes, void* stream, int64_t* pairs) {
  if (!ws || ws_bytes < sizeof(Status)) return PULSAR_ERR_INVALID_ARGUMENT;
  Status st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(&st, ws, sizeof(Status), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return fail_hip(e);
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail_hip(e);
  if (pairs) *pairs = int64_t(st.pairs);
  // the device writes the negated code: capacity, or an invalid device camera
  return st.code == 0u ? PULSAR_OK : -int(st.code);
}

const char* pulsar_status_string(int code) {
  switch (code) {
    case PULSAR_OK:
      return "success";
    case PULSAR_ERR_INVALID_ARGUMENT:
      return "invalid argument: a required pointer is NULL or a size or parameter is out of range";
    case PULSAR_ERR_WORKSPACE:
      return "workspace too small: allocate pulsar_workspace_size() bytes";
    case PULSAR_ERR_UNSUPPORTED:
      return "unsupported flag or size in this build";
    case PULSAR_ERR_HIP:
      return "HIP launch or runtime error (see pulsar_last_hip_error)";
    case PULSAR_ERR_CAPACITY:
      return "tile-pair capacity exceeded: raise params.max_pairs and render again";
    case PULSAR_ERR_SCRATCH:
      return "the call needs more than the static scratch buffer of pulsar_fwd_noalloc holds: "
             "use pulsar_fwd with a workspace";
    default:
      return "unknown status code";
  }
}

const char* pulsar_last_hip_error(void) { return g_last_hip_error.c_str(); }

int pulsar_timing_enable(int on) { return g_timing.exchange(on ? 1 : 0); }

int pulsar_timing_read(double* total_ms, int64_t* counts) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  int rc = PULSAR_OK;
  for (const Mark& m : g_marks) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(m.end);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.begin, m.end);
    if (e != hipSuccess) {
      rc = fail_hip(e);
    } else {
      if (total_ms) total_ms[m.stage] += double(ms);
      if (counts) counts[m.stage] += 1;
    }
    (void)hipEventDestroy(m.begin);
    (void)hipEventDestroy(m.end);
  }
  g_marks.clear();
  return rc;
}

const char* pulsar_stage_name(int stage) {
  static const char* names[PULSAR_NUM_STAGES] = {"project",    "binning",  "raster_fwd",
                                                 "zero",       "raster_bwd", "finalize",
                                                 "merge",      "raster_bwd_tiles"};
  return (stage >= 0 && stage < PULSAR_NUM_STAGES) ? names[stage] : "unknown";
}

int pulsar_version(void) { return 3; }

}  // extern "C"
