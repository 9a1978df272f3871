// K1: per-sphere projection and culling (paper App. B, Step 0).
//
// One lane per sphere. The camera transform and the projected bounds run in
// FP64 (the kernel is memory bound, FP64 costs nothing here and keeps the
// screen-space record exact enough for sub-pixel spheres). Outputs per sphere:
//   counts  number of 8x8 tiles its pixel rectangle touches (0 = culled)
//   trect   tile rectangle (tx0, ty0, tx1, ty1)
//   rec     four float4 per sphere, one 64-byte line:
//     [0]   (X_c - x0, Y_c - y0, kappa, x0 | y0 << 16): projected centre in
//           pixel units relative to the first pixel of its rectangle, and
//           kappa = (c_z pitch / R)^2 (high FP32 parts)
//     [1]   (c_x / c_z, c_y / c_z, c_z, R) (ratios as high parts)
//     [2]   low parts of X_c - x0, Y_c - y0, kappa, c_x / c_z
//     [3]   (low part of c_y / c_z, opacity, x1 | y1 << 16, first): x1, y1 is
//           the last pixel of its rectangle; first is the sum of the tile
//           counts of the spheres before it in its projection block, so its
//           first tile pair sits at (block offset + first) in emission order
//     [4-7] for payloads of at most 16 channels: the payload row, so that the
//           raster kernels' gather of a pair reads one 128-byte line
// and the per-block sum of counts for the tile-pair scan. High + low FP32
// parts carry the FP64 values to about 48 bits for the exact hit test.
#include <cstring>

#include "device_common.h"
#include "pulsar_internal.h"

namespace pulsar {

// Copies up to kUploadScenes scene descriptors from the launch arguments into
// the workspace table and its start arrays; the launch covering the last
// scene also writes the B-th (total) entry of each start array.
struct SceneUpload {
  int first, count, B;
  uint32_t total_spheres, total_tiles, total_blocks;
  SceneDev s[kUploadScenes];
};

__global__ __launch_bounds__(64) void k_upload_scenes(SceneUpload u, SceneDev* __restrict__ scenes,
                                                      uint32_t* __restrict__ starts,
                                                      Status* __restrict__ status) {
  const int k = threadIdx.x;
  const int B1 = u.B + 1;
  if (u.first == 0 && k == 0) status->bad_cam = 0u;
  if (k < u.count) {
    const int b = u.first + k;
    scenes[b] = u.s[k];
    starts[b] = u.s[k].sph_off;
    starts[B1 + b] = u.s[k].tile_off;
    starts[2 * B1 + b] = u.s[k].bgblk_off;
  }
  if (k == 0 && u.first + u.count == u.B) {
    starts[u.B] = u.total_spheres;
    starts[B1 + u.B] = u.total_tiles;
    starts[2 * B1 + u.B] = u.total_blocks;
  }
}

// Fills a SceneUpload with scenes first .. first + count - 1 of the table.
static SceneUpload make_upload(const Plan& q, const std::vector<SceneDev>& sc, int first) {
  SceneUpload u;
  std::memset(&u, 0, sizeof(u));
  u.first = first;
  u.count = q.B - first < kUploadScenes ? q.B - first : kUploadScenes;
  u.B = q.B;
  u.total_spheres = uint32_t(q.n);
  u.total_tiles = uint32_t(q.T);
  u.total_blocks = uint32_t(q.nbgblk);
  for (int k = 0; k < u.count; ++k) u.s[k] = sc[size_t(first + k)];
  return u;
}

void launch_upload_scenes(const Plan& q, const std::vector<SceneDev>& sc, char* ws,
                          hipStream_t stream) {
  SceneDev* scenes = ws_ptr<SceneDev>(ws, q.off_scenes);
  uint32_t* starts = ws_ptr<uint32_t>(ws, q.off_starts);
  for (int first = 0; first < q.B; first += kUploadScenes) {
    const SceneUpload u = make_upload(q, sc, first);
    hipLaunchKernelGGL(k_upload_scenes, dim3(1), dim3(64), 0, stream, u, scenes, starts,
                       ws_ptr<Status>(ws, q.off_status));
  }
}

// Cameras from device memory: scene b's camera and blend constants are
// rebuilt from d_cams[b] when the work runs, with the expressions the host
// uses (IEEE double, no contraction), so the table equals what the host would
// have uploaded for the same cameras. Image sizes, and with them the
// workspace plan, stay those of the host's scene array. An invalid camera
// (the checks pulsar_fwd makes on the host) is reported through the status;
// the call's outputs are then undefined, but every access stays in bounds
// (rectangles are clamped to the host's image sizes).
__global__ __launch_bounds__(256) void k_device_cameras(const pulsar_camera_t* __restrict__ d_cams,
                                                        int B, float gamma, float eps, int ortho,
                                                        SceneDev* __restrict__ scenes,
                                                        Status* __restrict__ status) {
#pragma clang fp contract(off)
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const pulsar_camera_t c = d_cams[b];
  bool ok = isfinite(c.focal) && c.focal > 0.f && isfinite(c.sensor_width) &&
            c.sensor_width > 0.f && isfinite(c.znear) && c.znear > 0.f && isfinite(c.zfar) &&
            c.zfar > c.znear;
  for (int i = 0; i < 9; ++i) ok = ok && isfinite(c.R[i]);
  for (int i = 0; i < 3; ++i) ok = ok && isfinite(c.t[i]);
  if (!ok) atomicOr(&status->bad_cam, 1u);
  SceneDev& sc = scenes[b];
  CamDev d = sc.cam;  // width, height and tile counts of the plan
  for (int i = 0; i < 9; ++i) d.R[i] = c.R[i];
  for (int i = 0; i < 3; ++i) d.t[i] = c.t[i];
  d.f = ortho ? 1.f : c.focal;
  d.s = c.sensor_width;
  d.znear = c.znear;
  d.zfar = c.zfar;
  const double W = double(d.W), H = double(d.H), s = double(c.sensor_width);
  d.pitch = float(s / W);
  d.sh = float(s * H / W);
  d.dpitch = s / W;
  d.dinv_pitch = W / s;
  d.dsh = s * H / W;
  d.dhalf_sh = 0.5 * s * H / W;
  d.ortho = ortho;
  sc.cam = d;
  const double log2e = 1.4426950408889634;
  const double span = double(c.zfar) - double(c.znear);
  BlendConst bc;
  bc.kz = float(log2e / (double(gamma) * span));
  bc.eps2 = float(double(eps) / double(gamma) * log2e);
  bc.zfar = c.zfar;
  bc.inv_gamma = float(1.0 / double(gamma));
  bc.inv_span = float(1.0 / span);
  sc.bc = bc;
}

// When the whole scene table fits in the launch arguments (`inline_scenes`),
// the projection reads its cameras from there and its first block also
// writes the workspace copy the later kernels use; otherwise the table was
// uploaded before and is read from the workspace.
__global__ __launch_bounds__(kProjectBlock) void k_project(
    int n, const float* __restrict__ pos, const float* __restrict__ radius,
    const float* __restrict__ opacity, SceneTable tab, SceneUpload u, int inline_scenes,
    SceneDev* __restrict__ tab_out, uint32_t* __restrict__ starts_out, float min_radius_px,
    uint32_t* __restrict__ counts, ushort4* __restrict__ trect, float4* __restrict__ rec,
    unsigned long long* __restrict__ partials, float* __restrict__ tmin_out,
    Status* __restrict__ status, const float* __restrict__ payload, int C, int rec4) {
  // no FMA contraction: the camera transform, the minimum size and the
  // earliest hit distance are the IEEE double evaluations of the same
  // expressions, term by term (early termination orders spheres by the
  // float32 of that distance)
#pragma clang fp contract(off)
  const int i = blockIdx.x * kProjectBlock + threadIdx.x;
  // the emission that follows flags spheres wider than kBigTiles tiles
  if (blockIdx.x == 0 && threadIdx.x == 0) status->big_spheres = 0u;
  if (inline_scenes && blockIdx.x == 0 && threadIdx.x < kWave) {
    const int k = threadIdx.x;
    const int B1 = u.B + 1;
    if (k == 0) status->bad_cam = 0u;
    if (k < u.count) {
      tab_out[k] = u.s[k];
      starts_out[k] = u.s[k].sph_off;
      starts_out[B1 + k] = u.s[k].tile_off;
      starts_out[2 * B1 + k] = u.s[k].bgblk_off;
    }
    if (k == 0) {
      starts_out[u.B] = u.total_spheres;
      starts_out[B1 + u.B] = u.total_tiles;
      starts_out[2 * B1 + u.B] = u.total_blocks;
    }
  }
  uint32_t count = 0;
  float4 r0, r1, r2, r3;
  // the payload row that goes into the record is requested first, so its
  // latency overlaps the projection below (16-byte rows: float4 loads)
  float4 pv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) pv[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (rec4 == 8 && i < n) {
    const float* f = payload + size_t(i) * size_t(C);
    if ((C & 3) == 0 && (reinterpret_cast<uintptr_t>(payload) & 15u) == 0u) {
      const float4* f4 = reinterpret_cast<const float4*>(f);
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (4 * q < C) pv[q] = f4[q];
    } else {
      float v[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = c < C ? f[c] : 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        pv[q] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    }
  }
  if (i < n) {
    int b = 0;
    if (inline_scenes) {
      for (int k = 1; k < u.count; ++k)
        if (u.s[k].sph_off <= uint32_t(i)) b = k;
    } else {
      b = find_scene(tab.sph_start, tab.B, uint32_t(i));
    }
    const CamDev cam = inline_scenes ? u.s[b].cam : tab.scenes[b].cam;
    const float px = pos[3 * i + 0], py = pos[3 * i + 1], pz = pos[3 * i + 2];
    const float r = radius[i];
    const float o = opacity ? opacity[i] : 1.f;
    bool ok = isfinite(px) && isfinite(py) && isfinite(pz) && isfinite(r) && isfinite(o) &&
              r > 0.f;
    const double cx = double(cam.R[0]) * px + double(cam.R[1]) * py + double(cam.R[2]) * pz +
                      double(cam.t[0]);
    const double cy = double(cam.R[3]) * px + double(cam.R[4]) * py + double(cam.R[5]) * pz +
                      double(cam.t[1]);
    const double cz = double(cam.R[6]) * px + double(cam.R[7]) * py + double(cam.R[8]) * pz +
                      double(cam.t[2]);
    const double f = cam.f;
    const double pitch = cam.dpitch;
    const double inv_pitch = cam.dinv_pitch;
    const double sh = cam.dsh;
    const bool ortho = cam.ortho != 0;
    double R = r;
    if (min_radius_px > 0.f) {
      // the minimum size in pixels: at depth c_z (pinhole) or at any depth
      const double rmin = ortho ? double(min_radius_px) * pitch
                                : double(min_radius_px) * pitch * cz / f;
      if (rmin > R) R = rmin;
    }
    ok = ok && (cz - R >= double(cam.znear));
    // the nearest point any ray can reach
    const double tmin = ortho ? cz - R : sqrt(cx * cx + cy * cy + cz * cz) - R;
    ok = ok && (tmin <= double(cam.zfar));
    if (tmin_out) tmin_out[i] = ok ? float(tmin) : INFINITY;
    if (ok) {
      // The cone of rays through the sphere lies between the two planes through
      // the camera centre tangent to it; on the plane z = f they bound
      // x in f (c_x c_z -+ R sqrt(c_x^2 + c_z^2 - R^2)) / (c_z^2 - R^2), same for y.
      // (orthographic: the sphere's shadow on the sensor is the disk of
      // radius R around (c_x, c_y))
      const double fden = f / (cz * cz - R * R);
      const double sx = R * sqrt(cx * cx + cz * cz - R * R);
      const double sy = R * sqrt(cy * cy + cz * cz - R * R);
      const double xlo = ortho ? cx - R : (cx * cz - sx) * fden;
      const double xhi = ortho ? cx + R : (cx * cz + sx) * fden;
      const double ylo = ortho ? cy - R : (cy * cz - sy) * fden;
      const double yhi = ortho ? cy + R : (cy * cz + sy) * fden;
      // pixel j has its centre at sensor x (j + 1/2) pitch - s/2; widen by a
      // small margin so rounding never drops a pixel the exact cone covers
      const double margin = 1e-3;
      double jlo = ceil((xlo + 0.5 * double(cam.s)) * inv_pitch - 0.5 - margin);
      double jhi = floor((xhi + 0.5 * double(cam.s)) * inv_pitch - 0.5 + margin);
      double ilo = ceil((ylo + 0.5 * sh) * inv_pitch - 0.5 - margin);
      double ihi = floor((yhi + 0.5 * sh) * inv_pitch - 0.5 + margin);
      jlo = fmax(jlo, 0.0);
      ilo = fmax(ilo, 0.0);
      jhi = fmin(jhi, double(cam.W - 1));
      ihi = fmin(ihi, double(cam.H - 1));
      if (jlo <= jhi && ilo <= ihi) {
        const int j0 = int(jlo), j1 = int(jhi), i0 = int(ilo), i1 = int(ihi);
        const int tx0 = j0 / kTileW, tx1 = j1 / kTileW, ty0 = i0 / kTileH, ty1 = i1 / kTileH;
        count = uint32_t(tx1 - tx0 + 1) * uint32_t(ty1 - ty0 + 1);
        trect[i] = make_ushort4(uint16_t(tx0), uint16_t(ty0), uint16_t(tx1), uint16_t(ty1));
        // the centre's pixel position and the pixel-space scale of the hit
        // test: q^2 / R^2 = kap (D_x^2 + D_y^2 + cross^2) / |v|^2 with the
        // pinhole ray direction v; orthographic rays have v = e_z and no
        // cross term, so q^2 / R^2 = (pitch / R)^2 (D_x^2 + D_y^2)
        const double inv_cz = 1.0 / cz;
        const double ax = ortho ? 0.0 : cx * inv_cz, ay = ortho ? 0.0 : cy * inv_cz;
        const double Xc = ((ortho ? cx : f * ax) + 0.5 * double(cam.s)) * inv_pitch - 0.5;
        const double Yc = ((ortho ? cy : f * ay) + 0.5 * sh) * inv_pitch - 0.5;
        const double kr = (ortho ? 1.0 : cz) * pitch / R;
        const double X = Xc - j0, Y = Yc - i0, kap = kr * kr;
        const float Xh = float(X), Yh = float(Y), kh = float(kap), axh = float(ax),
                    ayh = float(ay);
        const uint32_t packed = uint32_t(j0) | (uint32_t(i0) << 16);
        r0 = make_float4(Xh, Yh, kh, __uint_as_float(packed));
        r1 = make_float4(axh, ayh, float(cz), float(R));
        r2 = make_float4(float(X - Xh), float(Y - Yh), float(kap - kh), float(ax - axh));
        const uint32_t packed_end = uint32_t(j1) | (uint32_t(i1) << 16);
        r3 = make_float4(float(ay - ayh), o, __uint_as_float(packed_end), 0.f);
      }
    }
    counts[i] = count;
  }
  // exclusive prefix of tile counts inside the block, and the block sum
  __shared__ unsigned long long s_sum[kProjectBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  const unsigned long long incl = wave_incl_scan_u64(count, lane);
  if (lane == kWave - 1) s_sum[wid] = incl;
  __syncthreads();
  unsigned long long before = 0, total = 0;
#pragma unroll
  for (int k = 0; k < kProjectBlock / kWave; ++k) {
    if (k < wid) before += s_sum[k];
    total += s_sum[k];
  }
  if (count != 0) {
    // a prefix beyond 32 bits only belongs to pairs past any capacity
    const unsigned long long first = before + incl - count;
    r3.w = __uint_as_float(first < 0xffffffffull ? uint32_t(first) : 0xffffffffu);
    float4* r4 = rec + size_t(rec4) * size_t(i);
    r4[0] = r0;
    r4[1] = r1;
    r4[2] = r2;
    r4[3] = r3;
    if (rec4 == 8) {
      // the payload row after the geometry (unused channels zero)
#pragma unroll
      for (int q = 0; q < 4; ++q) r4[4 + q] = pv[q];
    }
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

// Uploads the scene table (unless the projection carries it) and projects.
// The projection runs even with no sphere (it then only writes the scene table).
void launch_project(const Plan& q, const std::vector<SceneDev>& sc, const FwdArgs& a, char* ws,
                    hipStream_t stream) {
  // device cameras replace those of the uploaded table, so the projection
  // reads the table from the workspace
  const bool inline_scenes = q.B <= kUploadScenes && !a.d_cams;
  if (!inline_scenes) launch_upload_scenes(q, sc, ws, stream);
  if (a.d_cams)
    hipLaunchKernelGGL(k_device_cameras, dim3(unsigned((q.B + 255) / 256)), dim3(256), 0, stream,
                       a.d_cams, q.B, a.gamma, a.eps, a.ortho ? 1 : 0,
                       ws_ptr<SceneDev>(ws, q.off_scenes), ws_ptr<Status>(ws, q.off_status));
  const SceneUpload u = make_upload(q, sc, 0);
  hipLaunchKernelGGL(k_project, dim3(q.nblk_proj > 0 ? q.nblk_proj : 1), dim3(kProjectBlock), 0,
                     stream, int(q.n), a.pos, a.radius, a.opacity, scene_table(q, ws), u,
                     inline_scenes ? 1 : 0, ws_ptr<SceneDev>(ws, q.off_scenes),
                     ws_ptr<uint32_t>(ws, q.off_starts), a.min_radius_px,
                     ws_ptr<uint32_t>(ws, q.off_counts), ws_ptr<ushort4>(ws, q.off_trect),
                     ws_ptr<float4>(ws, q.off_rec),
                     ws_ptr<unsigned long long>(ws, q.off_partials),
                     q.estop ? ws_ptr<float>(ws, q.off_tmin) : nullptr,
                     ws_ptr<Status>(ws, q.off_status), a.payload, a.C, q.rec4);
}

}  // namespace pulsar
