// Ray-sphere geometry shared by the raster kernels.
//
// A pixel ray is v = (x_s, y_s, f) through the pixel centre on the sensor
// plane z = f. With D = pixel - projected sphere centre in pixel units and
// (a_x, a_y) = (c_x, c_y) / c_z, the squared normalised distance of the centre
// from the ray is
//     r2 = q^2 / R^2 = kappa (D_x^2 + D_y^2 + (a_x D_y - a_y D_x)^2) / |v|^2,
//     kappa = (c_z pitch / R)^2,
// because |c x v| = c_z pitch |(-D_y, D_x, a_x D_y - a_y D_x)| (no cancellation).
//
// Near the silhouette the image depends on e = 1 - r2 with a gain of up to
// o exp(o z / gamma), far beyond what FP32 rounding of r2 allows. So a cheap
// FP32 test only rejects clear misses, and every candidate is decided and
// measured in FP64 from double-float records (hi + lo FP32 pairs), after which
// d = 1 - q/R = e / (1 + sqrt(1 - e)) keeps full relative accuracy.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_common.h"
#include "pulsar_internal.h"

namespace pulsar {

// FP32 rejection threshold on r2: generous against FP32 rounding of the
// record's high parts, so no hit of the exact test is ever rejected.
constexpr float kRejectR2 = 1.015625f;
// Below this FP32 r2 the pixel is well inside the disc: e = 1 - r2 >= 0.1 is
// then known to about 1e-5 relative in FP32 and the FP64 evaluation is skipped.
constexpr float kFastR2 = 0.9f;

struct PixelRay {
  int px, py;
  float xs, ys;       // sensor-plane coordinates of the pixel centre
  float ux, uy, uz;   // unit ray
  float inv_v2;       // 1 / |v|^2
  double inv_v2_d;    // the same in FP64
};

__device__ __forceinline__ PixelRay make_ray(const CamDev& cam, int px, int py) {
#pragma clang fp contract(off)
  PixelRay r;
  r.px = px;
  r.py = py;
  // the orthographic ray leaves its pixel centre along +z: in the
  // sphere's pixel-space record the offset is already taken into account
  r.xs = cam.ortho ? 0.f : (float(px) + 0.5f) * cam.pitch - 0.5f * cam.s;
  r.ys = cam.ortho ? 0.f : (float(py) + 0.5f) * cam.pitch - 0.5f * cam.sh;
  const float v2 = r.xs * r.xs + r.ys * r.ys + cam.f * cam.f;
  r.inv_v2 = 1.f / v2;
  const float inv_len = 1.f / sqrtf(v2);
  r.ux = r.xs * inv_len;
  r.uy = r.ys * inv_len;
  r.uz = cam.f * inv_len;
  const double pitch = cam.dpitch;
  const double xs = cam.ortho ? 0.0 : (double(px) + 0.5) * pitch - 0.5 * double(cam.s);
  const double ys = cam.ortho ? 0.0 : (double(py) + 0.5) * pitch - cam.dhalf_sh;
  r.inv_v2_d = 1.0 / (xs * xs + ys * ys + double(cam.f) * double(cam.f));
  return r;
}

// One sphere record in registers (uniform across the wave when broadcast).
struct SphereRec {
  int x0, y0;           // first pixel of its rectangle
  float xh, yh, kh;     // high parts: centre offset from (x0, y0), kappa
  float axh, ayh;       // high parts of c_x / c_z, c_y / c_z
  float cz, R, o;
  float xl, yl, kl, axl, ayl;  // low parts
};

struct Hit {
  float e;      // 1 - q^2/R^2, accurate to FP64 rounding
  float delta;  // 1 - q/R
  float sq;     // sqrt(1 - q^2/R^2) = sqrt(R^2 - q^2) / R
  float ratio;  // q / R
  float t;      // distance to the front intersection
  float dx, dy, cr;  // D and the cross term (pixel units), for the gradient direction
};

// Exact test. Returns true on a hit (q < R and t <= zfar) and fills h (h is
// meaningless on a miss). Deterministic: every kernel gets bitwise the same
// result for the same (pixel, sphere), which the K-th-nearest threshold
// relies on. Written predicated: the FP32 path runs on every lane and only
// the rare rim candidates branch into FP64, so a caller's loop has no
// divergent join around it.
__device__ __forceinline__ bool exact_hit(const PixelRay& ray, const SphereRec& s, float zfar,
                                          Hit& h) {
#pragma clang fp contract(off)
  const float dx32 = float(ray.px - s.x0) - s.xh;
  const float dy32 = float(ray.py - s.y0) - s.yh;
  const float cr32 = s.axh * dy32 - s.ayh * dx32;
  const float r2c = s.kh * (dx32 * dx32 + dy32 * dy32 + cr32 * cr32) * ray.inv_v2;
  bool ok = r2c < kRejectR2;
  float e = 1.f - r2c, ratio = fast_sqrt(r2c);
  h.dx = dx32;
  h.dy = dy32;
  h.cr = cr32;
  if (ok && !(r2c < kFastR2)) {
    const double X = double(s.xh) + double(s.xl);
    const double Y = double(s.yh) + double(s.yl);
    const double dx = double(ray.px - s.x0) - X;
    const double dy = double(ray.py - s.y0) - Y;
    const double ax = double(s.axh) + double(s.axl);
    const double ay = double(s.ayh) + double(s.ayl);
    const double cr = ax * dy - ay * dx;
    const double S = dx * dx + dy * dy + cr * cr;
    const double r2 = (double(s.kh) + double(s.kl)) * S * ray.inv_v2_d;
    ok = r2 < 1.0;
    e = float(1.0 - r2);
    ratio = fast_sqrt(float(r2));
    h.dx = float(dx);
    h.dy = float(dy);
    h.cr = float(cr);
  }
  const float sq = fast_sqrt(e);
  const float t = s.cz * (ray.ux * s.axh + ray.uy * s.ayh + ray.uz) - s.R * sq;
  h.e = e;
  h.sq = sq;
  h.ratio = ratio;
  h.delta = e * fast_rcp(1.f + ratio);
  h.t = t;
  return ok && (t <= zfar);
}

// A lower bound on the distance t of any front hit of the sphere: every ray
// meets the sphere no closer than its nearest point, |c| - R (for a ray at
// distance q from the centre, t = sqrt(|c|^2 - q^2) - sqrt(R^2 - q^2) grows
// with q). Lowered by 1e-4 |c|, far beyond the FP32 rounding of both this
// bound and exact_hit's t, so it never exceeds a computed t.
__device__ __forceinline__ float front_bound(const SphereRec& s) {
  const float cn = s.cz * fast_sqrt(s.axh * s.axh + s.ayh * s.ayh + 1.f);
  return (cn - s.R) - 1e-4f * cn;
}

// The same ray as make_ray, from per-tile LDS copies of its fields.
struct TileRays {
  float xs[kWave], ys[kWave], ux[kWave], uy[kWave], uz[kWave], iv2[kWave];
  double iv2d[kWave];
};

__device__ __forceinline__ void store_ray(TileRays& tr, int pl, const PixelRay& r) {
  tr.xs[pl] = r.xs;
  tr.ys[pl] = r.ys;
  tr.ux[pl] = r.ux;
  tr.uy[pl] = r.uy;
  tr.uz[pl] = r.uz;
  tr.iv2[pl] = r.inv_v2;
  tr.iv2d[pl] = r.inv_v2_d;
}

__device__ __forceinline__ PixelRay load_ray(const TileRays& tr, int pl, int px, int py) {
  PixelRay r;
  r.px = px;
  r.py = py;
  r.xs = tr.xs[pl];
  r.ys = tr.ys[pl];
  r.ux = tr.ux[pl];
  r.uy = tr.uy[pl];
  r.uz = tr.uz[pl];
  r.inv_v2 = tr.iv2[pl];
  r.inv_v2_d = tr.iv2d[pl];
  return r;
}

// The scene of a (global) tile, its camera and the tile's first pixel.
struct TileScene {
  int b;
  int tx0, ty0;
};

// The same from the scene arrays passed as restrict kernel parameters: the
// compiler then knows no store of the kernel can change them and reads them
// through the scalar cache, off the vector memory queue.
__device__ __forceinline__ TileScene tile_scene(const SceneDev* __restrict__ scenes,
                                                const uint32_t* __restrict__ tile_start, int B,
                                                uint32_t tile) {
  TileScene ts;
  ts.b = find_scene(tile_start, B, tile);
  const int lt = int(tile - scenes[ts.b].tile_off);
  const int tiles_x = scenes[ts.b].cam.tiles_x;
  ts.tx0 = (lt % tiles_x) * kTileW;
  ts.ty0 = (lt / tiles_x) * kTileH;
  return ts;
}

__device__ __forceinline__ TileScene tile_scene(const SceneTable& tab, uint32_t tile) {
  TileScene ts;
  ts.b = find_scene(tab.tile_start, tab.B, tile);
  const int lt = int(tile - tab.scenes[ts.b].tile_off);
  const int tiles_x = tab.scenes[ts.b].cam.tiles_x;
  ts.tx0 = (lt % tiles_x) * kTileW;
  ts.ty0 = (lt / tiles_x) * kTileH;
  return ts;
}

// Emission position of the pair (sphere, tile (tx, ty)), tile coordinates
// inside the sphere's scene: the sphere's first pair (its projection block's
// offset boff plus the in-block prefix in record word 3.w) plus the row-major
// index of the tile in the sphere's tile rectangle (derived from the pixel
// rectangle in words 0.w and 3.z). Unique per pair and ordered like the
// sphere index across spheres, so it serves as the K-nearest tie-break; it is
// also the pair's gradient slot. Integer arithmetic, identical everywhere.
__device__ __forceinline__ uint32_t pair_position(const float4& r0, const float4& r3,
                                                  uint32_t boff, int tx, int ty) {
  const uint32_t p0 = __float_as_uint(r0.w), p1 = __float_as_uint(r3.z);
  const int tx0 = int(p0 & 0xffffu) / kTileW, ty0 = int(p0 >> 16) / kTileH;
  const int tw = int(p1 & 0xffffu) / kTileW - tx0 + 1;
  return boff + __float_as_uint(r3.w) + uint32_t((ty - ty0) * tw + (tx - tx0));
}

// A sphere record is four float4 (see k_project for the layout).
__device__ __forceinline__ SphereRec unpack_rec(const float4& a, const float4& b,
                                                const float4& c, const float4& d) {
  SphereRec s;
  const uint32_t pk = __float_as_uint(a.w);
  s.x0 = int(pk & 0xffffu);
  s.y0 = int(pk >> 16);
  s.xh = a.x;
  s.yh = a.y;
  s.kh = a.z;
  s.axh = b.x;
  s.ayh = b.y;
  s.cz = b.z;
  s.R = b.w;
  s.xl = c.x;
  s.yl = c.y;
  s.kl = c.z;
  s.axl = c.w;
  s.ayl = d.x;
  s.o = d.y;
  return s;
}


}  // namespace pulsar
