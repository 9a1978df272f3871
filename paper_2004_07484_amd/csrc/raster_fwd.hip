// K6: per-tile forward raster (paper App. B, Steps 1-2; Eq. 1).
//
// One wave64 per 8x8 tile, one lane per pixel, so no two lanes ever write the
// same pixel. The wave walks its tile's depth-sorted sphere list in batches of
// 64: each lane gathers one sphere record (coalesced list read, 32-byte record
// gather), then the batch is broadcast record by record with v_readlane into
// scalar registers and every lane tests its own pixel ray.
//
// Hit test without cancellation: with D = pixel - projected centre in pixel
// units, (a_x, a_y) = (c_x, c_y) / c_z and v = (x_s, y_s, f) the unnormalised
// ray,  q^2 / R^2 = kappa (D_x^2 + D_y^2 + (a_x D_y - a_y D_x)^2) / |v|^2,
// kappa = (c_z pitch / R)^2, which follows from |c x v| = c_z pitch |(-D_y, D_x,
// a_x D_y - a_y D_x)|. The front hit is t = c_z (u . (a_x, a_y, 1)) - R sqrt(1 - q^2/R^2).
//
// Blending keeps a running maximum m of the exponents (base 2) and rescales
// the denominator and the numerator when it grows, so exp never overflows
// down to gamma = 1e-5. Every hit enters the sum (all spheres colour the pixel).
#include "device_common.h"
#include "pulsar_internal.h"

namespace pulsar {

template <int CM>
__global__ __launch_bounds__(kWave) void k_raster_fwd(
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ svals,
    const float4* __restrict__ recA, const float4* __restrict__ recB,
    const float* __restrict__ opacity, const float* __restrict__ payload, int C, int c0, int cn,
    const float* __restrict__ bg, CamDev cam, BlendConst bc, float* __restrict__ image,
    float* __restrict__ aux) {
  const int tile = blockIdx.x;
  const int lane = threadIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int px = tx * kTileW + (lane % kTileW);
  const int py = ty * kTileH + (lane / kTileW);
  const float xs = (float(px) + 0.5f) * cam.pitch - 0.5f * cam.s;
  const float ys = (float(py) + 0.5f) * cam.pitch - 0.5f * cam.sh;
  const float v2 = xs * xs + ys * ys + cam.f * cam.f;
  const float inv_v2 = 1.f / v2;
  const float inv_len = 1.f / sqrtf(v2);
  const float ux = xs * inv_len, uy = ys * inv_len, uz = cam.f * inv_len;

  float m2 = bc.eps2;  // running max exponent; the background's to start
  float D = 1.f;       // background weight exp2(eps2 - m2)
  float N[CM];
#pragma unroll
  for (int c = 0; c < CM; ++c) N[c] = c < cn ? bg[c0 + c] : 0.f;

  const uint32_t beg = ranges[tile], end = ranges[tile + 1];
  for (uint32_t base = beg; base < end; base += kWave) {
    const uint32_t j = base + uint32_t(lane);
    const bool valid = j < end;
    const uint32_t id = valid ? svals[j] : 0u;
    const float4 a = valid ? recA[id] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 b = valid ? recB[id] : make_float4(0.f, 0.f, 1.f, 1.f);
    const float o = valid ? (opacity ? opacity[id] : 1.f) : 0.f;
    const int cnt = int(min(uint32_t(kWave), end - base));
    for (int k = 0; k < cnt; ++k) {
      const uint32_t pk = rlu(__float_as_uint(a.w), k);
      const float dx = float(px - int(pk & 0xffffu)) - rl(a.x, k);
      const float dy = float(py - int(pk >> 16)) - rl(a.y, k);
      const float axf = rl(b.x, k), ayf = rl(b.y, k);
      const float cr = axf * dy - ayf * dx;
      const float S = dx * dx + dy * dy + cr * cr;
      const float r2 = rl(a.z, k) * S * inv_v2;
      if (r2 < 1.f) {
        const float cz = rl(b.z, k), R = rl(b.w, k);
        const float t = cz * (ux * axf + uy * ayf + uz) - R * fast_sqrt(1.f - r2);
        if (t <= bc.zfar) {
          const float ok = rl(o, k);
          const float s2 = ok * (bc.zfar - t) * bc.kz;
          if (s2 > m2) {
            const float sc = fast_exp2(m2 - s2);
            D *= sc;
#pragma unroll
            for (int c = 0; c < CM; ++c) N[c] *= sc;
            m2 = s2;
          }
          const float wgt = ok * (1.f - fast_sqrt(r2)) * fast_exp2(s2 - m2);
          D += wgt;
          const float* fp = payload + size_t(rlu(id, k)) * size_t(C) + c0;
#pragma unroll
          for (int c = 0; c < CM; ++c)
            if (c < cn) N[c] += wgt * fp[c];
        }
      }
    }
  }
  if (px < cam.W && py < cam.H) {
    const size_t p = size_t(py) * size_t(cam.W) + size_t(px);
    const float invD = 1.f / D;
#pragma unroll
    for (int c = 0; c < CM; ++c)
      if (c < cn) image[p * size_t(C) + c0 + c] = N[c] * invD;
    if (aux && c0 == 0) aux[p] = (m2 + fast_log2(D)) * 0.69314718055994531f;
  }
}

void launch_project(const Plan& q, const CamDev& cam, const FwdArgs& a, char* ws,
                    hipStream_t stream);
void launch_binning(const Plan& q, char* ws, hipStream_t stream);

template <int CM>
static void launch_raster_fwd_cm(const Plan& q, const CamDev& cam, const BlendConst& bc,
                                 const FwdArgs& a, char* ws, int c0, int cn,
                                 hipStream_t stream) {
  const uint32_t* svals =
      ws_ptr<uint32_t>(ws, sorted_in_a(q) ? q.off_valsA : q.off_valsB);
  hipLaunchKernelGGL(k_raster_fwd<CM>, dim3(unsigned(q.T)), dim3(kWave), 0, stream,
                     ws_ptr<uint32_t>(ws, q.off_ranges), svals, ws_ptr<float4>(ws, q.off_recA),
                     ws_ptr<float4>(ws, q.off_recB), a.opacity, a.payload, a.C, c0, cn, a.bg,
                     cam, bc, a.image, a.aux);
}

hipError_t launch_forward(const Plan& q, const CamDev& cam, const BlendConst& bc,
                          const FwdArgs& a, char* ws, hipStream_t stream) {
  stage_begin(PULSAR_STAGE_PROJECT, stream);
  launch_project(q, cam, a, ws, stream);
  stage_end(PULSAR_STAGE_PROJECT, stream);
  stage_begin(PULSAR_STAGE_BINNING, stream);
  launch_binning(q, ws, stream);
  stage_end(PULSAR_STAGE_BINNING, stream);
  stage_begin(PULSAR_STAGE_RASTER_FWD, stream);
  for (int c0 = 0; c0 < a.C; c0 += kFwdChannels) {
    const int cn = a.C - c0 < kFwdChannels ? a.C - c0 : kFwdChannels;
    if (cn <= 1)
      launch_raster_fwd_cm<1>(q, cam, bc, a, ws, c0, cn, stream);
    else if (cn <= 2)
      launch_raster_fwd_cm<2>(q, cam, bc, a, ws, c0, cn, stream);
    else if (cn <= 4)
      launch_raster_fwd_cm<4>(q, cam, bc, a, ws, c0, cn, stream);
    else if (cn <= 8)
      launch_raster_fwd_cm<8>(q, cam, bc, a, ws, c0, cn, stream);
    else if (cn <= 16)
      launch_raster_fwd_cm<16>(q, cam, bc, a, ws, c0, cn, stream);
    else
      launch_raster_fwd_cm<32>(q, cam, bc, a, ws, c0, cn, stream);
  }
  stage_end(PULSAR_STAGE_RASTER_FWD, stream);
  return hipGetLastError();
}

}  // namespace pulsar
