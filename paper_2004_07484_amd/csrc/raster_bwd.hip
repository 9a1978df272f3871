// K7/K8: backward pass (paper App. B, "The Backward Pass").
//
// K7, one wave64 per 8x8 tile, reuses the forward's sorted tile lists and
// recomputes each pixel's K nearest hits (ascending (t, sphere index)) into a
// register list instead of reading stored per-pixel hit lists. The walk stops
// as soon as the next sphere's depth lower bound exceeds the K-th distance of
// every lane. For each list entry it evaluates the derivatives of Eq. 1 and
// accumulates per sphere, in camera space, dL/dc (3), dL/dR, plus dL/do and
// dL/df straight into the caller's buffers, with float atomics (many pixels
// of one tile and of neighbouring tiles update the same sphere).
// The background gradient is reduced per tile into a partial buffer.
//
// K8 turns the camera-space accumulators into world-space position and
// radius gradients; K8b sums the per-tile background partials.
#include "device_common.h"
#include "pulsar_internal.h"

namespace pulsar {

__global__ void k_zero(float* __restrict__ p, size_t count) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0.f;
}

template <int KM>
__global__ __launch_bounds__(kWave) void k_raster_bwd(
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ skeys,
    const uint32_t* __restrict__ svals, const float4* __restrict__ recA,
    const float4* __restrict__ recB, const float* __restrict__ opacity,
    const float* __restrict__ payload, int C, int K, int depth_bits, float depth_step,
    CamDev cam, BlendConst bc, const float* __restrict__ image, const float* __restrict__ aux,
    const float* __restrict__ grad_image, float* __restrict__ gacc,
    float* __restrict__ grad_opacity, float* __restrict__ grad_payload,
    float* __restrict__ bgpart) {
  const int tile = blockIdx.x;
  const int lane = threadIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int px = tx * kTileW + (lane % kTileW);
  const int py = ty * kTileH + (lane / kTileW);
  const bool inside = px < cam.W && py < cam.H;
  const size_t p = inside ? size_t(py) * size_t(cam.W) + size_t(px) : 0;
  const float xs = (float(px) + 0.5f) * cam.pitch - 0.5f * cam.s;
  const float ys = (float(py) + 0.5f) * cam.pitch - 0.5f * cam.sh;
  const float v2 = xs * xs + ys * ys + cam.f * cam.f;
  const float inv_v2 = 1.f / v2;
  const float inv_len = 1.f / sqrtf(v2);
  const float ux = xs * inv_len, uy = ys * inv_len, uz = cam.f * inv_len;
  const float L2 = inside ? aux[p] * 1.4426950408889634f : 0.f;

  // Background: dL/dbg = sum_p exp(eps/gamma - L_p) G_p, one partial per tile.
  if (bgpart) {
    const float wbg = inside ? fast_exp2(bc.eps2 - L2) : 0.f;
    for (int c = 0; c < C; ++c) {
      const float g = inside ? grad_image[p * size_t(C) + c] : 0.f;
      const float s = wave_sum(wbg * g);
      if (lane == 0) bgpart[size_t(tile) * size_t(C) + c] = s;
    }
  }

  // K nearest hits. The list lives in the last K of KM slots, ascending; the
  // unused leading slots hold -inf and never move, so the K-th distance is
  // always kt[KM - 1].
  float kt[KM];
  uint32_t kid[KM];
#pragma unroll
  for (int i = 0; i < KM; ++i) {
    kt[i] = i < KM - K ? -INFINITY : INFINITY;
    kid[i] = 0xffffffffu;
  }
  const uint32_t beg = ranges[tile], end = ranges[tile + 1];
  const uint32_t qmask = (1u << depth_bits) - 1u;
  bool done = false;
  for (uint32_t base = beg; base < end && !done; base += kWave) {
    const uint32_t j = base + uint32_t(lane);
    const bool valid = j < end;
    const uint32_t id = valid ? svals[j] : 0u;
    const float lbv = valid ? cam.znear + float(skeys[j] & qmask) * depth_step : INFINITY;
    const float4 a = valid ? recA[id] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 b = valid ? recB[id] : make_float4(0.f, 0.f, 1.f, 1.f);
    const int cnt = int(min(uint32_t(kWave), end - base));
    for (int k = 0; k < cnt; ++k) {
      // every lane already holds K hits nearer than anything left in the list
      if (__all(!inside || kt[KM - 1] < rl(lbv, k))) {
        done = true;
        break;
      }
      const uint32_t pk = rlu(__float_as_uint(a.w), k);
      const float dx = float(px - int(pk & 0xffffu)) - rl(a.x, k);
      const float dy = float(py - int(pk >> 16)) - rl(a.y, k);
      const float axf = rl(b.x, k), ayf = rl(b.y, k);
      const float cr = axf * dy - ayf * dx;
      const float S = dx * dx + dy * dy + cr * cr;
      const float r2 = rl(a.z, k) * S * inv_v2;
      if (r2 < 1.f) {
        const float cz = rl(b.z, k), R = rl(b.w, k);
        float t = cz * (ux * axf + uy * ayf + uz) - R * fast_sqrt(1.f - r2);
        uint32_t idk = rlu(id, k);
        if (t <= bc.zfar && (t < kt[KM - 1] || (t == kt[KM - 1] && idk < kid[KM - 1]))) {
          // insertion: carry the new entry up the ascending list
#pragma unroll
          for (int i = 0; i < KM; ++i) {
            const bool lt = t < kt[i] || (t == kt[i] && idk < kid[i]);
            const float tt = kt[i];
            const uint32_t ti = kid[i];
            kt[i] = lt ? t : tt;
            kid[i] = lt ? idk : ti;
            t = lt ? tt : t;
            idk = lt ? ti : idk;
          }
        }
      }
    }
  }

  // Gradients of Eq. 1 for each of the K entries.
  const float* Gp = grad_image + p * size_t(C);
  const float* Fp = image + p * size_t(C);
#pragma unroll
  for (int i = 0; i < KM; ++i) {
    if (i < KM - K) continue;
    if (!(inside && kt[i] < INFINITY)) continue;
    const uint32_t id = kid[i];
    const float4 a = recA[id];
    const float4 b = recB[id];
    const float o = opacity ? opacity[id] : 1.f;
    const uint32_t pk = __float_as_uint(a.w);
    const float dx = float(px - int(pk & 0xffffu)) - a.x;
    const float dy = float(py - int(pk >> 16)) - a.y;
    const float axf = b.x, ayf = b.y, cz = b.z, R = b.w;
    const float cr = axf * dy - ayf * dx;
    const float S = dx * dx + dy * dy + cr * cr;
    // the list walk saw r2 < 1; keep it below 1 if this recomputation rounds differently
    const float r2 = fminf(a.z * S * inv_v2, 0.99999994f);
    const float sq = fast_sqrt(1.f - r2);  // sqrt(R^2 - q^2) / R
    const float ratio = fast_sqrt(r2);    // q / R
    const float t = cz * (ux * axf + uy * ayf + uz) - R * sq;
    const float s2 = o * (bc.zfar - t) * bc.kz;   // o z / gamma in base 2
    const float ex = fast_exp2(s2 - L2);          // exp(o z / gamma) / denominator
    const float e = (1.f - ratio) * ex;           // dw/do without the exponent term
    const float w = o * e;                        // blending weight of Eq. 1
    const float* fk = payload + size_t(id) * size_t(C);
    float h = 0.f;                                // G . (f_k - F)
    for (int c = 0; c < C; ++c) h += Gp[c] * (fk[c] - Fp[c]);
    if (grad_payload) {
      float* gf = grad_payload + size_t(id) * size_t(C);
      for (int c = 0; c < C; ++c) atomicAdd(gf + c, w * Gp[c]);
    }
    if (grad_opacity) {
      const float oz_g = o * (bc.zfar - t) * bc.inv_span * bc.inv_gamma;
      atomicAdd(grad_opacity + id, e * h * (1.f + oz_g));
    }
    if (gacc) {
      const float gt = -w * h * o * bc.inv_gamma * bc.inv_span;  // dL/dt
      const float gd = o * ex * h;                                // dL/d(1 - q/R)
      // d = c - (u.c) u = sqrt(kappa) (v x (-D_y, D_x, cr)) / |v|^2 * R
      const float sk = fast_sqrt(a.z) * inv_v2;
      const float dnx = (ys * cr - cam.f * dx) * sk;
      const float dny = (-cam.f * dy - xs * cr) * sk;
      const float dnz = (xs * dx + ys * dy) * sk;
      const float coef = gt / sq - (ratio > 0.f ? gd / (R * ratio) : 0.f);
      float* g = gacc + size_t(id) * 4;
      atomicAdd(g + 0, gt * ux + coef * dnx);
      atomicAdd(g + 1, gt * uy + coef * dny);
      atomicAdd(g + 2, gt * uz + coef * dnz);
      atomicAdd(g + 3, -gt / sq + gd * ratio / R);
    }
  }
}

// K8: camera-space (dL/dc, dL/dR) -> world-space position and radius gradients.
__global__ void k_finalize(int n, const float* __restrict__ pos, const float* __restrict__ radius,
                           CamDev cam, float min_radius_px, const float4* __restrict__ gacc,
                           float* __restrict__ grad_pos, float* __restrict__ grad_radius) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 g = gacc[i];
  float gx = g.x, gy = g.y, gz = g.z, gR = g.w;
  bool clamped = false;
  if (min_radius_px > 0.f) {
    const float px = pos[3 * i + 0], py = pos[3 * i + 1], pz = pos[3 * i + 2];
    const double cz = double(cam.R[6]) * px + double(cam.R[7]) * py + double(cam.R[8]) * pz +
                      double(cam.t[2]);
    const double pitch = double(cam.s) / double(cam.W);
    const double k = double(min_radius_px) * pitch / double(cam.f);
    clamped = k * cz > double(radius[i]);
    if (clamped) gz += float(double(gR) * k);  // R = k c_z depends on depth only
  }
  if (grad_radius) grad_radius[i] = clamped ? 0.f : gR;
  if (grad_pos) {
    // c = R p + t  =>  dL/dp = R^T dL/dc
    grad_pos[3 * i + 0] = cam.R[0] * gx + cam.R[3] * gy + cam.R[6] * gz;
    grad_pos[3 * i + 1] = cam.R[1] * gx + cam.R[4] * gy + cam.R[7] * gz;
    grad_pos[3 * i + 2] = cam.R[2] * gx + cam.R[5] * gy + cam.R[8] * gz;
  }
}

// K8b: grad_bg[c] = sum over tiles of the partials (one block per channel).
__global__ __launch_bounds__(256) void k_reduce_bg(const float* __restrict__ bgpart, int T, int C,
                                                   float* __restrict__ grad_bg) {
  __shared__ float s[256 / kWave];
  const int c = blockIdx.x;
  float acc = 0.f;
  for (int t = threadIdx.x; t < T; t += 256) acc += bgpart[size_t(t) * size_t(C) + c];
  acc = wave_sum(acc);
  if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float tsum = 0.f;
    for (int w = 0; w < 256 / kWave; ++w) tsum += s[w];
    grad_bg[c] = tsum;
  }
}

static void zero_async(float* p, size_t count, hipStream_t stream) {
  if (!p || count == 0) return;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_zero, dim3(unsigned(blocks)), dim3(256), 0, stream, p, count);
}

template <int KM>
static void launch_raster_bwd_km(const Plan& q, const CamDev& cam, const BlendConst& bc,
                                 const BwdArgs& a, char* ws, float* gacc, float* bgpart,
                                 hipStream_t stream) {
  const bool in_a = sorted_in_a(q);
  const float depth_step =
      float((double(cam.zfar) - double(cam.znear)) / double(1u << q.depth_bits));
  hipLaunchKernelGGL(k_raster_bwd<KM>, dim3(unsigned(q.T)), dim3(kWave), 0, stream,
                     ws_ptr<uint32_t>(ws, q.off_ranges),
                     ws_ptr<uint32_t>(ws, in_a ? q.off_keysA : q.off_keysB),
                     ws_ptr<uint32_t>(ws, in_a ? q.off_valsA : q.off_valsB),
                     ws_ptr<float4>(ws, q.off_recA), ws_ptr<float4>(ws, q.off_recB), a.opacity,
                     a.payload, a.C, a.K, q.depth_bits, depth_step, cam, bc, a.image, a.aux,
                     a.grad_image, gacc, a.grad_opacity, a.grad_payload, bgpart);
}

hipError_t launch_backward(const Plan& q, const CamDev& cam, const BlendConst& bc,
                           const BwdArgs& a, char* ws, hipStream_t stream) {
  const bool need_geo = a.grad_pos || a.grad_radius;
  float* gacc = need_geo ? ws_ptr<float>(ws, q.off_gacc) : nullptr;
  float* bgpart = a.grad_bg ? ws_ptr<float>(ws, q.off_bgpart) : nullptr;
  stage_begin(PULSAR_STAGE_ZERO, stream);
  zero_async(gacc, size_t(q.n) * 4, stream);
  zero_async(a.grad_opacity, size_t(q.n), stream);
  zero_async(a.grad_payload, size_t(q.n) * size_t(q.C), stream);
  stage_end(PULSAR_STAGE_ZERO, stream);
  stage_begin(PULSAR_STAGE_RASTER_BWD, stream);
  if (a.K <= 1)
    launch_raster_bwd_km<1>(q, cam, bc, a, ws, gacc, bgpart, stream);
  else if (a.K <= 2)
    launch_raster_bwd_km<2>(q, cam, bc, a, ws, gacc, bgpart, stream);
  else if (a.K <= 4)
    launch_raster_bwd_km<4>(q, cam, bc, a, ws, gacc, bgpart, stream);
  else if (a.K <= 8)
    launch_raster_bwd_km<8>(q, cam, bc, a, ws, gacc, bgpart, stream);
  else if (a.K <= 16)
    launch_raster_bwd_km<16>(q, cam, bc, a, ws, gacc, bgpart, stream);
  else
    launch_raster_bwd_km<32>(q, cam, bc, a, ws, gacc, bgpart, stream);
  stage_end(PULSAR_STAGE_RASTER_BWD, stream);
  stage_begin(PULSAR_STAGE_FINALIZE, stream);
  if (need_geo && q.n > 0)
    hipLaunchKernelGGL(k_finalize, dim3(unsigned((q.n + 255) / 256)), dim3(256), 0, stream,
                       int(q.n), a.pos, a.radius, cam, a.min_radius_px,
                       reinterpret_cast<const float4*>(gacc), a.grad_pos, a.grad_radius);
  if (a.grad_bg)
    hipLaunchKernelGGL(k_reduce_bg, dim3(unsigned(q.C)), dim3(256), 0, stream, bgpart,
                       int(q.T), int(q.C), a.grad_bg);
  stage_end(PULSAR_STAGE_FINALIZE, stream);
  return hipGetLastError();
}

}  // namespace pulsar
