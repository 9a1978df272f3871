// K7/K8: backward pass (paper App. B, "The Backward Pass").
//
// The forward left, per pixel, the K-th nearest hit (t_K, sphere index) and
// the log-normaliser L. A hit (t, k) of pixel p receives gradients iff it is
// among the K nearest, i.e. k is the K-th one or (t, k) < (t_K, k_K); nothing
// else per pixel is stored, every intersection is recomputed here.
//
// K7 runs over the same chunks as the forward with the roles turned around:
// lane l owns record l and walks the pixels of its rectangle inside the tile,
// so each lane accumulates its own sphere's derivatives of Eq. 1 in registers
// (camera-space dL/dc, dL/dR, dL/do, dL/df) and flushes them once per chunk
// with float atomics (a sphere meets several chunks only when its rectangle
// spans tiles or its tile list is split). The tile's G, F, L, thresholds and
// rays are staged once per chunk in LDS. The first chunk of each tile also
// writes the tile's background-gradient partial.
//
// K8 turns the camera-space accumulators into world-space position and
// radius gradients; K8b sums the per-tile background partials.
#include "hit_geometry.h"

namespace pulsar {

__global__ void k_zero(float* __restrict__ p, size_t count) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += size_t(gridDim.x) * blockDim.x)
    p[i] = 0.f;
}

struct BwdKernelArgs {
  const Status* status;
  const uint2* desc;
  const uint32_t* ranges;
  const uint32_t* svals;
  const float4* recA;
  const float4* recB;
  const float4* recC;
  const float4* recD;
  const float* payload;
  const float* image;
  const float* aux;
  const float* grad_image;
  const float2* thr;
  float* gacc;
  float* grad_opacity;
  float* grad_payload;
  float* bgpart;
  int C;
};

// CM >= C: channels kept in LDS and registers.
template <int CM>
__global__ __launch_bounds__(kWave) void k_bwd_chunks(BwdKernelArgs A, CamDev cam,
                                                      BlendConst bc) {
  __shared__ TileRays s_ray;
  __shared__ float s_G[CM][kWave], s_F[CM][kWave];
  __shared__ float s_L2[kWave], s_tk[kWave];
  __shared__ uint32_t s_ik[kWave];
  const int lane = threadIdx.x;
  const int C = A.C;
  const uint32_t nchunks = A.status->nchunks;
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const uint2 dsc = A.desc[chunk];
    const int tile = int(dsc.x), ci = int(dsc.y);
    const uint32_t beg = A.ranges[tile] + uint32_t(ci) * kChunk;
    const uint32_t end = min(A.ranges[tile + 1], beg + kChunk);
    const int tx0 = (tile % cam.tiles_x) * kTileW, ty0 = (tile / cam.tiles_x) * kTileH;
    if (beg >= end && !(ci == 0 && A.bgpart)) continue;  // empty tile, nothing to do
    // stage the tile's pixels (lane = pixel)
    const int px = tx0 + (lane % kTileW), py = ty0 + (lane / kTileW);
    const bool inside = px < cam.W && py < cam.H;
    const size_t p = inside ? size_t(py) * size_t(cam.W) + size_t(px) : 0;
    const float L2 = inside ? A.aux[p] * 1.4426950408889634f : 0.f;
    __syncthreads();  // the previous chunk's LDS reads are done
    store_ray(s_ray, lane, make_ray(cam, px, py));
    s_L2[lane] = L2;
    const float2 th = inside ? A.thr[p] : make_float2(-INFINITY, 0.f);
    s_tk[lane] = th.x;
    s_ik[lane] = __float_as_uint(th.y);
#pragma unroll
    for (int c = 0; c < CM; ++c) {
      s_G[c][lane] = (inside && c < C) ? A.grad_image[p * size_t(C) + c] : 0.f;
      s_F[c][lane] = (inside && c < C) ? A.image[p * size_t(C) + c] : 0.f;
    }
    if (ci == 0 && A.bgpart) {
      // dL/dbg = sum_p exp(eps/gamma - L_p) G_p
      const float wbg = inside ? fast_exp2(bc.eps2 - L2) : 0.f;
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        if (c < C) {
          const float sum = wave_sum(wbg * s_G[c][lane]);
          if (lane == 0) A.bgpart[size_t(tile) * size_t(C) + c] = sum;
        }
      }
    }
    __syncthreads();
    for (uint32_t b0 = beg; b0 < end; b0 += kWave) {
      const uint32_t j = b0 + uint32_t(lane);
      if (j >= end) continue;
      const uint32_t id = A.svals[j];
      const SphereRec s = load_rec(A.recA, A.recB, A.recC, A.recD, id);
      const uint32_t p1 = __float_as_uint(A.recD[id].z);
      float fk[CM];
      const float* fp = A.payload + size_t(id) * size_t(C);
#pragma unroll
      for (int c = 0; c < CM; ++c) fk[c] = c < C ? fp[c] : 0.f;
      float gcx = 0.f, gcy = 0.f, gcz = 0.f, gR = 0.f, go = 0.f, gf[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) gf[c] = 0.f;
      bool any = false;
      const int xa = max(s.x0, tx0), xb = min(int(p1 & 0xffffu), tx0 + kTileW - 1);
      const int ya = max(s.y0, ty0), yb = min(int(p1 >> 16), ty0 + kTileH - 1);
      for (int iy = ya; iy <= yb; ++iy) {
        for (int ix = xa; ix <= xb; ++ix) {
          const int pl = (iy - ty0) * kTileW + (ix - tx0);
          const PixelRay ray = load_ray(s_ray, pl, ix, iy);
          if (!(coarse_r2(ray, s.x0, s.y0, s.xh, s.yh, s.kh, s.axh, s.ayh) < kRejectR2)) continue;
          Hit h;
          if (!exact_hit(ray, s, bc.zfar, h)) continue;
          // among the pixel's K nearest hits?
          const float tk = s_tk[pl];
          const uint32_t ik = s_ik[pl];
          if (!(id == ik || h.t < tk || (h.t == tk && id < ik))) continue;
          any = true;
          const float o = s.o;
          const float s2 = o * (bc.zfar - h.t) * bc.kz;  // o z / gamma in base 2
          const float ex = fast_exp2(s2 - s_L2[pl]);      // exp(o z / gamma) / denominator
          const float e = h.delta * ex;                   // dw/do without the exponent term
          const float w = o * e;                          // blending weight of Eq. 1
          float hs = 0.f;                                 // G . (f_k - F)
#pragma unroll
          for (int c = 0; c < CM; ++c) hs += s_G[c][pl] * (fk[c] - s_F[c][pl]);
#pragma unroll
          for (int c = 0; c < CM; ++c) gf[c] += w * s_G[c][pl];
          go += e * hs * (1.f + o * (bc.zfar - h.t) * bc.inv_span * bc.inv_gamma);
          const float gt = -w * hs * o * bc.inv_gamma * bc.inv_span;  // dL/dt
          const float gd = o * ex * hs;                               // dL/d(1 - q/R)
          // (c - (u.c) u) / R = sqrt(kappa) (v x (-D_y, D_x, cr)) / |v|^2
          const float sk = fast_sqrt(s.kh) * ray.inv_v2;
          const float dnx = (ray.ys * h.cr - cam.f * h.dx) * sk;
          const float dny = (-cam.f * h.dy - ray.xs * h.cr) * sk;
          const float dnz = (ray.xs * h.dx + ray.ys * h.dy) * sk;
          const float coef = gt / h.sq - (h.ratio > 0.f ? gd / (s.R * h.ratio) : 0.f);
          gcx += gt * ray.ux + coef * dnx;
          gcy += gt * ray.uy + coef * dny;
          gcz += gt * ray.uz + coef * dnz;
          gR += -gt / h.sq + gd * h.ratio / s.R;
        }
      }
      if (any) {
        if (A.grad_payload) {
          float* g = A.grad_payload + size_t(id) * size_t(C);
#pragma unroll
          for (int c = 0; c < CM; ++c)
            if (c < C) atomicAdd(g + c, gf[c]);
        }
        if (A.grad_opacity) atomicAdd(A.grad_opacity + id, go);
        if (A.gacc) {
          float* g = A.gacc + size_t(id) * 4;
          atomicAdd(g + 0, gcx);
          atomicAdd(g + 1, gcy);
          atomicAdd(g + 2, gcz);
          atomicAdd(g + 3, gR);
        }
      }
    }
  }
}

// Channels beyond the register budget: same walk, the pixel terms read from
// global memory and payload gradients go out per hit.
__global__ __launch_bounds__(kWave) void k_bwd_chunks_wide(BwdKernelArgs A, CamDev cam,
                                                           BlendConst bc) {
  __shared__ TileRays s_ray;
  __shared__ float s_L2[kWave], s_tk[kWave];
  __shared__ uint32_t s_ik[kWave];
  const int lane = threadIdx.x;
  const int C = A.C;
  const uint32_t nchunks = A.status->nchunks;
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const uint2 dsc = A.desc[chunk];
    const int tile = int(dsc.x), ci = int(dsc.y);
    const uint32_t beg = A.ranges[tile] + uint32_t(ci) * kChunk;
    const uint32_t end = min(A.ranges[tile + 1], beg + kChunk);
    const int tx0 = (tile % cam.tiles_x) * kTileW, ty0 = (tile / cam.tiles_x) * kTileH;
    if (beg >= end && !(ci == 0 && A.bgpart)) continue;
    const int px = tx0 + (lane % kTileW), py = ty0 + (lane / kTileW);
    const bool inside = px < cam.W && py < cam.H;
    const size_t p = inside ? size_t(py) * size_t(cam.W) + size_t(px) : 0;
    const float L2 = inside ? A.aux[p] * 1.4426950408889634f : 0.f;
    __syncthreads();
    store_ray(s_ray, lane, make_ray(cam, px, py));
    s_L2[lane] = L2;
    const float2 th = inside ? A.thr[p] : make_float2(-INFINITY, 0.f);
    s_tk[lane] = th.x;
    s_ik[lane] = __float_as_uint(th.y);
    if (ci == 0 && A.bgpart) {
      const float wbg = inside ? fast_exp2(bc.eps2 - L2) : 0.f;
      for (int c = 0; c < C; ++c) {
        const float g = inside ? A.grad_image[p * size_t(C) + c] : 0.f;
        const float sum = wave_sum(wbg * g);
        if (lane == 0) A.bgpart[size_t(tile) * size_t(C) + c] = sum;
      }
    }
    __syncthreads();
    for (uint32_t b0 = beg; b0 < end; b0 += kWave) {
      const uint32_t j = b0 + uint32_t(lane);
      if (j >= end) continue;
      const uint32_t id = A.svals[j];
      const SphereRec s = load_rec(A.recA, A.recB, A.recC, A.recD, id);
      const uint32_t p1 = __float_as_uint(A.recD[id].z);
      const float* fk = A.payload + size_t(id) * size_t(C);
      float gcx = 0.f, gcy = 0.f, gcz = 0.f, gR = 0.f, go = 0.f;
      bool any = false;
      const int xa = max(s.x0, tx0), xb = min(int(p1 & 0xffffu), tx0 + kTileW - 1);
      const int ya = max(s.y0, ty0), yb = min(int(p1 >> 16), ty0 + kTileH - 1);
      for (int iy = ya; iy <= yb; ++iy) {
        for (int ix = xa; ix <= xb; ++ix) {
          const int pl = (iy - ty0) * kTileW + (ix - tx0);
          const PixelRay ray = load_ray(s_ray, pl, ix, iy);
          if (!(coarse_r2(ray, s.x0, s.y0, s.xh, s.yh, s.kh, s.axh, s.ayh) < kRejectR2)) continue;
          Hit h;
          if (!exact_hit(ray, s, bc.zfar, h)) continue;
          const float tk = s_tk[pl];
          const uint32_t ik = s_ik[pl];
          if (!(id == ik || h.t < tk || (h.t == tk && id < ik))) continue;
          any = true;
          const size_t pp = size_t(iy) * size_t(cam.W) + size_t(ix);
          const float* Gp = A.grad_image + pp * size_t(C);
          const float* Fp = A.image + pp * size_t(C);
          const float o = s.o;
          const float s2 = o * (bc.zfar - h.t) * bc.kz;
          const float ex = fast_exp2(s2 - s_L2[pl]);
          const float e = h.delta * ex;
          const float w = o * e;
          float hs = 0.f;
          for (int c = 0; c < C; ++c) hs += Gp[c] * (fk[c] - Fp[c]);
          if (A.grad_payload) {
            float* g = A.grad_payload + size_t(id) * size_t(C);
            for (int c = 0; c < C; ++c) atomicAdd(g + c, w * Gp[c]);
          }
          go += e * hs * (1.f + o * (bc.zfar - h.t) * bc.inv_span * bc.inv_gamma);
          const float gt = -w * hs * o * bc.inv_gamma * bc.inv_span;
          const float gd = o * ex * hs;
          const float sk = fast_sqrt(s.kh) * ray.inv_v2;
          const float dnx = (ray.ys * h.cr - cam.f * h.dx) * sk;
          const float dny = (-cam.f * h.dy - ray.xs * h.cr) * sk;
          const float dnz = (ray.xs * h.dx + ray.ys * h.dy) * sk;
          const float coef = gt / h.sq - (h.ratio > 0.f ? gd / (s.R * h.ratio) : 0.f);
          gcx += gt * ray.ux + coef * dnx;
          gcy += gt * ray.uy + coef * dny;
          gcz += gt * ray.uz + coef * dnz;
          gR += -gt / h.sq + gd * h.ratio / s.R;
        }
      }
      if (any) {
        if (A.grad_opacity) atomicAdd(A.grad_opacity + id, go);
        if (A.gacc) {
          float* g = A.gacc + size_t(id) * 4;
          atomicAdd(g + 0, gcx);
          atomicAdd(g + 1, gcy);
          atomicAdd(g + 2, gcz);
          atomicAdd(g + 3, gR);
        }
      }
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

hipError_t launch_backward(const Plan& q, const CamDev& cam, const BlendConst& bc,
                           const BwdArgs& a, char* ws, hipStream_t stream) {
  const bool need_geo = a.grad_pos || a.grad_radius;
  BwdKernelArgs A;
  A.status = ws_ptr<Status>(ws, q.off_status);
  A.desc = ws_ptr<uint2>(ws, q.off_desc);
  A.ranges = ws_ptr<uint32_t>(ws, q.off_ranges);
  A.svals = ws_ptr<uint32_t>(ws, sorted_in_a(q) ? q.off_valsA : q.off_valsB);
  A.recA = ws_ptr<float4>(ws, q.off_recA);
  A.recB = ws_ptr<float4>(ws, q.off_recB);
  A.recC = ws_ptr<float4>(ws, q.off_recC);
  A.recD = ws_ptr<float4>(ws, q.off_recD);
  A.payload = a.payload;
  A.image = a.image;
  A.aux = a.aux;
  A.grad_image = a.grad_image;
  A.thr = ws_ptr<float2>(ws, q.off_thr);
  A.gacc = need_geo ? ws_ptr<float>(ws, q.off_gacc) : nullptr;
  A.grad_opacity = a.grad_opacity;
  A.grad_payload = a.grad_payload;
  A.bgpart = a.grad_bg ? ws_ptr<float>(ws, q.off_bgpart) : nullptr;
  A.C = a.C;
  stage_begin(PULSAR_STAGE_ZERO, stream);
  zero_async(A.gacc, size_t(q.n) * 4, stream);
  zero_async(a.grad_opacity, size_t(q.n), stream);
  zero_async(a.grad_payload, size_t(q.n) * size_t(q.C), stream);
  stage_end(PULSAR_STAGE_ZERO, stream);
  stage_begin(PULSAR_STAGE_RASTER_BWD, stream);
  const dim3 grid(kRasterGrid), block(kWave);
  if (a.C <= 1)
    hipLaunchKernelGGL(k_bwd_chunks<1>, grid, block, 0, stream, A, cam, bc);
  else if (a.C <= 2)
    hipLaunchKernelGGL(k_bwd_chunks<2>, grid, block, 0, stream, A, cam, bc);
  else if (a.C <= 4)
    hipLaunchKernelGGL(k_bwd_chunks<4>, grid, block, 0, stream, A, cam, bc);
  else if (a.C <= 8)
    hipLaunchKernelGGL(k_bwd_chunks<8>, grid, block, 0, stream, A, cam, bc);
  else if (a.C <= 16)
    hipLaunchKernelGGL(k_bwd_chunks<16>, grid, block, 0, stream, A, cam, bc);
  else if (a.C <= kBwdChannels)
    hipLaunchKernelGGL(k_bwd_chunks<32>, grid, block, 0, stream, A, cam, bc);
  else
    hipLaunchKernelGGL(k_bwd_chunks_wide, grid, block, 0, stream, A, cam, bc);
  stage_end(PULSAR_STAGE_RASTER_BWD, stream);
  stage_begin(PULSAR_STAGE_FINALIZE, stream);
  if (need_geo && q.n > 0)
    hipLaunchKernelGGL(k_finalize, dim3(unsigned((q.n + 255) / 256)), dim3(256), 0, stream,
                       int(q.n), a.pos, a.radius, cam, a.min_radius_px,
                       reinterpret_cast<const float4*>(A.gacc), a.grad_pos, a.grad_radius);
  if (a.grad_bg)
    hipLaunchKernelGGL(k_reduce_bg, dim3(unsigned(q.C)), dim3(256), 0, stream, A.bgpart,
                       int(q.T), int(q.C), a.grad_bg);
  stage_end(PULSAR_STAGE_FINALIZE, stream);
  return hipGetLastError();
}

}  // namespace pulsar
