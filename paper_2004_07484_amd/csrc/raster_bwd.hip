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
// rays are staged once per chunk in LDS. Blocks take work items round-robin,
// full chunks first.
//
// K8 turns the camera-space accumulators into world-space position and
// radius gradients; the background gradient is a plain reduction over all
// pixels (k_bg_partial, k_reduce_bg).
#include "hit_geometry.h"

namespace pulsar {

// Backward raster by (tile, sphere) pair instead of by tile work item.
constexpr bool kPairBackward = false;

struct BwdKernelArgs {
  SceneTable tab;
  Status* status;
  const uint4* desc;
  const float4* srec;   // sphere records in sorted pair order (index | single-tile flag in .w)
  const float* spay;    // payload rows in sorted pair order
  const float* image;
  const float* aux;
  const float* grad_image;
  const float2* thr;
  float* gacc;
  float* grad_opacity;
  float* grad_payload;
  int C;
};

// Gradient terms of one hit (pixel ray, sphere s) that belongs to the K
// nearest: derivatives of Eq. 1 through t (depth), 1 - q/R (distance), o and f.
struct HitGrad {
  float gcx, gcy, gcz, gR, go, w;
};

__device__ __forceinline__ HitGrad hit_grad(const PixelRay& ray, const SphereRec& s,
                                            const Hit& h, const CamDev& cam, const BlendConst& bc,
                                            float L2, float hs) {
  HitGrad g;
  const float o = s.o;
  const float zg = o * (bc.zfar - h.t);             // o z (zfar - znear)
  const float ex = fast_exp2(zg * bc.kz - L2);      // exp(o z / gamma) / denominator
  const float e = h.delta * ex;                     // dw/do without the exponent term
  g.w = o * e;                                      // blending weight of Eq. 1
  g.go = e * hs * (1.f + zg * bc.inv_span * bc.inv_gamma);
  const float gt = -g.w * hs * o * bc.inv_gamma * bc.inv_span;  // dL/dt
  const float gd = o * ex * hs;                                 // dL/d(1 - q/R)
  // (c - (u.c) u) / R = sqrt(kappa) (v x (-D_y, D_x, cr)) / |v|^2
  const float sk = fast_sqrt(s.kh) * ray.inv_v2;
  const float dnx = (ray.ys * h.cr - cam.f * h.dx) * sk;
  const float dny = (-cam.f * h.dy - ray.xs * h.cr) * sk;
  const float dnz = (ray.xs * h.dx + ray.ys * h.dy) * sk;
  const float isq = fast_rcp(h.sq);
  const float coef = gt * isq - (h.ratio > 0.f ? gd * fast_rcp(s.R * h.ratio) : 0.f);
  g.gcx = gt * ray.ux + coef * dnx;
  g.gcy = gt * ray.uy + coef * dny;
  g.gcz = gt * ray.uz + coef * dnz;
  g.gR = -gt * isq + gd * h.ratio * fast_rcp(s.R);
  return g;
}

// CM >= C: channels kept in LDS. The (sphere, pixel) pairs of a batch (each
// sphere's rectangle inside the tile) are flattened by a wave prefix sum over
// rectangle sizes, so all 64 lanes stay busy whatever the sphere sizes; lane
// j handles pair j + 64 i and adds its terms to its sphere's LDS accumulator.
template <int CM>
__global__ __launch_bounds__(kWave) void k_bwd_chunks(BwdKernelArgs A) {
  constexpr int CQ = (CM + 3) / 4;
  constexpr int NA = 6 + CM;  // dL/dc (3), dL/dR, dL/do, hit count, dL/df (CM)
  __shared__ TileRays s_ray;
  __shared__ float s_G[CM][kWave];
  __shared__ float s_L2[kWave], s_GF[kWave], s_tk[kWave];
  __shared__ uint32_t s_ik[kWave];
  __shared__ float4 s_rec[kWave][4];
  __shared__ float4 s_pay[kWave][CQ];
  __shared__ uint32_t s_off[kWave], s_box[kWave], s_id[kWave];
  __shared__ float s_acc[kWave][NA + 1];
  const int lane = threadIdx.x;
  const int C = A.C;
  const uint32_t nchunks = A.status->nchunks;
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const uint4 dsc = A.desc[chunk];
    const uint32_t tile = dsc.x & ~kFirstChunk;
    const uint32_t beg = dsc.y, end = dsc.z;
    const TileScene ts = tile_scene(A.tab, tile);
    const SceneDev& sc = A.tab.scenes[ts.b];
    const CamDev cam = sc.cam;
    const BlendConst bc = sc.bc;
    const int tx0 = ts.tx0, ty0 = ts.ty0;
    // stage the tile's pixels (lane = pixel): ray, L, threshold, G and G . F
    {
      const int px = tx0 + (lane % kTileW), py = ty0 + (lane / kTileW);
      const bool inside = px < cam.W && py < cam.H;
      const size_t p =
          inside ? size_t(sc.pix_off) + size_t(py) * size_t(cam.W) + size_t(px) : 0;
      __syncthreads();  // the previous chunk's LDS reads are done
      store_ray(s_ray, lane, make_ray(cam, px, py));
      s_L2[lane] = inside ? A.aux[p] * 1.4426950408889634f : 0.f;
      const float2 th = inside ? A.thr[p] : make_float2(-INFINITY, 0.f);
      s_tk[lane] = th.x;
      s_ik[lane] = __float_as_uint(th.y);
      float gf = 0.f;
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const float g = (inside && c < C) ? A.grad_image[p * size_t(C) + c] : 0.f;
        const float f = (inside && c < C) ? A.image[p * size_t(C) + c] : 0.f;
        s_G[c][lane] = g;
        gf += g * f;
      }
      s_GF[lane] = gf;
    }
    for (uint32_t b0 = beg; b0 < end; b0 += kWave) {
      const uint32_t j = b0 + uint32_t(lane);
      const bool valid = j < end;
      uint32_t id = 0;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a, c = a, d = a;
      bool single = false;
      if (valid) {
        const float4* rp = A.srec + 4 * size_t(j);
        a = rp[0];
        b = rp[1];
        c = rp[2];
        d = rp[3];
        id = __float_as_uint(d.w) & ~kFirstChunk;
        single = (__float_as_uint(d.w) & kFirstChunk) != 0u;
      }
      // the sphere's rectangle inside this tile, in tile coordinates
      const uint32_t p0 = __float_as_uint(a.w), p1 = __float_as_uint(d.z);
      const int xa = max(int(p0 & 0xffffu), tx0) - tx0;
      const int xb = min(int(p1 & 0xffffu), tx0 + kTileW - 1) - tx0;
      const int ya = max(int(p0 >> 16), ty0) - ty0;
      const int yb = min(int(p1 >> 16), ty0 + kTileH - 1) - ty0;
      const uint32_t w = valid ? uint32_t(xb - xa + 1) : 1u;
      const uint32_t n = valid ? w * uint32_t(yb - ya + 1) : 0u;
      const uint32_t incl = wave_incl_scan_u32(n, lane);
      const uint32_t total = __builtin_amdgcn_readlane(incl, kWave - 1);
      const uint32_t magic = (65536u + w - 1u) / w;  // i / w = (i * magic) >> 16 for i < 64
      const float* fp = A.spay + size_t(valid ? j : 0u) * size_t(C);
      __syncthreads();  // the previous batch is done with the LDS below
      s_rec[lane][0] = a;
      s_rec[lane][1] = b;
      s_rec[lane][2] = c;
      s_rec[lane][3] = d;
#pragma unroll
      for (int q = 0; q < CQ; ++q) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (valid && 4 * q + u < C) ? fp[4 * q + u] : 0.f;
        s_pay[lane][q] = make_float4(v[0], v[1], v[2], v[3]);
      }
      s_id[lane] = id;
      s_off[lane] = incl - n;
      s_box[lane] = uint32_t(xa) | (uint32_t(ya) << 3) | (w << 6) | (magic << 10);
#pragma unroll
      for (int v = 0; v < NA; ++v) s_acc[lane][v] = 0.f;
      __syncthreads();
      for (uint32_t pb = 0; pb < total; pb += kWave) {
        const uint32_t pair = pb + uint32_t(lane);
        if (pair >= total) continue;
        // owner: the last sphere whose first pair is <= pair
        int lo = 0, hi = kWave - 1;
#pragma unroll
        for (int step = 0; step < 6; ++step) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_off[mid] <= pair)
            lo = mid;
          else
            hi = mid - 1;
        }
        const int r = lo;
        const uint32_t i = pair - s_off[r], box = s_box[r];
        const uint32_t bw = (box >> 6) & 15u, yy = (i * (box >> 10)) >> 16;
        const int x = int(box & 7u) + int(i - yy * bw), y = int((box >> 3) & 7u) + int(yy);
        const int pl = y * kTileW + x;
        const SphereRec s = unpack_rec(s_rec[r][0], s_rec[r][1], s_rec[r][2], s_rec[r][3]);
        const PixelRay ray = load_ray(s_ray, pl, tx0 + x, ty0 + y);
        Hit h;
        if (!exact_hit(ray, s, bc.zfar, h)) continue;
        // among the pixel's K nearest hits?
        const uint32_t sid = s_id[r];
        const float tk = s_tk[pl];
        const uint32_t ik = s_ik[pl];
        if (!(sid == ik || h.t < tk || (h.t == tk && sid < ik))) continue;
        float hs = -s_GF[pl];  // G . (f_k - F)
#pragma unroll
        for (int q = 0; q < CQ; ++q) {
          const float4 f = s_pay[r][q];
          const float fv[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (4 * q + u < CM) hs += s_G[4 * q + u][pl] * fv[u];
        }
        const HitGrad g = hit_grad(ray, s, h, cam, bc, s_L2[pl], hs);
        atomicAdd(&s_acc[r][0], g.gcx);
        atomicAdd(&s_acc[r][1], g.gcy);
        atomicAdd(&s_acc[r][2], g.gcz);
        atomicAdd(&s_acc[r][3], g.gR);
        atomicAdd(&s_acc[r][4], g.go);
        atomicAdd(&s_acc[r][5], 1.f);
#pragma unroll
        for (int cc = 0; cc < CM; ++cc) atomicAdd(&s_acc[r][6 + cc], g.w * s_G[cc][pl]);
      }
      __syncthreads();
      // A sphere that touches one tile appears in exactly one work item: it
      // stores its sums (zeros included). Others add into zeroed sums.
      if (valid && single) {
        if (A.grad_payload) {
          float* gp = A.grad_payload + size_t(id) * size_t(C);
#pragma unroll
          for (int cc = 0; cc < CM; ++cc)
            if (cc < C) gp[cc] = s_acc[lane][6 + cc];
        }
        if (A.grad_opacity) A.grad_opacity[id] = s_acc[lane][4];
        if (A.gacc)
          reinterpret_cast<float4*>(A.gacc)[id] =
              make_float4(s_acc[lane][0], s_acc[lane][1], s_acc[lane][2], s_acc[lane][3]);
      } else if (valid && s_acc[lane][5] > 0.f) {
        if (A.grad_payload) {
          float* gp = A.grad_payload + size_t(id) * size_t(C);
#pragma unroll
          for (int cc = 0; cc < CM; ++cc)
            if (cc < C) atomicAdd(gp + cc, s_acc[lane][6 + cc]);
        }
        if (A.grad_opacity) atomicAdd(A.grad_opacity + id, s_acc[lane][4]);
        if (A.gacc) {
          float* gg = A.gacc + size_t(id) * 4;
          atomicAdd(gg + 0, s_acc[lane][0]);
          atomicAdd(gg + 1, s_acc[lane][1]);
          atomicAdd(gg + 2, s_acc[lane][2]);
          atomicAdd(gg + 3, s_acc[lane][3]);
        }
      }
    }
  }
}

// Pair-parallel variant of K7: lane = one (tile, sphere) pair of the sorted
// lists. The lane walks its sphere's rectangle inside the tile, recomputes
// each hit from the pixel's ray, keeps those among the pixel's K nearest and
// adds their terms in registers; the pixel data (G, F, L, threshold) come
// straight from memory, where neighbouring lanes (pairs of the same tile)
// share them through the caches. No LDS, no barriers, so occupancy is set by
// registers alone and global-memory latency overlaps across many waves.
struct BwdPairArgs {
  SceneTable tab;
  const Status* status;
  const uint32_t* keys;  // sorted pair keys: tile << depth_bits | quantised depth
  int depth_bits;
  const float4* srec;
  const float* spay;
  const float* image;
  const float* aux;
  const float* grad_image;
  const float2* thr;
  float* gacc;
  float* grad_opacity;
  float* grad_payload;
  int C;
};

constexpr int kPairThreads = 256;

template <int CM>
__global__ __launch_bounds__(kPairThreads) void k_bwd_pairs(BwdPairArgs A) {
  const uint32_t used = A.status->used;
  const int C = A.C;
  for (uint32_t j = blockIdx.x * kPairThreads + threadIdx.x; j < used;
       j += gridDim.x * kPairThreads) {
    const uint32_t tile = A.keys[j] >> A.depth_bits;
    const TileScene ts = tile_scene(A.tab, tile);
    const SceneDev& sc = A.tab.scenes[ts.b];
    const CamDev cam = sc.cam;
    const BlendConst bc = sc.bc;
    const float4* rp = A.srec + 4 * size_t(j);
    const float4 rd = rp[3];
    const SphereRec s = unpack_rec(rp[0], rp[1], rp[2], rd);
    const uint32_t id = __float_as_uint(rd.w) & ~kFirstChunk;
    const bool single = (__float_as_uint(rd.w) & kFirstChunk) != 0u;
    const uint32_t p1 = __float_as_uint(rd.z);
    const int xa = max(s.x0, ts.tx0), xb = min(int(p1 & 0xffffu), ts.tx0 + kTileW - 1);
    const int ya = max(s.y0, ts.ty0), yb = min(int(p1 >> 16), ts.ty0 + kTileH - 1);
    float f[CM], gf[CM];
    const float* fp = A.spay + size_t(j) * size_t(C);
#pragma unroll
    for (int c = 0; c < CM; ++c) {
      f[c] = c < C ? fp[c] : 0.f;
      gf[c] = 0.f;
    }
    float gcx = 0.f, gcy = 0.f, gcz = 0.f, gR = 0.f, go = 0.f;
    uint32_t nh = 0;
    for (int py = ya; py <= yb; ++py) {
      for (int px = xa; px <= xb; ++px) {
        const PixelRay ray = make_ray(cam, px, py);
        Hit h;
        if (!exact_hit(ray, s, bc.zfar, h)) continue;
        const size_t p = size_t(sc.pix_off) + size_t(py) * size_t(cam.W) + size_t(px);
        const float2 th = A.thr[p];
        const float tk = th.x;
        const uint32_t ik = __float_as_uint(th.y);
        if (!(id == ik || h.t < tk || (h.t == tk && id < ik))) continue;
        float G[CM];
        float hs = 0.f;  // G . (f_k - F)
        const float* Gp = A.grad_image + p * size_t(C);
        const float* Fp = A.image + p * size_t(C);
#pragma unroll
        for (int c = 0; c < CM; ++c) {
          G[c] = c < C ? Gp[c] : 0.f;
          const float F = c < C ? Fp[c] : 0.f;
          hs += G[c] * (f[c] - F);
        }
        const HitGrad g = hit_grad(ray, s, h, cam, bc, A.aux[p] * 1.4426950408889634f, hs);
        gcx += g.gcx;
        gcy += g.gcy;
        gcz += g.gcz;
        gR += g.gR;
        go += g.go;
#pragma unroll
        for (int c = 0; c < CM; ++c) gf[c] += g.w * G[c];
        ++nh;
      }
    }
    // A sphere that touches one tile has exactly one pair: it stores its sums
    // (zeros included). Others add into zeroed sums.
    if (single) {
      if (A.grad_payload) {
        float* gp = A.grad_payload + size_t(id) * size_t(C);
#pragma unroll
        for (int c = 0; c < CM; ++c)
          if (c < C) gp[c] = gf[c];
      }
      if (A.grad_opacity) A.grad_opacity[id] = go;
      if (A.gacc) reinterpret_cast<float4*>(A.gacc)[id] = make_float4(gcx, gcy, gcz, gR);
    } else if (nh > 0) {
      if (A.grad_payload) {
        float* gp = A.grad_payload + size_t(id) * size_t(C);
#pragma unroll
        for (int c = 0; c < CM; ++c)
          if (c < C) atomicAdd(gp + c, gf[c]);
      }
      if (A.grad_opacity) atomicAdd(A.grad_opacity + id, go);
      if (A.gacc) {
        float* gg = A.gacc + size_t(id) * 4;
        atomicAdd(gg + 0, gcx);
        atomicAdd(gg + 1, gcy);
        atomicAdd(gg + 2, gcz);
        atomicAdd(gg + 3, gR);
      }
    }
  }
}

// Channels beyond the register budget: same walk, the pixel terms read from
// global memory and payload gradients go out per hit.
__global__ __launch_bounds__(kWave) void k_bwd_chunks_wide(BwdKernelArgs A) {
  __shared__ TileRays s_ray;
  __shared__ float s_L2[kWave], s_tk[kWave];
  __shared__ uint32_t s_ik[kWave];
  const int lane = threadIdx.x;
  const int C = A.C;
  const uint32_t nchunks = A.status->nchunks;
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const uint4 dsc = A.desc[chunk];
    const uint32_t tile = dsc.x & ~kFirstChunk;
    const uint32_t beg = dsc.y, end = dsc.z;
    const TileScene ts = tile_scene(A.tab, tile);
    const SceneDev& sc = A.tab.scenes[ts.b];
    const CamDev cam = sc.cam;
    const BlendConst bc = sc.bc;
    const int tx0 = ts.tx0, ty0 = ts.ty0;
    const int px = tx0 + (lane % kTileW), py = ty0 + (lane / kTileW);
    const bool inside = px < cam.W && py < cam.H;
    const size_t p = inside ? size_t(sc.pix_off) + size_t(py) * size_t(cam.W) + size_t(px) : 0;
    const float L2 = inside ? A.aux[p] * 1.4426950408889634f : 0.f;
    __syncthreads();
    store_ray(s_ray, lane, make_ray(cam, px, py));
    s_L2[lane] = L2;
    const float2 th = inside ? A.thr[p] : make_float2(-INFINITY, 0.f);
    s_tk[lane] = th.x;
    s_ik[lane] = __float_as_uint(th.y);
    __syncthreads();
    for (uint32_t b0 = beg; b0 < end; b0 += kWave) {
      const uint32_t j = b0 + uint32_t(lane);
      if (j >= end) continue;
      const float4* rp = A.srec + 4 * size_t(j);
      const float4 d = rp[3];
      const SphereRec s = unpack_rec(rp[0], rp[1], rp[2], d);
      const uint32_t id = __float_as_uint(d.w) & ~kFirstChunk;
      const uint32_t p1 = __float_as_uint(d.z);
      const float* fk = A.spay + size_t(j) * size_t(C);
      float gcx = 0.f, gcy = 0.f, gcz = 0.f, gR = 0.f, go = 0.f;
      bool any = false;
      const int xa = max(s.x0, tx0), xb = min(int(p1 & 0xffffu), tx0 + kTileW - 1);
      const int ya = max(s.y0, ty0), yb = min(int(p1 >> 16), ty0 + kTileH - 1);
      for (int iy = ya; iy <= yb; ++iy) {
        for (int ix = xa; ix <= xb; ++ix) {
          const int pl = (iy - ty0) * kTileW + (ix - tx0);
          const PixelRay ray = load_ray(s_ray, pl, ix, iy);
          Hit h;
          if (!exact_hit(ray, s, bc.zfar, h)) continue;
          const float tk = s_tk[pl];
          const uint32_t ik = s_ik[pl];
          if (!(id == ik || h.t < tk || (h.t == tk && id < ik))) continue;
          any = true;
          const size_t pp = size_t(sc.pix_off) + size_t(iy) * size_t(cam.W) + size_t(ix);
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

// Before K7: zero the sums of the spheres that K7 will add into (those that
// touch several tiles, or every visible one when K7 adds per hit).
__global__ void k_bwd_prep(int n, const uint32_t* __restrict__ counts, uint32_t min_count,
                           int C, float4* __restrict__ gacc, float* __restrict__ grad_opacity,
                           float* __restrict__ grad_payload) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || counts[i] < min_count) return;
  if (gacc) gacc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (grad_opacity) grad_opacity[i] = 0.f;
  if (grad_payload)
    for (int c = 0; c < C; ++c) grad_payload[size_t(i) * size_t(C) + c] = 0.f;
}

// K8: camera-space (dL/dc, dL/dR) -> world-space position and radius
// gradients; spheres that touch no tile get zeros everywhere.
__global__ void k_finalize(int n, const uint32_t* __restrict__ counts,
                           const float* __restrict__ pos, const float* __restrict__ radius,
                           SceneTable tab, float min_radius_px, int C,
                           const float4* __restrict__ gacc,
                           float* __restrict__ grad_pos, float* __restrict__ grad_radius,
                           float* __restrict__ grad_opacity, float* __restrict__ grad_payload) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (counts[i] == 0u) {
    if (grad_pos) {
      grad_pos[3 * i + 0] = 0.f;
      grad_pos[3 * i + 1] = 0.f;
      grad_pos[3 * i + 2] = 0.f;
    }
    if (grad_radius) grad_radius[i] = 0.f;
    if (grad_opacity) grad_opacity[i] = 0.f;
    if (grad_payload) {
      float* row = grad_payload + size_t(i) * size_t(C);
      if ((C & 3) == 0 && (reinterpret_cast<uintptr_t>(grad_payload) & 15u) == 0u) {
        for (int c = 0; c < C; c += 4)
          *reinterpret_cast<float4*>(row + c) = make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        for (int c = 0; c < C; ++c) row[c] = 0.f;
      }
    }
    return;
  }
  if (!gacc) return;
  const CamDev cam = tab.scenes[find_scene(tab.sph_start, tab.B, uint32_t(i))].cam;
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

// Background gradient, dL/dbg = sum_p exp(eps/gamma - L_p) G_p per scene:
// per-block partial sums [blocks][C]; every block covers kBgBlockPixels
// consecutive pixels of one scene. The block's pixel weights go to LDS, then
// the block reads its G rows as one flat run of floats: thread t takes
// elements t, t + S, t + 2S, ... with S the largest multiple of C <= 256, so
// its channel is always t % C and consecutive threads read consecutive floats.
constexpr int kBgThreads = 256;
constexpr int kBgMaxC = kBgThreads;  // wider images use k_bg_partial_wide
__global__ __launch_bounds__(kBgThreads) void k_bg_partial(SceneTable tab,
                                                           const float* __restrict__ aux,
                                                           const float* __restrict__ grad_image,
                                                           int C, float eps2,
                                                           float* __restrict__ bgsum) {
  __shared__ float s_w[kBgBlockPixels];
  __shared__ float s_acc[kBgThreads];
  const int tid = threadIdx.x;
  const int b = find_scene(tab.blk_start, tab.B, blockIdx.x);
  const SceneDev& sc = tab.scenes[b];
  const long long npix = (long long)sc.cam.W * sc.cam.H;
  const long long p0 = (long long)(blockIdx.x - sc.bgblk_off) * kBgBlockPixels;
  const int np = int(min((long long)kBgBlockPixels, npix - p0));
  const float* auxs = aux + sc.pix_off + p0;
  const float* gs = grad_image + (size_t(sc.pix_off) + size_t(p0)) * size_t(C);
  for (int k = tid; k < kBgBlockPixels; k += kBgThreads)
    s_w[k] = k < np ? fast_exp2(eps2 - auxs[k] * 1.4426950408889634f) : 0.f;
  __syncthreads();
  const int S = (kBgThreads / C) * C;  // threads in use, a multiple of C
  const int step = S / C;               // pixels advanced per round
  float acc = 0.f;
  if (tid < S) {
    const int total = np * C;
    int pix = tid / C;
    for (int f = tid; f < total; f += S, pix += step) acc += s_w[pix] * gs[f];
  }
  s_acc[tid] = acc;
  __syncthreads();
  if (tid < C) {
    float t = 0.f;
    for (int k = tid; k < S; k += C) t += s_acc[k];
    bgsum[size_t(blockIdx.x) * size_t(C) + tid] = t;
  }
}

// The same sums for C > kBgMaxC: one pixel per thread and a loop over channels.
__global__ __launch_bounds__(kBgThreads) void k_bg_partial_wide(SceneTable tab,
                                                                const float* __restrict__ aux,
                                                                const float* __restrict__ grad_image,
                                                                int C, float eps2,
                                                                float* __restrict__ bgsum) {
  __shared__ float s[kBgThreads / kWave];
  const int b = find_scene(tab.blk_start, tab.B, blockIdx.x);
  const SceneDev& sc = tab.scenes[b];
  const long long npix = (long long)sc.cam.W * sc.cam.H;
  const long long p0 = (long long)(blockIdx.x - sc.bgblk_off) * kBgBlockPixels;
  const float* auxs = aux + sc.pix_off;
  const float* gs = grad_image + size_t(sc.pix_off) * size_t(C);
  for (int c = 0; c < C; ++c) {
    float acc = 0.f;
    for (int k = threadIdx.x; k < kBgBlockPixels; k += kBgThreads) {
      const long long p = p0 + k;
      if (p < npix) acc += fast_exp2(eps2 - auxs[p] * 1.4426950408889634f) * gs[size_t(p) * C + c];
    }
    acc = wave_sum(acc);
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      float t = 0.f;
      for (int w = 0; w < kBgThreads / kWave; ++w) t += s[w];
      bgsum[size_t(blockIdx.x) * size_t(C) + c] = t;
    }
  }
}

// K8b: grad_bg[b][c] = sum of scene b's block partials (one block per (c, b)).
__global__ __launch_bounds__(256) void k_reduce_bg(SceneTable tab, const float* __restrict__ bgpart,
                                                   int C, float* __restrict__ grad_bg) {
  __shared__ float s[256 / kWave];
  const int c = blockIdx.x, b = blockIdx.y;
  const uint32_t k0 = tab.blk_start[b], k1 = tab.blk_start[b + 1];
  float acc = 0.f;
  for (uint32_t k = k0 + threadIdx.x; k < k1; k += 256) acc += bgpart[size_t(k) * size_t(C) + c];
  acc = wave_sum(acc);
  if ((threadIdx.x & (kWave - 1)) == 0) s[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    float tsum = 0.f;
    for (int w = 0; w < 256 / kWave; ++w) tsum += s[w];
    grad_bg[size_t(b) * size_t(C) + c] = tsum;
  }
}

hipError_t launch_backward(const Plan& q, const BwdArgs& a, char* ws, hipStream_t stream) {
  const bool need_geo = a.grad_pos || a.grad_radius;
  const SceneTable tab = scene_table(q, ws);
  BwdKernelArgs A;
  A.tab = tab;
  A.status = ws_ptr<Status>(ws, q.off_status);
  A.desc = ws_ptr<uint4>(ws, q.off_desc);
  A.srec = ws_ptr<float4>(ws, q.off_srec);
  A.spay = ws_ptr<float>(ws, q.off_spay);
  A.image = a.image;
  A.aux = a.aux;
  A.grad_image = a.grad_image;
  A.thr = ws_ptr<float2>(ws, q.off_thr);
  const uint32_t* counts = ws_ptr<uint32_t>(ws, q.off_counts);
  A.gacc = need_geo ? ws_ptr<float>(ws, q.off_gacc) : nullptr;
  A.grad_opacity = a.grad_opacity;
  A.grad_payload = a.grad_payload;
  A.C = a.C;
  float* bgsum = ws_ptr<float>(ws, q.off_bgsum);
  stage_begin(PULSAR_STAGE_ZERO, stream);
  // the narrow kernels store single-tile spheres directly, the wide one adds per hit
  const uint32_t min_count = a.C <= kBwdChannels ? 2u : 1u;
  if (q.n > 0)
    hipLaunchKernelGGL(k_bwd_prep, dim3(unsigned((q.n + 255) / 256)), dim3(256), 0, stream,
                       int(q.n), counts, min_count, a.C, reinterpret_cast<float4*>(A.gacc),
                       a.grad_opacity, a.grad_payload);
  stage_end(PULSAR_STAGE_ZERO, stream);
  stage_begin(PULSAR_STAGE_RASTER_BWD, stream);
  const dim3 grid(unsigned(q.raster_grid)), block(kWave);
  if (kPairBackward && a.C <= kBwdChannels) {
    BwdPairArgs P;
    P.tab = tab;
    P.status = A.status;
    P.keys = ws_ptr<uint32_t>(ws, sorted_in_a(q) ? q.off_keysA : q.off_keysB);
    P.depth_bits = q.depth_bits;
    P.srec = A.srec;
    P.spay = A.spay;
    P.image = A.image;
    P.aux = A.aux;
    P.grad_image = A.grad_image;
    P.thr = A.thr;
    P.gacc = A.gacc;
    P.grad_opacity = A.grad_opacity;
    P.grad_payload = A.grad_payload;
    P.C = A.C;
    long long pb = (q.cap + kPairThreads - 1) / kPairThreads;
    if (pb > 8192) pb = 8192;
    const dim3 pg{unsigned(pb), 1u, 1u}, pt{unsigned(kPairThreads), 1u, 1u};
    if (a.C <= 1)
      hipLaunchKernelGGL(k_bwd_pairs<1>, pg, pt, 0, stream, P);
    else if (a.C <= 2)
      hipLaunchKernelGGL(k_bwd_pairs<2>, pg, pt, 0, stream, P);
    else if (a.C <= 4)
      hipLaunchKernelGGL(k_bwd_pairs<4>, pg, pt, 0, stream, P);
    else if (a.C <= 8)
      hipLaunchKernelGGL(k_bwd_pairs<8>, pg, pt, 0, stream, P);
    else if (a.C <= 16)
      hipLaunchKernelGGL(k_bwd_pairs<16>, pg, pt, 0, stream, P);
    else
      hipLaunchKernelGGL(k_bwd_pairs<32>, pg, pt, 0, stream, P);
  } else if (a.C <= 1)
    hipLaunchKernelGGL(k_bwd_chunks<1>, grid, block, 0, stream, A);
  else if (a.C <= 2)
    hipLaunchKernelGGL(k_bwd_chunks<2>, grid, block, 0, stream, A);
  else if (a.C <= 4)
    hipLaunchKernelGGL(k_bwd_chunks<4>, grid, block, 0, stream, A);
  else if (a.C <= 8)
    hipLaunchKernelGGL(k_bwd_chunks<8>, grid, block, 0, stream, A);
  else if (a.C <= 16)
    hipLaunchKernelGGL(k_bwd_chunks<16>, grid, block, 0, stream, A);
  else if (a.C <= kBwdChannels)
    hipLaunchKernelGGL(k_bwd_chunks<32>, grid, block, 0, stream, A);
  else
    hipLaunchKernelGGL(k_bwd_chunks_wide, grid, block, 0, stream, A);
  stage_end(PULSAR_STAGE_RASTER_BWD, stream);
  stage_begin(PULSAR_STAGE_FINALIZE, stream);
  if (q.n > 0)
    hipLaunchKernelGGL(k_finalize, dim3(unsigned((q.n + 255) / 256)), dim3(256), 0, stream,
                       int(q.n), counts, a.pos, a.radius, tab, a.min_radius_px, a.C,
                       reinterpret_cast<const float4*>(A.gacc), a.grad_pos, a.grad_radius,
                       a.grad_opacity, a.grad_payload);
  if (a.grad_bg) {
    if (q.C <= kBgMaxC)
      hipLaunchKernelGGL(k_bg_partial, dim3(unsigned(q.nbgblk)), dim3(kBgThreads), 0, stream,
                         tab, a.aux, a.grad_image, int(q.C), a.eps2, bgsum);
    else
      hipLaunchKernelGGL(k_bg_partial_wide, dim3(unsigned(q.nbgblk)), dim3(kBgThreads), 0,
                         stream, tab, a.aux, a.grad_image, int(q.C), a.eps2, bgsum);
    hipLaunchKernelGGL(k_reduce_bg, dim3(unsigned(q.C), unsigned(q.B)), dim3(256), 0, stream, tab,
                       bgsum, int(q.C), a.grad_bg);
  }
  stage_end(PULSAR_STAGE_FINALIZE, stream);
  return hipGetLastError();
}

}  // namespace pulsar
