// K7/K8: backward pass (paper App. B, "The Backward Pass").
//
// The forward left, per pixel, the K-th nearest hit (t_K, sphere index) and
// the log-normaliser L. A hit (t, k) of pixel p receives gradients iff it is
// among the K nearest, i.e. k is the K-th one or (t, k) < (t_K, k_K); nothing
// else per pixel is stored, every intersection is recomputed here.
//
// K7 (k_bwd_items) runs over the forward's work items: a block takes one
// chunk of one tile's sorted list, stages the tile's 64 pixels in LDS and
// gives each thread one record. The thread walks its sphere's rectangle
// inside the tile and sums its sphere's derivatives of Eq. 1 (camera-space
// dL/dc, dL/dR, dL/do, dL/df) in registers, then writes them whole into the
// pair's slot (ps4 float4: dL/dc, dL/dR | dL/df[cm] | dL/do) with plain
// stores. A pair's slot is its emission position, so a sphere's slots are
// contiguous and in sphere order: no atomics and no zeroing pass, and the
// result does not depend on scheduling.
//
// K8 (k_finalize) runs in sphere order: it adds each sphere's slots (one per
// tile it touches, read sequentially), turns the camera-space sums into
// world-space position and radius gradients and writes every requested
// output contiguously. The background gradient is a
// plain reduction over all pixels: block sums at the end of K7 (k_bg_partial
// for the wide path), summed per scene by extra blocks of K8.
#include "hit_geometry.h"

namespace pulsar {

struct BwdKernelArgs {
  SceneTable tab;
  Status* status;
  const uint4* desc;
  uint32_t max_items;  // capacity of the work list (short items fill it from the back)
  const float4* rec;                // sphere records, rec4 float4 per sphere
  int rec4;                         // 8: the payload row follows the geometry
  const float* payload;             // the caller's payload rows [n, C]
  const unsigned long long* boff;   // first pair of each projection block
  const float* image;
  const float* aux;
  const float* grad_image;
  const float4* thr;  // per pixel: K-th nearest hit (t, sphere index), L, 0
  float4* pslot;        // per-pair sum slots at emission positions, ps4 float4 each
  int ps4;
  const uint32_t* svals;  // sphere index of every sorted pair
  uint32_t last_sph;      // n - 1: sorted indices are clamped to it
  float* grad_payload;  // caller's output, added per hit by the wide path only
  int C;
  int need_geo, need_op, need_pay, need_cam;
  float* bgsum;       // background-gradient block sums, or null
  uint32_t nbgblk;
  float eps2;
  // early termination: each sphere's earliest possible hit distance and per
  // pixel the first hit the forward skipped (hits from it on take no part)
  const float* tmin;
  const float2* stop;
  // PULSAR_STORE_HITS: per pixel the forward's K nearest (t bits, sphere index)
  const uint2* hits;
  const uint4* tinfo;  // per tile (first partial slot, work items)
  int K;
  uint32_t T;
  int only_if_big;  // the tile walk runs only when the emission flagged a very large sphere
};

constexpr int kBgThreads = 256;
constexpr int kBgMaxC = kBgThreads;  // wider images use k_bg_partial_wide
// LDS floats a background block sum works in (the caller's, so a kernel that
// also does other work can share it)
constexpr int kBgScratch = kBgBlockPixels + kBgThreads + 4 * kBgThreads;
__device__ void bg_partial_block(const SceneTable& tab, const float* __restrict__ aux,
                                 const float* __restrict__ grad_image, int C, float eps2,
                                 float* __restrict__ bgsum, uint32_t blk, float* scratch);

// Gradient terms of one hit (pixel ray, sphere s) that belongs to the K
// nearest: derivatives of Eq. 1 through t (depth), 1 - q/R (distance), o and f.
struct HitGrad {
  float gcx, gcy, gcz, gR, go, w;
  float gt, coef;  // dL/dt and the coefficient of (c - (u.c) u) / R in dL/dc
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
  g.gt = gt;
  g.coef = coef;
  return g;
}

// The same hit's derivative with respect to kappa = f / s, the only way the
// focal length and the sensor width enter a ray: u is the unit vector along
// (x_s, y_s, f) = s (a, b, kappa). With c fixed, t and 1 - q/R depend on u
// through b = u.c and q^2 = |c|^2 - b^2, which gives dL/du = (dL/dt - b
// coef / R) c, and c . du/dkappa = s (c_z - u_z b) / |v| = s c_z pitch
// (x_s D_x + y_s D_y) / |v|^3 (D in pixels: x_s - f c_x / c_z = pitch D_x),
// which stays accurate where c_z - u_z b cancels.
__device__ __forceinline__ float hit_grad_kappa(const PixelRay& ray, const SphereRec& s,
                                                const Hit& h, const CamDev& cam,
                                                const HitGrad& g) {
  const float b = h.t + s.R * h.sq;  // u . c
  const float du = g.gt - b * g.coef * fast_rcp(s.R);
  const float proj = (ray.xs * h.dx + ray.ys * h.dy) * (cam.pitch * cam.s);
  return du * s.cz * proj * ray.inv_v2 * fast_sqrt(ray.inv_v2);
}

// K7 by work item: a block of kBwdWaves waves takes one work item (a chunk of
// one tile's sorted list), so tile, scene and camera are uniform. The tile's
// 64 pixels are staged once in LDS (ray, L, K-th nearest threshold, G and
// G . F); then each thread owns one record of the chunk, walks the sphere's
// rectangle inside the tile, recomputes each hit, keeps those among the
// pixel's K nearest and adds their terms in registers. No global load sits
// inside the pixel loop and no barrier inside the record loop. CM >= C.
constexpr int kBwdWaves = 4;

// Up to 4 channels the item kernel fits 96 VGPRs without spilling, so 5
// blocks of 4 waves share a CU; with 8 it is held to 128 VGPRs (4 blocks):
// at 96 it spilled inside the record loop and measured 3 us slower. Wider
// instances keep the compiler's budget.
constexpr int bwd_waves_per_simd(int CM) { return CM <= 4 ? 5 : (CM <= 8 ? 4 : 1); }

// ES: early termination (hits from each pixel's first skipped one on take no part).
template <int CM, bool CAM, bool ES>
__device__ __forceinline__ void bwd_items_body(const BwdKernelArgs& A,
                                               const SceneDev* __restrict__ scenes,
                                               const uint32_t* __restrict__ tile_start,
                                               const uint4* __restrict__ desc) {
  __shared__ TileRays s_ray;
  __shared__ float s_G[CM][kWave];
  __shared__ float s_L2[kWave], s_GF[kWave], s_tk[kWave];
  __shared__ uint32_t s_ik[kWave];
  __shared__ uint64_t s_sk[ES ? kWave : 1];  // early termination: first skipped hit
  __shared__ float s_bg[kBgScratch];           // the background block sums at the end
  const int tid = threadIdx.x;
  const int C = A.C;
  const uint32_t nchunks = item_count(A.status), nfull = A.status->nfull;
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const uint4 dsc = desc[item_slot(chunk, nfull, A.max_items)];
    const uint32_t tile = dsc.x & ~kFirstChunk;
    const uint32_t beg = dsc.y, end = dsc.z;
    const TileScene ts = tile_scene(scenes, tile_start, A.tab.B, tile);
    const SceneDev& sc = scenes[ts.b];
    const CamDev cam = sc.cam;
    const BlendConst bc = sc.bc;
    // the thread's first record and payload row are requested before the
    // staging below, so the global round trips overlap; a sorted pair names
    // its sphere, whose record and payload row are read in place
    uint32_t j = beg + uint32_t(tid);
    float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra, rc = ra, rd = ra;
    uint32_t bo = 0, sph = 0;
    float tmin = 0.f;
    float f[CM];
#pragma unroll
    for (int c = 0; c < CM; ++c) f[c] = 0.f;
    auto load_record = [&](uint32_t jj) {
      sph = min(A.svals[jj], A.last_sph);
      const float4* rp = A.rec + size_t(A.rec4) * size_t(sph);
      ra = rp[0];
      rb = rp[1];
      rc = rp[2];
      rd = rp[3];
      if (ES) tmin = A.tmin[sph];
      bo = uint32_t(A.boff[sph / kProjectBlock]);
      // the payload row: in the record's second half when it fits there
      const float* fp = A.rec4 == 8 ? reinterpret_cast<const float*>(rp + 4)
                                    : A.payload + size_t(sph) * size_t(C);
      // unconditional loads (clamped to the row), so they issue together
#pragma unroll
      for (int c = 0; c < CM; ++c) f[c] = fp[min(c, C - 1)];
#pragma unroll
      for (int c = 0; c < CM; ++c) f[c] = c < C ? f[c] : 0.f;
    };
    const int ttx = ts.tx0 / kTileW, tty = ts.ty0 / kTileH;  // the tile, in tile units
    if (j < end) load_record(j);
    __syncthreads();  // the previous item's readers are done with the LDS
    if (tid < kWave) {
      // every load unconditional (pixels outside the image read one inside
      // it and are masked; channels are clamped), so they issue together
      const int px = ts.tx0 + (tid % kTileW), py = ts.ty0 + (tid / kTileW);
      const bool inside = px < cam.W && py < cam.H;
      const size_t p = size_t(sc.pix_off) + (inside ? size_t(py) * size_t(cam.W) + size_t(px)
                                                    : size_t(ts.ty0) * size_t(cam.W) +
                                                          size_t(ts.tx0));
      const float aux = A.aux[p];
      const float4 th = A.thr[p];
      if (ES) {
        const float2 st = A.stop[p];
        s_sk[tid] = inside ? (uint64_t(__float_as_uint(st.x)) << 32) | __float_as_uint(st.y) : 0ull;
      }
      float gi[CM], fi[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        gi[c] = A.grad_image[p * size_t(C) + size_t(min(c, C - 1))];
        fi[c] = A.image[p * size_t(C) + size_t(min(c, C - 1))];
      }
      store_ray(s_ray, tid, make_ray(cam, px, py));
      s_L2[tid] = inside ? aux * 1.4426950408889634f : 0.f;
      s_tk[tid] = inside ? th.x : -INFINITY;
      s_ik[tid] = inside ? __float_as_uint(th.y) : 0u;
      float gf = 0.f;
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const float g = (inside && c < C) ? gi[c] : 0.f;
        s_G[c][tid] = g;
        gf += g * ((inside && c < C) ? fi[c] : 0.f);
      }
      s_GF[tid] = gf;
    }
    __syncthreads();
    for (; j < end; j += kWave * kBwdWaves) {
      if (j != beg + uint32_t(tid)) load_record(j);
      const SphereRec s = unpack_rec(ra, rb, rc, rd);
      const uint32_t id = pair_position(ra, rd, bo, ttx, tty);  // the pair's slot
      const uint32_t p1 = __float_as_uint(rd.z);
      const int xa = max(s.x0, ts.tx0), xb = min(int(p1 & 0xffffu), ts.tx0 + kTileW - 1);
      const int ya = max(s.y0, ts.ty0), yb = min(int(p1 >> 16), ts.ty0 + kTileH - 1);
      float gf[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) gf[c] = 0.f;
      float gcx = 0.f, gcy = 0.f, gcz = 0.f, gR = 0.f, go = 0.f, gk = 0.f;
      uint32_t nh = 0;
      const float tlo = front_bound(s);
      // early termination: the sphere's place in the depth-sort order
      const uint64_t dkey = ES ? (uint64_t(__float_as_uint(tmin)) << 32) | sph : 0ull;
      for (int py = ya; py <= yb; ++py) {
        for (int px = xa; px <= xb; ++px) {
          const int pl = (py - ts.ty0) * kTileW + (px - ts.tx0);
          const float tk = s_tk[pl];
          // behind the pixel's K-th nearest hit: no gradient, no test needed
          if (tlo > tk) continue;
          // at or after the hit where the pixel stopped: never blended
          if (ES && dkey >= s_sk[pl]) continue;
          const PixelRay ray = load_ray(s_ray, pl, px, py);
          Hit h;
          if (!exact_hit(ray, s, bc.zfar, h)) continue;
          // among the pixel's K nearest: (t, sphere index) up to its K-th
          const uint32_t ik = s_ik[pl];
          if (!(sph == ik || h.t < tk || (h.t == tk && sph < ik))) continue;
          float hs = -s_GF[pl];  // G . (f_k - F)
#pragma unroll
          for (int c = 0; c < CM; ++c) hs += s_G[c][pl] * f[c];
          const HitGrad g = hit_grad(ray, s, h, cam, bc, s_L2[pl], hs);
          gcx += g.gcx;
          gcy += g.gcy;
          gcz += g.gcz;
          gR += g.gR;
          go += g.go;
          if (CAM) gk += hit_grad_kappa(ray, s, h, cam, g);
#pragma unroll
          for (int c = 0; c < CM; ++c) gf[c] += g.w * s_G[c][pl];
          ++nh;
        }
      }
      // the pair's sums go whole into its slot
      float4* sr = A.pslot + size_t(id) * size_t(A.ps4);
      // float4 holding dL/df[CM], then dL/do, dL/d(f/s) and the pixel count
      constexpr int NT = (CM + 6) / 4;
      sr[0] = make_float4(gcx, gcy, gcz, gR);
#pragma unroll
      for (int q = 0; q < NT; ++q) {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int k = 4 * q + u;
          v[u] = k < CM ? gf[k < CM ? k : 0]
                        : (k == CM ? go : (k == CM + 1 ? gk : (k == CM + 2 ? float(nh) : 0.f)));
        }
        sr[1 + q] = make_float4(v[0], v[1], v[2], v[3]);
      }
    }
  }
  // then the background-gradient block sums on the same grid (their reads
  // overlap the uneven end of the work-item loop)
  if (A.bgsum)
    for (uint32_t blk = blockIdx.x; blk < A.nbgblk; blk += gridDim.x)
      bg_partial_block(A.tab, A.aux, A.grad_image, C, A.eps2, A.bgsum, blk, s_bg);
}

template <int CM, bool CAM, bool ES>
__global__ __launch_bounds__(kWave * kBwdWaves, bwd_waves_per_simd(CM)) void k_bwd_items(
    BwdKernelArgs A, const SceneDev* __restrict__ scenes, const uint32_t* __restrict__ tile_start,
    const uint4* __restrict__ desc) {
  // beside the walk in sphere order: only for scenes with a very large sphere
  if (A.only_if_big && A.status->big_spheres == 0u) return;
  bwd_items_body<CM, CAM, ES>(A, scenes, tile_start, desc);
}

// Channels beyond the register budget: same walk, the pixel terms read from
// global memory and payload gradients go out per hit.
__global__ __launch_bounds__(kWave) void k_bwd_chunks_wide(BwdKernelArgs A,
                                                           const SceneDev* __restrict__ scenes,
                                                           const uint32_t* __restrict__ tile_start,
                                                           const uint4* __restrict__ desc) {
  __shared__ TileRays s_ray;
  __shared__ float s_L2[kWave], s_tk[kWave];
  __shared__ uint32_t s_ik[kWave];
  __shared__ uint64_t s_sk[kWave];  // early termination: first skipped hit
  const int lane = threadIdx.x;
  const int C = A.C;
  const uint32_t nchunks = item_count(A.status), nfull = A.status->nfull;
  for (uint32_t chunk = blockIdx.x; chunk < nchunks; chunk += gridDim.x) {
    const uint4 dsc = desc[item_slot(chunk, nfull, A.max_items)];
    const uint32_t tile = dsc.x & ~kFirstChunk;
    const uint32_t beg = dsc.y, end = dsc.z;
    const TileScene ts = tile_scene(scenes, tile_start, A.tab.B, tile);
    const SceneDev& sc = scenes[ts.b];
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
    const float4 th = inside ? A.thr[p] : make_float4(-INFINITY, 0.f, 0.f, 0.f);
    s_tk[lane] = th.x;
    s_ik[lane] = __float_as_uint(th.y);
    if (A.stop) {
      const float2 st = inside ? A.stop[p] : make_float2(0.f, 0.f);
      s_sk[lane] = (uint64_t(__float_as_uint(st.x)) << 32) | __float_as_uint(st.y);
    }
    __syncthreads();
    for (uint32_t b0 = beg; b0 < end; b0 += kWave) {
      const uint32_t j = b0 + uint32_t(lane);
      if (j >= end) continue;
      const uint32_t id = min(A.svals[j], A.last_sph);  // sphere index
      const float4* rp = A.rec + size_t(A.rec4) * size_t(id);
      const float4 a = rp[0], d = rp[3];
      const SphereRec s = unpack_rec(a, rp[1], rp[2], d);
      // the pair's slot
      const uint32_t slot =
          pair_position(a, d, uint32_t(A.boff[id / kProjectBlock]), tx0 / kTileW, ty0 / kTileH);
      const uint32_t p1 = __float_as_uint(d.z);
      const float* fk = A.payload + size_t(id) * size_t(C);
      float gcx = 0.f, gcy = 0.f, gcz = 0.f, gR = 0.f, go = 0.f, gk = 0.f, npx = 0.f;
      const int xa = max(s.x0, tx0), xb = min(int(p1 & 0xffffu), tx0 + kTileW - 1);
      const int ya = max(s.y0, ty0), yb = min(int(p1 >> 16), ty0 + kTileH - 1);
      const float tlo = front_bound(s);
      const uint64_t dkey =
          A.stop ? (uint64_t(__float_as_uint(A.tmin[id])) << 32) | id : 0ull;
      for (int iy = ya; iy <= yb; ++iy) {
        for (int ix = xa; ix <= xb; ++ix) {
          const int pl = (iy - ty0) * kTileW + (ix - tx0);
          const float tk = s_tk[pl];
          if (tlo > tk) continue;  // behind the K-th nearest hit
          if (A.stop && dkey >= s_sk[pl]) continue;  // after the pixel's early stop
          const PixelRay ray = load_ray(s_ray, pl, ix, iy);
          Hit h;
          if (!exact_hit(ray, s, bc.zfar, h)) continue;
          const uint32_t ik = s_ik[pl];
          if (!(id == ik || h.t < tk || (h.t == tk && id < ik))) continue;
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
          if (A.need_pay) {
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
          if (A.need_cam) {
            HitGrad g;
            g.gt = gt;
            g.coef = coef;
            gk += hit_grad_kappa(ray, s, h, cam, g);
          }
          npx += 1.f;
        }
      }
      // dL/dc, dL/dR, dL/do, dL/d(f/s) and the pixel count whole into the
      // pair's slot (the payload terms went out per hit)
      float4* sr = A.pslot + size_t(slot) * size_t(A.ps4);
      sr[0] = make_float4(gcx, gcy, gcz, gR);
      sr[1] = make_float4(go, gk, npx, 0.f);
    }
  }
}

// Before the wide K7: zero the caller's payload-gradient rows it adds into
// per hit (every visible sphere).
__global__ void k_bwd_prep(int n, const uint32_t* __restrict__ counts, int C,
                           float* __restrict__ grad_payload) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || counts[i] == 0u) return;
  for (int c = 0; c < C; ++c) grad_payload[size_t(i) * size_t(C) + c] = 0.f;
}

// A sphere's gradients from its camera-space sums g = (dL/dc, dL/dR), go =
// dL/do, gk = dL/dkappa (count: the tiles it touches, 0 when it is not
// visible; npx: the pixels it received gradients from). Writes its opacity,
// radius and camera-space camera terms and returns its position gradient
// (dL/dp = R^T dL/dc with the min-size clamp) and the factor of its payload
// gradient.
struct SphereGrad {
  float gx, gy, gz;  // dL/dp
  float scale;       // payload-gradient factor (the paper's per-pixel average)
};

__device__ __forceinline__ SphereGrad sphere_grad(int i, uint32_t count, float4 g, float go,
                                                  float gk, float npx, const CamDev& cam,
                                                  const float* __restrict__ pos,
                                                  const float* __restrict__ radius,
                                                  float min_radius_px,
                                                  float* __restrict__ grad_radius,
                                                  float* __restrict__ grad_opacity,
                                                  float4* __restrict__ camg, int paper_norm,
                                                  bool need_pos) {
  SphereGrad o;
  // the paper's optimisation-friendly variant (App. B normalisation, Sec. 7
  // limitation 1): every gradient of a sphere divided by the number of
  // pixels it received gradients from; position and radius gradients only
  // for spheres wider than 3 pixels in radius (R f / (c_z pitch))
  o.scale = (paper_norm && npx > 0.f) ? 1.f / npx : 1.f;
  o.gx = o.gy = o.gz = 0.f;
  if (grad_opacity) grad_opacity[i] = go * o.scale;
  if (!(need_pos || grad_radius || camg)) return o;
  float gx = g.x, gy = g.y, gz = g.z, gR = g.w;
  bool clamped = false, gated = false;
  float cam_scale = 1.f;  // the paper's camera-gradient normalisation
  if (count != 0u && (min_radius_px > 0.f || paper_norm)) {
    const float px = pos[3 * i + 0], py = pos[3 * i + 1], pz = pos[3 * i + 2];
    const double cz = double(cam.R[6]) * px + double(cam.R[7]) * py + double(cam.R[8]) * pz +
                      double(cam.t[2]);
    const double pitch = double(cam.s) / double(cam.W);
    // orthographic: the minimum radius min_radius_px pitch is constant
    const double k = cam.ortho ? 0.0 : double(min_radius_px) * pitch / double(cam.f);
    const double rmin = cam.ortho ? double(min_radius_px) * pitch : k * cz;
    clamped = min_radius_px > 0.f && rmin > double(radius[i]);
    if (clamped && !cam.ortho) {
      gz += float(double(gR) * k);  // R = k c_z depends on depth only
      // and on the camera through k = min_radius_px / (W kappa):
      // dR/dkappa = -R / kappa
      gk -= float(double(gR) * k * cz * double(cam.s) / double(cam.f));
    }
    const double reff = clamped ? rmin : double(radius[i]);
    const double rpx = cam.ortho ? reff / pitch : reff * double(cam.f) / (cz * pitch);
    gated = paper_norm && !(rpx > 3.0);
    // camera gradients: each sphere's part over its projected disk area
    // in pixels, times 1e-3 (App. B, normalisation)
    if (paper_norm) cam_scale = float(1e-3 / (3.141592653589793 * rpx * rpx));
  }
  if (camg) camg[i] = make_float4(gx * cam_scale, gy * cam_scale, gz * cam_scale, gk * cam_scale);
  if (grad_radius) grad_radius[i] = (clamped || gated) ? 0.f : gR * o.scale;
  // c = R p + t  =>  dL/dp = R^T dL/dc
  const float ps = gated ? 0.f : o.scale;
  o.gx = (cam.R[0] * gx + cam.R[3] * gy + cam.R[6] * gz) * ps;
  o.gy = (cam.R[1] * gx + cam.R[4] * gy + cam.R[7] * gz) * ps;
  o.gz = (cam.R[2] * gx + cam.R[5] * gy + cam.R[8] * gz) * ps;
  return o;
}

// The outputs of a block's spheres i0 .. i0 + nloc - 1, thread t holding
// sphere i0 + t (see sphere_grad). Opacity and payload gradients are copied
// out (CM > 0; with CM = 0, the wide path, the payload gradient was added in
// place). Rows wider than one float (positions, payloads) are staged in s_gp
// [3 kFinThreads] and s_pay [kFinThreads CS] and written as one contiguous
// run, so every store instruction covers consecutive addresses. Every thread
// of the block calls it (it holds a barrier).
constexpr int kFinThreads = 256;
template <int CM>
__device__ __forceinline__ void write_sphere_grads(
    int t, int i0, int nloc, uint32_t count, float4 g, float go, float gk, float npx,
    const float (&gf)[CM > 0 ? CM : 1], const CamDev& cam, const float* __restrict__ pos,
    const float* __restrict__ radius, float min_radius_px, int C, float* __restrict__ grad_pos,
    float* __restrict__ grad_radius, float* __restrict__ grad_opacity,
    float* __restrict__ grad_payload, float4* __restrict__ camg, int paper_norm,
    float* __restrict__ s_gp, float* __restrict__ s_pay) {
  constexpr int CS = CM > 0 ? CM : 1;
  const int i = i0 + t;
  float scale = 1.f;
  if (t < nloc) {
    const SphereGrad o = sphere_grad(i, count, g, go, gk, npx, cam, pos, radius, min_radius_px,
                                     grad_radius, grad_opacity, camg, paper_norm,
                                     grad_pos != nullptr);
    scale = o.scale;
    s_gp[3 * t + 0] = o.gx;
    s_gp[3 * t + 1] = o.gy;
    s_gp[3 * t + 2] = o.gz;
  }
  if (CM > 0) {
#pragma unroll
    for (int c = 0; c < CS; ++c) s_pay[t * CS + c] = gf[c] * scale;
  }
  __syncthreads();
  if (grad_pos) {
    float* dst = grad_pos + size_t(i0) * 3;
    for (int f = t; f < 3 * nloc; f += kFinThreads) dst[f] = s_gp[f];
  }
  if (!grad_payload) return;
  if (CM > 0) {
    // element f of the block's [nloc, C] rows: sphere f / C, channel f % C
    float* dst = grad_payload + size_t(i0) * size_t(C);
    const int total = nloc * C;
    const int dsph = kFinThreads / C, dch = kFinThreads % C;
    int sph = t / C, ch = t % C;
    for (int f = t; f < total; f += kFinThreads) {
      dst[f] = s_pay[sph * CS + ch];
      sph += dsph;
      ch += dch;
      if (ch >= C) {
        ch -= C;
        ++sph;
      }
    }
  } else if (t < nloc && count == 0u) {
    // the wide path added into the caller's rows; spheres without a tile get zeros
    for (int c = 0; c < C; ++c) grad_payload[size_t(i) * size_t(C) + c] = 0.f;
  } else if (t < nloc && scale != 1.f) {
    // ... and its per-hit sums take the pixel-count average here
    for (int c = 0; c < C; ++c) grad_payload[size_t(i) * size_t(C) + c] *= scale;
  }
}

// One projection block of K8 (every thread of the block calls it).
template <int CM>
__device__ __forceinline__ void finalize_block(
    uint32_t sb, int t, int n, const uint32_t* __restrict__ counts,
    const unsigned long long* __restrict__ boff, const Status* __restrict__ status,
    const float* __restrict__ pos, const float* __restrict__ radius, const SceneTable& tab,
    float min_radius_px, int C, const float4* __restrict__ pslot, int ps4,
    float* __restrict__ grad_pos, float* __restrict__ grad_radius,
    float* __restrict__ grad_opacity, float* __restrict__ grad_payload,
    float4* __restrict__ camg, int paper_norm, float* s_gp, float* s_pay) {
  constexpr int CS = CM > 0 ? CM : 1;
  __syncthreads();  // the previous block's readers of the LDS are done
  const int i0 = int(sb) * kFinThreads;
  const int nloc = min(kFinThreads, n - i0);
  const int i = i0 + t;
  // the first slot: the projection block's first emission position plus the
  // tile counts of the block's spheres before this one (a block here is a
  // projection block)
  static_assert(kFinThreads == kProjectBlock, "one finalize block per projection block");
  const uint32_t count = t < nloc ? counts[i] : 0u;
  __shared__ uint32_t s_wpre[kFinThreads / kWave];
  const int lane = t & (kWave - 1), wv = t / kWave;
  const uint32_t incl = wave_incl_scan_u32(count, lane);
  if (lane == kWave - 1) s_wpre[wv] = incl;
  __syncthreads();
  uint32_t first = incl - count;
#pragma unroll
  for (int w = 0; w < kFinThreads / kWave; ++w) first += w < wv ? s_wpre[w] : 0u;
  const uint32_t base = count != 0u ? uint32_t(boff[sb]) + first : 0u;
  float4 g = make_float4(0.f, 0.f, 0.f, 0.f);
  float go = 0.f, gk = 0.f, npx = 0.f;
  float gf[CS];
#pragma unroll
  for (int c = 0; c < CS; ++c) gf[c] = 0.f;
  if (count != 0u) {
    // after a capacity overflow (outputs invalid) the slots may be missing
    if (size_t(base) + count <= size_t(status->used)) {
      for (uint32_t k = 0; k < count; ++k) {
        const float4* sr = pslot + size_t(base + k) * size_t(ps4);
        const float4 a = sr[0];
        g.x += a.x;
        g.y += a.y;
        g.z += a.z;
        g.w += a.w;
        if (CM > 0) {
          constexpr int NT = (CM + 6) / 4;
#pragma unroll
          for (int q = 0; q < NT; ++q) {
            const float4 v = sr[1 + q];
            const float vv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int kk = 4 * q + u;
              if (kk < CM)
                gf[kk < CS ? kk : 0] += vv[u];
              else if (kk == CM)
                go += vv[u];
              else if (kk == CM + 1)
                gk += vv[u];
              else if (kk == CM + 2)
                npx += vv[u];
            }
          }
        } else {
          const float4 v = sr[1];
          go += v.x;
          gk += v.y;
          npx += v.z;
        }
      }
    }
  }
  // the sphere's own camera (a projection block may hold spheres of several scenes)
  const CamDev cam = tab.scenes[find_scene(tab.sph_start, tab.B, uint32_t(t < nloc ? i : i0))].cam;
  write_sphere_grads<CM>(t, i0, nloc, count, g, go, gk, npx, gf, cam, pos, radius, min_radius_px,
                         C, grad_pos, grad_radius, grad_opacity, grad_payload, camg, paper_norm,
                         s_gp, s_pay);
}

// K8 after the slot-based backward passes (the wide, stored-hits and
// tile-order ones): per sphere, in sphere order, kFinThreads spheres (a
// projection block) at a time, the first fin_grid blocks walking the nfin
// projection blocks. The camera-space sums are the sum of the sphere's pair
// slots sfirst .. sfirst + count - 1 (in that order; none when it touches no
// tile). With only_if_big those blocks do nothing unless the backward took
// the tile walk (a very large sphere). Blocks past them sum the background block
// sums, one block per (scene, channel).
template <int CM>
__global__ __launch_bounds__(kFinThreads) void k_finalize(
    int n, const uint32_t* __restrict__ counts, const unsigned long long* __restrict__ boff,
    const Status* __restrict__ status, const float* __restrict__ pos,
    const float* __restrict__ radius, SceneTable tab, float min_radius_px, int C,
    const float4* __restrict__ pslot, int ps4, float* __restrict__ grad_pos,
    float* __restrict__ grad_radius, float* __restrict__ grad_opacity,
    float* __restrict__ grad_payload, uint32_t nfin, uint32_t fin_grid, int only_if_big,
    const float* __restrict__ bgsum, float* __restrict__ grad_bg, float4* __restrict__ camg,
    int paper_norm) {
  constexpr int CS = CM > 0 ? CM : 1;
  __shared__ float s_gp[3 * kFinThreads];
  __shared__ float s_pay[kFinThreads * CS];
  const int t = threadIdx.x;
  if (blockIdx.x >= fin_grid) {
    const uint32_t k = blockIdx.x - fin_grid;
    const int c = int(k % uint32_t(C)), b = int(k / uint32_t(C));
    const uint32_t k0 = tab.blk_start[b], k1 = tab.blk_start[b + 1];
    float acc = 0.f;
    for (uint32_t j = k0 + t; j < k1; j += kFinThreads) acc += bgsum[size_t(j) * size_t(C) + c];
    acc = wave_sum(acc);
    __shared__ float s_red[kFinThreads / kWave];
    if ((t & (kWave - 1)) == 0) s_red[t / kWave] = acc;
    __syncthreads();
    if (t == 0) {
      float tsum = 0.f;
      for (int w = 0; w < kFinThreads / kWave; ++w) tsum += s_red[w];
      grad_bg[size_t(b) * size_t(C) + c] = tsum;
    }
    return;
  }
  if (only_if_big && status->big_spheres == 0u) return;
  for (uint32_t sb = blockIdx.x; sb < nfin; sb += fin_grid)
    finalize_block<CM>(sb, t, n, counts, boff, status, pos, radius, tab, min_radius_px, C, pslot,
                       ps4, grad_pos, grad_radius, grad_opacity, grad_payload, camg, paper_norm,
                       s_gp, s_pay);
}


// ---------------------------------------------------------------- K7 by sphere
// The default backward (up to kBwdChannels channels): one thread per sphere,
// in sphere order, kSphThreads spheres of one scene per block. A sphere's
// record, payload row and every output row are read and written as
// contiguous runs, and its gradient never goes through per-pair slots: the
// thread ends with the sphere's sums and writes its outputs itself.
//
// The (sphere, pixel of its rectangle) pairs of a wave are flattened over its
// lanes, 64 at a time, by a prefix sum over rectangle sizes (a pair's sphere
// is found by binary search in that sum), so a wave takes as many rounds as
// its spheres have pixels in all / 64, whatever the size of each. A lane
// gathers its pixel's L, K-th nearest hit and (for a hit among the K
// nearest) G and F, recomputes the hit exactly as the forward did and forms
// its terms; a segmented scan over the lanes adds the terms of each sphere's
// pixels in a fixed order, and the sphere's own lane takes the sum. No
// atomics: the gradients are reproducible bit for bit. The pixels that
// spheres touch lie in the non-empty tiles, which stay in cache. Blocks past
// the spheres compute the background-gradient block sums.
struct BwdSphArgs {
  const Status* status;
  const uint32_t* counts;  // tiles per sphere (0: not visible)
  const float4* rec;       // sphere records, rec4 float4 each
  int rec4;
  const float* payload;
  int C;
  int vec4;  // C % 4 == 0 and 16-byte aligned image rows: float4 row loads
  int pay4;  // the same for the payload rows
  int gpay4;  // ... and for the payload-gradient rows
  const float* pos;
  const float* radius;
  const float* image;
  const float* aux;
  const float* grad_image;
  const float4* thr;  // per pixel: K-th nearest hit (t, sphere index), L, 0
  int l_in_thr;       // thr holds the image's L (else it is read from aux)
  // early termination: each sphere's earliest possible hit distance and per
  // pixel the first hit the forward skipped (hits from it on take no part)
  const float* tmin;
  const float2* stop;
  float* grad_pos;
  float* grad_radius;
  float* grad_opacity;
  float* grad_payload;
  float4* camg;
  float min_radius_px;
  int paper_norm;
  int B;
  uint32_t nsph_blocks;  // blocks of spheres; the blocks after them sum the background
  uint32_t nbgblk;       // background-gradient blocks
  SceneTable tab;
  float* bgsum;  // background-gradient block sums, or null
  float eps2;
};

constexpr int kSphThreads = kFinThreads;
constexpr int kSphPerLane = 1;  // spheres per lane of the sphere-order backward
constexpr uint32_t kFinGridAuto = 1024;  // K8 blocks for the tile walk beside the sphere walk
constexpr long long kBwdGridAuto = 1024;  // tile-walk blocks beside the sphere walk
static_assert(kSphThreads == kBgThreads, "the background blocks share the launch");

// With `span` spheres per block, scene b owns blocks b + sph_off_b / span
// onwards, as many as its spheres need, so a block never spans two scenes (a
// block right after a scene's last may have nothing to do).
__device__ __forceinline__ uint32_t sph_first_block(const SceneDev& sc, int b, uint32_t span) {
  return uint32_t(b) + sc.sph_off / span;
}

// The terms of one (sphere, pixel) pair, added into v = (dL/dc, dL/dR, dL/do,
// dL/dkappa, pixel count, dL/df[CM]) when the pixel's ray hits the sphere
// among its K nearest hits (the same tests, in the same precision, as every
// other raster kernel).
template <int CM, bool CAM, bool ES>
__device__ __forceinline__ void sphere_pixel_terms(const BwdSphArgs& A, const CamDev& cam,
                                                   const BlendConst& bc,
                                                   unsigned long long pix_off,
                                                   const SphereRec& s, const float (&f)[CM],
                                                   uint32_t sph, float tmin, int px, int py,
                                                   float (&v)[7 + CM]) {
  const size_t p = size_t(pix_off) + size_t(py) * size_t(cam.W) + size_t(px);
  // the K-th nearest hit and L in one record (after a rebuild of the
  // thresholds, L from the caller's image)
  const float4 th = A.thr[p];
  const float aux = A.l_in_thr ? th.z : A.aux[p];
  float2 st = make_float2(0.f, 0.f);
  if (ES) st = A.stop[p];
  // behind the pixel's K-th nearest hit: no gradient, no test needed
  if (front_bound(s) > th.x) return;
  // at or after the hit where the pixel stopped: never blended
  if (ES) {
    const uint64_t sk = (uint64_t(__float_as_uint(st.x)) << 32) | __float_as_uint(st.y);
    if (((uint64_t(__float_as_uint(tmin)) << 32) | sph) >= sk) return;
  }
  const PixelRay ray = make_ray(cam, px, py);
  Hit h;
  if (!exact_hit(ray, s, bc.zfar, h)) return;
  // among the pixel's K nearest: (t, sphere index) up to its K-th
  const uint32_t ik = __float_as_uint(th.y);
  if (!(sph == ik || h.t < th.x || (h.t == th.x && sph < ik))) return;
  const int C = A.C;
  float G[CM], F[CM];
  if (A.vec4) {
    const float4* g4 = reinterpret_cast<const float4*>(A.grad_image + p * size_t(C));
    const float4* f4 = reinterpret_cast<const float4*>(A.image + p * size_t(C));
#pragma unroll
    for (int q = 0; q < (CM + 3) / 4; ++q) {
      const int qq = min(q, C / 4 - 1);  // rows hold C / 4 float4
      const float4 a = g4[qq], b = f4[qq];
      const float ga[4] = {a.x, a.y, a.z, a.w}, fa[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (4 * q + u < CM) {
          G[4 * q + u] = 4 * q + u < C ? ga[u] : 0.f;
          F[4 * q + u] = 4 * q + u < C ? fa[u] : 0.f;
        }
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < CM; ++c) {
      G[c] = A.grad_image[p * size_t(C) + size_t(min(c, C - 1))];
      F[c] = A.image[p * size_t(C) + size_t(min(c, C - 1))];
    }
#pragma unroll
    for (int c = 0; c < CM; ++c) {
      G[c] = c < C ? G[c] : 0.f;
      F[c] = c < C ? F[c] : 0.f;
    }
  }
  // G . (f_k - F), as G . f_k - G . F
  float gfp = 0.f;
#pragma unroll
  for (int c = 0; c < CM; ++c) gfp += G[c] * F[c];
  float hs = -gfp;
#pragma unroll
  for (int c = 0; c < CM; ++c) hs += G[c] * f[c];
  const HitGrad g = hit_grad(ray, s, h, cam, bc, aux * 1.4426950408889634f, hs);
  v[0] += g.gcx;
  v[1] += g.gcy;
  v[2] += g.gcz;
  v[3] += g.gR;
  v[4] += g.go;
  if (CAM) v[5] += hit_grad_kappa(ray, s, h, cam, g);
  v[6] += 1.f;
#pragma unroll
  for (int c = 0; c < CM; ++c) v[7 + c] += g.w * G[c];
}

// SPL spheres per lane: a block covers SPL kSphThreads spheres, lane t of
// wave w taking spheres t, t + kSphThreads, ... of it, and a wave's pairs are
// flattened over its SPL 64 spheres at once.
template <int CM, bool CAM, bool ES, int SPL>
__device__ __forceinline__ void bwd_spheres_body(const BwdSphArgs& A,
                                                 const SceneDev* __restrict__ scenes) {
  constexpr int NV = 7 + CM;                   // dL/dc (3), dL/dR, dL/do, dL/dkappa, count, dL/df
  constexpr int RW = 16 + CM + (ES ? 1 : 0);   // staged words per sphere: record, payload, t_min
  constexpr int RS = (RW + 3) & ~3;            // row stride in floats (16-byte rows)
  constexpr int SB = SPL * kSphThreads;        // spheres per block
  constexpr int NVL = SPL * kWave;             // a wave's spheres
  static_assert(RS * SB >= kBgScratch, "the background sums fit the stage");
  __shared__ float4 s_stage4[RS / 4 * SB];
  float* s_stage = reinterpret_cast<float*>(s_stage4);
  const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
  const uint32_t g = blockIdx.x;
  if (g >= A.nsph_blocks) {
    if (A.bgsum && g - A.nsph_blocks < A.nbgblk)
      bg_partial_block(A.tab, A.aux, A.grad_image, A.C, A.eps2, A.bgsum, g - A.nsph_blocks,
                       s_stage);
    return;
  }
  // the block's scene (uniform: its camera comes in through scalar loads)
  int lo = 0, hi = A.B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sph_first_block(scenes[mid], mid, SB) <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const SceneDev& sc = scenes[lo];
  const uint32_t local = g - sph_first_block(sc, lo, SB);
  if (local >= (sc.n + uint32_t(SB) - 1u) / uint32_t(SB)) return;  // the whole block
  const int i0 = int(sc.sph_off + local * uint32_t(SB));
  const int nloc = int(min(uint32_t(SB), sc.sph_off + sc.n - uint32_t(i0)));
  const CamDev cam = sc.cam;
  const BlendConst bc = sc.bc;
  const unsigned long long pix_off = sc.pix_off;
  const int C = A.C;
  const bool ok = A.status->code == 0u;
  // the spheres: their tile counts (none after a capacity overflow, whose
  // outputs are invalid anyway), then the record and payload row of each
  // visible one (an invisible sphere has no record; most spheres of a scene
  // can be invisible, and skipping their reads saves more than the extra
  // round trip costs), staged in LDS
  uint32_t count[SPL];
#pragma unroll
  for (int u = 0; u < SPL; ++u) {
    const int ts = u * kSphThreads + t;
    count[u] = A.counts[ts < nloc ? i0 + ts : i0];
    count[u] = (ts < nloc && ok) ? count[u] : 0u;
  }
  uint32_t npx[SPL];
#pragma unroll
  for (int u = 0; u < SPL; ++u) {
    const int ts = u * kSphThreads + t;
    const int i = ts < nloc ? i0 + ts : i0;
    float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb = ra, rc = ra, rd = ra;
    float f[CM];
#pragma unroll
    for (int c = 0; c < CM; ++c) f[c] = 0.f;
    float tm = 0.f;
    if (count[u] != 0u) {
      const float4* rp = A.rec + size_t(A.rec4) * size_t(i);
      ra = rp[0];
      rb = rp[1];
      rc = rp[2];
      rd = rp[3];
      if (A.pay4) {
        const float4* f4 = reinterpret_cast<const float4*>(A.payload + size_t(i) * size_t(C));
#pragma unroll
        for (int q = 0; q < (CM + 3) / 4; ++q) {
          const float4 v = f4[min(q, C / 4 - 1)];
          const float va[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int w = 0; w < 4; ++w)
            if (4 * q + w < CM) f[4 * q + w] = va[w];
        }
      } else {
#pragma unroll
        for (int c = 0; c < CM; ++c)
          f[c] = A.payload[size_t(i) * size_t(C) + size_t(min(c, C - 1))];
      }
      if (ES) tm = A.tmin[i];
    }
    float* my = s_stage + ts * RS;
    reinterpret_cast<float4*>(my)[0] = ra;
    reinterpret_cast<float4*>(my)[1] = rb;
    reinterpret_cast<float4*>(my)[2] = rc;
    reinterpret_cast<float4*>(my)[3] = rd;
#pragma unroll
    for (int c = 0; c < CM; ++c) my[16 + c] = c < C ? f[c] : 0.f;
    if (ES) my[16 + CM] = tm;
    const uint32_t p0 = __float_as_uint(ra.w), p1 = __float_as_uint(rd.z);
    npx[u] = count[u] != 0u ? ((p1 & 0xffffu) - (p0 & 0xffffu) + 1u) *
                                  ((p1 >> 16) - (p0 >> 16) + 1u)
                            : 0u;
  }
  // each wave reads only its own rows of the stage: a wave-level barrier
  // (LDS operations of one wave complete in order)
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // this wave's pairs: sphere v = u 64 + lane owns pairs start[u] ..
  // start[u] + npx[u] - 1 (all of slot 0's spheres, then slot 1's, ...)
  uint32_t incl[SPL], start[SPL];
  uint32_t total = 0;
#pragma unroll
  for (int u = 0; u < SPL; ++u) {
    incl[u] = total + wave_incl_scan_u32(npx[u], lane);
    start[u] = incl[u] - npx[u];
    total = __builtin_amdgcn_readlane(incl[u], kWave - 1);
  }
  // a wave-level value of sphere v (v < NVL) from its lane
  auto at_sphere = [&](const uint32_t (&x)[SPL], int v) {
    uint32_t r = 0;
#pragma unroll
    for (int u = 0; u < SPL; ++u) {
      const uint32_t y = __shfl(x[u], v & (kWave - 1), kWave);
      r = (v >> 6) == u ? y : r;
    }
    return r;
  };
  float acc[SPL][NV];
#pragma unroll
  for (int u = 0; u < SPL; ++u)
#pragma unroll
    for (int q = 0; q < NV; ++q) acc[u][q] = 0.f;
  for (uint32_t pb = 0; pb < total; pb += kWave) {
    const uint32_t j = pb + uint32_t(lane);
    const bool act = j < total;
    // the pair's sphere: the number of spheres whose pairs end at or before it
    int o = 0;
#pragma unroll
    for (int step = NVL / 2; step > 0; step >>= 1) {
      const uint32_t e = at_sphere(incl, o + step - 1);
      if (e <= j) o += step;
    }
    o = min(o, NVL - 1);  // lanes past the end
    const uint32_t ostart = at_sphere(start, o);
    const int orow = (o >> 6) * kSphThreads + wv * kWave + (o & (kWave - 1));
    float v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = 0.f;
    if (act) {
      const float* r = s_stage + orow * RS;
      const float4 a = reinterpret_cast<const float4*>(r)[0];
      const float4 b = reinterpret_cast<const float4*>(r)[1];
      const float4 c = reinterpret_cast<const float4*>(r)[2];
      const float4 d = reinterpret_cast<const float4*>(r)[3];
      float fo[CM];
#pragma unroll
      for (int q = 0; q < CM; ++q) fo[q] = r[16 + q];
      const float to = ES ? r[16 + CM] : 0.f;
      const SphereRec s = unpack_rec(a, b, c, d);
      const uint32_t q1 = __float_as_uint(d.z);
      const uint32_t w = (q1 & 0xffffu) - uint32_t(s.x0) + 1u;
      const uint32_t k = j - ostart;
      const uint32_t yy = k / w;
      const int px = s.x0 + int(k - yy * w), py = s.y0 + int(yy);
      sphere_pixel_terms<CM, CAM, ES>(A, cam, bc, pix_off, s, fo, uint32_t(i0 + orow), to, px,
                                      py, v);
    }
    // segmented inclusive scan over the lanes: a lane adds the partial sum of
    // the lane `off` below while both belong to the same sphere
    const uint32_t key = act ? uint32_t(o) : uint32_t(NVL + lane);
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t ku = __shfl_up(key, off, kWave);
      const bool add = lane >= off && ku == key;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const float x = __shfl_up(v[q], off, kWave);
        v[q] = add ? v[q] + x : v[q];
      }
    }
    // each sphere takes the sum at the last lane of its run in this round
#pragma unroll
    for (int u = 0; u < SPL; ++u) {
      const bool has = npx[u] != 0u && start[u] < pb + kWave && start[u] + npx[u] > pb;
      const int tail = has ? int(min(start[u] + npx[u], pb + kWave) - 1u - pb) : lane;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const float x = __shfl(v[q], tail, kWave);
        acc[u][q] = has ? acc[u][q] + x : acc[u][q];
      }
    }
  }
  // the spheres' outputs, each lane its own rows (a wave's position rows are
  // one run of 768 bytes, its payload rows one of 256 C bytes)
#pragma unroll
  for (int u = 0; u < SPL; ++u) {
    const int ts = u * kSphThreads + t;
    if (ts >= nloc) continue;
    const int i = i0 + ts;
    const SphereGrad o = sphere_grad(i, count[u], make_float4(acc[u][0], acc[u][1], acc[u][2],
                                                              acc[u][3]),
                                     acc[u][4], acc[u][5], acc[u][6], cam, A.pos, A.radius,
                                     A.min_radius_px, A.grad_radius, A.grad_opacity, A.camg,
                                     A.paper_norm, A.grad_pos != nullptr);
    if (A.grad_pos) {
      A.grad_pos[3 * size_t(i) + 0] = o.gx;
      A.grad_pos[3 * size_t(i) + 1] = o.gy;
      A.grad_pos[3 * size_t(i) + 2] = o.gz;
    }
    if (A.grad_payload) {
      float* gp = A.grad_payload + size_t(i) * size_t(C);
      if (A.gpay4) {
#pragma unroll
        for (int q = 0; q < (CM + 3) / 4; ++q)
          if (4 * q < C)
            reinterpret_cast<float4*>(gp)[q] =
                make_float4(acc[u][7 + min(4 * q, CM - 1)] * o.scale,
                            acc[u][7 + min(4 * q + 1, CM - 1)] * o.scale,
                            acc[u][7 + min(4 * q + 2, CM - 1)] * o.scale,
                            acc[u][7 + min(4 * q + 3, CM - 1)] * o.scale);
      } else {
#pragma unroll
        for (int c = 0; c < CM; ++c)
          if (c < C) gp[c] = acc[u][7 + c] * o.scale;
      }
    }
  }
}

// The default backward launches both walks; each reads on the device whether
// the emission found a sphere wider than kBigTiles tiles (whose pixels the
// walk in sphere order would all give to one wave) and returns at once when
// the other walk is the one to run, so one launch sequence (and one graph)
// serves every scene. With such a sphere the walk over the tile lists runs,
// and k_finalize adds its per-pair slots.
template <int CM, bool CAM, bool ES, int SPL>
__global__ __launch_bounds__(kSphThreads) void k_bwd_spheres(BwdSphArgs A,
                                                             const SceneDev* __restrict__ scenes) {
  if (A.status->big_spheres != 0u) return;
  bwd_spheres_body<CM, CAM, ES, SPL>(A, scenes);
}

// The block sum for background block `blk`, by a whole block of kBgThreads
// threads (called uniformly; it starts with a barrier so a block can run it
// for several blocks in a row).
__device__ void bg_partial_block(const SceneTable& tab, const float* __restrict__ aux,
                                 const float* __restrict__ grad_image, int C, float eps2,
                                 float* __restrict__ bgsum, uint32_t blk, float* scratch) {
  float* s_w = scratch;                          // [kBgBlockPixels]
  float* s_acc = scratch + kBgBlockPixels;       // [kBgThreads]
  float* s_acc4_buf = s_acc + kBgThreads;        // [4 kBgThreads]
  const int tid = threadIdx.x;
  __syncthreads();  // the previous call's readers are done with the LDS
  const int b = find_scene(tab.blk_start, tab.B, blk);
  const SceneDev& sc = tab.scenes[b];
  const long long npix = (long long)sc.cam.W * sc.cam.H;
  const long long p0 = (long long)(blk - sc.bgblk_off) * kBgBlockPixels;
  const int np = int(min((long long)kBgBlockPixels, npix - p0));
  const float* auxs = aux + sc.pix_off + p0;
  const float* gs = grad_image + (size_t(sc.pix_off) + size_t(p0)) * size_t(C);
  for (int k = tid; k < kBgBlockPixels; k += kBgThreads)
    s_w[k] = k < np ? fast_exp2(eps2 - auxs[k] * 1.4426950408889634f) : 0.f;
  __syncthreads();
  const int cq = C / 4;
  if ((C & 3) == 0 && cq <= kWave && (cq & (cq - 1)) == 0 &&
      (reinterpret_cast<uintptr_t>(gs) & 15u) == 0u) {
    // the same in float4 units: thread t always sees channels 4 (t mod C/4) ..
    // 4 (t mod C/4) + 3; C/4 is a power of two, so lanes of one channel group
    // stay together under xor shuffles by multiples of C/4
    const int S4 = (kBgThreads / cq) * cq;
    const int step4 = S4 / cq;
    float4 acc4 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (tid < S4) {
      const float4* g4 = reinterpret_cast<const float4*>(gs);
      const int total4 = np * cq;
      int pix = tid / cq;
      int f = tid;
      for (; f + 3 * S4 < total4; f += 4 * S4, pix += 4 * step4) {
        float4 g[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) g[u] = g4[f + u * S4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float w = s_w[pix + u * step4];
          acc4.x += w * g[u].x;
          acc4.y += w * g[u].y;
          acc4.z += w * g[u].z;
          acc4.w += w * g[u].w;
        }
      }
      for (; f < total4; f += S4, pix += step4) {
        const float4 g = g4[f];
        const float w = s_w[pix];
        acc4.x += w * g.x;
        acc4.y += w * g.y;
        acc4.z += w * g.z;
        acc4.w += w * g.w;
      }
    }
    for (int off = kWave / 2; off >= cq; off >>= 1) {
      acc4.x += __shfl_xor(acc4.x, off, kWave);
      acc4.y += __shfl_xor(acc4.y, off, kWave);
      acc4.z += __shfl_xor(acc4.z, off, kWave);
      acc4.w += __shfl_xor(acc4.w, off, kWave);
    }
    // lane l < C/4 of each wave now holds its wave's sums for group l
    const int lane = tid % kWave, wv = tid / kWave;
    if (lane < cq) {
      float* dst = s_acc4_buf + (wv * cq + lane) * 4;
      dst[0] = acc4.x;
      dst[1] = acc4.y;
      dst[2] = acc4.z;
      dst[3] = acc4.w;
    }
    __syncthreads();
    if (tid < C) {
      float t = 0.f;
      for (int w = 0; w < kBgThreads / kWave; ++w) t += s_acc4_buf[(w * cq + tid / 4) * 4 + (tid & 3)];
      bgsum[size_t(blk) * size_t(C) + tid] = t;
    }
    return;
  }
  const int S = (kBgThreads / C) * C;  // threads in use, a multiple of C
  const int step = S / C;               // pixels advanced per round
  float acc = 0.f;
  if (tid < S) {
    const int total = np * C;
    int pix = tid / C;
    int f = tid;
    // eight independent loads in flight per round
    for (; f + 7 * S < total; f += 8 * S, pix += 8 * step) {
      float g[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) g[u] = gs[f + u * S];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += s_w[pix + u * step] * g[u];
    }
    for (; f < total; f += S, pix += step) acc += s_w[pix] * gs[f];
  }
  s_acc[tid] = acc;
  __syncthreads();
  // two-stage per-channel sum of the S partials: `split` runs per channel
  // (split * C <= kBgThreads), then one thread per channel adds its runs
  const int split = min(16, kBgThreads / C);
  float part = 0.f;
  if (tid < C * split) {
    const int c = tid % C, r = tid / C;
    for (int k = c + C * r; k < S; k += C * split) part += s_acc[k];
  }
  __syncthreads();
  if (tid < C * split) s_acc[tid] = part;
  __syncthreads();
  if (tid < C) {
    float t = 0.f;
    for (int r = 0; r < split; ++r) t += s_acc[tid + C * r];
    bgsum[size_t(blk) * size_t(C) + tid] = t;
  }
}

__global__ __launch_bounds__(kBgThreads) void k_bg_partial(SceneTable tab,
                                                           const float* __restrict__ aux,
                                                           const float* __restrict__ grad_image,
                                                           int C, float eps2,
                                                           float* __restrict__ bgsum) {
  __shared__ float s_bg[kBgScratch];
  bg_partial_block(tab, aux, grad_image, C, eps2, bgsum, blockIdx.x, s_bg);
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

// PULSAR_STORE_HITS: every slot of the call starts at zero (the hits add
// into them).
__global__ __launch_bounds__(256) void k_zero_slots(const Status* __restrict__ status,
                                                    float4* __restrict__ pslot, int ps4) {
  if (status->code != 0u) return;
  const size_t total = size_t(status->used) * size_t(ps4);
  for (size_t k = size_t(blockIdx.x) * 256 + threadIdx.x; k < total; k += size_t(gridDim.x) * 256)
    pslot[k] = make_float4(0.f, 0.f, 0.f, 0.f);
}

// PULSAR_STORE_HITS backward (App. B keeps each pixel's nearest hits from the
// forward): one wave per non-empty tile, lane p = pixel p. Each of the pixel's stored K
// nearest hits names its sphere; the hit's geometry is recomputed from the
// sphere's record with the same hit test and gradient terms as k_bwd_items,
// and its terms are added with float atomics into the slot of its (tile,
// sphere) pair, which k_finalize then sums per sphere. CM = 0: payloads wider
// than the register budget, whose terms go into the caller's rows (zeroed by
// k_bwd_prep) and whose slots hold dL/dc, dL/dR | dL/do, dL/d(f/s), count.
template <int CM, bool CAM>
__global__ __launch_bounds__(kWave) void k_bwd_hits(BwdKernelArgs A,
                                                    const SceneDev* __restrict__ scenes,
                                                    const uint32_t* __restrict__ tile_start) {
  constexpr int CS = CM > 0 ? CM : 1;
  const int lane = threadIdx.x;
  // a workspace whose forward stored no hits (or other ones): nothing is read
  if (A.status->code != 0u) return;
  if (A.status->hits_k != uint32_t(A.K)) {
    if (blockIdx.x == 0 && lane == 0)
      A.status->code = uint32_t(-PULSAR_ERR_INVALID_ARGUMENT);
    return;
  }
  const int C = A.C;
  for (uint32_t tile = blockIdx.x; tile < A.T; tile += gridDim.x) {
    // a tile no sphere touches was filled with the background, and its
    // pixels' hit entries were never written: nothing to read there
    if (A.tinfo[tile].y == 0u) continue;
    const TileScene ts = tile_scene(scenes, tile_start, A.tab.B, tile);
    const SceneDev& sc = scenes[ts.b];
    const CamDev cam = sc.cam;
    const BlendConst bc = sc.bc;
    const int px = ts.tx0 + lane % kTileW, py = ts.ty0 + lane / kTileW;
    if (px >= cam.W || py >= cam.H) continue;
    const size_t p = size_t(sc.pix_off) + size_t(py) * size_t(cam.W) + size_t(px);
    const uint2* hp = A.hits + p * size_t(A.K);
    if (hp[0].y == 0xffffffffu) continue;  // no hit at all
    const int ttx = ts.tx0 / kTileW, tty = ts.ty0 / kTileH;
    const PixelRay ray = make_ray(cam, px, py);
    const float L2 = A.aux[p] * 1.4426950408889634f;
    const float* Gp = A.grad_image + p * size_t(C);
    const float* Fp = A.image + p * size_t(C);
    float G[CS], gf0 = 0.f;
    if (CM > 0) {
#pragma unroll
      for (int c = 0; c < CS; ++c) G[c] = c < C ? Gp[c] : 0.f;
#pragma unroll
      for (int c = 0; c < CS; ++c) gf0 += c < C ? G[c] * Fp[c] : 0.f;
    }
    for (int j = 0; j < A.K; ++j) {
      const uint2 e = hp[j];
      if (e.y == 0xffffffffu) break;  // fewer than K hits
      const uint32_t sph = min(e.y, A.last_sph);
      const float4* rp = A.rec + size_t(A.rec4) * size_t(sph);
      const float4 ra = rp[0], rd = rp[3];
      const SphereRec s = unpack_rec(ra, rp[1], rp[2], rd);
      Hit h;
      if (!exact_hit(ray, s, bc.zfar, h)) continue;  // never, for a stored hit
      const float* fk = A.payload + size_t(sph) * size_t(C);
      float hs = 0.f;
      if (CM > 0) {
        hs = -gf0;
#pragma unroll
        for (int c = 0; c < CS; ++c) hs += c < C ? G[c] * fk[c] : 0.f;
      } else {
        for (int c = 0; c < C; ++c) hs += Gp[c] * (fk[c] - Fp[c]);
      }
      const HitGrad g = hit_grad(ray, s, h, cam, bc, L2, hs);
      const float gk = CAM ? hit_grad_kappa(ray, s, h, cam, g) : 0.f;
      const uint32_t slot =
          pair_position(ra, rd, uint32_t(A.boff[sph / kProjectBlock]), ttx, tty);
      float* sr = reinterpret_cast<float*>(A.pslot + size_t(slot) * size_t(A.ps4));
      atomicAdd(sr + 0, g.gcx);
      atomicAdd(sr + 1, g.gcy);
      atomicAdd(sr + 2, g.gcz);
      atomicAdd(sr + 3, g.gR);
      if (CM > 0) {
#pragma unroll
        for (int c = 0; c < CS; ++c)
          if (c < C) atomicAdd(sr + 4 + c, g.w * G[c]);
        atomicAdd(sr + 4 + CM, g.go);
        if (CAM) atomicAdd(sr + 5 + CM, gk);
        atomicAdd(sr + 6 + CM, 1.f);
      } else {
        if (A.need_pay) {
          float* gp = A.grad_payload + size_t(sph) * size_t(C);
          for (int c = 0; c < C; ++c) atomicAdd(gp + c, g.w * Gp[c]);
        }
        atomicAdd(sr + 4, g.go);
        if (CAM) atomicAdd(sr + 5, gk);
        atomicAdd(sr + 6, 1.f);
      }
    }
  }
}

template <int CM>
static void launch_hits(const BwdKernelArgs& A, unsigned grid, hipStream_t stream) {
  if (A.need_cam)
    hipLaunchKernelGGL((k_bwd_hits<CM, true>), dim3(grid), dim3(kWave), 0, stream, A,
                       A.tab.scenes, A.tab.tile_start);
  else
    hipLaunchKernelGGL((k_bwd_hits<CM, false>), dim3(grid), dim3(kWave), 0, stream, A,
                       A.tab.scenes, A.tab.tile_start);
}

template <int CM, bool ES>
static void launch_items_es(const BwdKernelArgs& A, dim3 grid, dim3 block, hipStream_t stream) {
  if (A.need_cam)
    hipLaunchKernelGGL((k_bwd_items<CM, true, ES>), grid, block, 0, stream, A, A.tab.scenes,
                       A.tab.tile_start, A.desc);
  else
    hipLaunchKernelGGL((k_bwd_items<CM, false, ES>), grid, block, 0, stream, A, A.tab.scenes,
                       A.tab.tile_start, A.desc);
}

template <int CM>
static void launch_items(const BwdKernelArgs& A, dim3 grid, dim3 block, hipStream_t stream) {
  if (A.stop)
    launch_items_es<CM, true>(A, grid, block, stream);
  else
    launch_items_es<CM, false>(A, grid, block, stream);
}

template <int CM>
static void launch_finalize(const Plan& q, const BwdArgs& a, char* ws, hipStream_t stream,
                            uint32_t nfin, uint32_t fin_grid, int only_if_big, uint32_t nred) {
  hipLaunchKernelGGL((k_finalize<CM>), dim3(fin_grid + nred), dim3(kFinThreads), 0, stream,
                     int(q.n), ws_ptr<uint32_t>(ws, q.off_counts),
                     ws_ptr<unsigned long long>(ws, q.off_boff), ws_ptr<Status>(ws, q.off_status),
                     a.pos, a.radius, scene_table(q, ws), a.min_radius_px, a.C,
                     ws_ptr<float4>(ws, q.off_pslot), q.bwd_ps4, a.grad_pos, a.grad_radius,
                     a.grad_opacity, a.grad_payload, nfin, fin_grid, only_if_big,
                     ws_ptr<float>(ws, q.off_bgsum), a.grad_bg,
                     a.grad_cam ? ws_ptr<float4>(ws, q.off_camg) : nullptr, a.paper_norm ? 1 : 0);
}

template <int CM, bool CAM>
static void launch_spheres_cam(const BwdSphArgs& S, unsigned grid, const SceneDev* scenes,
                               hipStream_t stream) {
  if (S.stop)
    hipLaunchKernelGGL((k_bwd_spheres<CM, CAM, true, kSphPerLane>), dim3(grid),
                       dim3(kSphThreads), 0, stream, S, scenes);
  else
    hipLaunchKernelGGL((k_bwd_spheres<CM, CAM, false, kSphPerLane>), dim3(grid),
                       dim3(kSphThreads), 0, stream, S, scenes);
}

template <int CM>
static void launch_spheres(const BwdSphArgs& S, bool cam, unsigned grid, const SceneDev* scenes,
                           hipStream_t stream) {
  if (cam)
    launch_spheres_cam<CM, true>(S, grid, scenes, stream);
  else
    launch_spheres_cam<CM, false>(S, grid, scenes, stream);
}

// Camera gradients: dL/dR = sum_i dL/dc_i p_i^T, dL/dt = sum_i dL/dc_i and
// dL/dkappa = sum_i dL/dkappa_i over each scene's spheres (c = R p + t),
// in FP64 and in a fixed order. K9a: block g adds kCamSpan spheres of one
// scene (scene b owns blocks b + sph_off_b / kCamSpan onwards, as many as
// its spheres need; blocks in the gaps do nothing). K9b: one block per scene
// adds its block sums (strided over threads, then a fixed tree) and maps
// dL/dkappa to the focal length and the sensor width (kappa = f / s).
constexpr int kCamThreads = 256;
constexpr int kCamVals = 13;  // R (9), t (3), kappa

__device__ __forceinline__ uint32_t cam_first_block(const SceneDev& sc, int b) {
  return uint32_t(b) + sc.sph_off / uint32_t(kCamSpan);
}

__global__ __launch_bounds__(kCamThreads) void k_cam_partial(const SceneDev* __restrict__ scenes,
                                                             int B, const float4* __restrict__ camg,
                                                             const float* __restrict__ pos,
                                                             double* __restrict__ part) {
  __shared__ double s_acc[kCamVals][kCamThreads];
  const uint32_t g = blockIdx.x;
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cam_first_block(scenes[mid], mid) <= g)
      lo = mid;
    else
      hi = mid - 1;
  }
  const SceneDev& sc = scenes[lo];
  const uint32_t local = g - cam_first_block(sc, lo);
  const uint32_t nblk = (sc.n + uint32_t(kCamSpan) - 1u) / uint32_t(kCamSpan);
  if (local >= nblk) return;  // the whole block: no barrier is reached
  const uint32_t i0 = sc.sph_off + local * uint32_t(kCamSpan);
  const uint32_t i1 = min(i0 + uint32_t(kCamSpan), sc.sph_off + sc.n);
  double acc[kCamVals];
#pragma unroll
  for (int k = 0; k < kCamVals; ++k) acc[k] = 0.0;
  for (uint32_t i = i0 + threadIdx.x; i < i1; i += kCamThreads) {
    const float4 gc = camg[i];
    const double c[3] = {gc.x, gc.y, gc.z};
    const double p[3] = {pos[3 * size_t(i)], pos[3 * size_t(i) + 1], pos[3 * size_t(i) + 2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int b = 0; b < 3; ++b) acc[3 * a + b] += c[a] * p[b];
      acc[9 + a] += c[a];
    }
    acc[12] += double(gc.w);
  }
  const int t = threadIdx.x;
#pragma unroll
  for (int k = 0; k < kCamVals; ++k) s_acc[k][t] = acc[k];
  __syncthreads();
  for (int w = kCamThreads / 2; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int k = 0; k < kCamVals; ++k) s_acc[k][t] += s_acc[k][t + w];
    __syncthreads();
  }
  if (t < kCamVals) part[size_t(g) * 16 + size_t(t)] = s_acc[t][0];
}

__global__ __launch_bounds__(kCamThreads) void k_cam_final(const SceneDev* __restrict__ scenes,
                                                          const double* __restrict__ part,
                                                          float* __restrict__ grad_cam) {
  __shared__ double s_acc[kCamVals][kCamThreads];
  const int b = blockIdx.x, t = threadIdx.x;
  const SceneDev& sc = scenes[b];
  const uint32_t first = cam_first_block(sc, b);
  const uint32_t nblk = (sc.n + uint32_t(kCamSpan) - 1u) / uint32_t(kCamSpan);
  // thread t adds block sums t, t + kCamThreads, ...; then a fixed tree
  double acc[kCamVals];
#pragma unroll
  for (int k = 0; k < kCamVals; ++k) acc[k] = 0.0;
  for (uint32_t j = uint32_t(t); j < nblk; j += kCamThreads) {
    const double* pj = part + size_t(first + j) * 16;
#pragma unroll
    for (int k = 0; k < kCamVals; ++k) acc[k] += pj[k];
  }
#pragma unroll
  for (int k = 0; k < kCamVals; ++k) s_acc[k][t] = acc[k];
  __syncthreads();
  for (int w = kCamThreads / 2; w > 0; w >>= 1) {
    if (t < w)
#pragma unroll
      for (int k = 0; k < kCamVals; ++k) s_acc[k][t] += s_acc[k][t + w];
    __syncthreads();
  }
  if (t < 14) {
    const double f = sc.cam.f, s = sc.cam.s, gk = s_acc[12][0];
    // kappa = f / s: dL/df = dL/dkappa / s, dL/ds = -dL/dkappa f / s^2
    const double v = t < 12 ? s_acc[t][0] : (t == 12 ? gk / s : -gk * f / (s * s));
    grad_cam[size_t(b) * 14 + size_t(t)] = float(v);
  }
}

hipError_t launch_backward(const Plan& q, const BwdArgs& a, char* ws, hipStream_t stream) {
  const bool wide = a.C > kBwdChannels;
  const SceneTable tab = scene_table(q, ws);
  BwdKernelArgs A;
  A.only_if_big = 0;
  A.tab = tab;
  A.status = ws_ptr<Status>(ws, q.off_status);
  A.desc = ws_ptr<uint4>(ws, q.off_desc);
  A.max_items = uint32_t(q.max_chunks);
  A.rec = ws_ptr<float4>(ws, q.off_rec);
  A.rec4 = q.rec4;
  A.payload = a.payload;
  A.boff = ws_ptr<unsigned long long>(ws, q.off_boff);
  A.image = a.image;
  A.aux = a.aux;
  A.grad_image = a.grad_image;
  A.thr = ws_ptr<float4>(ws, q.off_thr);
  A.pslot = ws_ptr<float4>(ws, q.off_pslot);
  A.ps4 = q.bwd_ps4;
  A.svals = ws_ptr<uint32_t>(ws, q.off_vals);
  A.last_sph = q.n > 0 ? uint32_t(q.n - 1) : 0u;
  A.grad_payload = a.grad_payload;
  A.C = a.C;
  A.need_geo = (a.grad_pos || a.grad_radius || a.grad_cam) ? 1 : 0;
  A.need_cam = a.grad_cam ? 1 : 0;
  A.need_op = a.grad_opacity ? 1 : 0;
  A.need_pay = a.grad_payload ? 1 : 0;
  // the narrow raster kernel also computes the background block sums
  A.bgsum = (a.grad_bg && !wide) ? ws_ptr<float>(ws, q.off_bgsum) : nullptr;
  A.nbgblk = uint32_t(q.nbgblk);
  A.eps2 = a.eps2;
  A.tmin = q.estop ? ws_ptr<float>(ws, q.off_tmin) : nullptr;
  A.stop = q.estop ? ws_ptr<float2>(ws, q.off_stop) : nullptr;
  A.hits = q.store_hits ? ws_ptr<uint2>(ws, q.off_hits) : nullptr;
  A.tinfo = ws_ptr<uint4>(ws, q.off_tinfo);
  A.K = q.K;
  A.T = uint32_t(q.T);
  const bool store = q.store_hits != 0;
  // the default: the walk in sphere order, which writes the outputs itself
  const bool by_sphere = !wide && !store && !q.bwd_tiles;
  // the pair-parallel kernel also computes the background block sums
  if (store) A.bgsum = nullptr;
  float* bgsum = ws_ptr<float>(ws, q.off_bgsum);
  const uint32_t* counts = ws_ptr<uint32_t>(ws, q.off_counts);
  // clearing before the raster pass (only the wide and stored-hits passes add into memory)
  const bool prep = wide && a.grad_payload && q.n > 0;
  if (prep || store) {
    stage_begin(PULSAR_STAGE_ZERO, stream);
    if (prep)
      hipLaunchKernelGGL(k_bwd_prep, dim3(unsigned((q.n + 255) / 256)), dim3(256), 0, stream,
                         int(q.n), counts, a.C, a.grad_payload);
    if (store)
      hipLaunchKernelGGL(k_zero_slots, dim3(1024), dim3(256), 0, stream, A.status, A.pslot,
                         A.ps4);
    stage_end(PULSAR_STAGE_ZERO, stream);
  }
  stage_begin(PULSAR_STAGE_RASTER_BWD, stream);
  if (store) {
    const unsigned hg = unsigned(q.T < q.raster_grid ? q.T : q.raster_grid);
    if (a.C <= 1)
      launch_hits<1>(A, hg, stream);
    else if (a.C <= 2)
      launch_hits<2>(A, hg, stream);
    else if (a.C <= 4)
      launch_hits<4>(A, hg, stream);
    else if (a.C <= 8)
      launch_hits<8>(A, hg, stream);
    else if (a.C <= 16)
      launch_hits<16>(A, hg, stream);
    else if (!wide)
      launch_hits<32>(A, hg, stream);
    else
      launch_hits<0>(A, hg, stream);
  } else if (by_sphere) {
    BwdSphArgs S;
    S.status = A.status;
    S.counts = counts;
    S.rec = A.rec;
    S.rec4 = q.rec4;
    S.payload = a.payload;
    S.C = a.C;
    S.vec4 = (a.C % 4 == 0 && (reinterpret_cast<uintptr_t>(a.image) & 15u) == 0u &&
              (reinterpret_cast<uintptr_t>(a.grad_image) & 15u) == 0u)
                 ? 1
                 : 0;
    S.pay4 = (a.C % 4 == 0 && (reinterpret_cast<uintptr_t>(a.payload) & 15u) == 0u) ? 1 : 0;
    S.gpay4 =
        (a.C % 4 == 0 && (reinterpret_cast<uintptr_t>(a.grad_payload) & 15u) == 0u) ? 1 : 0;
    S.pos = a.pos;
    S.radius = a.radius;
    S.image = a.image;
    S.aux = a.aux;
    S.grad_image = a.grad_image;
    S.thr = A.thr;
    S.l_in_thr = a.rebinned ? 0 : 1;
    S.tmin = A.tmin;
    S.stop = A.stop;
    S.grad_pos = a.grad_pos;
    S.grad_radius = a.grad_radius;
    S.grad_opacity = a.grad_opacity;
    S.grad_payload = a.grad_payload;
    S.camg = a.grad_cam ? ws_ptr<float4>(ws, q.off_camg) : nullptr;
    S.min_radius_px = a.min_radius_px;
    S.paper_norm = a.paper_norm ? 1 : 0;
    S.B = q.B;
    // scene b's blocks start at b + sph_off_b / (spheres per block)
    constexpr int64_t sb = int64_t(kSphPerLane) * kSphThreads;
    S.nsph_blocks = uint32_t(q.B + (q.n + sb - 1) / sb);
    S.nbgblk = uint32_t(q.nbgblk);
    S.tab = tab;
    S.bgsum = a.grad_bg ? bgsum : nullptr;
    S.eps2 = a.eps2;
    const unsigned grid = unsigned(S.nsph_blocks + (a.grad_bg ? uint32_t(q.nbgblk) : 0u));
    const bool cam = a.grad_cam != nullptr;
    if (a.C <= 1)
      launch_spheres<1>(S, cam, grid, tab.scenes, stream);
    else if (a.C <= 2)
      launch_spheres<2>(S, cam, grid, tab.scenes, stream);
    else if (a.C <= 4)
      launch_spheres<4>(S, cam, grid, tab.scenes, stream);
    else if (a.C <= 8)
      launch_spheres<8>(S, cam, grid, tab.scenes, stream);
    else if (a.C <= 16)
      launch_spheres<16>(S, cam, grid, tab.scenes, stream);
    else
      launch_spheres<32>(S, cam, grid, tab.scenes, stream);
    // the tile walk beside it, on a small persistent grid (it returns at once
    // unless a very large sphere needs it), timed as a stage of its own
    stage_end(PULSAR_STAGE_RASTER_BWD, stream);
    stage_begin(PULSAR_STAGE_RASTER_BWD_TILES, stream);
    BwdKernelArgs Ab = A;
    Ab.only_if_big = 1;
    const long long ig = q.raster_grid / kBwdWaves < kBwdGridAuto ? q.raster_grid / kBwdWaves
                                                                    : kBwdGridAuto;
    const dim3 igrid{unsigned(ig > 0 ? ig : 1), 1u, 1u}, iblock{unsigned(kWave * kBwdWaves), 1u, 1u};
    if (a.C <= 1)
      launch_items<1>(Ab, igrid, iblock, stream);
    else if (a.C <= 2)
      launch_items<2>(Ab, igrid, iblock, stream);
    else if (a.C <= 4)
      launch_items<4>(Ab, igrid, iblock, stream);
    else if (a.C <= 8)
      launch_items<8>(Ab, igrid, iblock, stream);
    else if (a.C <= 16)
      launch_items<16>(Ab, igrid, iblock, stream);
    else
      launch_items<32>(Ab, igrid, iblock, stream);
    stage_end(PULSAR_STAGE_RASTER_BWD_TILES, stream);
  } else {
    // as many waves as the forward's grid of one-wave blocks: blocks past the
    // work items would only be dispatched after them to find nothing to do
    const long long bg = q.raster_grid / kBwdWaves > 0 ? q.raster_grid / kBwdWaves : 1;
    const dim3 ig{unsigned(bg), 1u, 1u}, it{unsigned(kWave * kBwdWaves), 1u, 1u};
    if (a.C <= 1)
      launch_items<1>(A, ig, it, stream);
    else if (a.C <= 2)
      launch_items<2>(A, ig, it, stream);
    else if (a.C <= 4)
      launch_items<4>(A, ig, it, stream);
    else if (a.C <= 8)
      launch_items<8>(A, ig, it, stream);
    else if (a.C <= 16)
      launch_items<16>(A, ig, it, stream);
    else if (!wide)
      launch_items<32>(A, ig, it, stream);
    else
      hipLaunchKernelGGL(k_bwd_chunks_wide, dim3(unsigned(q.raster_grid)), dim3(kWave), 0, stream,
                         A, A.tab.scenes, A.tab.tile_start, A.desc);
  }
  if (!by_sphere) stage_end(PULSAR_STAGE_RASTER_BWD, stream);
  stage_begin(PULSAR_STAGE_FINALIZE, stream);
  if (a.grad_bg && (wide || store)) {
    if (q.C <= kBgMaxC)
      hipLaunchKernelGGL(k_bg_partial, dim3(unsigned(q.nbgblk)), dim3(kBgThreads), 0, stream,
                         tab, a.aux, a.grad_image, int(q.C), a.eps2, bgsum);
    else
      hipLaunchKernelGGL(k_bg_partial_wide, dim3(unsigned(q.nbgblk)), dim3(kBgThreads), 0,
                         stream, tab, a.aux, a.grad_image, int(q.C), a.eps2, bgsum);
  }
  // after the walk in sphere order only the per-scene background sums remain;
  // its per-sphere blocks (a grid of at most kFinGridAuto walking the
  // spheres) then return at once
  const uint32_t nfin = uint32_t((q.n + kFinThreads - 1) / kFinThreads);
  const uint32_t fin_grid = by_sphere ? (nfin < kFinGridAuto ? nfin : kFinGridAuto) : nfin;
  const uint32_t nred = a.grad_bg ? uint32_t(q.C) * uint32_t(q.B) : 0u;
  if (fin_grid + nred > 0) {
    if (a.C <= 1)
      launch_finalize<1>(q, a, ws, stream, nfin, fin_grid, by_sphere ? 1 : 0, nred);
    else if (a.C <= 2)
      launch_finalize<2>(q, a, ws, stream, nfin, fin_grid, by_sphere ? 1 : 0, nred);
    else if (a.C <= 4)
      launch_finalize<4>(q, a, ws, stream, nfin, fin_grid, by_sphere ? 1 : 0, nred);
    else if (a.C <= 8)
      launch_finalize<8>(q, a, ws, stream, nfin, fin_grid, by_sphere ? 1 : 0, nred);
    else if (a.C <= 16)
      launch_finalize<16>(q, a, ws, stream, nfin, fin_grid, by_sphere ? 1 : 0, nred);
    else if (!wide)
      launch_finalize<32>(q, a, ws, stream, nfin, fin_grid, by_sphere ? 1 : 0, nred);
    else
      launch_finalize<0>(q, a, ws, stream, nfin, fin_grid, by_sphere ? 1 : 0, nred);
  }
  if (a.grad_cam) {
    hipLaunchKernelGGL(k_cam_partial, dim3(unsigned(q.ncampart)), dim3(kCamThreads), 0, stream,
                       tab.scenes, q.B, ws_ptr<float4>(ws, q.off_camg), a.pos,
                       ws_ptr<double>(ws, q.off_campart));
    hipLaunchKernelGGL(k_cam_final, dim3(unsigned(q.B)), dim3(kCamThreads), 0, stream, tab.scenes,
                       ws_ptr<double>(ws, q.off_campart), a.grad_cam);
  }
  stage_end(PULSAR_STAGE_FINALIZE, stream);
  return hipGetLastError();
}

}  // namespace pulsar
