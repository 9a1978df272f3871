/*
 * FP64 brute-force oracle for the sphere renderer of Pulsar (Lassner and
 * Zollhoefer, "Pulsar: Efficient Sphere-based Neural Rendering").
 *
 * TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library. It shares no code, header, table or
 * constant with the HIP renderer, and the renderer never calls it.
 *
 * What it computes (paper Sec. 3.1, Sec. 3.2 Eq. 1, App. A):
 *   scene S = {(p_i, f_i, r_i, o_i)}; camera x_cam = R x_world + t, pinhole with
 *   focal length f and sensor width s, principal point at the sensor centre.
 *   For every pixel ray and EVERY sphere (no binning, no culling structure):
 *     w_i = o_i d_i exp(o_i z_i / gamma) / (exp(eps/gamma) + sum_k o_k d_k exp(o_k z_k / gamma))
 *     F   = sum_i w_i f_i + exp(eps/gamma) / (...) * background
 *   The sum runs over all spheres the ray intersects.
 *
 * Readings of points the paper leaves open:
 *   - pixel (row i, col j) centre on the plane z = f at
 *       x_s = (j + 1/2) s/W - s/2,  y_s = (i + 1/2) s/W - (s H/W)/2,
 *     camera axes x right, y down, z forward; unit ray u = (x_s, y_s, f)/|.|.
 *   - the intersection depth is the distance along u to the FRONT intersection,
 *     t = b - sqrt(R^2 - q^2) with b = u.c, d = c - b u, q = |d|;
 *     a hit needs q < R and t <= far.
 *   - z = (far - t)/(far - near) in [0, 1], 0 at the far plane (Sec. 3.2).
 *   - d_i is used as delta = 1 - min(1, q/R): the weight is largest on the
 *     ray through the centre and falls continuously to 0 at the silhouette.
 *   - a sphere takes part iff its inputs are finite, r > 0 and c_z - R >= near.
 *   - optional minimum size (App. B, Step 0): R = max(r, rho c_z / f), with
 *     rho = min_radius_px * pitch; off when min_radius_px = 0.
 *   - gradients flow through the first min(K, #hits) hits of a pixel in
 *     ascending (t, sphere index) order (App. B, Step 2 and backward prep);
 *     the image blends every hit (Sec. 2, point-based representations: an
 *     unlimited number of spheres colour a pixel, the first few get gradients).
 *   - the sums are shifted by m = max(eps/gamma, max_i o_i z_i / gamma), which
 *     leaves Eq. 1 unchanged and keeps exp() finite down to gamma = 1e-5.
 *
 * All arithmetic is IEEE double. Threads split work over pixels in the
 * forward; the backward accumulates serially in pixel order, so it is
 * deterministic.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_OK 0
#define ORACLE_BAD_ARG -1
#define ORACLE_NEG_OPACITY -2

/* cam[17] = R (row-major 9), t (3), f, s, near, far, projection (0 pinhole, 1 orthographic) */
typedef struct {
  double R[9], t[3];
  double f, s, znear, zfar;
  int W, H;
  double pitch, sh;
  int ortho; /* orthographic projection: parallel rays along +z from the sensor plane */
} camera_t;

typedef struct {
  double c[3];  /* camera-space centre */
  double R;     /* effective radius */
  float tmin;   /* earliest possible hit distance |c| - R (c_z - R orthographic), in float */
  int take_part;
  int clamped;  /* effective radius comes from the minimum size */
} sphere_cam_t;

typedef struct {
  double t;
  int k;
  int is_hit;     /* 1: a hit; 0: a near miss kept only for the ambiguity flag */
  int uncertain;  /* within rounding distance of the silhouette or the far plane */
  float tmin;     /* the sphere's earliest possible hit distance (early stop order) */
} hit_key_t;

static void make_camera(camera_t* cam, const double* c16, int W, int H) {
  memcpy(cam->R, c16, 9 * sizeof(double));
  memcpy(cam->t, c16 + 9, 3 * sizeof(double));
  cam->f = c16[12];
  cam->s = c16[13];
  cam->znear = c16[14];
  cam->zfar = c16[15];
  cam->W = W;
  cam->H = H;
  cam->pitch = cam->s / (double)W;
  cam->sh = cam->s * (double)H / (double)W;
  cam->ortho = c16[16] != 0.0;
}

/* ray through the centre of pixel (i, j): origin o, unit direction u. The
 * pinhole ray starts at the camera centre; the orthographic one starts at the
 * pixel centre on the sensor plane z = 0 and runs along +z (Sec. 3.1 names
 * both projection models). */
static void pixel_ray(const camera_t* cam, int i, int j, double u[3], double o[3]) {
  double xs = (j + 0.5) * cam->pitch - 0.5 * cam->s;
  double ys = (i + 0.5) * cam->pitch - 0.5 * cam->sh;
  if (cam->ortho) {
    o[0] = xs;
    o[1] = ys;
    o[2] = 0.0;
    u[0] = 0.0;
    u[1] = 0.0;
    u[2] = 1.0;
    return;
  }
  double len = sqrt(xs * xs + ys * ys + cam->f * cam->f);
  o[0] = o[1] = o[2] = 0.0;
  u[0] = xs / len;
  u[1] = ys / len;
  u[2] = cam->f / len;
}

static void sphere_to_camera(const camera_t* cam, const double* pos, double r, double o,
                             double min_radius_px, sphere_cam_t* sc) {
  for (int a = 0; a < 3; ++a)
    sc->c[a] = cam->R[3 * a + 0] * pos[0] + cam->R[3 * a + 1] * pos[1] +
               cam->R[3 * a + 2] * pos[2] + cam->t[a];
  /* the minimum size in pixels: at depth c_z for the pinhole, at any depth
     for the orthographic projection */
  double rmin = cam->ortho ? min_radius_px * cam->pitch
                           : min_radius_px * cam->pitch * sc->c[2] / cam->f;
  sc->clamped = (min_radius_px > 0.0) && (rmin > r);
  sc->R = sc->clamped ? rmin : r;
  /* no ray meets the sphere before its nearest point: |c| - R from the
     camera centre, c_z - R from the orthographic sensor plane */
  sc->tmin = cam->ortho ? (float)(sc->c[2] - sc->R)
                        : (float)(sqrt(sc->c[0] * sc->c[0] + sc->c[1] * sc->c[1] +
                                       sc->c[2] * sc->c[2]) -
                                  sc->R);
  int finite = isfinite(pos[0]) && isfinite(pos[1]) && isfinite(pos[2]) && isfinite(r) &&
               isfinite(o);
  sc->take_part = finite && r > 0.0 && (sc->c[2] - sc->R >= cam->znear);
}

/* Ray-sphere test along unit direction u. Returns 1 on a hit and fills
 * t (front intersection distance), q (distance of the centre from the ray),
 * b (projection of the centre on the ray) and d (vector from the ray to the centre). */
static int ray_sphere(const camera_t* cam, const double u[3], const double o[3],
                      const sphere_cam_t* sc, double* t, double* q, double* b, double d[3]) {
  if (!sc->take_part) return 0;
  double c[3] = {sc->c[0] - o[0], sc->c[1] - o[1], sc->c[2] - o[2]};
  double bb = u[0] * c[0] + u[1] * c[1] + u[2] * c[2];
  double dd[3] = {c[0] - bb * u[0], c[1] - bb * u[1], c[2] - bb * u[2]};
  double qq = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  if (!(qq < sc->R)) return 0;
  double tt = bb - sqrt(sc->R * sc->R - qq * qq);
  if (!(tt <= cam->zfar)) return 0;
  *t = tt;
  *q = qq;
  *b = bb;
  d[0] = dd[0];
  d[1] = dd[1];
  d[2] = dd[2];
  return 1;
}

/* Distance along u to the point of closest approach when the ray misses the
 * sphere by less than rel * R (q in [R, R (1 + rel))); used only to flag
 * pixels whose K nearest hits could change under float32 rounding. */
static int near_miss(const camera_t* cam, const double u[3], const double o[3],
                     const sphere_cam_t* sc, double rel, double* t) {
  if (!sc->take_part) return 0;
  double c[3] = {sc->c[0] - o[0], sc->c[1] - o[1], sc->c[2] - o[2]};
  double bb = u[0] * c[0] + u[1] * c[1] + u[2] * c[2];
  double dd[3] = {c[0] - bb * u[0], c[1] - bb * u[1], c[2] - bb * u[2]};
  double qq = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  if (!(qq >= sc->R && qq < sc->R * (1.0 + rel))) return 0;
  if (!(bb <= cam->zfar * (1.0 + rel))) return 0;
  *t = bb;
  return 1;
}

/* order of the early stop: earliest possible hit distance (in float), then index */
static int cmp_tmin(const void* pa, const void* pb) {
  const hit_key_t* a = (const hit_key_t*)pa;
  const hit_key_t* b = (const hit_key_t*)pb;
  if (a->tmin < b->tmin) return -1;
  if (a->tmin > b->tmin) return 1;
  return (a->k > b->k) - (a->k < b->k);
}

static int cmp_hit(const void* pa, const void* pb) {
  const hit_key_t* a = (const hit_key_t*)pa;
  const hit_key_t* b = (const hit_key_t*)pb;
  if (a->t < b->t) return -1;
  if (a->t > b->t) return 1;
  return (a->k > b->k) - (a->k < b->k);
}

static sphere_cam_t* transform_all(const camera_t* cam, int n, const double* pos,
                                   const double* radius, const double* opacity,
                                   double min_radius_px) {
  sphere_cam_t* sc = (sphere_cam_t*)malloc(sizeof(sphere_cam_t) * (size_t)(n > 0 ? n : 1));
  if (!sc) return NULL;
  for (int k = 0; k < n; ++k)
    sphere_to_camera(cam, pos + 3 * (size_t)k, radius[k], opacity ? opacity[k] : 1.0,
                     min_radius_px, &sc[k]);
  return sc;
}

/*
 * Forward pass over the pixels of the listed rows (all rows when rows == NULL).
 *   F [H,W,C], L [H,W] (log of the Eq. 1 denominator, L = m + ln D),
 *   nhits [H,W], klist_t / klist_id [H,W,K] (ascending (t, index); id -1 and
 *   t = +inf where a pixel has fewer than K hits), t_next [H,W] (distance of
 *   hit K+1, +inf if none), ambiguous [H,W].
 * A pixel is ambiguous when float32 rounding could change its K nearest hits:
 * hit K and hit K+1 lie closer than amb_rel * t_K, or, among the first K+1
 * entries of the depth-sorted list of hits and near misses, one lies within
 * amb_rel of the silhouette (1 - q/R < amb_rel or a miss by less than
 * amb_rel R) or of the far plane. It only serves the parity harness.
 * Entries of rows that are not listed are left untouched.
 *
 * Early stop (stop_share > 0; Sec. 3.2 and App. B, Step 2): the hits of a
 * pixel are taken in ascending order of their sphere's earliest possible hit
 * distance (float32, then index), the order of the paper's device-wide depth
 * sort. Before a hit is blended, the largest weight any sphere starting at
 * that depth could have, exp(z(t_min) / gamma) (opacity <= 1 and d <= 1), is
 * compared with the running denominator D of Eq. 1: if it is below
 * stop_share / (1 - stop_share) D, no such sphere can reach a share of
 * stop_share of the pixel, and this hit and every later one are skipped.
 * Only the blended hits enter F, L, nhits and the K nearest. A pixel whose
 * decision lies within 1e-3 (natural-log units, relative above 1) of the
 * threshold is flagged ambiguous.
 */
int oracle_forward(int n, int C, const double* pos, const double* radius, const double* opacity,
                   const double* payload, const double* bg, const double* cam16, int W, int H,
                   double gamma, double eps, double min_radius_px, int K, double amb_rel,
                   int n_rows, const int* rows, double* F, double* L, int* nhits,
                   double* klist_t, int* klist_id, double* t_next, uint8_t* ambiguous,
                   int n_threads, int blend_topk, double stop_share) {
  if (stop_share < 0.0 || stop_share >= 1.0 || (stop_share > 0.0 && blend_topk))
    return ORACLE_BAD_ARG;
  if (n < 0 || C < 1 || W < 1 || H < 1 || K < 1 || !(gamma > 0.0)) return ORACLE_BAD_ARG;
  if (n > 0 && (!pos || !radius || !payload)) return ORACLE_BAD_ARG;
  if (opacity)
    for (int k = 0; k < n; ++k)
      if (opacity[k] < 0.0) return ORACLE_NEG_OPACITY;
  camera_t cam;
  make_camera(&cam, cam16, W, H);
  sphere_cam_t* sc = transform_all(&cam, n, pos, radius, opacity, min_radius_px);
  if (!sc) return ORACLE_BAD_ARG;
  int nr = rows ? n_rows : H;
  long long npix = (long long)nr * W;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel
  {
    hit_key_t* hits = (hit_key_t*)malloc(sizeof(hit_key_t) * (size_t)(n > 0 ? n : 1));
    double* acc = (double*)malloc(sizeof(double) * (size_t)C);
#pragma omp for schedule(dynamic, 16)
    for (long long pix = 0; pix < npix; ++pix) {
      int i = rows ? rows[pix / W] : (int)(pix / W);
      int j = (int)(pix % W);
      size_t p = (size_t)i * W + j;
      double u[3], ro[3];
      pixel_ray(&cam, i, j, u, ro);
      /* collect every intersected sphere */
      int nh = 0;
      double m = eps / gamma;
      for (int k = 0; k < n; ++k) {
        double t, q, b, d[3];
        if (ray_sphere(&cam, u, ro, &sc[k], &t, &q, &b, d)) {
          hits[nh].t = t;
          hits[nh].k = k;
          hits[nh].tmin = sc[k].tmin;
          hits[nh].is_hit = 1;
          hits[nh].uncertain = (1.0 - q / sc[k].R < amb_rel) || (t > cam.zfar * (1.0 - amb_rel));
          ++nh;
          double o = opacity ? opacity[k] : 1.0;
          double z = (cam.zfar - t) / (cam.zfar - cam.znear);
          double s = o * z / gamma;
          if (s > m) m = s;
        }
      }
      /* the top-K variant blends only the K nearest hits, in (t, index)
         order, with the shift m taken over those */
      int nb = nh;
      if (blend_topk && nh > K) {
        qsort(hits, (size_t)nh, sizeof(hit_key_t), cmp_hit);
        nb = K;
        m = eps / gamma;
        for (int h = 0; h < nb; ++h) {
          int k = hits[h].k;
          double o = opacity ? opacity[k] : 1.0;
          double s = o * ((cam.zfar - hits[h].t) / (cam.zfar - cam.znear)) / gamma;
          if (s > m) m = s;
        }
      }
      /* early stop: walk the hits in the order of the depth sort, keeping the
         log of the running denominator; drop the stopping hit and the rest */
      int stop_amb = 0;
      if (stop_share > 0.0 && nh > 0) {
        qsort(hits, (size_t)nh, sizeof(hit_key_t), cmp_tmin);
        const double span = cam.zfar - cam.znear;
        const double lrho = log(stop_share / (1.0 - stop_share));
        double Lc = eps / gamma; /* log of the background weight */
        m = eps / gamma;
        nb = 0;
        for (int h = 0; h < nh; ++h) {
          const int k = hits[h].k;
          const double bound = (cam.zfar - (double)hits[h].tmin) / span / gamma;
          const double thr = lrho + Lc;
          if (fabs(bound - thr) < 1e-3 * fmax(1.0, fabs(thr))) stop_amb = 1;
          if (bound < thr) break;
          double t = 0.0, q = 0.0, b = 0.0, d[3];
          ray_sphere(&cam, u, ro, &sc[k], &t, &q, &b, d);
          const double o = opacity ? opacity[k] : 1.0;
          const double lw = log(o * (1.0 - q / sc[k].R)) + o * ((cam.zfar - t) / span) / gamma;
          /* log(exp(Lc) + exp(lw)) */
          if (lw > -INFINITY) Lc = lw > Lc ? lw + log1p(exp(Lc - lw)) : Lc + log1p(exp(lw - Lc));
          const double s = o * ((cam.zfar - t) / span) / gamma;
          if (s > m) m = s;
          ++nb;
        }
        nh = nb; /* the skipped hits take no part in anything below */
      }
      /* near misses go after the hits; the blend below reads only hits[0 .. nb) */
      int nall = nh;
      for (int k = 0; k < n; ++k) {
        double t;
        if (near_miss(&cam, u, ro, &sc[k], amb_rel, &t)) {
          hits[nall].t = t;
          hits[nall].k = k;
          hits[nall].is_hit = 0;
          hits[nall].uncertain = 1;
          ++nall;
        }
      }
      /* Eq. 1 with all hits, shifted by m */
      double wbg = exp(eps / gamma - m);
      double D = wbg;
      for (int c = 0; c < C; ++c) acc[c] = wbg * bg[c];
      for (int h = 0; h < nb; ++h) {
        int k = hits[h].k;
        double t = 0.0, q = 0.0, b = 0.0, d[3];
        ray_sphere(&cam, u, ro, &sc[k], &t, &q, &b, d);
        double o = opacity ? opacity[k] : 1.0;
        double z = (cam.zfar - t) / (cam.zfar - cam.znear);
        double delta = 1.0 - q / sc[k].R;
        double a = o * delta * exp(o * z / gamma - m);
        D += a;
        for (int c = 0; c < C; ++c) acc[c] += a * payload[(size_t)k * C + c];
      }
      for (int c = 0; c < C; ++c) F[p * C + c] = acc[c] / D;
      L[p] = m + log(D);
      /* the K nearest hits in ascending (t, index) */
      qsort(hits, (size_t)nall, sizeof(hit_key_t), cmp_hit);
      nhits[p] = nh;
      int r = 0;
      double tk = INFINITY, tk1 = INFINITY;
      for (int h = 0; h < nall; ++h) {
        if (!hits[h].is_hit) continue;
        if (r < K) {
          klist_t[p * K + r] = hits[h].t;
          klist_id[p * K + r] = hits[h].k;
          tk = hits[h].t;
        } else if (r == K) {
          tk1 = hits[h].t;
        }
        ++r;
      }
      for (; r < K; ++r) {
        klist_t[p * K + r] = INFINITY;
        klist_id[p * K + r] = -1;
      }
      t_next[p] = tk1;
      int amb = stop_amb || ((nh > K) && (tk1 - tk < amb_rel * tk));
      if (nall > K)
        for (int h = 0; h <= K && h < nall; ++h) amb |= hits[h].uncertain;
      ambiguous[p] = (uint8_t)amb;
    }
    free(hits);
    free(acc);
  }
  free(sc);
  return ORACLE_OK;
}

/*
 * Backward pass for upstream dLoss/dF = G [H,W,C] over the listed rows, using
 * F, L and the K-lists of oracle_forward. Derivatives of Eq. 1 (in the
 * readings above) with respect to the camera-space centre c, the effective
 * radius, opacity and features of each sphere in a pixel's K-list, then chained
 * to world position (dLoss/dp = R^T dLoss/dc) and radius. Outputs are overwritten.
 * grad_opacity may be NULL (no opacity input).
 *
 * Camera gradients (Sec. 3.1: the render map is differentiable in the camera
 * too), written when grad_cam is not NULL, as 14 values: dLoss/dR (row-major
 * 3x3, R taken as a free matrix), dLoss/dt, dLoss/df, dLoss/ds. R and t act
 * only through c = R p + t, so they collect dLoss/dc of every sphere. f and s
 * act through every pixel ray u (its direction (x_s, y_s, f), with x_s, y_s
 * proportional to s) and through the minimum-size radius rho c_z / f with
 * rho proportional to s. grad_cam_abs (may be NULL) receives, per value, the
 * sum of the absolute values of the terms added into it, a scale for
 * comparing sums that cancel. grad_cam_sphere (may be NULL) receives [n, 14]:
 * row k holds the part of those 14 values that comes from sphere k (its
 * centre through R and t, its hits through f and s, its minimum-size radius);
 * the rows add up to grad_cam.
 */
int oracle_backward(int n, int C, const double* pos, const double* radius, const double* opacity,
                    const double* payload, const double* bg, const double* cam16, int W, int H,
                    double gamma, double eps, double min_radius_px, int K, int n_rows,
                    const int* rows, const double* G, const double* F, const double* L,
                    const int* klist_id, double* grad_pos, double* grad_radius,
                    double* grad_opacity, double* grad_payload, double* grad_bg,
                    double* grad_cam, double* grad_cam_abs, double* grad_cam_sphere) {
  (void)bg;
  if (n < 0 || C < 1 || W < 1 || H < 1 || K < 1 || !(gamma > 0.0)) return ORACLE_BAD_ARG;
  camera_t cam;
  make_camera(&cam, cam16, W, H);
  sphere_cam_t* sc = transform_all(&cam, n, pos, radius, opacity, min_radius_px);
  double* gc = (double*)calloc((size_t)(n > 0 ? n : 1) * 3, sizeof(double));
  double* gR = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  /* per sphere: its f and s terms from the pixel rays */
  double* gfs = (double*)calloc((size_t)(n > 0 ? n : 1) * 2, sizeof(double));
  if (!sc || !gc || !gR || !gfs) return ORACLE_BAD_ARG;
  memset(grad_pos, 0, sizeof(double) * 3 * (size_t)n);
  memset(grad_radius, 0, sizeof(double) * (size_t)n);
  if (grad_opacity) memset(grad_opacity, 0, sizeof(double) * (size_t)n);
  memset(grad_payload, 0, sizeof(double) * (size_t)n * C);
  memset(grad_bg, 0, sizeof(double) * (size_t)C);
  double gcam[14] = {0}, gabs[14] = {0};
  int nr = rows ? n_rows : H;
  const double span = cam.zfar - cam.znear;
  for (int ri = 0; ri < nr; ++ri) {
    int i = rows ? rows[ri] : ri;
    for (int j = 0; j < W; ++j) {
      size_t p = (size_t)i * W + j;
      const double* Gp = G + p * C;
      const double* Fp = F + p * C;
      /* background weight exp(eps/gamma) / denominator */
      double wbg = exp(eps / gamma - L[p]);
      for (int c = 0; c < C; ++c) grad_bg[c] += wbg * Gp[c];
      double u[3], ro[3];
      pixel_ray(&cam, i, j, u, ro);
      /* the ray's unnormalised direction v = (x_s, y_s, f) and its
         derivatives: dv/df = e_z, dv/ds = (x_s / s, y_s / s, 0); then
         du/dx = (dv/dx - u (u . dv/dx)) / |v| */
      double xs = (j + 0.5) * cam.pitch - 0.5 * cam.s;
      double ys = (i + 0.5) * cam.pitch - 0.5 * cam.sh;
      double vlen = sqrt(xs * xs + ys * ys + cam.f * cam.f);
      double du_df[3], du_ds[3];
      {
        double dvs[3] = {xs / cam.s, ys / cam.s, 0.0};
        double uf = u[2], us = u[0] * dvs[0] + u[1] * dvs[1];
        for (int a = 0; a < 3; ++a) {
          du_df[a] = ((a == 2 ? 1.0 : 0.0) - u[a] * uf) / vlen;
          du_ds[a] = (dvs[a] - u[a] * us) / vlen;
        }
      }
      for (int r = 0; r < K; ++r) {
        int k = klist_id[p * K + r];
        if (k < 0) break;
        double t = 0.0, q = 0.0, b = 0.0, d[3];
        if (!ray_sphere(&cam, u, ro, &sc[k], &t, &q, &b, d)) continue; /* cannot happen */
        double o = opacity ? opacity[k] : 1.0;
        double Rk = sc[k].R;
        double z = (cam.zfar - t) / span;
        double delta = 1.0 - q / Rk;
        double ex = exp(o * z / gamma - L[p]); /* exp(s) / denominator */
        double e = delta * ex;                 /* d w / d o-linear factor */
        double w = o * e;                      /* blending weight w_k of Eq. 1 */
        double h = 0.0;                        /* G . (f_k - F) */
        for (int c = 0; c < C; ++c) h += Gp[c] * (payload[(size_t)k * C + c] - Fp[c]);
        for (int c = 0; c < C; ++c) grad_payload[(size_t)k * C + c] += w * Gp[c];
        if (grad_opacity) grad_opacity[k] += e * h * (1.0 + o * z / gamma);
        double g_t = -(w * h * o / gamma) / span; /* dLoss/dt */
        double g_delta = o * ex * h;              /* dLoss/d delta */
        double root = sqrt(Rk * Rk - q * q);
        for (int a = 0; a < 3; ++a) {
          double dt_dc = u[a] + d[a] / root;               /* t = b - sqrt(R^2 - q^2) */
          double ddelta_dc = q > 0.0 ? -d[a] / (q * Rk) : 0.0; /* delta = 1 - q/R */
          gc[3 * (size_t)k + a] += g_t * dt_dc + g_delta * ddelta_dc;
        }
        gR[k] += g_t * (-Rk / root) + g_delta * (q / (Rk * Rk));
        if (grad_cam && !cam.ortho) {
          /* with c fixed: b = u . c, q^2 = |c|^2 - b^2, so db/du = c,
             dt/du = c - (b / root) c, d delta/du = (b / (q R)) c */
          double sdu = g_t * (1.0 - b / root) + (q > 0.0 ? g_delta * b / (q * Rk) : 0.0);
          double cf = 0.0, cs = 0.0;
          for (int a = 0; a < 3; ++a) {
            cf += sc[k].c[a] * du_df[a];
            cs += sc[k].c[a] * du_ds[a];
          }
          gcam[12] += sdu * cf;
          gabs[12] += fabs(sdu * cf);
          gcam[13] += sdu * cs;
          gabs[13] += fabs(sdu * cs);
          gfs[2 * (size_t)k] += sdu * cf;
          gfs[2 * (size_t)k + 1] += sdu * cs;
        }
      }
    }
  }
  for (int k = 0; k < n; ++k) {
    double g[3] = {gc[3 * (size_t)k], gc[3 * (size_t)k + 1], gc[3 * (size_t)k + 2]};
    double* row = grad_cam_sphere ? grad_cam_sphere + 14 * (size_t)k : NULL;
    if (row) {
      memset(row, 0, 14 * sizeof(double));
      if (!cam.ortho) {
        row[12] = gfs[2 * (size_t)k];
        row[13] = gfs[2 * (size_t)k + 1];
      }
    }
    if (sc[k].clamped && cam.ortho) {
      /* R = min_radius_px pitch depends on neither the sphere nor its depth */
      grad_radius[k] = 0.0;
    } else if (sc[k].clamped) {
      /* R = rho c_z / f depends on the depth, not on r */
      g[2] += gR[k] * min_radius_px * cam.pitch / cam.f;
      grad_radius[k] = 0.0;
      /* and on the camera: rho = min_radius_px s / W, so dR/df = -R/f, dR/ds = R/s */
      gcam[12] += gR[k] * (-sc[k].R / cam.f);
      gabs[12] += fabs(gR[k] * sc[k].R / cam.f);
      gcam[13] += gR[k] * (sc[k].R / cam.s);
      gabs[13] += fabs(gR[k] * sc[k].R / cam.s);
      if (row) {
        row[12] += gR[k] * (-sc[k].R / cam.f);
        row[13] += gR[k] * (sc[k].R / cam.s);
      }
    } else {
      grad_radius[k] = gR[k];
    }
    /* c = R p + t: dLoss/dR_ab = dLoss/dc_a p_b, dLoss/dt = dLoss/dc */
    for (int a = 0; a < 3; ++a) {
      for (int b2 = 0; b2 < 3; ++b2) {
        gcam[3 * a + b2] += g[a] * pos[3 * (size_t)k + b2];
        gabs[3 * a + b2] += fabs(g[a] * pos[3 * (size_t)k + b2]);
      }
      gcam[9 + a] += g[a];
      gabs[9 + a] += fabs(g[a]);
      if (row) {
        for (int b2 = 0; b2 < 3; ++b2) row[3 * a + b2] = g[a] * pos[3 * (size_t)k + b2];
        row[9 + a] = g[a];
      }
    }
    /* c = R p + t  =>  dLoss/dp = R^T dLoss/dc */
    for (int a = 0; a < 3; ++a)
      grad_pos[3 * (size_t)k + a] =
          cam.R[0 * 3 + a] * g[0] + cam.R[1 * 3 + a] * g[1] + cam.R[2 * 3 + a] * g[2];
  }
  if (grad_cam) memcpy(grad_cam, gcam, sizeof(gcam));
  if (grad_cam_abs) memcpy(grad_cam_abs, gabs, sizeof(gabs));
  free(sc);
  free(gc);
  free(gR);
  free(gfs);
  return ORACLE_OK;
}

/*
 * Per-sphere intersection dump for one pixel: hit [n] (0/1), t, q, b [n]
 * (valid where hit), and the camera-space centre c [n,3] and effective radius
 * [n] of every sphere.
 */
int oracle_pixel_hits(int n, const double* pos, const double* radius, const double* opacity,
                      const double* cam16, int W, int H, double min_radius_px, int i, int j,
                      uint8_t* hit, double* t_out, double* q_out, double* b_out, double* c_out,
                      double* reff_out, double* u_out) {
  if (n < 0 || W < 1 || H < 1 || i < 0 || i >= H || j < 0 || j >= W) return ORACLE_BAD_ARG;
  camera_t cam;
  make_camera(&cam, cam16, W, H);
  double u[3], ro[3];
  pixel_ray(&cam, i, j, u, ro);
  for (int a = 0; a < 3; ++a) u_out[a] = u[a];
  for (int k = 0; k < n; ++k) {
    sphere_cam_t sc;
    sphere_to_camera(&cam, pos + 3 * (size_t)k, radius[k], opacity ? opacity[k] : 1.0,
                     min_radius_px, &sc);
    double t = NAN, q = NAN, b = NAN, d[3];
    hit[k] = (uint8_t)ray_sphere(&cam, u, ro, &sc, &t, &q, &b, d);
    t_out[k] = t;
    q_out[k] = q;
    b_out[k] = b;
    for (int a = 0; a < 3; ++a) c_out[3 * (size_t)k + a] = sc.c[a];
    reff_out[k] = sc.R;
  }
  return ORACLE_OK;
}

int oracle_version(void) { return 1; }
