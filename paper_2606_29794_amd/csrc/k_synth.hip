// k_synth.hip -- image synthesis between the HEALPix grid and camera images:
// the final step of rendering, I_C(u, v) = Interp_H(I_H, P_C(u, v))
// (Eq. camera_synthesis), and the reverse sampling of a camera image at the
// HEALPix pixel centres used for ground truth (supp. Eq.
// supp_image_to_healpix), with the camera mappings of the supplementary
// section on camera models (pinhole; anisotropic equidistant fisheye,
// Eq. fish_weff; equirectangular panorama).
//
// Conventions shared with the rest of the library: one camera frame for all
// models with +z the optical axis, +x right and +y up (the image's v axis
// points down, so v is negated for pinhole and fisheye); pixel (i, j) of a
// W x H image is centred at (u, v) = (i + 1/2, j + 1/2); the HEALPix pole is
// camera +y and its longitude is atan2(t_x, t_z).
//
// Interp_H: the two rings that enclose the point's colatitude, in each the
// two pixels that enclose its longitude; linear in longitude along each ring,
// linear in colatitude between the rings.  Above the first ring (below the
// last) the pole value is the mean of that ring's four pixels.  Neighbours
// outside the camera's active set get weight zero and the others are
// renormalised.  Geometry runs in double precision (CDNA4 issues FP64 vector
// FMAs at the FP32 rate), the colours in float.
//
// Both kernels are gathers over small, L2-resident inputs with coalesced
// outputs: one thread per output sample.
#include "hp_common.h"

namespace {

enum { CAM_FULL = 0, CAM_FISHEYE = 1, CAM_PINHOLE = 2 };

struct SynthCam {
  int type, W, H;
  double fx, fy;        // focal lengths in pixels
  double wx, wy;        // fisheye FoV / pi
  double cx, cy;        // principal point (image centre)
};

SynthCam synth_cam(const hp_view* v, int W, int H) {
  SynthCam c;
  c.type = v->cam_type;
  c.W = W;
  c.H = H;
  c.cx = 0.5 * W;
  c.cy = 0.5 * H;
  if (c.type == CAM_PINHOLE) {
    c.fx = W / (2.0 * tan(0.5 * (double)v->fov_x));
    c.fy = H / (2.0 * tan(0.5 * (double)v->fov_y));
  } else {
    c.fx = W / M_PI;
    c.fy = H / M_PI;
  }
  c.wx = (double)v->fov_x / M_PI;
  c.wy = (double)v->fov_y / M_PI;
  return c;
}

// ray through image position (u, v); false outside the camera's domain
__device__ bool synth_ray(const SynthCam& c, double u, double v, double d[3]) {
  if (c.type == CAM_FULL) {
    const double om = 2.0 * M_PI * u / c.W - M_PI, ph = 0.5 * M_PI - M_PI * v / c.H;
    double so, co, sp, cp;
    sincos(om, &so, &co);
    sincos(ph, &sp, &cp);
    d[0] = cp * so;
    d[1] = sp;
    d[2] = cp * co;
    return true;
  }
  const double mx = (u - c.cx) / c.fx, my = -(v - c.cy) / c.fy;
  if (c.type == CAM_PINHOLE) {
    const double n = rsqrt(mx * mx + my * my + 1.0);
    d[0] = mx * n;
    d[1] = my * n;
    d[2] = n;
    return true;
  }
  const double rm = sqrt(mx * mx + my * my);
  const double gam = atan2(my, mx);
  double sg, cg;
  sincos(gam, &sg, &cg);
  const double weff = sqrt(c.wx * cg * c.wx * cg + c.wy * sg * c.wy * sg);
  double sps, cps;
  sincos(rm * weff, &sps, &cps);
  d[0] = sps * cg;
  d[1] = sps * sg;
  d[2] = cps;
  return rm <= 0.5 * M_PI;
}

// image position of direction d; false outside the camera's domain
__device__ bool synth_project(const SynthCam& c, const double d[3], double* u, double* v) {
  if (c.type == CAM_FULL) {
    const double om = atan2(d[0], d[2]);
    const double ph = asin(fmin(1.0, fmax(-1.0, d[1])));
    *u = (om + M_PI) * c.W / (2.0 * M_PI);
    *v = (0.5 * M_PI - ph) * c.H / M_PI;
    return true;
  }
  if (c.type == CAM_PINHOLE) {
    if (!(d[2] > 0.0)) return false;
    *u = c.cx + c.fx * (d[0] / d[2]);
    *v = c.cy - c.fy * (d[1] / d[2]);
    return *u >= 0.0 && *u <= c.W && *v >= 0.0 && *v <= c.H;
  }
  const double psi = acos(fmin(1.0, fmax(-1.0, d[2])));
  const double gam = atan2(d[1], d[0]);
  double sg, cg;
  sincos(gam, &sg, &cg);
  const double weff = sqrt(c.wx * cg * c.wx * cg + c.wy * sg * c.wy * sg);
  const double rm = psi / weff;
  *u = c.cx + c.fx * rm * cg;
  *v = c.cy - c.fy * rm * sg;
  return rm <= 0.5 * M_PI;
}

// ---- ring structure of the grid (Gorski et al. 2005) -----------------------
// colatitude of ring i (1 .. 4N-1); 0 and pi for the poles (i = 0, 4N).  In
// the caps 1 - |z| = 2 sin^2(theta / 2) = i^2 / (3 N^2), taken through the
// half-angle sine to avoid cancellation.
__device__ double ring_theta(int64_t N, int64_t i) {
  const double r6 = 2.449489742783178098197284;  // sqrt(6)
  if (i <= 0) return 0.0;
  if (i >= 4 * N) return M_PI;
  if (i < N) return 2.0 * asin((double)i / ((double)N * r6));
  if (i > 3 * N) return M_PI - 2.0 * asin((double)(4 * N - i) / ((double)N * r6));
  return acos((double)(2 * N - i) * 2.0 / (3.0 * (double)N));
}

// pixels in ring i and the longitude offset (in pixels) of its pixel 0's centre
__device__ void ring_len(int64_t N, int64_t i, int64_t* n, double* off) {
  if (i < N) { *n = 4 * i; *off = 0.5; }
  else if (i > 3 * N) { *n = 4 * (4 * N - i); *off = 0.5; }
  else { *n = 4 * N; *off = ((i - N) & 1) ? 0.0 : 0.5; }
}

// NESTED index of pixel j (0-based) of ring i.  Polar caps: face column
// j / nr, then the face-local (x, y) from the ring's position on the face.
// Equatorial belt: the ring crosses faces of two rows; the face is the one
// whose (x, y) = ((s + dxy) / 2, (s - dxy) / 2) falls inside it, with
// s = x + y fixed by the row and dxy = x - y by the position along the ring.
__device__ int64_t ring_nest(int order, int64_t i, int64_t j) {
  const int64_t N = (int64_t)1 << order;
  if (i < N || i > 3 * N) {
    const bool north = i < N;
    const int64_t nr = north ? i : 4 * N - i;
    const int64_t col = j / nr, q = j - col * nr;
    const int64_t x = north ? N - nr + q : q;
    const int64_t y = north ? N - 1 - q : nr - 1 - q;
    return hp_xyf_nest(order, (int)x, (int)y, (int)((north ? 0 : 8) + col));
  }
  const int64_t ks = (i - N) & 1;
  for (int r = 0; r < 3; ++r) {
    const int64_t s = (int64_t)(r + 2) * N - 1 - i;
    if (s < 0 || s > 2 * N - 2) continue;
    for (int col = 0; col < 4; ++col) {
      const int64_t L = r == 1 ? 2 * col : 2 * col + 1;
      int64_t dxy = 2 * (j + 1) - 1 - ks - L * N;  // defined modulo 8N
      dxy = ((dxy + 4 * N) % (8 * N) + 8 * N) % (8 * N) - 4 * N;
      if ((s + dxy) & 1) continue;
      const int64_t x = (s + dxy) / 2, y = (s - dxy) / 2;
      if (x >= 0 && x < N && y >= 0 && y < N) return hp_xyf_nest(order, (int)x, (int)y, 4 * r + col);
    }
  }
  return -1;
}

// the four (ring, position) samples of Interp_H and their weights
__device__ void interp4(int order, const double d[3], int64_t ring[4], int64_t pos[4], double w[4]) {
  const int64_t N = (int64_t)1 << order;
  const double xh = d[2], yh = d[0], zh = d[1];
  const double theta = atan2(sqrt(xh * xh + yh * yh), zh);
  double phi = atan2(yh, xh);
  if (phi < 0.0) phi += 2.0 * M_PI;
  // first guess of the ring above from the closed forms, then exact fix-up
  // against the ring colatitudes
  const double z = cos(theta);
  double ic;
  if (z > 2.0 / 3.0) ic = (double)N * 2.449489742783178098197284 * sin(0.5 * theta);
  else if (z < -2.0 / 3.0) ic = 4.0 * N - (double)N * 2.449489742783178098197284 * sin(0.5 * (M_PI - theta));
  else ic = 2.0 * N - 1.5 * N * z;
  int64_t i1 = (int64_t)floor(ic);
  i1 = i1 < 0 ? 0 : (i1 > 4 * N - 1 ? 4 * N - 1 : i1);
  while (i1 < 4 * N - 1 && ring_theta(N, i1 + 1) <= theta) ++i1;
  while (i1 > 0 && ring_theta(N, i1) > theta) --i1;
  const int64_t i2 = i1 + 1;
  auto pair = [&](int64_t i, int64_t* ja, int64_t* jb, double* f) {
    int64_t n;
    double off;
    ring_len(N, i, &n, &off);
    const double t = phi / (2.0 * M_PI / (double)n) - off;
    const double j1 = floor(t);
    *f = t - j1;
    int64_t a = (int64_t)j1 % n;
    if (a < 0) a += n;
    *ja = a;
    *jb = a + 1 == n ? 0 : a + 1;
  };
  if (i1 >= 1 && i2 <= 4 * N - 1) {
    const double t1 = ring_theta(N, i1), t2 = ring_theta(N, i2);
    const double wt = (theta - t1) / (t2 - t1);
    double f1, f2;
    pair(i1, &pos[0], &pos[1], &f1);
    pair(i2, &pos[2], &pos[3], &f2);
    ring[0] = ring[1] = i1;
    ring[2] = ring[3] = i2;
    w[0] = (1.0 - wt) * (1.0 - f1);
    w[1] = (1.0 - wt) * f1;
    w[2] = wt * (1.0 - f2);
    w[3] = wt * f2;
    return;
  }
  const int64_t ir = i1 == 0 ? 1 : 4 * N - 1;
  const double tr = ring_theta(N, ir);
  const double wr = i1 == 0 ? theta / tr : (M_PI - theta) / (M_PI - tr);
  int64_t a, b;
  double f;
  pair(ir, &a, &b, &f);
  for (int k = 0; k < 4; ++k) {
    ring[k] = ir;
    pos[k] = k;
    w[k] = 0.25 * (1.0 - wr);
  }
  w[a] += wr * (1.0 - f);
  w[b] += wr * f;
}

// compact slot of nested pixel q in the mask, or -1 (inactive or invalid q)
__device__ int64_t synth_slot(const HpMaskView& m, const HpGeom& g, int64_t q) {
  if (q < 0 || q >= g.npix) return -1;
  const int per_b = 2 * g.b;
  const int64_t t = q >> per_b;
  const int loc = (int)(q - (t << per_b));
  // a fully active tile holds its pixels in nested order: no rank to count
  if (m.tile_count[t] == (1 << per_b)) return (int64_t)m.tile_start[t] + loc;
  const uint32_t* bits = m.tile_bits + 8 * t;
  const uint32_t word = bits[loc >> 5];
  if (!((word >> (loc & 31)) & 1u)) return -1;
  int rank = __popc(word & ((1u << (loc & 31)) - 1u));
  for (int k = 0; k < (loc >> 5); ++k) rank += __popc(bits[k]);
  return (int64_t)m.tile_start[t] + rank;
}

__global__ __launch_bounds__(256) void k_sphere_to_image(HpGeom g, HpMaskView m, int64_t n_active, SynthCam c,
                                                         const float* __restrict__ img, float* __restrict__ out,
                                                         uint8_t* __restrict__ valid) {
  const int64_t HW = (int64_t)c.W * c.H;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= HW) return;
  const int i = (int)(k % c.W), j = (int)(k / c.W);
  double d[3];
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  double ws = 0.0;
  if (synth_ray(c, i + 0.5, j + 0.5, d)) {
    int64_t ring[4], pos[4];
    double w[4];
    interp4(g.order, d, ring, pos, w);
    for (int q = 0; q < 4; ++q) {
      const int64_t s = synth_slot(m, g, ring_nest(g.order, ring[q], pos[q]));
      if (s < 0 || s >= n_active) continue;
      const float wf = (float)w[q];
      a0 += wf * img[s];
      a1 += wf * img[n_active + s];
      a2 += wf * img[2 * n_active + s];
      ws += w[q];
    }
  }
  const bool ok = ws > 0.0;
  const float inv = ok ? (float)(1.0 / ws) : 0.f;
  out[k] = a0 * inv;
  out[HW + k] = a1 * inv;
  out[2 * HW + k] = a2 * inv;
  if (valid) valid[k] = ok ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_image_to_sphere(HpGeom g, HpMaskView m, int64_t n_active, SynthCam c,
                                                         const float* __restrict__ img, float* __restrict__ out,
                                                         uint8_t* __restrict__ valid) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_active) return;
  double t[3], u = 0.5 * c.W, v = 0.5 * c.H;
  hp_pix_dir(g.order, m.active_pix[k], t);
  const bool ok = synth_project(c, t, &u, &v);
  const double x = u - 0.5, y = v - 0.5;
  const double x0 = floor(x), y0 = floor(y);
  const float fx = (float)(x - x0), fy = (float)(y - y0);
  int64_t xs[2] = {(int64_t)x0, (int64_t)x0 + 1}, ys[2] = {(int64_t)y0, (int64_t)y0 + 1};
  for (int a = 0; a < 2; ++a) {
    if (c.type == CAM_FULL) xs[a] = ((xs[a] % c.W) + c.W) % c.W;
    else xs[a] = xs[a] < 0 ? 0 : (xs[a] >= c.W ? c.W - 1 : xs[a]);
    ys[a] = ys[a] < 0 ? 0 : (ys[a] >= c.H ? c.H - 1 : ys[a]);
  }
  const int64_t HW = (int64_t)c.W * c.H;
  const int64_t o00 = ys[0] * c.W + xs[0], o01 = ys[0] * c.W + xs[1], o10 = ys[1] * c.W + xs[0],
                o11 = ys[1] * c.W + xs[1];
  const float w00 = (1.f - fx) * (1.f - fy), w01 = fx * (1.f - fy), w10 = (1.f - fx) * fy, w11 = fx * fy;
  for (int ch = 0; ch < 3; ++ch) {
    const float* p = img + ch * HW;
    const float s = w00 * p[o00] + w01 * p[o01] + w10 * p[o10] + w11 * p[o11];
    out[ch * n_active + k] = ok ? s : 0.f;
  }
  if (valid) valid[k] = ok ? 1 : 0;
}

hp_status synth_check(const hp_view* view, const hp_params* prm, const void* mask, int32_t W, int32_t H) {
  HP_TRY(hp_check_view(view, prm));
  if (!mask || W <= 0 || H <= 0 || (int64_t)W * H > ((int64_t)1 << 31)) return HP_ERR_INVALID_ARG;
  return HP_OK;
}

}  // namespace

extern "C" hp_status hp_sphere_to_image(const void* mask, const hp_view* view, const hp_params* prm, int64_t n_active,
                                        const float* img, int32_t W, int32_t H, float* out, uint8_t* valid,
                                        void* stream) {
  HP_TRY(synth_check(view, prm, mask, W, H));
  const HpGeom g = hp_geom(view->order, prm->tile_log2);
  if (n_active < 0 || n_active > g.npix || !out || (n_active > 0 && !img)) return HP_ERR_INVALID_ARG;
  const int64_t HW = (int64_t)W * H;
  hipLaunchKernelGGL(k_sphere_to_image, dim3(hp_blocks(HW, 256)), dim3(256), 0, (hipStream_t)stream, g,
                     hp_mask_view((char*)const_cast<void*>(mask), g), n_active, synth_cam(view, W, H), img, out,
                     valid);
  HP_CHECK_LAUNCH();
  return HP_OK;
}

extern "C" hp_status hp_image_to_sphere(const void* mask, const hp_view* view, const hp_params* prm, int64_t n_active,
                                        const float* img, int32_t W, int32_t H, float* out, uint8_t* valid,
                                        void* stream) {
  HP_TRY(synth_check(view, prm, mask, W, H));
  const HpGeom g = hp_geom(view->order, prm->tile_log2);
  if (n_active < 0 || n_active > g.npix || !img || (n_active > 0 && !out)) return HP_ERR_INVALID_ARG;
  if (n_active == 0) return HP_OK;
  hipLaunchKernelGGL(k_image_to_sphere, dim3(hp_blocks(n_active, 256)), dim3(256), 0, (hipStream_t)stream, g,
                     hp_mask_view((char*)const_cast<void*>(mask), g), n_active, synth_cam(view, W, H), img, out,
                     valid);
  HP_CHECK_LAUNCH();
  return HP_OK;
}
