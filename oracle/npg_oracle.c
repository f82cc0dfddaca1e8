/*
 * npg_oracle.c -- plain, slow CPU reference of photon-driven neural path
 * guiding's data-parallel hot path (Zhu et al., "Photon-Driven Neural Path
 * Guiding", arXiv 2010.01775).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; it shares no code, header, table or constant with the
 * GPU implementation.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.
 *
 * Every floating-point quantity is computed in binary64 (FP64) with plain
 * loops in the order the definitions state them.  Where the paper is silent
 * the readings used are the ones listed in the design notes (bin rule,
 * mean-1 input scaling, network topology, CDF storage, sampling rule,
 * octree rule); each function below names its reading.
 *
 * Pins: every function is checked by the CPU test-suite against closed
 * forms, invariants, brute force on tiny inputs or an independent library
 * routine (see tests/test_oracle_*.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_ARG -1
#define OR_E_RANGE -2
#define OR_E_CAPACITY -3

static int is_pow2_in(int v, int lo, int hi) {
  return v >= lo && v <= hi && (v & (v - 1)) == 0;
}

/* ------------------------------------------------------------------------
 * Direction -> bin (Sec. 5 "Computing sampling maps from photons",
 * paragraph "Spherical function representation").
 *
 * The map is cylindrical and equal-area: rows are uniform slabs of z,
 * columns uniform slices of the azimuth phi.  The paper writes
 * phi = arctan(y/x); read as the full-circle azimuth in [0, 2pi).
 *
 * Exact rule (so that FP32 and FP64 implementations agree on every photon):
 *  row:    iz = #{ b in 1..H-1 : z >= -1 + 2b/H }  (boundaries exact in FP32)
 *  column: boundary rays e_b, b = 0..W-1, with e_{qW/4 + r} = Rot90^q(c_r, s_r),
 *          c_r = RN32(cos t_r), s_r = RN32(sin t_r), t_r = fl64(2*pi*r)/W;
 *          v = (x, y) lies in sector b iff cross(e_b, v) >= 0 and
 *          cross(e_{b+1 mod W}, v) < 0, cross(e, v) = e.x*y - e.y*x taken in
 *          FP64 from FP32 operands (both products exact); x = y = 0 -> 0.
 *  bin:    k = iz*W + iphi (row-major [z][phi]).
 * The oracle finds the sector by scanning all W sectors.
 * ---------------------------------------------------------------------- */
void or_boundaries(int W, float *ex, float *ey) {
  int Q = W / 4;
  for (int r = 0; r < Q; r++) {
    double t = (2.0 * M_PI * (double)r) / (double)W;
    float c = (float)cos(t), s = (float)sin(t);
    /* Rot90(x, y) = (-y, x), applied q times. */
    ex[r] = c;          ey[r] = s;
    ex[Q + r] = -s;     ey[Q + r] = c;
    ex[2 * Q + r] = -c; ey[2 * Q + r] = -s;
    ex[3 * Q + r] = s;  ey[3 * Q + r] = -c;
  }
}

static double cross_fp64(float ex, float ey, float x, float y) {
  double a = (double)ex * (double)y; /* exact: 24x24-bit product */
  double b = (double)ey * (double)x; /* exact */
  return a - b;                       /* correctly rounded: sign exact */
}

static int phi_sector(float x, float y, int W, const float *ex, const float *ey) {
  if (x == 0.0f && y == 0.0f) return 0;
  for (int b = 0; b < W; b++) {
    int b1 = (b + 1) % W;
    if (cross_fp64(ex[b], ey[b], x, y) >= 0.0 && cross_fp64(ex[b1], ey[b1], x, y) < 0.0)
      return b;
  }
  return -1; /* not reached for finite (x, y) */
}

static int z_row(float z, int H) {
  int iz = 0;
  for (int b = 1; b < H; b++)
    if ((double)z >= -1.0 + 2.0 * (double)b / (double)H) iz++;
  return iz;
}

static int dir_finite(const float *d) {
  return isfinite(d[0]) && isfinite(d[1]) && isfinite(d[2]);
}

/* Bin of each direction; -1 for a non-finite one. */
int or_bin_dirs(const float *dirs, int64_t n, int H, int W, int32_t *bin_out) {
  if (!is_pow2_in(H, 4, 1024) || !is_pow2_in(W, 4, 1024)) return OR_E_ARG;
  float *ex = malloc(sizeof(float) * W), *ey = malloc(sizeof(float) * W);
  or_boundaries(W, ex, ey);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t i = 0; i < n; i++) {
    const float *d = dirs + 3 * i;
    if (!dir_finite(d)) { bin_out[i] = -1; bad |= 1; continue; }
    bin_out[i] = z_row(d[2], H) * W + phi_sector(d[0], d[1], W, ex, ey);
  }
  free(ex); free(ey);
  return bad ? OR_E_RANGE : OR_OK;
}

/* ------------------------------------------------------------------------
 * Photon binning (Eq. "photon": Phi_{j,k} = sum of photon energies over the
 * photons of voxel j whose direction falls in bin k), plus the per-bin photon
 * count P (Sec. 6, the photon-count input channels).  Nearest-bin binning.  Weights are
 * integers in units of 2^-16, so sums are exact and order-independent.
 * perm == NULL: photon i of leaf l is i itself (leaf-sorted input);
 * otherwise photon perm[i].  accumulate != 0 adds into the existing maps
 * (progressive accumulation, Sec. 5 "Computing incident energy").
 * ---------------------------------------------------------------------- */
int or_splat(const float *dirs, const uint32_t *w, const uint32_t *perm,
             const uint32_t *leaf_off, int64_t L, int H, int W,
             uint64_t *energy, uint32_t *count, int accumulate) {
  if (!is_pow2_in(H, 4, 1024) || !is_pow2_in(W, 4, 1024)) return OR_E_ARG;
  int64_t HW = (int64_t)H * W;
  if (!accumulate) {
    memset(energy, 0, sizeof(uint64_t) * (size_t)(L * HW));
    if (count) memset(count, 0, sizeof(uint32_t) * (size_t)(L * HW));
  }
  float *ex = malloc(sizeof(float) * W), *ey = malloc(sizeof(float) * W);
  or_boundaries(W, ex, ey);
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : bad)
  for (int64_t l = 0; l < L; l++) {
    for (uint64_t i = leaf_off[l]; i < leaf_off[l + 1]; i++) {
      uint64_t p = perm ? perm[i] : i;
      const float *d = dirs + 3 * p;
      if (!dir_finite(d)) { bad |= 1; continue; }
      int64_t k = (int64_t)z_row(d[2], H) * W + phi_sector(d[0], d[1], W, ex, ey);
      energy[l * HW + k] += (uint64_t)w[p];
      if (count) count[l * HW + k] += 1u;
    }
  }
  free(ex); free(ey);
  return bad ? OR_E_RANGE : OR_OK;
}

/* ------------------------------------------------------------------------
 * Raw sampling map (Sec. 7.2 "Sampling map reconstruction": the energy map
 * is normalised before it is fed to the network).  The scale is not stated;
 * reading: mean-1 scaling, x_k = H*W*E_k / sum_j E_j, zero map if the sum is
 * zero.
 * ---------------------------------------------------------------------- */
void or_normalize_input(const uint64_t *energy, int64_t L, int H, int W, double *x) {
  int64_t HW = (int64_t)H * W;
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < L; l++) {
    uint64_t tot = 0;
    for (int64_t k = 0; k < HW; k++) tot += energy[l * HW + k];
    for (int64_t k = 0; k < HW; k++)
      x[l * HW + k] = tot ? (double)HW * (double)energy[l * HW + k] / (double)tot : 0.0;
  }
}

/* ------------------------------------------------------------------------
 * Network (Sec. 6.1 describes a compact U-Net; its figure and weights are
 * not published, so the networks evaluated are the stand-ins of the weight
 * file):
 *   arch 1 (CNN): 3x3 convs in sequence, ReLU after each but the last,
 *                 softplus after the last.
 *   arch 2 (U-Net, D levels): encoder level d = two 3x3 conv + ReLU
 *                 (level input is the previous level's output after a 2x2
 *                 average pool); decoder level d = nearest x2 upsample of
 *                 the level below, concatenated as [upsampled, skip],
 *                 two 3x3 conv + ReLU; head = 1x1 conv to one channel,
 *                 softplus.
 * Zero "same" padding.  softplus(x) = max(x,0) + log1p(exp(-|x|)).
 * Per-leaf planar [C][H][W] FP64 buffers, direct 7-deep loops.
 * ---------------------------------------------------------------------- */
typedef struct {
  int cout, cin, k;
  double *w; /* [cout][cin][k][k] */
  double *b; /* [cout] */
} or_layer;

typedef struct {
  int arch, levels, n;
  int in_ch; /* input channels: 1, or 5 for the five-channel U-Net */
  or_layer *layer;
} or_net;

static uint32_t rd_u32(const unsigned char *p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

static double rd_f32(const unsigned char *p) {
  uint32_t u = rd_u32(p);
  float f;
  memcpy(&f, &u, 4);
  return (double)f;
}

static void net_free(or_net *net) {
  if (!net->layer) return;
  for (int i = 0; i < net->n; i++) { free(net->layer[i].w); free(net->layer[i].b); }
  free(net->layer);
  net->layer = NULL;
}

/* Parse an NPGW v1 weight file; checks the topology of the declared arch. */
static int net_parse(const unsigned char *buf, size_t len, or_net *net) {
  memset(net, 0, sizeof(*net));
  if (len < 20 || memcmp(buf, "NPGW", 4) != 0 || rd_u32(buf + 4) != 1) return OR_E_ARG;
  net->arch = (int)rd_u32(buf + 8);
  net->levels = (int)rd_u32(buf + 12);
  net->n = (int)rd_u32(buf + 16);
  if (net->n <= 0 || net->n > 256) return OR_E_ARG;
  net->layer = calloc((size_t)net->n, sizeof(or_layer));
  size_t o = 20;
  for (int i = 0; i < net->n; i++) {
    if (o + 12 > len) { net_free(net); return OR_E_ARG; }
    or_layer *y = &net->layer[i];
    y->cout = (int)rd_u32(buf + o);
    y->cin = (int)rd_u32(buf + o + 4);
    y->k = (int)rd_u32(buf + o + 8);
    o += 12;
    if (y->cout <= 0 || y->cin <= 0 || (y->k != 1 && y->k != 3)) { net_free(net); return OR_E_ARG; }
    size_t nw = (size_t)y->cout * y->cin * y->k * y->k;
    if (o + 4 * (nw + (size_t)y->cout) > len) { net_free(net); return OR_E_ARG; }
    y->w = malloc(sizeof(double) * nw);
    y->b = malloc(sizeof(double) * (size_t)y->cout);
    for (size_t j = 0; j < nw; j++) y->w[j] = rd_f32(buf + o + 4 * j);
    o += 4 * nw;
    for (int j = 0; j < y->cout; j++) y->b[j] = rd_f32(buf + o + 4 * (size_t)j);
    o += 4 * (size_t)y->cout;
  }
  if (o != len) { net_free(net); return OR_E_ARG; }
  /* topology checks */
  net->in_ch = 1;
  if (net->arch == 1) {
    int c = 1;
    for (int i = 0; i < net->n; i++) {
      if (net->layer[i].cin != c || net->layer[i].k != 3) { net_free(net); return OR_E_ARG; }
      c = net->layer[i].cout;
    }
    if (c != 1) { net_free(net); return OR_E_ARG; }
  } else if (net->arch == 2) {
    int D = net->levels;
    if (D < 1 || net->n != 4 * D - 1) { net_free(net); return OR_E_ARG; }
    /* the first layer takes the one-channel raw map, or the five channels of
     * Sec. 6 (then as a masked convolution) */
    net->in_ch = net->layer[0].cin == 5 ? 5 : 1;
    int prev = net->in_ch;
    for (int d = 0; d < D; d++) {
      or_layer *a = &net->layer[2 * d], *b = &net->layer[2 * d + 1];
      if (a->cin != prev || a->k != 3 || b->cin != a->cout || b->cout != a->cout || b->k != 3) {
        net_free(net); return OR_E_ARG;
      }
      prev = a->cout;
    }
    int li = 2 * D;
    for (int d = D - 2; d >= 0; d--) {
      int cd = net->layer[2 * d].cout, cu = net->layer[2 * (d + 1)].cout;
      or_layer *a = &net->layer[li], *b = &net->layer[li + 1];
      if (a->cin != cu + cd || a->cout != cd || a->k != 3 || b->cin != cd || b->cout != cd || b->k != 3) {
        net_free(net); return OR_E_ARG;
      }
      li += 2;
    }
    or_layer *h = &net->layer[li];
    if (h->k != 1 || h->cout != 1 || h->cin != net->layer[0].cout) { net_free(net); return OR_E_ARG; }
  } else if (net->arch == 3) {
    /* the paper-style U-Net: five input channels, per level two 3x3 convs
     * (the deepest: one 3x3 conv and two dilated ones), decoder levels of two
     * convs on [upsampled, skip], a 1x1 head */
    int D = net->levels;
    if (D < 2 || net->n != 4 * D) { net_free(net); return OR_E_ARG; }
    net->in_ch = 5;
    int prev = 5, li = 0;
    for (int d = 0; d < D; d++) {
      int nconv = d == D - 1 ? 3 : 2;
      or_layer *a = &net->layer[li];
      if (a->cin != prev || a->k != 3) { net_free(net); return OR_E_ARG; }
      for (int j = 1; j < nconv; j++) {
        or_layer *b = &net->layer[li + j];
        if (b->cin != a->cout || b->cout != a->cout || b->k != 3) { net_free(net); return OR_E_ARG; }
      }
      prev = a->cout;
      li += nconv;
    }
    for (int d = D - 2; d >= 0; d--) {
      int cd = net->layer[2 * d].cout, cu = net->layer[d == D - 2 ? 2 * (D - 1) : 2 * (d + 1)].cout;
      or_layer *a = &net->layer[li], *b = &net->layer[li + 1];
      if (a->cin != cu + cd || a->cout != cd || a->k != 3 || b->cin != cd || b->cout != cd || b->k != 3) {
        net_free(net); return OR_E_ARG;
      }
      li += 2;
    }
    or_layer *h = &net->layer[li];
    if (h->k != 1 || h->cout != 1 || h->cin != net->layer[0].cout) { net_free(net); return OR_E_ARG; }
  } else {
    net_free(net);
    return OR_E_ARG;
  }
  return OR_OK;
}

/* out[co][y][x] = b[co] + sum_{ci,ky,kx} w[co][ci][ky][kx] * in[ci][y+ky-r][x+kx-r]
 * with zero padding (r = k/2). */
static void conv2d(const or_layer *y, const double *in, int H, int W, double *out) {
  int k = y->k, r = k / 2;
  for (int co = 0; co < y->cout; co++)
    for (int yy = 0; yy < H; yy++)
      for (int xx = 0; xx < W; xx++) {
        double acc = y->b[co];
        for (int ci = 0; ci < y->cin; ci++)
          for (int ky = 0; ky < k; ky++)
            for (int kx = 0; kx < k; kx++) {
              int sy = yy + ky - r, sx = xx + kx - r;
              if (sy < 0 || sy >= H || sx < 0 || sx >= W) continue;
              acc += y->w[((co * y->cin + ci) * k + ky) * k + kx] * in[((size_t)ci * H + sy) * W + sx];
            }
        out[((size_t)co * H + yy) * W + xx] = acc;
      }
}

/* Masked (partial) convolution, Liu et al. 2018, as the paper's first layer
 * (Sec. 6.1: only valid bins contribute): with the mask M = in[mask_ch]
 * (1 where the bin holds photons) and S = number of in-map taps of the
 * k x k window with M = 1 (outside the map M = 0),
 *   out = b + (k*k / S) * sum_{ci, taps} w * in * M   if S > 0, else 0. */
static void pconv2d(const or_layer *y, const double *in, int mask_ch, int H, int W, double *out) {
  int k = y->k, r = k / 2;
  const double *M = in + (size_t)mask_ch * H * W;
  for (int co = 0; co < y->cout; co++)
    for (int yy = 0; yy < H; yy++)
      for (int xx = 0; xx < W; xx++) {
        double acc = 0.0;
        int S = 0;
        for (int ky = 0; ky < k; ky++)
          for (int kx = 0; kx < k; kx++) {
            int sy = yy + ky - r, sx = xx + kx - r;
            if (sy < 0 || sy >= H || sx < 0 || sx >= W) continue;
            double m = M[(size_t)sy * W + sx];
            if (m != 0.0) S++;
            for (int ci = 0; ci < y->cin; ci++)
              acc += y->w[((co * y->cin + ci) * k + ky) * k + kx] * in[((size_t)ci * H + sy) * W + sx] * m;
          }
        out[((size_t)co * H + yy) * W + xx] = S > 0 ? y->b[co] + (double)(k * k) / (double)S * acc : 0.0;
      }
}

/* 3x3 (or 1x1) convolution with dilation `dil`: taps at offsets
 * (ky - r) * dil, (kx - r) * dil, zero padding. */
static void conv2d_dil(const or_layer *y, const double *in, int H, int W, int dil, double *out) {
  int k = y->k, r = k / 2;
  for (int co = 0; co < y->cout; co++)
    for (int yy = 0; yy < H; yy++)
      for (int xx = 0; xx < W; xx++) {
        double acc = y->b[co];
        for (int ci = 0; ci < y->cin; ci++)
          for (int ky = 0; ky < k; ky++)
            for (int kx = 0; kx < k; kx++) {
              int sy = yy + (ky - r) * dil, sx = xx + (kx - r) * dil;
              if (sy < 0 || sy >= H || sx < 0 || sx >= W) continue;
              acc += y->w[((co * y->cin + ci) * k + ky) * k + kx] * in[((size_t)ci * H + sy) * W + sx];
            }
        out[((size_t)co * H + yy) * W + xx] = acc;
      }
}

/* ELU (Clevert et al. 2016): x for x > 0, e^x - 1 otherwise. */
static void elu(double *a, size_t n) {
  for (size_t i = 0; i < n; i++) a[i] = a[i] > 0.0 ? a[i] : expm1(a[i]);
}

static void add_to(double *a, const double *b, size_t n) {
  for (size_t i = 0; i < n; i++) a[i] += b[i];
}

static void relu(double *a, size_t n) {
  for (size_t i = 0; i < n; i++) a[i] = a[i] > 0.0 ? a[i] : 0.0;
}

static double softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }

/* 2x2 average pool: mean of the four inputs. */
static void avgpool2(const double *in, int C, int H, int W, double *out) {
  int h = H / 2, w = W / 2;
  for (int c = 0; c < C; c++)
    for (int y = 0; y < h; y++)
      for (int x = 0; x < w; x++) {
        const double *p = in + ((size_t)c * H + 2 * y) * W + 2 * x;
        out[((size_t)c * h + y) * w + x] = (p[0] + p[1] + p[W] + p[W + 1]) / 4.0;
      }
}

/* nearest x2 upsample of lo [Cu][H/2][W/2] then channel concat with skip
 * [Cs][H][W]: out = [up(lo), skip]. */
static void upcat(const double *lo, int Cu, const double *skip, int Cs, int H, int W, double *out) {
  int h = H / 2, w = W / 2;
  for (int c = 0; c < Cu; c++)
    for (int y = 0; y < H; y++)
      for (int x = 0; x < W; x++)
        out[((size_t)c * H + y) * W + x] = lo[((size_t)c * h + y / 2) * w + x / 2];
  memcpy(out + (size_t)Cu * H * W, skip, sizeof(double) * (size_t)Cs * H * W);
}

/* The paper-style U-Net (Sec. 6.1: masked first convolution on the five
 * channels, ELU activations, residual links, a dilated bottleneck, skip
 * connections, at most 64 channels in the paper).  Encoder level d < D-1:
 * a = ELU(conv(x)), o = ELU(conv(a)) + a (residual), skip_d = o, next input
 * avgpool2(o).  Deepest level: a = ELU(conv(x)), b = ELU(conv_dil2(a)) + a,
 * o = ELU(conv_dil4(b)) + b.  Decoder level d: c = [up(o), skip_d],
 * a = ELU(conv(c)), o = ELU(conv(a)) + a.  Head: softplus(conv1x1(o)).  The
 * first conv is the masked (partial) convolution on the valid-bin mask. */
static void paper_forward_leaf(const or_net *net, const double *x, int H, int W, double *s) {
  size_t HW = (size_t)H * W;
  int D = net->levels;
  double **skip = calloc((size_t)D, sizeof(double *));
  int *hs = calloc((size_t)D, sizeof(int)), *wsz = calloc((size_t)D, sizeof(int));
  const double *cur = x;
  double *owned = NULL;
  int h = H, w = W, li = 0;
  for (int d = 0; d < D; d++) {
    const or_layer *la = &net->layer[li];
    double *pooled = NULL;
    if (d > 0) {
      pooled = malloc(sizeof(double) * (size_t)la->cin * (h / 2) * (w / 2));
      avgpool2(cur, la->cin, h, w, pooled);
      h /= 2; w /= 2;
      cur = pooled;
    }
    size_t n = (size_t)la->cout * h * w;
    double *a = malloc(sizeof(double) * n);
    if (d == 0)
      pconv2d(la, cur, 4, h, w, a);
    else
      conv2d(la, cur, h, w, a);
    elu(a, n);
    free(pooled);
    int nres = d == D - 1 ? 2 : 1;
    for (int j = 1; j <= nres; j++) {
      double *o = malloc(sizeof(double) * n);
      conv2d_dil(&net->layer[li + j], a, h, w, d == D - 1 ? 2 * j : 1, o);
      elu(o, n);
      add_to(o, a, n);
      free(a);
      a = o;
    }
    li += 1 + nres;
    if (d < D - 1) {
      skip[d] = a;
    } else {
      owned = a;
    }
    hs[d] = h; wsz[d] = w;
    cur = a;
  }
  for (int d = D - 2; d >= 0; d--) {
    const or_layer *la = &net->layer[li], *lb = &net->layer[li + 1];
    li += 2;
    h = hs[d]; w = wsz[d];
    int cs = net->layer[2 * d].cout, cu = la->cin - cs;
    double *cat = malloc(sizeof(double) * (size_t)la->cin * h * w);
    upcat(cur, cu, skip[d], cs, h, w, cat);
    size_t n = (size_t)la->cout * h * w;
    double *a = malloc(sizeof(double) * n);
    conv2d(la, cat, h, w, a);
    elu(a, n);
    double *o = malloc(sizeof(double) * n);
    conv2d(lb, a, h, w, o);
    elu(o, n);
    add_to(o, a, n);
    free(cat); free(a);
    free(owned);
    owned = o;
    cur = o;
  }
  double *head = malloc(sizeof(double) * HW);
  conv2d(&net->layer[li], cur, H, W, head);
  for (size_t k = 0; k < HW; k++) s[k] = softplus(head[k]);
  free(head);
  free(owned);
  for (int d = 0; d < D - 1; d++) free(skip[d]);
  free(skip); free(hs); free(wsz);
}

static void net_forward_leaf(const or_net *net, const double *x, int H, int W, double *s) {
  size_t HW = (size_t)H * W;
  if (net->arch == 3) {
    paper_forward_leaf(net, x, H, W, s);
    return;
  }
  if (net->arch == 1) {
    size_t cmax = 1;
    for (int i = 0; i < net->n; i++) if ((size_t)net->layer[i].cout > cmax) cmax = net->layer[i].cout;
    double *a = malloc(sizeof(double) * cmax * HW), *b = malloc(sizeof(double) * cmax * HW);
    memcpy(a, x, sizeof(double) * HW);
    for (int i = 0; i < net->n; i++) {
      conv2d(&net->layer[i], a, H, W, b);
      if (i + 1 < net->n) relu(b, (size_t)net->layer[i].cout * HW);
      double *t = a; a = b; b = t;
    }
    for (size_t k = 0; k < HW; k++) s[k] = softplus(a[k]);
    free(a); free(b);
    return;
  }
  int D = net->levels;
  double **skip = calloc((size_t)D, sizeof(double *));
  int *hs = calloc((size_t)D, sizeof(int)), *wsz = calloc((size_t)D, sizeof(int));
  const double *cur = x;
  double *owned = NULL;
  int h = H, w = W;
  for (int d = 0; d < D; d++) {
    const or_layer *la = &net->layer[2 * d], *lb = &net->layer[2 * d + 1];
    double *pooled = NULL;
    if (d > 0) {
      pooled = malloc(sizeof(double) * (size_t)la->cin * (h / 2) * (w / 2));
      avgpool2(cur, la->cin, h, w, pooled);
      h /= 2; w /= 2;
      cur = pooled;
    }
    double *t = malloc(sizeof(double) * (size_t)la->cout * h * w);
    if (d == 0 && net->in_ch == 5)
      pconv2d(la, cur, 4, h, w, t); /* channel 4 is the valid-bin mask */
    else
      conv2d(la, cur, h, w, t);
    relu(t, (size_t)la->cout * h * w);
    double *o = malloc(sizeof(double) * (size_t)lb->cout * h * w);
    conv2d(lb, t, h, w, o);
    relu(o, (size_t)lb->cout * h * w);
    free(t);
    free(pooled);
    skip[d] = o; hs[d] = h; wsz[d] = w;
    cur = o;
  }
  int li = 2 * D;
  for (int d = D - 2; d >= 0; d--) {
    const or_layer *la = &net->layer[li], *lb = &net->layer[li + 1];
    li += 2;
    h = hs[d]; w = wsz[d];
    int cs = net->layer[2 * d].cout, cu = la->cin - cs;
    double *cat = malloc(sizeof(double) * (size_t)la->cin * h * w);
    upcat(cur, cu, skip[d], cs, h, w, cat);
    double *t = malloc(sizeof(double) * (size_t)la->cout * h * w);
    conv2d(la, cat, h, w, t);
    relu(t, (size_t)la->cout * h * w);
    double *o = malloc(sizeof(double) * (size_t)lb->cout * h * w);
    conv2d(lb, t, h, w, o);
    relu(o, (size_t)lb->cout * h * w);
    free(cat); free(t);
    free(owned);
    owned = o;
    cur = o;
  }
  double *head = malloc(sizeof(double) * HW);
  conv2d(&net->layer[li], cur, H, W, head);
  for (size_t k = 0; k < HW; k++) s[k] = softplus(head[k]);
  free(head);
  free(owned);
  for (int d = 0; d < D; d++) free(skip[d]);
  free(skip); free(hs); free(wsz);
}

/* s[L][H][W] = network(x[L][H][W]) for a parsed NPGW file. */
int or_net_forward(const unsigned char *model, size_t model_len, const double *x,
                   int64_t L, int H, int W, double *s) {
  or_net net;
  int rc = net_parse(model, model_len, &net);
  if (rc) return rc;
  if (net.arch == 2) {
    int D = net.levels;
    if ((H >> (D - 1)) < 1 || (W >> (D - 1)) < 1 || (H % (1 << (D - 1))) || (W % (1 << (D - 1)))) {
      net_free(&net);
      return OR_E_ARG;
    }
  }
  size_t HW = (size_t)H * W;
  if (net.in_ch != 1) {
    net_free(&net);
    return OR_E_ARG;
  }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t l = 0; l < L; l++) net_forward_leaf(&net, x + (size_t)l * HW, H, W, s + (size_t)l * HW);
  net_free(&net);
  return OR_OK;
}

/* s[L][H][W] = five-channel network(x[L][5][H][W]). */
int or_net_forward5(const unsigned char *model, size_t model_len, const double *x,
                    int64_t L, int H, int W, double *s) {
  or_net net;
  int rc = net_parse(model, model_len, &net);
  if (rc) return rc;
  int D = net.levels;
  if ((net.arch != 2 && net.arch != 3) || net.in_ch != 5 || (H % (1 << (D - 1))) || (W % (1 << (D - 1)))) {
    net_free(&net);
    return OR_E_ARG;
  }
  size_t HW = (size_t)H * W;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t l = 0; l < L; l++) net_forward_leaf(&net, x + (size_t)l * 5 * HW, H, W, s + (size_t)l * HW);
  net_free(&net);
  return OR_OK;
}

/* The five input channels of Sec. 6 for each leaf: the raw sampling maps of
 * iterations t and t-1 (energies E, mean 1: H*W*E/sum(E) in FP64, 0 for an
 * empty map), their photon-count maps normalised the same way, and the mask
 * of bins holding photons at iteration t.  x[L][5][H][W], FP64 throughout. */
void or_input5(const uint64_t *e_t, const uint64_t *e_p, const uint32_t *p_t, const uint32_t *p_p,
               int64_t L, int H, int W, double *x) {
  size_t HW = (size_t)H * W;
#pragma omp parallel for schedule(static)
  for (int64_t l = 0; l < L; l++) {
    const uint64_t *E[2] = {e_t + l * HW, e_p + l * HW};
    const uint32_t *P[2] = {p_t + l * HW, p_p + l * HW};
    double *xl = x + (size_t)l * 5 * HW;
    for (int c = 0; c < 2; c++) {
      double S = 0.0, T = 0.0;
      for (size_t k = 0; k < HW; k++) {
        S += (double)E[c][k];
        T += (double)P[c][k];
      }
      for (size_t k = 0; k < HW; k++) {
        xl[(size_t)c * HW + k] = S > 0.0 ? (double)HW * (double)E[c][k] / S : 0.0;
        xl[(size_t)(2 + c) * HW + k] = T > 0.0 ? (double)HW * (double)P[c][k] / T : 0.0;
      }
    }
    for (size_t k = 0; k < HW; k++) xl[4 * HW + k] = P[0][k] > 0 ? 1.0 : 0.0;
  }
}

/* One masked convolution layer (weights OIHW f32, bias f32) on in[C][H][W]
 * with the mask in channel mask_ch, for pins. */
void or_pconv2d(const float *w, const float *b, int cout, int cin, int k, const double *in, int mask_ch,
                int H, int W, double *out) {
  or_layer y;
  size_t nw = (size_t)cout * cin * k * k;
  y.cout = cout; y.cin = cin; y.k = k;
  y.w = malloc(sizeof(double) * nw);
  y.b = malloc(sizeof(double) * (size_t)cout);
  for (size_t i = 0; i < nw; i++) y.w[i] = (double)w[i];
  for (int i = 0; i < cout; i++) y.b[i] = b ? (double)b[i] : 0.0;
  pconv2d(&y, in, mask_ch, H, W, out);
  free(y.w); free(y.b);
}

/* Raw layer access for brute-force conv checks: one conv of a single
 * layer (weights OIHW f32, bias f32) on in[C][H][W] (FP64). */
void or_conv2d_dil(const float *w, const float *b, int cout, int cin, int k, const double *in, int dil, int H,
                   int W, double *out) {
  or_layer y = {cout, cin, k, malloc(sizeof(double) * (size_t)cout * cin * k * k), malloc(sizeof(double) * cout)};
  for (size_t i = 0; i < (size_t)cout * cin * k * k; i++) y.w[i] = (double)w[i];
  for (int i = 0; i < cout; i++) y.b[i] = b ? (double)b[i] : 0.0;
  conv2d_dil(&y, in, H, W, dil, out);
  free(y.w);
  free(y.b);
}

void or_conv2d(const float *w, const float *b, int cout, int cin, int k,
               const double *in, int H, int W, double *out) {
  or_layer y;
  size_t nw = (size_t)cout * cin * k * k;
  y.cout = cout; y.cin = cin; y.k = k;
  y.w = malloc(sizeof(double) * nw);
  y.b = malloc(sizeof(double) * (size_t)cout);
  for (size_t i = 0; i < nw; i++) y.w[i] = (double)w[i];
  for (int i = 0; i < cout; i++) y.b[i] = b ? (double)b[i] : 0.0;
  conv2d(&y, in, H, W, out);
  free(y.w); free(y.b);
}

/* ------------------------------------------------------------------------
 * Sampling density and CDF tables (Eq. "energy_target": the guide pdf is
 * proportional to the map value over the bin's solid angle; Sec. 7.3:
 * the map is sampled like an environment map from a CDF built by a
 * cumulative sum over pixels).
 *   p_k = s_k / sum_j s_j (FP64); pdf_k = p_k * H*W / (4 pi) [1/sr], since
 *   every bin covers 4pi/(HW) sr.
 *   m_i = sum_j p_{i,j}; M_0 = 0, M_i = sum_{i'<i} m_{i'}, M_H := 1.
 *   C_{i,0} = 0, C_{i,j} = sum_{j'<j} p_{i,j'} / m_i, C_{i,W} := 1;
 *   a row with m_i = 0 gets C_{i,j} = j/W.
 * Tables are stored as float32 rounded from the FP64 prefixes; total in FP64.
 * A leaf whose density sums to zero (or is not finite) is an error: its
 * tables are written as NaN and the total as 0.
 * ---------------------------------------------------------------------- */
int or_build_cdf(const double *s, int64_t L, int H, int W, float *pdf, float *marg,
                 float *cond, double *total) {
  int64_t HW = (int64_t)H * W;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t l = 0; l < L; l++) {
    const double *sl = s + l * HW;
    double S = 0.0;
    int ok = 1;
    for (int64_t k = 0; k < HW; k++) {
      if (!(sl[k] >= 0.0) || !isfinite(sl[k])) ok = 0;
      S += sl[k];
    }
    if (!ok || !(S > 0.0) || !isfinite(S)) {
      bad |= 1;
      total[l] = 0.0;
      for (int64_t k = 0; k < HW; k++) pdf[l * HW + k] = NAN;
      for (int i = 0; i <= H; i++) marg[l * (H + 1) + i] = NAN;
      for (int64_t k = 0; k < (int64_t)H * (W + 1); k++) cond[l * H * (W + 1) + k] = NAN;
      continue;
    }
    total[l] = S;
    double M = 0.0;
    for (int i = 0; i < H; i++) {
      marg[l * (H + 1) + i] = (float)M;
      double m = 0.0;
      for (int j = 0; j < W; j++) {
        double p = sl[i * W + j] / S;
        pdf[l * HW + i * W + j] = (float)(p * (double)HW / (4.0 * M_PI));
        m += p;
      }
      float *c = cond + (l * H + i) * (W + 1);
      if (m > 0.0) {
        double C = 0.0;
        for (int j = 0; j < W; j++) {
          c[j] = (float)(C / m);
          C += sl[i * W + j] / S;
        }
      } else {
        for (int j = 0; j < W; j++) c[j] = (float)((double)j / (double)W);
      }
      c[W] = 1.0f;
      M += m;
    }
    marg[l * (H + 1) + H] = 1.0f;
  }
  return bad ? OR_E_RANGE : OR_OK;
}

/* ------------------------------------------------------------------------
 * Guided direction sampling by inversion of the tables (Sec. 7.3;
 * Algorithm 1, guided-sampling step).  Reading: piecewise-constant map, the two caller
 * uniforms select the row and column and are reused for the offset inside
 * the bin.
 *   i = max{ i in [0,H-1] : M_i <= u1 },  j = max{ j in [0,W-1] : C_{i,j} <= u2 }
 *   t1 = (u1 - M_i)/(M_{i+1} - M_i), t2 likewise, clamped to [0, 1)
 *   z = -1 + 2(i + t1)/H, phi = 2pi (j + t2)/W,
 *   w = (sqrt(1-z^2) cos phi, sqrt(1-z^2) sin phi, z), pdf = pdf table[i][j].
 * Leaf >= L or u outside [0,1): error; outputs NaN direction, pdf NaN,
 * bin 0xffffffff.
 * ---------------------------------------------------------------------- */
int or_sample(const float *pdf, const float *marg, const float *cond, int64_t L, int H, int W,
              const uint32_t *leaf, const float *u, int64_t n,
              double *dir_out, float *pdf_out, uint32_t *bin_out) {
  int bad = 0;
  const double below1 = nextafter(1.0, 0.0);
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t q = 0; q < n; q++) {
    uint32_t l = leaf[q];
    float u1 = u[2 * q], u2 = u[2 * q + 1];
    if ((int64_t)l >= L || !(u1 >= 0.0f && u1 < 1.0f) || !(u2 >= 0.0f && u2 < 1.0f)) {
      bad |= 1;
      dir_out[3 * q] = dir_out[3 * q + 1] = dir_out[3 * q + 2] = NAN;
      pdf_out[q] = NAN;
      if (bin_out) bin_out[q] = 0xffffffffu;
      continue;
    }
    const float *M = marg + (int64_t)l * (H + 1);
    int i = 0;
    for (int r = 0; r < H; r++) if (M[r] <= u1) i = r;
    const float *C = cond + ((int64_t)l * H + i) * (W + 1);
    int j = 0;
    for (int c = 0; c < W; c++) if (C[c] <= u2) j = c;
    double t1 = ((double)u1 - (double)M[i]) / ((double)M[i + 1] - (double)M[i]);
    double t2 = ((double)u2 - (double)C[j]) / ((double)C[j + 1] - (double)C[j]);
    if (!(t1 >= 0.0)) t1 = 0.0;
    if (t1 > below1) t1 = below1;
    if (!(t2 >= 0.0)) t2 = 0.0;
    if (t2 > below1) t2 = below1;
    double z = -1.0 + 2.0 * ((double)i + t1) / (double)H;
    double phi = 2.0 * M_PI * ((double)j + t2) / (double)W;
    double r = sqrt(fmax(0.0, 1.0 - z * z));
    dir_out[3 * q] = r * cos(phi);
    dir_out[3 * q + 1] = r * sin(phi);
    dir_out[3 * q + 2] = z;
    pdf_out[q] = pdf[(int64_t)l * H * W + (int64_t)i * W + j];
    if (bin_out) bin_out[q] = (uint32_t)(i * W + j);
  }
  return bad ? OR_E_RANGE : OR_OK;
}

/* pdf of a direction under a leaf's map: the table value of its bin (the
 * guide term of the one-sample MIS pdf, Eq. "mis_coef").  Leaf >= L or a
 * non-finite direction: error, pdf 0. */
int or_eval_pdf(const float *pdf, int64_t L, int H, int W, const uint32_t *leaf,
                const float *dirs, int64_t n, float *pdf_out) {
  float *ex = malloc(sizeof(float) * W), *ey = malloc(sizeof(float) * W);
  or_boundaries(W, ex, ey);
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t q = 0; q < n; q++) {
    const float *d = dirs + 3 * q;
    if ((int64_t)leaf[q] >= L || !dir_finite(d)) { bad |= 1; pdf_out[q] = 0.0f; continue; }
    int64_t k = (int64_t)z_row(d[2], H) * W + phi_sector(d[0], d[1], W, ex, ey);
    pdf_out[q] = pdf[(int64_t)leaf[q] * H * W + k];
  }
  free(ex); free(ey);
  return bad ? OR_E_RANGE : OR_OK;
}

/* ------------------------------------------------------------------------
 * Adaptive spatial hierarchy (Sec. 7.1, "Voxel subdivision": a voxel is
 * split when its photon count exceeds a threshold, recursively).  Stand-in
 * read as an octree over the unit box: the root [0,1)^3 has depth 0; a cell
 * splits into its 8 octants iff count > T and depth < Dmax; the octants are
 * the midpoint halves on every axis.  Leaves are the unsplit cells holding
 * at least one photon, numbered in ascending Morton order (child index =
 * x | y<<1 | z<<2 of the upper-half flags).  Within a leaf the photons keep
 * their input order, so perm is unique.  Leaf key = Morton code of the
 * cell's lowest corner on the 2^21 lattice (x in the lowest bit of every
 * bit triple), shifted to 63 bits.
 * Built here by literal recursion with explicit coordinate comparisons
 * against the cell bounds (exact: bounds are dyadic).
 * ---------------------------------------------------------------------- */
typedef struct {
  const float *pos;
  uint32_t T;
  int Dmax;
  uint32_t *perm, *leaf_of, *leaf_off;
  uint64_t *key;
  uint8_t *depth;
  int64_t max_leaves, nleaves, written;
  int overflow;
} tree_ctx;

static uint64_t morton_of_corner(uint32_t ix, uint32_t iy, uint32_t iz) {
  uint64_t k = 0;
  for (int b = 0; b < 21; b++) {
    k |= (uint64_t)((ix >> b) & 1u) << (3 * b);
    k |= (uint64_t)((iy >> b) & 1u) << (3 * b + 1);
    k |= (uint64_t)((iz >> b) & 1u) << (3 * b + 2);
  }
  return k;
}

/* cell = [lo, lo + 2^-d)^3 with lo = (ix, iy, iz) * 2^-d */
static void tree_rec(tree_ctx *t, const uint32_t *idx, int64_t n, int d,
                     uint32_t ix, uint32_t iy, uint32_t iz) {
  if (n == 0) return;
  if (n > (int64_t)t->T && d < t->Dmax) {
    /* split at the cell midpoint on every axis; photons keep their order */
    double half = ldexp(1.0, -(d + 1));
    double mx = (2.0 * ix + 1.0) * half, my = (2.0 * iy + 1.0) * half, mz = (2.0 * iz + 1.0) * half;
    unsigned char *child = malloc((size_t)n);
    int64_t cnt[8] = {0}, at[8];
    for (int64_t i = 0; i < n; i++) {
      const float *p = t->pos + 3 * (size_t)idx[i];
      int c = ((double)p[0] >= mx) | (((double)p[1] >= my) << 1) | (((double)p[2] >= mz) << 2);
      child[i] = (unsigned char)c;
      cnt[c]++;
    }
    at[0] = 0;
    for (int c = 1; c < 8; c++) at[c] = at[c - 1] + cnt[c - 1];
    uint32_t *sub = malloc(sizeof(uint32_t) * (size_t)n);
    int64_t fill[8];
    memcpy(fill, at, sizeof(fill));
    for (int64_t i = 0; i < n; i++) sub[fill[child[i]]++] = idx[i];
    free(child);
    for (int c = 0; c < 8; c++)
      tree_rec(t, sub + at[c], cnt[c], d + 1, 2 * ix + (c & 1), 2 * iy + ((c >> 1) & 1),
               2 * iz + ((c >> 2) & 1));
    free(sub);
    return;
  }
  int64_t id = t->nleaves++;
  if (id >= t->max_leaves) { t->overflow = 1; return; }
  t->leaf_off[id] = (uint32_t)t->written;
  uint32_t sh = (uint32_t)(21 - d);
  t->key[id] = morton_of_corner(ix << sh, iy << sh, iz << sh);
  t->depth[id] = (uint8_t)d;
  for (int64_t i = 0; i < n; i++) {
    t->perm[t->written + i] = idx[i];
    t->leaf_of[idx[i]] = (uint32_t)id;
  }
  t->written += n;
  t->leaf_off[id + 1] = (uint32_t)t->written;
}

int or_build_tree(const float *pos, int64_t n, uint32_t T, int Dmax, uint32_t *perm,
                  uint32_t *leaf_of, uint32_t *leaf_off, uint64_t *key, uint8_t *depth,
                  int64_t max_leaves, int64_t *n_leaves) {
  if (Dmax < 0 || Dmax > 21 || n < 0 || n > 0xffffffffLL) return OR_E_ARG;
  for (int64_t i = 0; i < 3 * n; i++)
    if (!(pos[i] >= 0.0f && pos[i] < 1.0f)) return OR_E_RANGE;
  uint32_t *idx = malloc(sizeof(uint32_t) * (size_t)(n ? n : 1));
  for (int64_t i = 0; i < n; i++) idx[i] = (uint32_t)i;
  tree_ctx t = {pos, T, Dmax, perm, leaf_of, leaf_off, key, depth, max_leaves, 0, 0, 0};
  leaf_off[0] = 0;
  tree_rec(&t, idx, n, 0, 0, 0, 0);
  free(idx);
  *n_leaves = t.nleaves;
  return t.overflow ? OR_E_CAPACITY : OR_OK;
}
