// Network evaluation: weight-file loading and repacking, the convolution
// kernels, and the per-chunk CNN / U-Net schedule.
//
// Activations are channel-last per leaf, [leaf][y][x][c].  3x3 convolutions
// with at least 16 output channels run as implicit GEMMs on the matrix cores.
// FP32 mode: the float32 weights as loaded, binary64 activations, products
// and sums (v_mfma_f64_16x16x4f64), softplus in binary64, float32 densities.
// A float32 accumulation chain over K = 9*Cin terms and 15 layers loses ~3e-5
// relative accuracy in the output pdf, and float32 activation storage alone
// ~1e-5 on spiky leaves; with binary64 activations (and the normalised input
// map formed in binary64 as well) the only rounding left is that of the
// float32 output densities.  BF16 mode: bf16 activations
// and weights, float32 accumulation (v_mfma_f32_16x16x32_bf16).
//   M = output pixels of a tile, N = output channels, K = 9 taps x input
//   channels.
// A workgroup (4 wavefronts) owns a tile of 64*MW pixels (rows of one leaf)
// and all output channels.  For each chunk of KC input channels it stages
// the tile's input patch with a one-pixel halo in LDS, plus the chunk's
// weights, and the nine taps read shifted windows of the patch, so each
// input element is fetched from memory once per chunk.  The 2x2 average pool
// (encoder) and the nearest upsample + skip concatenation (decoder) are
// folded into the patch loads; bias and ReLU into the epilogue; the 1x1 head
// and softplus into the epilogue of the last decoder convolution.  The first
// layer (one input channel) is computed into the second layer's patch, or
// runs as a direct convolution like any layer the tiling does not fit; it
// computes the normalised input map from the energy map on the fly.  FP8
// mode: e4m3 activations and weights with static per-layer scales.
// Five-channel models (maps and photon counts of two iterations and the
// valid-bin mask) start with a masked (partial) convolution kernel; the
// paper-style U-Net adds ELU, residual links and dilated convolutions, which
// the tiles take in an extended form (a wider halo, the activation and the
// residual add in the epilogue) compiled only for the layers that use it.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <string>
#include <mutex>
#include <vector>

#include "npg_internal.h"

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef long fp8x8;  // eight e4m3 bytes

// ------------------------------------------------------------------ model
struct LayerDev {
  int cout = 0, cin = 0, k = 0;
  float *w = nullptr;          // OIHW float32
  float *b = nullptr;          // [cout]
  float *pk32 = nullptr;       // [chunk][tap][kc16][cout]
  double *pkp = nullptr;       // [chunk][phase][tap 2x2][kc16][cout]: weights of a 3x3 conv on a
                               // nearest-upsampled input, merged per output phase (exact sums)
  double *pk64 = nullptr;      // pk32 in binary64 (read by some FP64 tiles)
  uint16_t *pk16 = nullptr;    // [chunk][tap][cout][kc32] (bf16 bits)
  uint16_t *pk16s = nullptr;   // [chunk][tap][cout][kc16] (bf16 bits)
  // FP8 (after calibration): e4m3 weights with the input channels' activation
  // scales folded in, and one dequantisation scale per output channel
  uint8_t *pk8 = nullptr;      // [chunk][tap][cout][kc32]
  uint8_t *pk8s = nullptr;     // [chunk][tap][cout][kc16]
  float *wsc8 = nullptr;       // [cout]
  float a8 = 1.0f;             // value of one e4m3 unit of this layer's output
  int dil = 1;                 // dilation of a 3x3 layer (the paper-style bottleneck: 2, 4)
};

struct npg_model {
  npg_ctx *ctx = nullptr;
  int arch = 0, levels = 0;
  int in_ch = 1;  // 1, or 5: the five-channel U-Net (masked first layer)
  std::vector<LayerDev> layer;
  std::vector<std::vector<float>> host_w, host_b;
  void *blob = nullptr;  // one device allocation holding every array
  size_t blob_bytes = 0;
  void *blob8 = nullptr;  // FP8 weights and scales (calibration)
  size_t blob8_bytes = 0;
  bool fp8_ready = false;
};

namespace {

uint32_t rd32(const unsigned char *p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

uint16_t f32_to_bf16_host(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

constexpr int KC32 = 16;  // input channels per chunk, FP32 path
constexpr int KC16 = 32;  // input channels per chunk, BF16 path
constexpr int KC16S = 16; // BF16 path for 16- and 48-channel inputs: one 32-wide
                          // MFMA K slice covers two taps of 16 channels
constexpr int KC8 = 32;   // FP8 path, as BF16
constexpr int KC8S = 16;
constexpr float E4M3_MAX = 448.0f;

}  // namespace

// OCP FP8 e4m3: 1 sign, 4 exponent bits (bias 7), 3 mantissa bits, no
// infinities, 0x7f / 0xff NaN, largest finite 448, subnormal step 2^-9.
// Encoding rounds to nearest even and saturates at +-448.
__host__ __device__ inline uint8_t e4m3_enc(float x) {
  if (x != x) return 0x7f;
  uint8_t s = 0;
  if (x < 0.0f) {
    s = 0x80;
    x = -x;
  }
  if (x >= E4M3_MAX) return s | 0x7e;
  if (x < 0.015625f) return s | (uint8_t)rintf(x * 512.0f);  // subnormal (8 -> 0x08, the smallest normal)
  int e;
  (void)frexpf(x, &e);                          // x in [2^(e-1), 2^e)
  int m = (int)rintf(ldexpf(x, 4 - e)) - 8;     // mantissa steps of 2^(e-4), in [0, 8]
  int E = e - 1 + 7;
  if (m == 8) {
    m = 0;
    ++E;
  }
  return s | (uint8_t)((E << 3) | m);  // x < 448 keeps (E, m) <= (15, 6)
}
__host__ __device__ inline float e4m3_dec(uint8_t v) {
  const int e = (v >> 3) & 15, m = v & 7;
  float mag = e ? ldexpf((float)(8 + m), e - 10) : ldexpf((float)m, -9);
  if ((v & 0x7f) == 0x7f) mag = NAN;
  return (v & 0x80) ? -mag : mag;
}

// Device forms on the conversion instructions (gfx950 converts to OCP e4m3
// with round to nearest even; out-of-range inputs, which would give NaN,
// are clamped first so that both forms saturate alike).
__device__ __forceinline__ uint8_t e4m3_enc_d(float x) {
  const float c = x != x ? x : fminf(fmaxf(x, -E4M3_MAX), E4M3_MAX);
  return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(c, c, 0, false) & 0xff);
}
__device__ __forceinline__ float e4m3_dec_d(uint8_t v) { return __builtin_amdgcn_cvt_f32_fp8((int)v, 0); }
// Four values as four e4m3 bytes (first value in the low byte), each clamped
// and rounded as e4m3_enc_d does: two conversion instructions.
__device__ __forceinline__ float e4m3_clamp_d(float x) { return x != x ? x : fminf(fmaxf(x, -E4M3_MAX), E4M3_MAX); }
__device__ __forceinline__ uint32_t e4m3_pack4_d(float a, float b, float c, float d) {
  const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp_d(a), e4m3_clamp_d(b), 0, false);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(e4m3_clamp_d(c), e4m3_clamp_d(d), lo, true);
}

// Parses the NPGW v1 file and checks the declared topology.
static int parse_model(npg_ctx *ctx, const unsigned char *buf, size_t len, npg_model *m) {
  if (len < 20 || memcmp(buf, "NPGW", 4) != 0 || rd32(buf + 4) != 1)
    return npg_fail(ctx, NPG_E_ARG, "model: not an NPGW v1 file");
  m->arch = (int)rd32(buf + 8);
  m->levels = (int)rd32(buf + 12);
  const int n = (int)rd32(buf + 16);
  if (n <= 0 || n > 256) return npg_fail(ctx, NPG_E_ARG, "model: bad layer count %d", n);
  size_t o = 20;
  m->layer.resize(n);
  m->host_w.resize(n);
  m->host_b.resize(n);
  for (int i = 0; i < n; ++i) {
    if (o + 12 > len) return npg_fail(ctx, NPG_E_ARG, "model: truncated");
    LayerDev &y = m->layer[i];
    y.cout = (int)rd32(buf + o);
    y.cin = (int)rd32(buf + o + 4);
    y.k = (int)rd32(buf + o + 8);
    o += 12;
    if (y.cout <= 0 || y.cin <= 0 || y.cout > 4096 || y.cin > 4096 || (y.k != 1 && y.k != 3))
      return npg_fail(ctx, NPG_E_ARG, "model: bad layer %d shape", i);
    const size_t nw = (size_t)y.cout * y.cin * y.k * y.k;
    if (o + 4 * (nw + y.cout) > len) return npg_fail(ctx, NPG_E_ARG, "model: truncated weights");
    m->host_w[i].resize(nw);
    m->host_b[i].resize(y.cout);
    memcpy(m->host_w[i].data(), buf + o, 4 * nw);
    o += 4 * nw;
    memcpy(m->host_b[i].data(), buf + o, 4 * (size_t)y.cout);
    o += 4 * (size_t)y.cout;
  }
  if (o != len) return npg_fail(ctx, NPG_E_ARG, "model: %zu trailing bytes", len - o);
  if (m->arch == 1) {
    int c = 1;
    for (int i = 0; i < n; ++i) {
      if (m->layer[i].cin != c || m->layer[i].k != 3) return npg_fail(ctx, NPG_E_ARG, "model: CNN layer %d", i);
      c = m->layer[i].cout;
    }
    if (c != 1) return npg_fail(ctx, NPG_E_ARG, "model: CNN must end with one channel");
  } else if (m->arch == 2) {
    const int D = m->levels;
    if (D < 1 || D > 10 || n != 4 * D - 1) return npg_fail(ctx, NPG_E_ARG, "model: U-Net layer count");
    // one input channel (the raw map), or the five of the paper's input
    m->in_ch = m->layer[0].cin == 5 ? 5 : 1;
    int prev = m->in_ch;
    for (int d = 0; d < D; ++d) {
      const LayerDev &a = m->layer[2 * d], &b = m->layer[2 * d + 1];
      if (a.cin != prev || a.k != 3 || b.cin != a.cout || b.cout != a.cout || b.k != 3)
        return npg_fail(ctx, NPG_E_ARG, "model: U-Net encoder level %d", d);
      prev = a.cout;
    }
    int li = 2 * D;
    for (int d = D - 2; d >= 0; --d) {
      const int cd = m->layer[2 * d].cout, cu = m->layer[2 * (d + 1)].cout;
      const LayerDev &a = m->layer[li], &b = m->layer[li + 1];
      if (a.cin != cu + cd || a.cout != cd || a.k != 3 || b.cin != cd || b.cout != cd || b.k != 3)
        return npg_fail(ctx, NPG_E_ARG, "model: U-Net decoder level %d", d);
      li += 2;
    }
    const LayerDev &h = m->layer[li];
    if (h.k != 1 || h.cout != 1 || h.cin != m->layer[0].cout)
      return npg_fail(ctx, NPG_E_ARG, "model: U-Net head");
  } else if (m->arch == 3) {
    // the paper-style U-Net: five input channels; encoder levels of two 3x3
    // convs, the deepest of one 3x3 conv and two convs of dilation 2 and 4;
    // decoder levels of two convs on [upsampled, skip]; a 1x1 head
    const int D = m->levels;
    if (D < 2 || D > 10 || n != 4 * D) return npg_fail(ctx, NPG_E_ARG, "model: paper U-Net layer count");
    m->in_ch = 5;
    int prev = 5, li = 0;
    for (int d = 0; d < D; ++d) {
      const int nconv = d == D - 1 ? 3 : 2;
      const LayerDev &a = m->layer[li];
      if (a.cin != prev || a.k != 3) return npg_fail(ctx, NPG_E_ARG, "model: paper U-Net encoder level %d", d);
      for (int j = 1; j < nconv; ++j) {
        LayerDev &b = m->layer[li + j];
        if (b.cin != a.cout || b.cout != a.cout || b.k != 3)
          return npg_fail(ctx, NPG_E_ARG, "model: paper U-Net encoder level %d", d);
        if (d == D - 1) b.dil = 2 * j;
      }
      prev = a.cout;
      li += nconv;
    }
    for (int d = D - 2; d >= 0; --d) {
      const int cd = m->layer[2 * d].cout, cu = m->layer[2 * (d + 1)].cout;
      const LayerDev &a = m->layer[li], &b = m->layer[li + 1];
      if (a.cin != cu + cd || a.cout != cd || a.k != 3 || b.cin != cd || b.cout != cd || b.k != 3)
        return npg_fail(ctx, NPG_E_ARG, "model: paper U-Net decoder level %d", d);
      li += 2;
    }
    const LayerDev &h = m->layer[li];
    if (h.k != 1 || h.cout != 1 || h.cin != m->layer[0].cout)
      return npg_fail(ctx, NPG_E_ARG, "model: paper U-Net head");
  } else {
    return npg_fail(ctx, NPG_E_ARG, "model: unknown arch %d", m->arch);
  }
  return NPG_OK;
}

extern "C" int npg_model_load(npg_ctx *ctx, const void *host_bytes, size_t n_bytes, npg_model **out) {
  if (!ctx || !out) return NPG_E_ARG;
  *out = nullptr;
  if (!host_bytes) return npg_fail(ctx, NPG_E_ARG, "model: null buffer");
  npg_model *m = new npg_model();
  m->ctx = ctx;
  int rc = parse_model(ctx, static_cast<const unsigned char *>(host_bytes), n_bytes, m);
  if (rc) {
    delete m;
    return rc;
  }
  // host-side repacking into one blob
  std::vector<char> blob;
  struct Off { size_t w, b, p32, p16, p16s, pp, p64; };
  std::vector<Off> offs(m->layer.size());
  auto put = [&](const void *src, size_t bytes) {
    size_t at = npg_align(blob.size());
    blob.resize(at + npg_align(bytes));
    memcpy(blob.data() + at, src, bytes);
    return at;
  };
  for (size_t i = 0; i < m->layer.size(); ++i) {
    const LayerDev &y = m->layer[i];
    const std::vector<float> &w = m->host_w[i];
    offs[i].w = put(w.data(), 4 * w.size());
    offs[i].b = put(m->host_b[i].data(), 4 * (size_t)y.cout);
    offs[i].p32 = offs[i].p16 = offs[i].p16s = offs[i].pp = offs[i].p64 = (size_t)-1;
    if (y.k == 3) {
      const int nch32 = (y.cin + KC32 - 1) / KC32, nch16 = (y.cin + KC16 - 1) / KC16;
      const int nch16s = (y.cin + KC16S - 1) / KC16S;
      std::vector<float> p32((size_t)nch32 * 9 * KC32 * y.cout, 0.0f);
      std::vector<uint16_t> p16((size_t)nch16 * 9 * y.cout * KC16, 0);
      std::vector<uint16_t> p16s((size_t)nch16s * 9 * y.cout * KC16S, 0);
      for (int co = 0; co < y.cout; ++co)
        for (int ci = 0; ci < y.cin; ++ci)
          for (int t = 0; t < 9; ++t) {
            const float v = w[((size_t)co * y.cin + ci) * 9 + t];
            const int c32 = ci / KC32, k32 = ci % KC32;
            p32[(((size_t)c32 * 9 + t) * KC32 + k32) * y.cout + co] = v;
            const int c16 = ci / KC16, k16 = ci % KC16;
            p16[(((size_t)c16 * 9 + t) * y.cout + co) * KC16 + k16] = f32_to_bf16_host(v);
            const int c16s = ci / KC16S, k16s = ci % KC16S;
            p16s[(((size_t)c16s * 9 + t) * y.cout + co) * KC16S + k16s] = f32_to_bf16_host(v);
          }
      offs[i].p32 = put(p32.data(), 4 * p32.size());
      if (y.cin >= 16) {
        // On a nearest-upsampled input, output pixel (2i + a, 2j + b) reads
        // low-resolution rows {i - 1, i} (a = 0: kernel row 0, then rows
        // 1 + 2) or {i, i + 1} (a = 1: rows 0 + 1, then row 2), and columns
        // likewise: per phase (a, b) a 2x2 conv whose taps are sums of the
        // 3x3 taps; the sums of float32 weights are exact in binary64.
        static const int lo[2][2] = {{0, 1}, {0, 2}}, hi[2][2] = {{0, 2}, {1, 2}};  // [a][i]: rows lo..hi
        std::vector<double> pp((size_t)nch32 * 16 * KC32 * y.cout, 0.0);
        for (int co = 0; co < y.cout; ++co)
          for (int ci = 0; ci < y.cin; ++ci)
            for (int ph = 0; ph < 4; ++ph)
              for (int t = 0; t < 4; ++t) {
                const int pa = ph >> 1, pb = ph & 1, ti = t >> 1, tj = t & 1;
                double v = 0.0;
                for (int r = lo[pa][ti]; r <= hi[pa][ti]; ++r)
                  for (int c = lo[pb][tj]; c <= hi[pb][tj]; ++c) v += (double)w[((size_t)co * y.cin + ci) * 9 + r * 3 + c];
                const int c32 = ci / KC32, k32 = ci % KC32;
                pp[((((size_t)c32 * 4 + ph) * 4 + t) * KC32 + k32) * y.cout + co] = v;
              }
        offs[i].pp = put(pp.data(), 8 * pp.size());
      }
      // binary64 copy (exact), read by the FP64 tiles that take binary64 weights
      const std::vector<double> p64(p32.begin(), p32.end());
      offs[i].p64 = put(p64.data(), 8 * p64.size());
      offs[i].p16 = put(p16.data(), 2 * p16.size());
      offs[i].p16s = put(p16s.data(), 2 * p16s.size());
    }
  }
  rc = npg_set_device(ctx);
  if (!rc) rc = npg_device_alloc(ctx, blob.size(), &m->blob);
  if (rc) {
    delete m;
    return rc;
  }
  m->blob_bytes = blob.size();
  if (hipMemcpy(m->blob, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
    npg_device_free(ctx, m->blob, m->blob_bytes);
    delete m;
    return npg_fail(ctx, NPG_E_HIP, "model: upload failed");
  }
  char *base = static_cast<char *>(m->blob);
  for (size_t i = 0; i < m->layer.size(); ++i) {
    LayerDev &y = m->layer[i];
    y.w = reinterpret_cast<float *>(base + offs[i].w);
    y.b = reinterpret_cast<float *>(base + offs[i].b);
    if (offs[i].p32 != (size_t)-1) {
      y.pk32 = reinterpret_cast<float *>(base + offs[i].p32);
      if (offs[i].pp != (size_t)-1) y.pkp = reinterpret_cast<double *>(base + offs[i].pp);
      if (offs[i].p64 != (size_t)-1) y.pk64 = reinterpret_cast<double *>(base + offs[i].p64);
      y.pk16 = reinterpret_cast<uint16_t *>(base + offs[i].p16);
      y.pk16s = reinterpret_cast<uint16_t *>(base + offs[i].p16s);
    }
  }
  *out = m;
  return NPG_OK;
}

extern "C" void npg_model_free(npg_model *m) {
  if (!m) return;
  if (m->ctx) {
    (void)hipSetDevice(m->ctx->device);
    npg_device_free(m->ctx, m->blob, m->blob_bytes);
    if (m->blob8) npg_device_free(m->ctx, m->blob8, m->blob8_bytes);
  }
  delete m;
}

// ------------------------------------------------------------- kernels
namespace {

enum SrcMode : int { SRC_PLAIN = 0, SRC_POOL = 1, SRC_UPCAT = 2, SRC_ENERGY = 3, SRC_FIVE = 4 };
enum Act : int { ACT_RELU = 0, ACT_SOFTPLUS = 1, ACT_ELU = 2 };

// ReLU, or ELU (Clevert et al. 2016: x for x > 0, e^x - 1 otherwise).
template <class A>
__device__ __forceinline__ A act_fn(A v, int act) {
  if (act == ACT_ELU) {
    if constexpr (sizeof(A) == 8)
      return v > (A)0 ? v : (A)expm1((double)v);
    else
      return v > (A)0 ? v : (A)expm1f((float)v);
  }
  return v > (A)0 ? v : (A)0;
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float -> bf16 bits, round to nearest even (one conversion instruction)
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float softplus_f(float x) { return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x))); }
__device__ __forceinline__ double softplus_f(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }

// activation storage types: double (FP32 mode) and bf16 bits (BF16 mode)
template <class T> __device__ __forceinline__ double to_d(T v);
template <> __device__ __forceinline__ double to_d<double>(double v) { return v; }
template <> __device__ __forceinline__ double to_d<float>(float v) { return v; }
template <> __device__ __forceinline__ double to_d<uint16_t>(uint16_t v) { return bf2f(v); }
template <> __device__ __forceinline__ double to_d<uint8_t>(uint8_t v) { return e4m3_dec_d(v); }
template <class T> __device__ __forceinline__ T from_d(double v);
template <> __device__ __forceinline__ double from_d<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_d<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ uint16_t from_d<uint16_t>(double v) { return f2bf((float)v); }
template <> __device__ __forceinline__ uint8_t from_d<uint8_t>(double v) { return e4m3_enc_d((float)v); }

// Source tensors of one convolution's (virtual) input.
struct Src {
  int mode;
  const void *s0;      // PLAIN: [L][H][W][C0]; POOL: [L][2H][2W][C0]; UPCAT: [L][H/2][W/2][C0];
                       // ENERGY: uint64 [L][H][W]
  const void *s1;      // UPCAT: skip [L][H][W][C1]
  const double *tot;   // ENERGY: per-leaf energy totals
  int C0, C1;
  float dq0 = 1.0f, dq1 = 1.0f;  // FP8: value of one e4m3 unit of s0 / s1
  // FIVE: s0, s1 = energies of iterations t and t-1 (uint64), s2, s3 = their
  // photon counts (uint32), tot = [L][4] sums of the four maps
  const void *s2 = nullptr, *s3 = nullptr;
};

// One input element (leaf, y, x, c) in storage units; (y, x) inside the map.
template <class T>
__device__ __forceinline__ double src_raw(const Src &s, int leaf, int y, int x, int c, int H, int W) {
  switch (s.mode) {
    case SRC_ENERGY: {
      // the normalised energy: binary64 in FP32 mode, else rounded to
      // float32 (as npg_normalize_input stores it)
      const double t = s.tot[leaf];
      const uint64_t e = static_cast<const uint64_t *>(s.s0)[((size_t)leaf * H + y) * W + x];
      const double v = t > 0.0 ? (double)(H * W) * (double)e / t : 0.0;
      return sizeof(T) == sizeof(double) ? v : (double)(float)v;
    }
    case SRC_POOL: {
      const T *p = static_cast<const T *>(s.s0);
      const int W2 = 2 * W;
      const size_t b = (((size_t)leaf * 2 * H + 2 * y) * W2 + 2 * x) * s.C0 + c;
      return to_d<T>(from_d<T>((to_d<T>(p[b]) + to_d<T>(p[b + s.C0]) + to_d<T>(p[b + (size_t)W2 * s.C0]) +
                                to_d<T>(p[b + (size_t)W2 * s.C0 + s.C0])) * 0.25));
    }
    case SRC_UPCAT:
      if (c < s.C0)
        return to_d<T>(static_cast<const T *>(s.s0)[(((size_t)leaf * (H / 2) + y / 2) * (W / 2) + x / 2) * s.C0 + c]);
      return to_d<T>(static_cast<const T *>(s.s1)[(((size_t)leaf * H + y) * W + x) * s.C1 + (c - s.C0)]);
    default:
      return to_d<T>(static_cast<const T *>(s.s0)[(((size_t)leaf * H + y) * W + x) * s.C0 + c]);
  }
}

// The element's value (FP8 storage units times the source's scale).
template <class T>
__device__ __forceinline__ double src_at(const Src &s, int leaf, int y, int x, int c, int H, int W) {
  const double v = src_raw<T>(s, leaf, y, x, c, H, W);
  if constexpr (sizeof(T) == 1) {
    if (s.mode == SRC_ENERGY) return v;
    return v * (double)((s.mode == SRC_UPCAT && c >= s.C0) ? s.dq1 : s.dq0);
  }
  return v;
}

// The paper's first layer on its five input channels (Sec. 6): raw maps of
// iterations t and t-1 (mean-1 energies), their photon counts normalised the
// same way, and the mask B of bins with photons at t, as a masked (partial)
// convolution: only taps with B = 1 contribute, and the sum is rescaled by
// 9/S for the S valid in-map taps (zero output where S = 0), then bias and
// the activation.
//
// One workgroup per tile of TR x TW output pixels of one leaf (TW = min(W,
// 256), TR = min(H, 256 / TW); grid = (tiles per leaf, leaves)).  The tile
// and its one-pixel halo are normalised once into LDS as four values of the
// accumulation type (binary64 in FP32 mode, so the normalised maps are never
// rounded to float32; float in BF16 mode); bins without photons at t and
// bins outside the map hold zeros, so their taps add exact zeros, and B =
// [x2 > 0] (a bin with P > 0 has x2 >= H*W / 2^32 > 0).  Each thread then
// sums its nine taps from LDS in tap-major, channel-minor order and writes
// its COUT outputs as 16-byte stores; out T [L][H][W][COUT].
constexpr int F5_LDS = 774;  // (TR + 2) * (TW + 2) for TR * TW = 256, at most 3 * 258

template <class A>
struct alignas(16) Quad {
  A x, y, z, w;
};

template <class T, class Acc, int COUT, int ACT>
__global__ __launch_bounds__(256) void conv_first5_kernel(Src s, const float *__restrict__ w,
                                                          const float *__restrict__ b, int H, int W, int TW,
                                                          int TR, void *out) {
  __shared__ Quad<Acc> tile[F5_LDS];
  const int tiles_x = W / TW;
  const int tx0 = (int)(blockIdx.x % (unsigned)tiles_x) * TW, ty0 = (int)(blockIdx.x / (unsigned)tiles_x) * TR;
  const size_t leaf = blockIdx.y, HW = (size_t)H * W, base = leaf * HW;
  const double *tl = s.tot + 4 * leaf;
  double inv[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) inv[k] = tl[k] > 0.0 ? (double)HW / tl[k] : 0.0;
  const uint64_t *e_t = static_cast<const uint64_t *>(s.s0) + base;
  const uint64_t *e_p = static_cast<const uint64_t *>(s.s1) + base;
  const uint32_t *p_t = static_cast<const uint32_t *>(s.s2) + base;
  const uint32_t *p_p = static_cast<const uint32_t *>(s.s3) + base;
  const int LW = TW + 2, n_in = (TR + 2) * LW, nj = (n_in + 255) / 256;
  // all loads of the staging first (coordinates clamped into the map, so
  // every load is in bounds and none waits on another), then the selects
  uint64_t ve[4][2];
  uint32_t vp[4][2];
  bool ok[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (j < nj) {
      const int i = min((int)threadIdx.x + 256 * j, n_in - 1);
      const int ly = i / LW, lx = i - ly * LW, sy = ty0 + ly - 1, sx = tx0 + lx - 1;
      ok[j] = sy >= 0 && sy < H && sx >= 0 && sx < W;
      const size_t k = (size_t)min(max(sy, 0), H - 1) * W + min(max(sx, 0), W - 1);
      ve[j][0] = e_t[k];
      ve[j][1] = e_p[k];
      vp[j][0] = p_t[k];
      vp[j][1] = p_p[k];
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int i = (int)threadIdx.x + 256 * j;
    if (j < nj && i < n_in) {
      Quad<Acc> v{(Acc)0, (Acc)0, (Acc)0, (Acc)0};
      if (ok[j] && vp[j][0] != 0)
        v = Quad<Acc>{(Acc)((double)ve[j][0] * inv[0]), (Acc)((double)ve[j][1] * inv[1]),
                      (Acc)((double)vp[j][0] * inv[2]), (Acc)((double)vp[j][1] * inv[3])};
      tile[i] = v;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x >= TR * TW) return;
  const int ly = (int)threadIdx.x / TW, lx = (int)threadIdx.x - ly * TW;
  Acc acc[COUT];
#pragma unroll
  for (int c = 0; c < COUT; ++c) acc[c] = (Acc)0;
  int S = 0;
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const Quad<Acc> v = tile[(ly + t / 3) * LW + lx + t % 3];
    const int m = v.z > (Acc)0;
    S += m;
    const Acc xv[5] = {v.x, v.y, v.z, v.w, (Acc)m};
#pragma unroll
    for (int c = 0; c < COUT; ++c)
#pragma unroll
      for (int ch = 0; ch < 5; ++ch) acc[c] = fma((Acc)w[(c * 5 + ch) * 9 + t], xv[ch], acc[c]);
  }
  const Acc sc = S > 0 ? (Acc)(9.0 / (double)S) : (Acc)0;
  T o[COUT];
#pragma unroll
  for (int c = 0; c < COUT; ++c) {
    const Acc v = S > 0 ? (Acc)b[c] + sc * acc[c] : (Acc)0;
    o[c] = from_d<T>((double)act_fn(v, ACT));
  }
  const size_t pix = base + (size_t)(ty0 + ly) * W + tx0 + lx;
  T *dst = static_cast<T *>(out) + pix * COUT;
  if constexpr (sizeof(o) % 16 == 0) {
#pragma unroll
    for (int k = 0; k < (int)(sizeof(o) / 16); ++k) {
      uint4 q;
      __builtin_memcpy(&q, reinterpret_cast<const char *>(o) + 16 * k, 16);
      reinterpret_cast<uint4 *>(dst)[k] = q;
    }
  } else {
#pragma unroll
    for (int c = 0; c < COUT; ++c) dst[c] = o[c];
  }
}

// The 1x1 head + softplus on a C-channel activation (channel-last, type T)
// when it is not fused into the previous layer (the paper-style network,
// whose last conv adds a residual after its activation): one thread per
// pixel, the pixel's channels in 16-byte loads, the bias plus the products
// in channel order in binary64 (as the direct convolution sums them).
template <class T, int C>
__global__ __launch_bounds__(256) void head_kernel(const T *__restrict__ in, const float *__restrict__ w,
                                                   const float *__restrict__ b, size_t npix,
                                                   float *__restrict__ out) {
  const size_t pix = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (pix >= npix) return;
  constexpr int NV = C * (int)sizeof(T) / 16;
  T v[C];
  const uint4 *src = reinterpret_cast<const uint4 *>(in + pix * C);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const uint4 q = src[k];
    __builtin_memcpy(reinterpret_cast<char *>(v) + 16 * k, &q, 16);
  }
  double acc = (double)b[0];
#pragma unroll
  for (int c = 0; c < C; ++c) acc = fma((double)w[c], to_d<T>(v[c]), acc);
  out[pix] = (float)softplus_f(acc);
}

// Sums of the four maps of the five-channel input per leaf (exact integer
// sums, stored as binary64): tot[L][4] = (E_t, E_t-1, P_t, P_t-1).
__global__ __launch_bounds__(256) void leaf_totals5_kernel(const uint64_t *__restrict__ e_t,
                                                           const uint64_t *__restrict__ e_p,
                                                           const uint32_t *__restrict__ p_t,
                                                           const uint32_t *__restrict__ p_p, int HW,
                                                           double *__restrict__ tot) {
  __shared__ unsigned long long part[4][4];
  const int leaf = blockIdx.x, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t o = (size_t)leaf * HW;
  unsigned long long v[4] = {0, 0, 0, 0};
  for (int k = threadIdx.x; k < HW; k += 256) {
    v[0] += e_t[o + k];
    v[1] += e_p[o + k];
    v[2] += p_t[o + k];
    v[3] += p_p[o + k];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off);
    if (lane == 0) part[j][wave] = v[j];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int j = threadIdx.x;
    tot[4 * (size_t)leaf + j] = (double)(part[j][0] + part[j][1] + part[j][2] + part[j][3]);
  }
}

// Direct convolution, one thread per output pixel, binary64 sums; taps
// `dil` pixels apart.  out: T [L][H][W][Cout] (ACT_RELU / ACT_ELU, plus the
// residual res of the same layout if given) or float [L][H][W]
// (ACT_SOFTPLUS, Cout 1).
template <class T>
__global__ __launch_bounds__(256) void conv_direct_kernel(Src src, const float *__restrict__ w,
                                                          const float *__restrict__ bias, int Cin, int Cout,
                                                          int k, int H, int W, size_t npix, int act,
                                                          float oinv, void *out, int dil, const void *res) {
  const size_t pix = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (pix >= npix) return;
  const int HW = H * W;
  const int leaf = (int)(pix / HW);
  const int rem = (int)(pix - (size_t)leaf * HW);
  const int y = rem / W, x = rem - y * W;
  const int r = k / 2;
  for (int co0 = 0; co0 < Cout; co0 += 16) {
    const int nco = min(16, Cout - co0);
    double acc[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) acc[j] = j < nco ? (double)bias[co0 + j] : 0.0;
    for (int ci = 0; ci < Cin; ++ci)
      for (int ky = 0; ky < k; ++ky) {
        const int sy = y + (ky - r) * dil;
        if (sy < 0 || sy >= H) continue;
        for (int kx = 0; kx < k; ++kx) {
          const int sx = x + (kx - r) * dil;
          if (sx < 0 || sx >= W) continue;
          const double v = (double)src_at<T>(src, leaf, sy, sx, ci, H, W);
          const float *wp = w + ((size_t)co0 * Cin + ci) * k * k + ky * k + kx;
#pragma unroll
          for (int j = 0; j < 16; ++j)
            if (j < nco) acc[j] = fma((double)wp[(size_t)j * Cin * k * k], v, acc[j]);
        }
      }
    if (act == ACT_SOFTPLUS) {
      static_cast<float *>(out)[pix] = (float)softplus_f(acc[0]);
    } else {
      T *o = static_cast<T *>(out) + pix * Cout + co0;
      const T *rs = res ? static_cast<const T *>(res) + pix * Cout + co0 : nullptr;
      for (int j = 0; j < nco; ++j) {
        double r = act_fn(acc[j], act);
        if (rs) r = to_d<T>(from_d<T>(r)) + to_d<T>(rs[j]);  // the stored activation plus the residual
        o[j] = from_d<T>(sizeof(T) == 1 ? r * (double)oinv : r);
      }
    }
  }
}

// First layer: one input channel (the normalised energy map) to C0 <= 16
// channels, 3x3, ReLU.  A workgroup owns 256 output pixels (whole rows of
// one leaf); it computes the normalised input x = H*W*E/total once per pixel
// of the tile and its halo into LDS, then each thread evaluates its pixel's
// C0 outputs from the nine LDS values.  FP32 mode accumulates in binary64.
template <class T, class Acc>
__global__ __launch_bounds__(256) void conv_first_kernel(const uint64_t *__restrict__ energy,
                                                         const double *__restrict__ tot,
                                                         const float *__restrict__ w,
                                                         const float *__restrict__ bias, int C0, int H,
                                                         int W, int TW, int TR, float oinv, void *out) {
  __shared__ Acc xs[800];  // (TR+2) x (TW+2) <= 3 x 258 for TR*TW = 256
  const int tiles_x = W / TW;
  const int tpl = (H / TR) * tiles_x;
  const int leaf = blockIdx.x / tpl;
  const int t = blockIdx.x - leaf * tpl;
  const int ty0 = (t / tiles_x) * TR, tx0 = (t % tiles_x) * TW;
  const int PW = TW + 2, PH = TR + 2;
  const double tl = tot[leaf];
  const double hw = (double)H * (double)W;
  const uint64_t *e = energy + (size_t)leaf * H * W;
  for (int i = threadIdx.x; i < PH * PW; i += 256) {
    const int py = i / PW, px = i - py * PW;
    const int y = ty0 - 1 + py, x = tx0 - 1 + px;
    // the normalised energy in the accumulation type: binary64 in FP32 mode,
    // float32 otherwise (as npg_normalize_input stores it)
    Acc v = (Acc)0;
    if (y >= 0 && y < H && x >= 0 && x < W && tl > 0.0) v = (Acc)(hw * (double)e[(size_t)y * W + x] / tl);
    xs[i] = v;
  }
  __syncthreads();
  const int m = threadIdx.x;
  const int ty = m / TW, tx = m - ty * TW;
  Acc xv[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) xv[k] = xs[(ty + k / 3) * PW + tx + k % 3];
  T res[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    if (c < C0) {
      Acc a = (Acc)bias[c];
#pragma unroll
      for (int k = 0; k < 9; ++k) a = fma((Acc)w[c * 9 + k], (Acc)xv[k], a);
      const Acc r = a > (Acc)0 ? a : (Acc)0;
      res[c] = from_d<T>(sizeof(T) == 1 ? (double)(r * (Acc)oinv) : (double)r);
    }
  }
  T *o = static_cast<T *>(out) + (((size_t)leaf * H + ty0 + ty) * W + tx0 + tx) * C0;
  if (C0 == 16) {
    constexpr int NV = 16 * sizeof(T) / 16;  // 16-byte pieces per pixel
#pragma unroll
    for (int v = 0; v < NV; ++v) reinterpret_cast<uint4 *>(o)[v] = reinterpret_cast<const uint4 *>(res)[v];
  } else {
    for (int c = 0; c < C0; ++c) o[c] = res[c];
  }
}

// Largest element of a non-negative (post-ReLU) activation buffer, as float
// bits (ordered like the values for non-negative floats).
template <class T>
__global__ __launch_bounds__(256) void amax_kernel(const T *__restrict__ x, size_t n, unsigned *out) {
  float m = 0.0f;
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    m = fmaxf(m, (float)x[i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// ---------------------------------------------------------- MFMA conv
// Output fragment of a 16x16 MFMA block: lane l holds column l % 16 and four
// rows.  The f32 instructions give rows 4*(l/16) + r, r = 0..3; the f64
// instruction gives rows 4*r + l/16.
struct F32P {
  using T = double;   // activations
  using WT = float;   // weights
  using Acc = f64x4;
  static constexpr bool F64 = true, Q8 = false;
  static constexpr int KC = KC32, VEC = 2, PSTR = KC + 2, KCP = 0, MAX_TILES = 8;
  // pooling windows (four loads each) in flight per thread in the pooled
  // staging, the one staging that goes through registers
  static constexpr int SBP = 2;
  // B fragments straight from the packed weights in global memory (L2/L1
  // resident, shared by every workgroup), a few K steps ahead in registers;
  // the LDS then holds the patch only, which leaves room for more workgroups
  static constexpr bool WGLB = true;
  __device__ static int row(int lg, int r) { return 4 * r + lg; }
  __device__ static int swz(int) { return 0; }
};
// 8-bit and 16-bit traits: a lane's A or B fragment is 8 consecutive K
// values (channels) of one pixel or output channel; PSTR / KCP are the LDS
// row strides (elements) of the patch and of the weight tile, whole 16-byte
// slots (they are written by LDS loads slot by slot).  The 16 rows of a
// fragment read would share LDS banks at a 64-byte pitch (32-channel BF16
// chunks) and at a 32-byte pitch read 8 bytes at a time (32-channel FP8
// chunks): there the 16-byte pieces of row p are stored in the order
// piece ^ swz(p), which spreads them over the banks (the 16-channel chunks,
// read two taps at a time, need no such order).  SBP: pooling windows in
// flight per thread in the pooled staging, which goes through registers.
struct BF16P {
  using T = uint16_t;
  using WT = uint16_t;
  using Acc = f32x4;
  using Frag = bf16x8;
  static constexpr bool F64 = false, Q8 = false, WGLB = false;
  static constexpr int KC = KC16, VEC = 8, PSTR = KC, KCP = KC, MAX_TILES = 16;
  static constexpr int SBP = 1;
  __device__ static int row(int lg, int r) { return 4 * lg + r; }
  __device__ static int swz(int p) { return (p >> 1) & 3; }
  __device__ static Acc mma(Frag a, Frag b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
struct BF16S : BF16P {
  static constexpr int KC = KC16S, PSTR = KC, KCP = KC;
  __device__ static int swz(int) { return 0; }
};
struct FP8P {
  using T = uint8_t;
  using WT = uint8_t;
  using Acc = f32x4;
  using Frag = fp8x8;
  static constexpr bool F64 = false, Q8 = true, WGLB = false;
  static constexpr int KC = KC8, VEC = 16, PSTR = KC, KCP = KC, MAX_TILES = 16;
  static constexpr int SBP = 2;
  __device__ static int row(int lg, int r) { return 4 * lg + r; }
  __device__ static int swz(int p) { return (p >> 2) & 1; }
  __device__ static Acc mma(Frag a, Frag b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a, b, c, 0, 0, 0); }
};
struct FP8S : FP8P {
  static constexpr int KC = KC8S, PSTR = KC, KCP = KC;
  __device__ static int swz(int) { return 0; }
};

// n / d for 2 <= d and n * d < 2^32, as a multiply-high by m = ceil(2^32 / d).
struct FastDiv {
  uint32_t d, m;
};
static inline FastDiv make_fastdiv(uint32_t d) { return FastDiv{d, (uint32_t)((0x100000000ull + d - 1) / d)}; }
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv f) { return __umulhi(n, f.m); }

struct ConvArgs {
  Src src;
  int Cin, Cout, H, W, TW, TR, TL, nchunk;
  FastDiv fPW, fPP;       // divisions by the patch row length and patch size
  FastDiv fTW, fTPX;      // divisions by the tile row length and pixels per leaf
  int Lc;                 // leaves in this launch
  int tiles_x, tiles_per_leaf;
  const void *wpk;
  const void *wpp = nullptr;   // phase-merged weights (upsampled chunks, staging mode 3)
  const void *wpk64 = nullptr; // binary64 packed weights (FP64 tiles: mode 3, 64 output channels)
  const float *bias;
  const float *head_w;   // non-null: fuse the 1x1 head + softplus (Cout == 16)
  float head_b;
  const float *wsc;      // FP8: per-output-channel weight scales
  float oinv, asc;       // FP8: output quantisation multiplier (1/asc) and unit value
  void *out;
  // first layer fused into the patch (staging mode 2): its weights [16][9],
  // biases [16] and FP8 output quantisation multiplier; src is the energy
  const float *w0, *b0;
  float oinv0;
  int wbytes;            // LDS bytes of the weight tile (the energy tile follows it)
  int dil = 1;           // tap spacing (dilated convolutions); the patch halo is dil pixels
  int act = 0;           // ACT_RELU or ACT_ELU (8/16-bit and FP64 tiles without a fused head)
  const void *res = nullptr;  // residual added after the activation, same layout as out
  // non-null (plain tile order, no residual, even TR and TW): also store the
  // 2x2 means of the stored tile, [leaf][H/2][W/2][Cout], the next level's
  // pooled input, with the pooled staging's arithmetic
  void *pool_out = nullptr;
};

// The input channels of one K chunk (plain or upsampled + concatenated
// input) as a buffer resource over the tile's leaves.  Loads at offsets past
// its end return zeros, so the zero padding outside the map and past the last
// leaf of the launch needs no branches.
template <class T>
struct ChunkSrc {
  __amdgpu_buffer_rsrc_t rs;
  int shift;       // 1: the half-resolution input read through nearest upsampling
  int Ws, C;       // source row length and channels per pixel
  int plane;       // source elements per leaf
  uint32_t cbyte;  // byte offset of the chunk's first channel within a pixel
  int cleft;       // source channels from the chunk's first on (<= 0: padding)
  // byte offset of pixel (y, x) of tile leaf ls, out of range outside the map
  __device__ __forceinline__ uint32_t off(int ls, int y, int x, int H, int W) const {
    const bool in = (uint32_t)y < (uint32_t)H && (uint32_t)x < (uint32_t)W;
    const uint32_t o = (uint32_t)(ls * plane + ((y >> shift) * Ws + (x >> shift)) * C) * (uint32_t)sizeof(T) + cbyte;
    return in ? o : 0x80000000u;
  }
  __device__ __forceinline__ uint4 load(uint32_t o) const {
    return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0));
  }
};
// Buffer-resource word 3 for raw (unswizzled, untyped) buffers on gfx9.
constexpr int BUF_WORD3 = 0x00020000;

template <class T>
__device__ __forceinline__ ChunkSrc<T> chunk_src(const ConvArgs &a, int leaf0, int c0) {
  ChunkSrc<T> cs;
  const void *base = nullptr;
  int C = 0, shift = 0, cl = 0, coff = 0;
  if (a.src.mode == SRC_UPCAT) {
    if (c0 < a.src.C0) {
      base = a.src.s0, C = a.src.C0, shift = 1, cl = a.src.C0 - c0, coff = c0;
    } else if (c0 - a.src.C0 < a.src.C1) {
      base = a.src.s1, C = a.src.C1, cl = a.src.C1 - (c0 - a.src.C0), coff = c0 - a.src.C0;
    }
  } else if (c0 < a.src.C0) {
    base = a.src.s0, C = a.src.C0, cl = a.src.C0 - c0, coff = c0;
  }
  cs.shift = shift;
  cs.Ws = a.W >> shift;
  cs.C = C;
  cs.plane = (a.H >> shift) * cs.Ws * C;
  cs.cbyte = (uint32_t)coff * (uint32_t)sizeof(T);
  cs.cleft = cl;
  const int nl = min(a.TL, a.Lc - leaf0);
  const T *b = base ? static_cast<const T *>(base) + (size_t)leaf0 * cs.plane : nullptr;
  cs.rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(b), (short)0, b ? nl * cs.plane * (int)sizeof(T) : 0,
                                            BUF_WORD3);
  return cs;
}

// 16-byte LDS slots [0, nslots) of region lds written straight from global
// memory (buffer loads with the LDS bit): instruction k of the workgroup,
// issued by wavefront k % 4, fills slots 64k .. 64k + 63, lane l slot 64k + l,
// whose source is byte offset off(s) of resource rs (offsets out of range,
// and slots past nslots, write zeros).  The region is a whole number of
// 1 KiB blocks.  No registers hold the data, so every load of a chunk is in
// flight at once; the caller waits on vmcnt and a barrier before reading.
typedef __attribute__((address_space(3))) void lds_void;
constexpr size_t DMA_BLOCK = 1024;
template <class F>
__device__ __forceinline__ void dma_slots(__amdgpu_buffer_rsrc_t rs, char *lds, int nslots, int wave, int lane, F off) {
  const int ninst = (nslots + 63) >> 6;
  for (int k = wave; k < ninst; k += 4) {
    const int s = k * 64 + lane;
    const uint32_t o = s < nslots ? off(s) : 0x80000000u;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)(lds + (size_t)k * DMA_BLOCK), 16, o, 0, 0, 0);
  }
}

// Mean of four 16-byte pieces (the pooling window), rounded to storage.
template <class P>
__device__ __forceinline__ uint4 pool_combine(const uint4 &a, const uint4 &b, const uint4 &cc, const uint4 &d) {
  using T = typename P::T;
  constexpr int VEC = P::VEC;
  uint4 r;
  if constexpr (sizeof(T) == 1) {
    // sums of four e4m3 values are exact in float32; two bytes per conversion
    const uint32_t *wa = &a.x, *wb = &b.x, *wc = &cc.x, *wd = &d.x;
    uint32_t *wr = &r.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // means of e4m3 values stay in range: no clamp needed
      const auto la = __builtin_amdgcn_cvt_pk_f32_fp8((int)wa[k], false), lb = __builtin_amdgcn_cvt_pk_f32_fp8((int)wb[k], false);
      const auto lc = __builtin_amdgcn_cvt_pk_f32_fp8((int)wc[k], false), ld = __builtin_amdgcn_cvt_pk_f32_fp8((int)wd[k], false);
      const auto ha = __builtin_amdgcn_cvt_pk_f32_fp8((int)wa[k], true), hb = __builtin_amdgcn_cvt_pk_f32_fp8((int)wb[k], true);
      const auto hc = __builtin_amdgcn_cvt_pk_f32_fp8((int)wc[k], true), hd = __builtin_amdgcn_cvt_pk_f32_fp8((int)wd[k], true);
      int o = __builtin_amdgcn_cvt_pk_fp8_f32((la[0] + lb[0] + lc[0] + ld[0]) * 0.25f,
                                              (la[1] + lb[1] + lc[1] + ld[1]) * 0.25f, 0, false);
      o = __builtin_amdgcn_cvt_pk_fp8_f32((ha[0] + hb[0] + hc[0] + hd[0]) * 0.25f,
                                          (ha[1] + hb[1] + hc[1] + hd[1]) * 0.25f, o, true);
      wr[k] = (uint32_t)o;
    }
    return r;
  }
  const T *ta = reinterpret_cast<const T *>(&a), *tb = reinterpret_cast<const T *>(&b);
  const T *tc = reinterpret_cast<const T *>(&cc), *td = reinterpret_cast<const T *>(&d);
  T *tr = reinterpret_cast<T *>(&r);
#pragma unroll
  for (int i = 0; i < VEC; ++i)
    tr[i] = from_d<T>((to_d<T>(ta[i]) + to_d<T>(tb[i]) + to_d<T>(tc[i]) + to_d<T>(td[i])) * 0.25);
  return r;
}


// One workgroup (4 wavefronts) computes BM = 64*MW output pixels x all Cout
// channels.  A tile is TR rows x TW columns of one leaf, or TL whole leaves
// when a map has fewer than BM pixels (the weights staged for a chunk are
// then shared by TL leaves).
// Staging modes: 0 plain or upsampled+concatenated input, 1 2x2-pooled
// input, 2 the first layer (one input channel, 16 outputs, ReLU) computed
// into the patch from the energy map, as conv_first_kernel would store it,
// 3 (FP64 tiles) upsampled+concatenated input with the output pixels in
// phase order: wavefront w holds the pixels of row parity w / 2 and column
// parity w % 2, and the upsampled channels take four phase-merged taps
// instead of nine (the concatenated ones keep nine).
// 16 bytes of stored activations plus 16 bytes of the residual, element by
// element in binary64, rounded once to the storage type.
template <class T>
__device__ __forceinline__ uint4 add_res(uint4 v, uint4 r) {
  constexpr int N = 16 / (int)sizeof(T);
  T x[N], y[N];
  __builtin_memcpy(x, &v, 16);
  __builtin_memcpy(y, &r, 16);
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = from_d<T>(to_d<T>(x[i]) + to_d<T>(y[i]));
  __builtin_memcpy(&v, x, 16);
  return v;
}

// The 2x2 means of a stored output tile staged in LDS (rows of op elements,
// tile pixel m = leaf * TR * TW + row * TW + column): pool_combine of the
// four stored 16-byte pieces, exactly what the pooled staging of the next
// layer would compute from them, stored [leaf][H/2][W/2][BN].
template <class P, int BN>
__device__ __forceinline__ void store_pooled(const ConvArgs &a, const typename P::T *ol, int op, int leaf0, int ty0,
                                             int tx0) {
  using T = typename P::T;
  constexpr int EPP = 16 / (int)sizeof(T), PPR = BN / EPP;
  const int TW2 = a.TW >> 1, Q = (a.TR >> 1) * TW2, TPX = a.TR * a.TW;
  T *po = static_cast<T *>(a.pool_out);
  for (int i = threadIdx.x; i < a.TL * Q * PPR; i += 256) {
    const int q = i / PPR, pc = i - q * PPR;
    const int ls = q / Q, r = q - ls * Q, qy = r / TW2, qx = r - qy * TW2;
    if (leaf0 + ls >= a.Lc) continue;
    const int m = ls * TPX + 2 * qy * a.TW + 2 * qx;
    auto at = [&](int mm) { return *reinterpret_cast<const uint4 *>(ol + mm * op + pc * EPP); };
    const uint4 v = pool_combine<P>(at(m), at(m + 1), at(m + a.TW), at(m + a.TW + 1));
    const long g = ((long)(leaf0 + ls) * (a.H >> 1) + (ty0 >> 1) + qy) * (a.W >> 1) + (tx0 >> 1) + qx;
    *reinterpret_cast<uint4 *>(po + g * BN + pc * EPP) = v;
  }
}

// no work to run late in a chunk's taps
struct NoLate {
  __device__ void operator()() const {}
};

// X: the extended form (dilation, ELU, residual link); without it the
// layer is a plain 3x3 conv + ReLU and none of that code is compiled in.
template <class P, int MW, int NW, int MODE, bool X = false>
__global__ __launch_bounds__(256) void conv_mfma_kernel(ConvArgs a) {
  using T = typename P::T;
  using AccV = typename P::Acc;
  using AS = std::remove_cv_t<std::remove_reference_t<decltype(AccV{}[0])>>;
  constexpr int KC = P::KC, VEC = P::VEC, PSTR = P::PSTR, G = KC / VEC;
  constexpr int BN = 16 * NW;
  using WT = typename P::WT;
  constexpr bool IS_F32 = P::F64;                // FP32 weights, FP64 activations and sums
  constexpr bool WGLB = P::WGLB;                 // B fragments from global memory
  static_assert(WGLB == IS_F32, "FP64 tiles read their weights from global memory, 8/16-bit tiles from LDS");
  constexpr bool TWO_TAP = !IS_F32 && KC == 16;  // K slice = 2 taps x 16 channels
  constexpr int NTAPW = TWO_TAP ? 10 : 9;        // weight taps in LDS (10th = zeros)
  constexpr int KCP = P::KCP;  // 8/16-bit B tile: [tap][n][KCP]
  static_assert(IS_F32 || (PSTR * sizeof(T) % 16 == 0 && KCP * sizeof(WT) % 16 == 0),
                "8/16-bit LDS rows are whole 16-byte slots");
  extern __shared__ __attribute__((aligned(16))) char smem[];
  const int DIL = X ? a.dil : 1, TW = a.TW, TR = a.TR, TL = a.TL, PW = TW + 2 * DIL, PH = TR + 2 * DIL;
  const int ACT = X ? a.act : ACT_RELU;
  const void *const RES = X ? a.res : nullptr;
  const int H = a.H, W = a.W;
  T *patch = reinterpret_cast<T *>(smem);
  // the patch (and the 8/16-bit weights) staged by whole 1 KiB blocks
  const size_t patch_bytes = npg_align((size_t)TL * PH * PW * PSTR * sizeof(T), DMA_BLOCK);
  WT *wl = reinterpret_cast<WT *>(smem + patch_bytes);
  const int wave_u = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  const int tile = blockIdx.x;
  const int grp = tile / a.tiles_per_leaf;
  const int t = tile - grp * a.tiles_per_leaf;
  const int leaf0 = grp * TL;
  const int ty0 = (t / a.tiles_x) * TR, tx0 = (t - (t / a.tiles_x) * a.tiles_x) * TW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int TPX = TR * TW;  // pixels per leaf in the tile

  int bp[MW];
#pragma unroll
  for (int mi = 0; mi < MW; ++mi) {
    if constexpr (MODE == 3) {
      // pixel mi * 16 + lr of the wavefront's phase: TPX / 4 per leaf
      const int m = mi * 16 + lr, Q = TPX >> 2, hw2 = TW >> 1;
      const int ls = m / Q, rem = m - ls * Q, qy = rem / hw2;
      bp[mi] = ls * PH * PW + (2 * qy + (wave >> 1)) * PW + 2 * (rem - qy * hw2) + (wave & 1);
    } else {
      const int m = wave * 16 * MW + mi * 16 + lr;
      const int ls = (int)fdiv((uint32_t)m, a.fTPX), rem = m - ls * TPX;
      const int ry = (int)fdiv((uint32_t)rem, a.fTW);
      bp[mi] = ls * PH * PW + ry * PW + (rem - ry * TW);
    }
  }
  AccV acc[MW][NW];
#pragma unroll
  for (int mi = 0; mi < MW; ++mi)
#pragma unroll
    for (int ni = 0; ni < NW; ++ni) acc[mi][ni] = AccV{0, 0, 0, 0};
  // 8/16-bit tiles: element offset of this lane's fragment (K values lg*8 ..
  // lg*8 + 7) in LDS row p of the patch or weight tile, whose 16-byte pieces
  // are stored in the order piece ^ swz(p)
  constexpr int EPP = 16 / (int)sizeof(T);  // elements per 16-byte piece
  auto frag_at = [&](int p, int stride) {
    const int e = lg * 8;
    return p * stride + (((e / EPP) ^ P::swz(p)) * EPP) + e % EPP;
  };

  // WGLB: this lane's B values for the next R K steps (a K step
  // is 4 channels of one tap) in a ring of R slots: step s sits in slot
  // s % R until its matrix products are issued, then the slot is reloaded
  // with step s + R.  R divides the K steps of a tap, so every slot is
  // known at compile time and no register copies (which would wait for the
  // loads in flight) are needed.  A chunk's first R steps (wfirst) are
  // loaded before its patch is staged, so they arrive with it.  Mode 3
  // reads binary64 weights (its phase-merged taps are binary64 sums); so do
  // the 64-channel tiles (binary64 copies of the float32 weights), which
  // spares them a conversion on the vector ALUs per weight (every vector
  // instruction delays the FP64 matrix products of its SIMD) at no cost in
  // wavefronts per SIMD; the other tiles would lose a wavefront to the
  // wider registers and keep float32.
  using WR = std::conditional_t<WGLB && (MODE == 3 || NW == 4), double, float>;
  constexpr int KS = KC / 4;
  constexpr int R = NW >= 4 ? 2 : KS;
  static_assert(KS % R == 0, "ring slots repeat every tap");
  WR wr[WGLB ? R : 1][WGLB ? NW : 1];
  auto wfetch = [&](const WR *wg, int step, WR (&dst)[WGLB ? NW : 1]) {
#pragma unroll
    for (int ni = 0; ni < NW; ++ni) dst[ni] = wg[(4 * step + lg) * BN + ni * 16 + lr];
  };
  auto wfirst = [&](const WR *wg) {
    if constexpr (WGLB) {
#pragma unroll
      for (int r = 0; r < R; ++r) wfetch(wg, r, wr[r]);
    }
  };
  // the weights and the number of taps of chunk ch: phase-merged taps for
  // upsampled channels in mode 3
  struct ChunkW {
    const WR *wg;
    int nt;
  };
  auto chunk_w = [&](int ch) -> ChunkW {
    if constexpr (std::is_same_v<WR, double>) {
      if constexpr (MODE == 3) {
        if (ch * KC < a.src.C0) return {static_cast<const double *>(a.wpp) + ((size_t)ch * 4 + wave) * 4 * KC * BN, 4};
      }
      return {static_cast<const double *>(a.wpk64) + (size_t)ch * 9 * KC * BN, 9};
    } else {
      return {static_cast<const float *>(a.wpk) + (size_t)ch * 9 * KC * BN, 9};
    }
  };

  // the nine taps of one K chunk on the staged patch (weights wg of the
  // chunk, its first R steps already in the ring); NT = 4: the four
  // phase-merged taps of an upsampled chunk (mode 3).  late() runs once per
  // chunk, right after the loads of its last step: vector loads retire in
  // order, so a load issued there holds up no weight of the chunk
  auto taps = [&](const WR *wg, int NT, auto &&late) {
    constexpr int LKS = R < KS ? KS - 1 - R : KS - 1;  // K step and tap (from the end)
    constexpr int LT = R < KS ? 1 : 2;                 // after which late() runs
    auto one_tap = [&](int tap, auto has_late) {
      int toff;
      if constexpr (MODE == 3)
        toff = NT == 4 ? (tap >> 1) * PW + (tap & 1) + (wave >> 1) * PW + (wave & 1) : (tap / 3) * PW + (tap % 3);
      else
        toff = ((tap / 3) * PW + (tap % 3)) * DIL;
      if constexpr (IS_F32) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          double av[MW], bv[NW];
#pragma unroll
          for (int mi = 0; mi < MW; ++mi)
            av[mi] = (double)patch[(bp[mi] + toff) * PSTR + ks * 4 + lg];
#pragma unroll
          for (int ni = 0; ni < NW; ++ni) bv[ni] = (double)wr[ks % R][ni];
          // the step R ahead into the slot just read (steps past the chunk's
          // last are not loaded)
          if (ks + R < KS || tap + 1 < NT) wfetch(wg, tap * KS + ks + R, wr[ks % R]);
          if constexpr (decltype(has_late)::value)
            if (ks == LKS) late();
#pragma unroll
          for (int mi = 0; mi < MW; ++mi)
#pragma unroll
            for (int ni = 0; ni < NW; ++ni)
              acc[mi][ni] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mi], bv[ni], acc[mi][ni], 0, 0, 0);
        }
      } else if constexpr (!TWO_TAP) {
        using Frag = typename P::Frag;
        Frag av[MW], bv[NW];
#pragma unroll
        for (int mi = 0; mi < MW; ++mi) av[mi] = *reinterpret_cast<const Frag *>(patch + frag_at(bp[mi] + toff, PSTR));
#pragma unroll
        for (int ni = 0; ni < NW; ++ni)
          bv[ni] = *reinterpret_cast<const Frag *>(wl + frag_at(tap * BN + ni * 16 + lr, KCP));
#pragma unroll
        for (int mi = 0; mi < MW; ++mi)
#pragma unroll
          for (int ni = 0; ni < NW; ++ni) acc[mi][ni] = P::mma(bv[ni], av[mi], acc[mi][ni]);
      } else {
        if (tap & 1) return;  // taps handled in pairs (tap, tap + 1)
        // lanes 0-31 read tap `tap`, lanes 32-63 tap `tap + 1` (the tenth
        // tap has zero weights; its patch reads stay inside the patch)
        const int tl = tap + (lg >> 1);
        const int tofl = tl < 9 ? ((tl / 3) * PW + (tl % 3)) * DIL : 0;
        const int cofs = (lg & 1) * 8;
        using Frag = typename P::Frag;
        Frag av[MW], bv[NW];
#pragma unroll
        for (int mi = 0; mi < MW; ++mi)
          av[mi] = *reinterpret_cast<const Frag *>(patch + (bp[mi] + tofl) * PSTR + cofs);
#pragma unroll
        for (int ni = 0; ni < NW; ++ni)
          bv[ni] = *reinterpret_cast<const Frag *>(wl + (tl * BN + ni * 16 + lr) * KCP + cofs);
#pragma unroll
        for (int mi = 0; mi < MW; ++mi)
#pragma unroll
          for (int ni = 0; ni < NW; ++ni) acc[mi][ni] = P::mma(bv[ni], av[mi], acc[mi][ni]);
      }
    };
    // with a late() to run, the last LT taps are peeled off the loop, so the
    // loads it issues are not pending (for the compiler's waits) at the top
    // of the loop
    constexpr bool HAS_LATE = !std::is_same_v<std::decay_t<decltype(late)>, NoLate>;
    if constexpr (IS_F32 && HAS_LATE) {
#pragma unroll 1
      for (int tap = 0; tap < NT - LT; ++tap) one_tap(tap, std::false_type{});
      if constexpr (LT == 2) one_tap(NT - 2, std::true_type{});
      one_tap(NT - 1, std::bool_constant<LT == 1>{});
    } else {
#pragma unroll 1
      for (int tap = 0; tap < NT; ++tap) one_tap(tap, std::false_type{});
    }
  };

  auto chunk_taps = [&](int ch, auto &&late) {
    const ChunkW c = chunk_w(ch);
    taps(c.wg, c.nt, late);  // one call site: one copy of the tap loop
  };

  // FP64 tiles on plain or concatenated inputs whose patch has at most one
  // pixel per thread: the next chunk's pixel is loaded into registers while
  // the matrix cores work on the current chunk's last K steps, after its
  // last weight loads (the weights come straight from global memory, so the
  // patch is all there is to stage; issued at the start of the chunk, the
  // load would hold up the first tap's weights behind it)
  bool piped = false;
  if constexpr (WGLB && (MODE == 0 || MODE == 3)) {
    const int npx = TL * PH * PW;
    if (npx <= 256) {
      piped = true;
      // this thread's patch pixel (the same in every chunk)
      const int ls = (int)fdiv((uint32_t)tid, a.fPP), pr = tid - ls * PH * PW;
      const int py = (int)fdiv((uint32_t)pr, a.fPW), px = pr - py * PW;
      auto load_px = [&](int ch, uint4 (&v)[G]) {
        const ChunkSrc<T> cs = chunk_src<T>(a, leaf0, ch * KC);
        const uint32_t o = tid < npx ? cs.off(ls, ty0 - DIL + py, tx0 - DIL + px, H, W) : 0x80000000u;
#pragma unroll
        for (int g = 0; g < G; ++g) v[g] = g * VEC < cs.cleft ? cs.load(o + 16 * g) : make_uint4(0, 0, 0, 0);
      };
      auto store_px = [&](const uint4 (&v)[G]) {
        if (tid < npx) {
#pragma unroll
          for (int g = 0; g < G; ++g) *reinterpret_cast<uint4 *>(patch + tid * PSTR + g * VEC) = v[g];
        }
      };
      uint4 nv[G];
      wfirst(chunk_w(0).wg);
      load_px(0, nv);
      store_px(nv);
      __syncthreads();
      for (int ch = 0; ch < a.nchunk; ++ch) {
        chunk_taps(ch, [&] {
          if (ch + 1 < a.nchunk) load_px(ch + 1, nv);
        });
        // the next chunk's first weights, in flight across the barriers
        if (ch + 1 < a.nchunk) wfirst(chunk_w(ch + 1).wg);
        __syncthreads();
        if (ch + 1 < a.nchunk) {
          store_px(nv);
          __syncthreads();
        }
      }
    }
  }
  const int items = TL * PH * PW * G;
  // staging mode 2 reads the first layer's 16 channels: a single chunk, as
  // a trip count the compiler sees (with a loop around them, the LDS loads
  // would turn the first layer's weight reads into vector loads held in
  // many registers)
  const int nch = piped ? 0 : MODE == 2 ? 16 / KC : a.nchunk;
  for (int ch = 0; ch < nch; ++ch) {
    const int c0 = ch * KC;
    const WT *wg = static_cast<const WT *>(a.wpk) + (size_t)ch * 9 * KC * BN;
    // 8/16-bit weights [tap][n][KCP] straight into LDS (slot g of row r holds
    // piece g ^ swz(r); the tenth tap of two-tap chunks and any row padding
    // are written as zeros), issued before the patch loads so that both
    // arrive in one global round trip
    auto stage_w = [&]() {
      if constexpr (!IS_F32) {
        constexpr int SPW = KCP * (int)sizeof(WT) / 16, RW = KC * (int)sizeof(WT) / 16;
        const auto wrs = __builtin_amdgcn_make_buffer_rsrc(const_cast<WT *>(wg), (short)0,
                                                           9 * BN * KC * (int)sizeof(WT), BUF_WORD3);
        dma_slots(wrs, reinterpret_cast<char *>(wl), NTAPW * BN * SPW, wave_u, lane, [&](int s) -> uint32_t {
          const int row = s / SPW, g = s - row * SPW;
          return g < RW ? (uint32_t)(row * KC * (int)sizeof(WT) + (g ^ P::swz(row)) * 16) : 0x80000000u;
        });
      }
    };
    stage_w();
    wfirst(chunk_w(ch).wg);
    // input patch with halo: straight into LDS for 8/16-bit tiles on plain
    // or concatenated inputs; otherwise through registers, in batches of SB
    // loads per thread, then the stores (pooled inputs, four loads per piece,
    // one piece at a time)
    if constexpr (MODE == 2) {
      // normalised energy x = HW*E/total (binary64 in FP32 mode, float32
      // otherwise; zero outside the map) on the patch plus one more pixel of
      // border, then the first layer's 16 outputs per patch pixel (zero
      // where the pixel is outside the map: the second layer's zero padding)
      using A0 = std::conditional_t<P::F64, double, float>;
      // the first layer's weights read as constant memory: scalar loads,
      // although the LDS loads issued above are in flight
      using CF = const __attribute__((address_space(4))) float;
      CF *w0 = (CF *)a.w0, *b0 = (CF *)a.b0;
      const int EW = TW + 4, EH = TR + 4;
      A0 *xt = reinterpret_cast<A0 *>(smem + npg_align(patch_bytes + (size_t)a.wbytes, 16));
      const int ne = TL * EH * EW;
      const double hw = (double)H * (double)W;
      for (int i = tid; i < ne; i += 256) {
        const int ls = i / (EH * EW), r = i - ls * EH * EW;
        const int ey = r / EW, ex = r - ey * EW;
        const int y = ty0 - 2 + ey, x = tx0 - 2 + ex, leaf = leaf0 + ls;
        A0 v = (A0)0;
        if (leaf < a.Lc && y >= 0 && y < H && x >= 0 && x < W) {
          const double tl = a.src.tot[leaf];
          if (tl > 0.0)
            v = (A0)(hw * (double)static_cast<const uint64_t *>(a.src.s0)[((size_t)leaf * H + y) * W + x] / tl);
        }
        xt[i] = v;
      }
      __syncthreads();
      const int np = TL * PH * PW;
      for (int pp = tid; pp < np; pp += 256) {
        const int ls = pp / (PH * PW), r = pp - ls * PH * PW;
        const int py = r / PW, px = r - py * PW;
        const int y = ty0 - DIL + py, x = tx0 - DIL + px, leaf = leaf0 + ls;
        T res[KC];  // the pixel's KC channels, written as 16-byte pieces
        if (leaf < a.Lc && y >= 0 && y < H && x >= 0 && x < W) {
          const A0 *xp = xt + ls * EH * EW + py * EW + px;
          A0 xv[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) xv[k] = (A0)xp[(k / 3) * EW + k % 3];
#pragma unroll
          for (int cc = 0; cc < KC; ++cc) {  // this chunk's channels c0 .. c0 + KC - 1
            const int c = c0 + cc;
            A0 acc0 = (A0)b0[c];
#pragma unroll
            for (int k = 0; k < 9; ++k) acc0 = fma((A0)w0[c * 9 + k], xv[k], acc0);
            const A0 rl = acc0 > (A0)0 ? acc0 : (A0)0;
            res[cc] = from_d<T>(sizeof(T) == 1 ? (double)(rl * (A0)a.oinv0) : (double)rl);
          }
        } else {
#pragma unroll
          for (int c = 0; c < KC; ++c) res[c] = from_d<T>(0.0);
        }
#pragma unroll
        for (int v = 0; v < KC * (int)sizeof(T) / 16; ++v)
          reinterpret_cast<uint4 *>(patch + pp * PSTR)[v ^ P::swz(pp)] = reinterpret_cast<const uint4 *>(res)[v];
      }
    } else if constexpr (MODE == 1) {
      constexpr int SBP = P::SBP;  // pooling windows (four loads each) in flight per thread
      // the full-resolution input of the tile's leaves as a buffer resource
      // (out-of-range offsets read zeros: padding outside the map)
      const int C0 = a.src.C0, W2 = 2 * W, plane = 4 * H * W * C0;
      const int nl = min(TL, a.Lc - leaf0);
      const T *pb = static_cast<const T *>(a.src.s0) + (size_t)leaf0 * plane;
      const auto prs = __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(pb), (short)0, nl * plane * (int)sizeof(T),
                                                         BUF_WORD3);
      const uint32_t dcb = (uint32_t)(C0 * sizeof(T)), drb = (uint32_t)W2 * dcb;
      auto pld = [&](uint32_t o) {
        return __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(prs, o, 0, 0));
      };
      for (int base = 0; base < items; base += 256 * SBP) {
        uint4 q[SBP][4];
#pragma unroll
        for (int k = 0; k < SBP; ++k) {
          const int it = base + k * 256 + tid;
          const int pp = it / G, g = it - pp * G;
          const int ls = (int)fdiv((uint32_t)pp, a.fPP), pr = pp - ls * PH * PW;
          const int py = (int)fdiv((uint32_t)pr, a.fPW), px = pr - py * PW;
          const int y = ty0 - DIL + py, x = tx0 - DIL + px, c = c0 + g * VEC;
          const bool in = it < items && (uint32_t)y < (uint32_t)H && (uint32_t)x < (uint32_t)W && c < C0;
          const uint32_t o = in ? (uint32_t)(ls * plane + (2 * y * W2 + 2 * x) * C0 + c) * (uint32_t)sizeof(T)
                                : 0x80000000u;
          q[k][0] = pld(o);
          q[k][1] = pld(o + dcb);
          q[k][2] = pld(o + drb);
          q[k][3] = pld(o + drb + dcb);
        }
#pragma unroll
        for (int k = 0; k < SBP; ++k) {
          const int it = base + k * 256 + tid;
          if (it < items) {
            const int pp = it / G, g = it - pp * G;
            *reinterpret_cast<uint4 *>(patch + pp * PSTR + (g ^ P::swz(pp)) * VEC) =
                pool_combine<P>(q[k][0], q[k][1], q[k][2], q[k][3]);
          }
        }
      }
    } else {
      // the patch straight into LDS: slot g of pixel p holds the source's
      // piece g ^ swz(p); slots past the first G of a pixel (row padding,
      // none at present) are written as zeros.  A chunk's channels come from
      // one source: the concatenation boundary is a multiple of KC.
      constexpr int SPP = PSTR * (int)sizeof(T) / 16;
      const ChunkSrc<T> cs = chunk_src<T>(a, leaf0, c0);
      dma_slots(cs.rs, reinterpret_cast<char *>(patch), TL * PH * PW * SPP, wave_u, lane, [&](int s) -> uint32_t {
        const int pp = s / SPP, g = s - pp * SPP;
        const int ls = (int)fdiv((uint32_t)pp, a.fPP), pr = pp - ls * PH * PW;
        const int py = (int)fdiv((uint32_t)pr, a.fPW), px = pr - py * PW;
        if (g >= G) return 0x80000000u;
        const int gs = g ^ P::swz(pp);  // the source piece this slot holds
        if (gs * VEC >= cs.cleft) return 0x80000000u;
        return cs.off(ls, ty0 - DIL + py, tx0 - DIL + px, H, W) + 16u * (uint32_t)gs;
      });
    }
    // the LDS loads of this wavefront have landed; the barrier covers the others'
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    chunk_taps(ch, NoLate{});
    __syncthreads();
  }

  // epilogue: bias + ReLU (+ head), staged through LDS (free after the last
  // barrier) so that global stores are whole 16-byte pieces of output rows
  const int BM = 64 * MW;
  auto gpix = [&](int m) -> long {  // global pixel index of tile pixel m, -1 if past the last leaf
    if constexpr (MODE == 3) {
      const int w = m / (16 * MW), mp = m - w * 16 * MW, Q = TPX >> 2, hw2 = TW >> 1;
      const int ls = mp / Q, rem = mp - ls * Q, qy = rem / hw2;
      if (leaf0 + ls >= a.Lc) return -1;
      return ((long)(leaf0 + ls) * H + ty0 + 2 * qy + (w >> 1)) * W + tx0 + 2 * (rem - qy * hw2) + (w & 1);
    }
    const int ls = (int)fdiv((uint32_t)m, a.fTPX), rem = m - ls * TPX;
    if (leaf0 + ls >= a.Lc) return -1;
    const int ry = (int)fdiv((uint32_t)rem, a.fTW);
    return ((long)(leaf0 + ls) * H + ty0 + ry) * W + tx0 + (rem - ry * TW);
  };
  if constexpr (!P::F64) {
    // 8/16-bit tiles hold the transposed product (weights as the A operand):
    // lane (lr, lg) has channels 16 ni + 4 lg + r, r = 0..3, of pixel
    // 16 mi + lr of its wavefront's block
    if (a.head_w) {
      float *dl = reinterpret_cast<float *>(smem);  // [BM] densities
      AS bn[4], hw[4], ws[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        bn[r] = (AS)a.bias[4 * lg + r];
        hw[r] = (AS)a.head_w[4 * lg + r];
        ws[r] = (AS)1;
        if constexpr (P::Q8) ws[r] = (AS)a.wsc[4 * lg + r];
      }
      AS mine = 0;
#pragma unroll
      for (int mi = 0; mi < MW; ++mi) {
        AS v = 0;
        // the values the unfused path would store (type T) feed the head
        if constexpr (P::Q8) {
          float q[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const AS v0 = acc[mi][0][r] * ws[r] + bn[r];
            q[r] = (v0 > (AS)0 ? v0 : (AS)0) * a.oinv;
          }
          const int pk = (int)e4m3_pack4_d(q[0], q[1], q[2], q[3]);
          const auto d01 = __builtin_amdgcn_cvt_pk_f32_fp8(pk, false), d23 = __builtin_amdgcn_cvt_pk_f32_fp8(pk, true);
          const float dq[4] = {d01[0], d01[1], d23[0], d23[1]};
#pragma unroll
          for (int r = 0; r < 4; ++r) v += (AS)(dq[r] * a.asc) * hw[r];
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const AS v0 = acc[mi][0][r] + bn[r];
            v += (AS)bf2f(f2bf(v0 > (AS)0 ? v0 : (AS)0)) * hw[r];
          }
        }
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        if (lg == mi) mine = v;
      }
      if (lg < MW) dl[wave * 16 * MW + lg * 16 + lr] = (float)softplus_f(mine + (AS)a.head_b);
      __syncthreads();
      // four consecutive tile pixels are contiguous in the output (TW >= 4)
      for (int i = tid; i < BM / 4; i += 256) {
        const long g = gpix(i * 4);
        if (g >= 0)
          *reinterpret_cast<float4 *>(static_cast<float *>(a.out) + g) = *reinterpret_cast<const float4 *>(dl + i * 4);
      }
      return;
    }
    // [BM][OP]: the row padding puts the 16 lanes of a group, which hold
    // 16 pixels of the same channels, in different LDS banks
    constexpr int OP = BN + 16 / (int)sizeof(T);
    T *ol = reinterpret_cast<T *>(smem);
#pragma unroll
    for (int ni = 0; ni < NW; ++ni) {
      AS bn[4], ws[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        bn[r] = (AS)a.bias[16 * ni + 4 * lg + r];
        ws[r] = (AS)1;
        if constexpr (P::Q8) ws[r] = (AS)a.wsc[16 * ni + 4 * lg + r];
      }
#pragma unroll
      for (int mi = 0; mi < MW; ++mi) {
        const int m = wave * 16 * MW + mi * 16 + lr;
        float q[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if constexpr (P::Q8) {
            const AS v = acc[mi][ni][r] * ws[r] + bn[r];
            q[r] = (v > (AS)0 ? v : (AS)0) * a.oinv;
          } else {
            q[r] = act_fn(acc[mi][ni][r] + bn[r], ACT);
          }
        }
        T *o = ol + m * OP + 16 * ni + 4 * lg;  // four consecutive channels: one store
        if constexpr (sizeof(T) == 2)
          *reinterpret_cast<uint2 *>(o) = make_uint2((uint32_t)f2bf(q[0]) | ((uint32_t)f2bf(q[1]) << 16),
                                                     (uint32_t)f2bf(q[2]) | ((uint32_t)f2bf(q[3]) << 16));
        else
          *reinterpret_cast<uint32_t *>(o) = e4m3_pack4_d(q[0], q[1], q[2], q[3]);
      }
    }
    __syncthreads();
    constexpr int PPR = BN * (int)sizeof(T) / 16;  // 16-byte pieces per pixel
    T *out = static_cast<T *>(a.out);
    for (int i = tid; i < BM * PPR; i += 256) {
      const int m = i / PPR, pc = i - m * PPR;
      const long g = gpix(m);
      if (g >= 0) {
        uint4 v = *reinterpret_cast<const uint4 *>(ol + m * OP + pc * (16 / sizeof(T)));
        if (RES)
          v = add_res<T>(v, *reinterpret_cast<const uint4 *>(static_cast<const T *>(RES) + g * BN +
                                                             pc * (16 / sizeof(T))));
        *reinterpret_cast<uint4 *>(out + g * BN + pc * (16 / sizeof(T))) = v;
      }
    }
    if constexpr (MODE != 3)
      if (a.pool_out) store_pooled<P, BN>(a, ol, OP, leaf0, ty0, tx0);
    return;
  }
  if (a.head_w) {
    float *dl = reinterpret_cast<float *>(smem);  // [BM] densities
    const AS bn = (AS)a.bias[lr];
    const AS hw = (AS)a.head_w[lr];
    AS ws = (AS)1;
    if constexpr (P::Q8) ws = (AS)a.wsc[lr];
    // after the 16-lane reductions every lane of group lg holds the sum of
    // pixel (mi, r); lane lr keeps pixel (lr / 4, lr % 4) so one softplus per
    // lane covers the wavefront's pixels
    AS mine = 0;
#pragma unroll
    for (int mi = 0; mi < MW; ++mi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // the value the unfused path would store (type T) feeds the head
        AS v0;
        double act;
        if constexpr (P::Q8) {
          v0 = acc[mi][0][r] * ws + bn;
          act = (double)(e4m3_dec_d(e4m3_enc_d((v0 > (AS)0 ? v0 : (AS)0) * a.oinv)) * a.asc);
        } else {
          v0 = acc[mi][0][r] + bn;
          act = to_d<T>(from_d<T>((double)(v0 > (AS)0 ? v0 : (AS)0)));
        }
        AS v = (AS)act * hw;
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        if (lr == mi * 4 + r) mine = v;
      }
    if (lr < 4 * MW) {
      const int mi = lr >> 2, r = lr & 3;
      dl[wave * 16 * MW + mi * 16 + P::row(lg, r)] = (float)softplus_f(mine + (AS)a.head_b);
    }
    __syncthreads();
    // four consecutive tile pixels are contiguous in the output (TW >= 4)
    for (int i = tid; i < BM / 4; i += 256) {
      const long g = gpix(i * 4);
      if (g >= 0)
        *reinterpret_cast<float4 *>(static_cast<float *>(a.out) + g) = *reinterpret_cast<const float4 *>(dl + i * 4);
    }
    return;
  }
  T *ol = reinterpret_cast<T *>(smem);  // [BM][BN]
#pragma unroll
  for (int ni = 0; ni < NW; ++ni) {
    const int n = ni * 16 + lr;
    const AS bn = (AS)a.bias[n];
    AS ws = (AS)1;
    if constexpr (P::Q8) ws = (AS)a.wsc[n];
#pragma unroll
    for (int mi = 0; mi < MW; ++mi)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = wave * 16 * MW + mi * 16 + P::row(lg, r);
        if constexpr (P::Q8) {
          const AS v = acc[mi][ni][r] * ws + bn;
          ol[m * BN + n] = e4m3_enc_d((v > (AS)0 ? v : (AS)0) * a.oinv);
        } else {
          ol[m * BN + n] = from_d<T>((double)act_fn(acc[mi][ni][r] + bn, ACT));
        }
      }
  }
  __syncthreads();
  constexpr int PPR = BN * (int)sizeof(T) / 16;  // 16-byte pieces per pixel
  T *out = static_cast<T *>(a.out);
  for (int i = tid; i < BM * PPR; i += 256) {
    const int m = i / PPR, pc = i - m * PPR;
    const long g = gpix(m);
    if (g >= 0) {
      uint4 v = *reinterpret_cast<const uint4 *>(ol + m * BN + pc * (16 / sizeof(T)));
      if (RES)
        v = add_res<T>(v, *reinterpret_cast<const uint4 *>(static_cast<const T *>(RES) + g * BN +
                                                           pc * (16 / sizeof(T))));
      *reinterpret_cast<uint4 *>(out + g * BN + pc * (16 / sizeof(T))) = v;
    }
  }
  if constexpr (MODE != 3)
    if (a.pool_out) store_pooled<P, BN>(a, ol, BN, leaf0, ty0, tx0);
}

// Tiling of a layer: returns false if the MFMA kernel does not fit it.
struct Tiling {
  int MW, NW, TW, TR, TL;
  int dil = 1;  // patch halo (dilated convolutions)
};

// Bytes of the weight tile a workgroup stages in LDS.
template <class P>
size_t conv_wts_bytes(const Tiling &t) {
  using WT = typename P::WT;
  const int BN = 16 * t.NW;
  if (P::F64) return 0;  // FP64 tiles read their weights from global memory
  return npg_align((size_t)(P::KC == 16 ? 10 : 9) * BN * P::KCP * sizeof(WT), DMA_BLOCK);
}

// first: the energy tile of a fused first layer follows the weights
template <class P>
size_t conv_lds_bytes(const Tiling &t, bool first = false) {
  using T = typename P::T;
  const int BN = 16 * t.NW;
  // patch (and 8/16-bit weights) in whole blocks (their LDS loads)
  const size_t patch = npg_align((size_t)t.TL * (t.TR + 2 * t.dil) * (t.TW + 2 * t.dil) * P::PSTR * sizeof(T),
                                 DMA_BLOCK);
  const size_t wts = conv_wts_bytes<P>(t);
  // output tile staging (8/16-bit rows padded by 16 bytes)
  const size_t epi = (size_t)64 * t.MW * (BN * sizeof(T) + (P::F64 ? 0 : 16));
  const size_t xt = first ? npg_align(patch + wts, 16) - patch - wts +
                                (size_t)t.TL * (t.TR + 4) * (t.TW + 4) * (P::F64 ? sizeof(double) : sizeof(float))
                          : 0;
  return std::max(patch + wts + xt, epi);
}

// Largest pixel tile (64*MW pixels) whose accumulators and LDS fit; maps
// smaller than the tile are batched TL whole leaves per tile.
template <class P>
bool pick_tiling(int Cout, int H, int W, Tiling *t, int mw_max = 4, int dil = 1) {
  if (Cout % 16 || Cout > 128) return false;
  const int NW = Cout / 16;
  if (NW & (NW - 1)) return false;  // 1, 2, 4 or 8 tiles of 16 output channels (the launched forms)
  if (NW > P::MAX_TILES) return false;
  const int HW = H * W;
  for (int MW = 8; MW >= 1; MW >>= 1) {
    if (MW > mw_max) continue;
    if (MW * NW > P::MAX_TILES || (MW == 8 && NW > 2)) continue;
    const int BM = 64 * MW;
    Tiling c{MW, NW, 0, 0, 1, dil};
    if (BM <= HW) {
      // the TR x TW shape (TW >= 8, a power of two like W and H) with the
      // smallest halo patch (TR + 2 dil) x (TW + 2 dil): fewer bytes staged per pixel
      c.TW = std::min(W, BM);
      c.TR = BM / c.TW;
      for (int tw = c.TW / 2; tw >= 8; tw /= 2) {
        const int tr = BM / tw;
        if (tr > H) break;
        if ((tr + 2 * dil) * (tw + 2 * dil) < (c.TR + 2 * dil) * (c.TW + 2 * dil)) {
          c.TW = tw;
          c.TR = tr;
        }
      }
    } else if (BM % HW == 0 && BM / HW <= 8 && W >= 4) {
      c.TW = W;
      c.TR = H;
      c.TL = BM / HW;
    } else {
      continue;
    }
    if (conv_lds_bytes<P>(c) > 160 * 1024) continue;
    *t = c;
    return true;
  }
  return false;
}

template <class P, int MW, int NW, int MODE, bool X>
hipError_t launch_mfma_kx(const ConvArgs &a, size_t lds, unsigned tiles, hipStream_t s) {
  static std::atomic<uint64_t> attr{0};
  if (npg_first_on_device(attr)) {
    hipError_t e = hipFuncSetAttribute((const void *)conv_mfma_kernel<P, MW, NW, MODE, X>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((conv_mfma_kernel<P, MW, NW, MODE, X>), dim3(tiles), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <class P, int MW, int NW, int MODE>
hipError_t launch_mfma_k(const ConvArgs &a, size_t lds, unsigned tiles, hipStream_t s) {
  // the extended form only for the layers that need it (8/16-bit and FP64
  // tiles on plain, concatenated or pooled inputs; never FP8)
  if (a.dil != 1 || a.act != ACT_RELU || a.res) {
    if constexpr (MODE != 2 && !P::Q8) return launch_mfma_kx<P, MW, NW, MODE, true>(a, lds, tiles, s);
    return hipErrorInvalidValue;
  }
  return launch_mfma_kx<P, MW, NW, MODE, false>(a, lds, tiles, s);
}

template <class P, int MW, int NW>
hipError_t launch_mfma_t(const ConvArgs &a, size_t lds, unsigned tiles, hipStream_t s) {
  if (a.src.mode == SRC_POOL) return launch_mfma_k<P, MW, NW, 1>(a, lds, tiles, s);
  if (a.wpp) {
    if constexpr (P::F64) return launch_mfma_k<P, MW, NW, 3>(a, lds, tiles, s);
    return hipErrorInvalidValue;
  }
  if (a.src.mode == SRC_ENERGY) {
    if constexpr (NW == 1 && P::KC <= 16 && 16 % P::KC == 0) return launch_mfma_k<P, MW, NW, 2>(a, lds, tiles, s);
    return hipErrorInvalidValue;
  }
  return launch_mfma_k<P, MW, NW, 0>(a, lds, tiles, s);
}

template <class P>
hipError_t launch_mfma(const ConvArgs &a0, const Tiling &t, unsigned tiles, hipStream_t s) {
  const bool first = a0.src.mode == SRC_ENERGY;
  const size_t lds = conv_lds_bytes<P>(t, first);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  if (P::F64 && !a0.wpk64) return hipErrorInvalidValue;  // the FP64 tiles read the binary64 weights
  ConvArgs a = a0;
  a.wbytes = (int)conv_wts_bytes<P>(t);
  switch (t.NW * 10 + t.MW) {
    case 11: return launch_mfma_t<P, 1, 1>(a, lds, tiles, s);
    case 12: return launch_mfma_t<P, 2, 1>(a, lds, tiles, s);
    case 14: return launch_mfma_t<P, 4, 1>(a, lds, tiles, s);
    case 21: return launch_mfma_t<P, 1, 2>(a, lds, tiles, s);
    case 22: return launch_mfma_t<P, 2, 2>(a, lds, tiles, s);
    case 24: return launch_mfma_t<P, 4, 2>(a, lds, tiles, s);
    case 41: return launch_mfma_t<P, 1, 4>(a, lds, tiles, s);
    case 42: return launch_mfma_t<P, 2, 4>(a, lds, tiles, s);
    case 44: return launch_mfma_t<P, 4, 4>(a, lds, tiles, s);
    case 81: return launch_mfma_t<P, 1, 8>(a, lds, tiles, s);
    case 82: return launch_mfma_t<P, 2, 8>(a, lds, tiles, s);
    case 18: return launch_mfma_t<P, 8, 1>(a, lds, tiles, s);
    case 28:
      if constexpr (P::MAX_TILES >= 16) return launch_mfma_t<P, 8, 2>(a, lds, tiles, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// ---------------------------------------------------------------- runner
namespace {

struct Runner {
  npg_ctx *ctx;
  const npg_model *m;
  npg_precision prec;
  hipStream_t s;
  size_t esz;  // bytes per activation element
  int force_direct = 0;
  int upsample_taps9 = 0;                    // 1: upsampled channels with nine taps (testing)
  const std::vector<int> *mw_cap = nullptr;  // per conv call of a chunk (autotuned)
  int mw_all = 4;                            // cap for every call (autotuner probes)
  std::vector<hipEvent_t> *ev = nullptr;     // per-call begin/end events (autotuner)
  int call = 0;                              // conv call index within a chunk
  int fuse_first = 1;                        // first layer inside the second layer's staging
  int pool_outputs = 1;                      // U-Net levels store their output's 2x2 means too
  unsigned *amax = nullptr;                  // calibration: per-call max of the stored output
                                             // (float bits); the head is then not fused
  bool pooled = false;                       // the last conv also stored its output's 2x2 means

  int cap() const {
    int c = mw_all;
    if (mw_cap && call < (int)mw_cap->size()) c = std::min(c, (*mw_cap)[call]);
    return c;
  }
  // mw_lim: 4 for a fused head (its epilogue keeps one pixel per lane of a
  // 16-lane group, 4*MW <= 16)
  bool tiling(const LayerDev &y, int H, int W, Tiling *t, int mw_lim = 8) const {
    const int c = std::min(cap(), mw_lim);
    if (prec == NPG_FP32) return pick_tiling<F32P>(y.cout, H, W, t, c, y.dil);
    if (prec == NPG_FP8) {
      if (y.cin % KC8 == 0) return pick_tiling<FP8P>(y.cout, H, W, t, c, y.dil);
      return pick_tiling<FP8S>(y.cout, H, W, t, c, y.dil);
    }
    if (y.cin % KC16 == 0) return pick_tiling<BF16P>(y.cout, H, W, t, c, y.dil);
    return pick_tiling<BF16S>(y.cout, H, W, t, c, y.dil);
  }
  // channel granularity of the tiled kernel's 16-byte input loads
  int vec() const { return prec == NPG_FP32 ? 2 : prec == NPG_FP8 ? 16 : 8; }
  bool mfma_fits(const LayerDev &y, const Src &src, int H, int W, Tiling *t, int mw_lim = 8) const {
    const int v = vec();
    if (force_direct || y.k != 3 || src.mode == SRC_ENERGY || src.mode == SRC_FIVE || y.cin % v) return false;
    if (src.mode == SRC_UPCAT && (src.C0 % v || src.C1 % v)) return false;
    // the tiled kernel takes each K chunk's channels from one source
    const int kc = prec == NPG_FP32 ? KC32 : (y.cin % 32 == 0 ? 32 : 16);
    if (src.mode == SRC_UPCAT && src.C0 % kc) return false;
    if (!tiling(y, H, W, t, mw_lim)) return false;
    // the tiles read their input through buffer resources: the bytes of one
    // tile's leaves must stay below 2^31 (offsets at or past 2^31 mean padding)
    const size_t esz = prec == NPG_FP32 ? sizeof(double) : prec == NPG_FP8 ? 1 : 2;
    const size_t px = src.mode == SRC_POOL ? (size_t)4 * H * W : (size_t)H * W;
    const size_t ch = (size_t)std::max(src.C0, src.C1);
    return (size_t)t->TL * px * ch * esz < ((size_t)1 << 31);
  }

  // The first layer (energy -> 16 channels, 3x3, ReLU) can be computed inside
  // the second layer's patch staging (16 -> 16, 3x3, ReLU) when the tiles fit.
  bool first_fusable(const LayerDev &l0, const LayerDev &l1, int H, int W, Tiling *t) const {
    if (force_direct || amax || !fuse_first) return false;
    if (l0.k != 3 || l0.cin != 1 || l0.cout != 16 || l1.k != 3 || l1.cin != 16 || l1.cout != 16) return false;
    if (!tiling(l1, H, W, t)) return false;
    const size_t lds = prec == NPG_FP32  ? conv_lds_bytes<F32P>(*t, true)
                       : prec == NPG_FP8 ? conv_lds_bytes<FP8S>(*t, true)
                                         : conv_lds_bytes<BF16S>(*t, true);
    return lds <= 160 * 1024;
  }

  int conv_first_fused(const LayerDev &l0, const LayerDev &l1, const Src &energy, int Lc, int H, int W,
                       void *out, void *pool_out = nullptr) {
    pooled = false;
    if (ev) {
      if (hipEventRecord((*ev)[2 * call], s) != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "event record");
    }
    Tiling t;
    if (!first_fusable(l0, l1, H, W, &t)) return npg_fail(ctx, NPG_E_ARG, "internal: first layer not fusable");
    ConvArgs a{};
    a.src = energy;
    a.Cin = 16;
    a.Cout = 16;
    a.H = H;
    a.W = W;
    a.TW = t.TW;
    a.TR = t.TR;
    a.TL = t.TL;
    a.Lc = Lc;
    a.fPW = make_fastdiv((uint32_t)(t.TW + 2));
    a.fPP = make_fastdiv((uint32_t)((t.TW + 2) * (t.TR + 2)));
    a.fTW = make_fastdiv((uint32_t)t.TW);
    a.fTPX = make_fastdiv((uint32_t)(t.TW * t.TR));
    a.tiles_x = W / t.TW;
    a.tiles_per_leaf = (H / t.TR) * a.tiles_x;
    a.nchunk = prec == NPG_FP32 ? 16 / KC32 : 1;
    a.bias = l1.b;
    a.head_w = nullptr;
    a.wsc = l1.wsc8;
    a.oinv = 1.0f / l1.a8;
    a.asc = l1.a8;
    a.w0 = l0.w;
    a.b0 = l0.b;
    a.oinv0 = prec == NPG_FP8 ? 1.0f / l0.a8 : 1.0f;
    a.out = out;
    if (pool_out && t.TR % 2 == 0 && t.TW % 2 == 0) {
      a.pool_out = pool_out;
      pooled = true;
    }
    const unsigned tiles = (unsigned)((Lc + t.TL - 1) / t.TL) * a.tiles_per_leaf;
    // layer 1 on the matrix cores; layer 0 recomputed on the vector ALUs for
    // every patch pixel (the tile and its one-pixel halo)
    ctx->conv_flops[0] += 2.0 * Lc * H * W * 16.0 * 9.0 * 16.0;
    ctx->conv_flops[1] += 2.0 * tiles * t.TL * (t.TR + 2.0) * (t.TW + 2.0) * 16.0 * 9.0;
    hipError_t e;
    if (prec == NPG_FP32) {
      a.wpk = l1.pk32;
      a.wpk64 = l1.pk64;
      e = launch_mfma<F32P>(a, t, tiles, s);
    } else if (prec == NPG_FP8) {
      a.wpk = l1.pk8s;
      e = launch_mfma<FP8S>(a, t, tiles, s);
    } else {
      a.wpk = l1.pk16s;
      e = launch_mfma<BF16S>(a, t, tiles, s);
    }
    if (e != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "fused first conv launch: %s", hipGetErrorString(e));
    if (ev) {
      if (hipEventRecord((*ev)[2 * call + 1], s) != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "event record");
    }
    ++call;
    return NPG_OK;
  }

  // res: a tensor of the output's layout added after the activation (a
  // residual link), or null
  // the pooled output of a plain-order tile (no phase order, head or
  // residual) with even TR and TW
  void set_pool(ConvArgs &a, const Tiling &t, void *pool_out) {
    if (pool_out && !a.wpp && !a.head_w && !a.res && t.TR % 2 == 0 && t.TW % 2 == 0) {
      a.pool_out = pool_out;
      pooled = true;
    }
  }
  // pool_out: where to store the 2x2 means of the output as well (the next
  // level's pooled input), if the layer's tiles can; `pooled` tells whether
  // they did
  int conv(const LayerDev &y, const Src &src, int Lc, int H, int W, void *out, const LayerDev *head,
           int act, const void *res = nullptr, void *pool_out = nullptr) {
    pooled = false;
    if (ev) {
      if (hipEventRecord((*ev)[2 * call], s) != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "event record");
    }
    int rc = conv_impl(y, src, Lc, H, W, out, head, act, res, pool_out);
    if (ev && !rc) {
      if (hipEventRecord((*ev)[2 * call + 1], s) != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "event record");
    }
    if (amax && !rc && act == ACT_RELU && !head) {
      const size_t n = (size_t)Lc * H * W * y.cout;
      const unsigned blocks = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
      if (prec == NPG_FP32)
        hipLaunchKernelGGL(amax_kernel<double>, dim3(blocks), dim3(256), 0, s, static_cast<const double *>(out), n,
                           amax + call);
      else
        return npg_fail(ctx, NPG_E_ARG, "internal: calibration runs in FP32");
      if (hipGetLastError() != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "amax launch");
    }
    ++call;
    return rc;
  }

  // One 3x3 conv (+ReLU / ELU, + residual) or the last layer (+head / softplus).
  int conv_impl(const LayerDev &y, const Src &src, int Lc, int H, int W, void *out, const LayerDev *head,
                int act, const void *res, void *pool_out) {
    if ((act == ACT_ELU || res || y.dil != 1) && (prec == NPG_FP8 || head))
      return npg_fail(ctx, NPG_E_ARG, "internal: ELU, residual and dilated layers run in FP32 or BF16, unfused");
    Tiling t;
    const bool mfma_ok = (act == ACT_RELU || act == ACT_ELU) && mfma_fits(y, src, H, W, &t, head ? 4 : 8) &&
                         (!head || y.cout == 16);
    if (mfma_ok) {
      ConvArgs a;
      a.src = src;
      a.Cin = y.cin;
      a.Cout = y.cout;
      a.H = H;
      a.W = W;
      a.TW = t.TW;
      a.TR = t.TR;
      a.TL = t.TL;
      a.Lc = Lc;
      a.dil = y.dil;
      a.act = act;
      a.res = res;
      a.fPW = make_fastdiv((uint32_t)(t.TW + 2 * y.dil));
      a.fPP = make_fastdiv((uint32_t)((t.TW + 2 * y.dil) * (t.TR + 2 * y.dil)));
      a.fTW = make_fastdiv((uint32_t)t.TW);
      a.fTPX = make_fastdiv((uint32_t)(t.TW * t.TR));
      a.tiles_x = W / t.TW;
      a.tiles_per_leaf = (H / t.TR) * a.tiles_x;
      a.bias = y.b;
      a.head_w = head ? head->w : nullptr;
      a.head_b = head ? m->host_b[&*head - &m->layer[0]][0] : 0.0f;
      a.wsc = y.wsc8;
      a.oinv = 1.0f / y.a8;
      a.asc = y.a8;
      a.out = out;
      const unsigned tiles = (unsigned)((Lc + t.TL - 1) / t.TL) * a.tiles_per_leaf;
      const double px = (double)Lc * H * W;
      double taps_x_cin = 9.0 * y.cin;  // multiply-adds per output channel and pixel
      hipError_t e;
      if (prec == NPG_FP32) {
        a.nchunk = (y.cin + KC32 - 1) / KC32;
        a.wpk = y.pk32;
        a.wpk64 = y.pk64;
        // upsampled channels by phase (every tile here has even TR and TW)
        if (src.mode == SRC_UPCAT && !head && y.dil == 1 && y.pkp && !upsample_taps9 && t.TR % 2 == 0 &&
            t.TW % 2 == 0 && t.TL * t.TR * t.TW == 64 * t.MW) {
          a.wpp = y.pkp;
          taps_x_cin = 4.0 * src.C0 + 9.0 * src.C1;
        }
        ctx->conv_flops[0] += 2.0 * px * y.cout * taps_x_cin;
        set_pool(a, t, pool_out);
        e = launch_mfma<F32P>(a, t, tiles, s);
      } else if (prec == NPG_FP8 && y.cin % KC8 == 0) {
        ctx->conv_flops[0] += 2.0 * px * y.cout * taps_x_cin;
        a.nchunk = y.cin / KC8;
        a.wpk = y.pk8;
        set_pool(a, t, pool_out);
        e = launch_mfma<FP8P>(a, t, tiles, s);
      } else if (prec == NPG_FP8) {
        ctx->conv_flops[0] += 2.0 * px * y.cout * taps_x_cin;
        a.nchunk = (y.cin + KC8S - 1) / KC8S;
        a.wpk = y.pk8s;
        set_pool(a, t, pool_out);
        e = launch_mfma<FP8S>(a, t, tiles, s);
      } else if (y.cin % KC16 == 0) {
        ctx->conv_flops[0] += 2.0 * px * y.cout * taps_x_cin;
        a.nchunk = y.cin / KC16;
        a.wpk = y.pk16;
        set_pool(a, t, pool_out);
        e = launch_mfma<BF16P>(a, t, tiles, s);
      } else {
        ctx->conv_flops[0] += 2.0 * px * y.cout * taps_x_cin;
        a.nchunk = (y.cin + KC16S - 1) / KC16S;
        a.wpk = y.pk16s;
        set_pool(a, t, pool_out);
        e = launch_mfma<BF16S>(a, t, tiles, s);
      }
      if (head) ctx->conv_flops[1] += 2.0 * px * head->cin;  // 1x1 head in the epilogue
      if (e != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "conv launch: %s", hipGetErrorString(e));
      return NPG_OK;
    }
    if (src.mode == SRC_FIVE) {
      ctx->conv_flops[1] += 2.0 * Lc * H * W * y.cout * 5.0 * 9.0;
      if (y.k != 3 || y.cin != 5 || (act != ACT_RELU && act != ACT_ELU) || head || res || prec == NPG_FP8)
        return npg_fail(ctx, NPG_E_ARG, "internal: five-channel first layer");
      // tile of TR x TW pixels per workgroup (H, W powers of two, 4..1024)
      const int TW = std::min(W, 256), TR = std::min(H, 256 / TW);
      if ((TR + 2) * (TW + 2) > F5_LDS || H % TR || W % TW)
        return npg_fail(ctx, NPG_E_ARG, "internal: five-channel tile %dx%d", TR, TW);
      const dim3 grid((unsigned)((H / TR) * (W / TW)), (unsigned)Lc);
      auto go = [&](auto tag_t, auto tag_acc, auto tag_c) {
        using TT = decltype(tag_t);
        using AA = decltype(tag_acc);
        constexpr int C = decltype(tag_c)::value;
        if (act == ACT_ELU)
          hipLaunchKernelGGL((conv_first5_kernel<TT, AA, C, ACT_ELU>), grid, dim3(256), 0, s, src, y.w, y.b, H, W,
                             TW, TR, out);
        else
          hipLaunchKernelGGL((conv_first5_kernel<TT, AA, C, ACT_RELU>), grid, dim3(256), 0, s, src, y.w, y.b, H,
                             W, TW, TR, out);
      };
      auto by_c = [&](auto tag_t, auto tag_acc) {
        switch (y.cout) {
          case 4: go(tag_t, tag_acc, std::integral_constant<int, 4>{}); return true;
          case 8: go(tag_t, tag_acc, std::integral_constant<int, 8>{}); return true;
          case 16: go(tag_t, tag_acc, std::integral_constant<int, 16>{}); return true;
          case 32: go(tag_t, tag_acc, std::integral_constant<int, 32>{}); return true;
          default: return false;
        }
      };
      const bool ok = prec == NPG_FP32 ? by_c(double{}, double{}) : by_c(uint16_t{}, float{});
      if (!ok) return npg_fail(ctx, NPG_E_ARG, "five-channel first layer: %d outputs (4, 8, 16 or 32)", y.cout);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "five-channel conv launch: %s", hipGetErrorString(e));
      return NPG_OK;
    }
    if (!force_direct && src.mode == SRC_ENERGY && y.k == 3 && y.cin == 1 && y.cout <= 16 && act == ACT_RELU &&
        H * W >= 256 && !head && !res) {
      const int TW = std::min(W, 256), TR = 256 / TW;
      if (TR <= H) {
        ctx->conv_flops[1] += 2.0 * Lc * H * W * y.cout * 9.0;
        const unsigned blocks = (unsigned)Lc * (H / TR) * (W / TW);
        if (prec == NPG_FP32)
          hipLaunchKernelGGL((conv_first_kernel<double, double>), dim3(blocks), dim3(256), 0, s,
                             static_cast<const uint64_t *>(src.s0), src.tot, y.w, y.b, y.cout, H, W, TW, TR, 1.0f,
                             out);
        else if (prec == NPG_FP8)
          hipLaunchKernelGGL((conv_first_kernel<uint8_t, float>), dim3(blocks), dim3(256), 0, s,
                             static_cast<const uint64_t *>(src.s0), src.tot, y.w, y.b, y.cout, H, W, TW, TR,
                             1.0f / y.a8, out);
        else
          hipLaunchKernelGGL((conv_first_kernel<uint16_t, float>), dim3(blocks), dim3(256), 0, s,
                             static_cast<const uint64_t *>(src.s0), src.tot, y.w, y.b, y.cout, H, W, TW, TR, 1.0f,
                             out);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "first conv launch: %s", hipGetErrorString(e));
        return NPG_OK;
      }
    }
    const size_t npix = (size_t)Lc * H * W;
    // an unfused 1x1 head on 16 or 32 channels (FP32 or BF16 activations)
    if (!force_direct && act == ACT_SOFTPLUS && y.k == 1 && y.cout == 1 && src.mode == SRC_PLAIN && !res &&
        !head && prec != NPG_FP8 && (y.cin == 16 || y.cin == 32)) {
      ctx->conv_flops[1] += 2.0 * npix * y.cin;
      const unsigned blocks = (unsigned)((npix + 255) / 256);
      float *o = static_cast<float *>(out);
      if (prec == NPG_FP32) {
        const double *in = static_cast<const double *>(src.s0);
        if (y.cin == 16) hipLaunchKernelGGL((head_kernel<double, 16>), dim3(blocks), dim3(256), 0, s, in, y.w, y.b, npix, o);
        else hipLaunchKernelGGL((head_kernel<double, 32>), dim3(blocks), dim3(256), 0, s, in, y.w, y.b, npix, o);
      } else {
        const uint16_t *in = static_cast<const uint16_t *>(src.s0);
        if (y.cin == 16) hipLaunchKernelGGL((head_kernel<uint16_t, 16>), dim3(blocks), dim3(256), 0, s, in, y.w, y.b, npix, o);
        else hipLaunchKernelGGL((head_kernel<uint16_t, 32>), dim3(blocks), dim3(256), 0, s, in, y.w, y.b, npix, o);
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "head launch: %s", hipGetErrorString(e));
      return NPG_OK;
    }
    // direct path; a fused head becomes a separate 1x1 direct layer
    void *dst = out;
    if (head) {
      // intermediate activation is written into the head's output region's
      // companion buffer provided by the caller through `out` of this call:
      return npg_fail(ctx, NPG_E_ARG, "internal: head fusion without MFMA tiling");
    }
    ctx->conv_flops[1] += 2.0 * npix * y.cout * y.cin * y.k * y.k;
    const unsigned blocks = (unsigned)((npix + 255) / 256);
    if (prec == NPG_FP32)
      hipLaunchKernelGGL(conv_direct_kernel<double>, dim3(blocks), dim3(256), 0, s, src, y.w, y.b, y.cin,
                         y.cout, y.k, H, W, npix, act, 1.0f, dst, y.dil, res);
    else if (prec == NPG_FP8)
      hipLaunchKernelGGL(conv_direct_kernel<uint8_t>, dim3(blocks), dim3(256), 0, s, src, y.w, y.b, y.cin,
                         y.cout, y.k, H, W, npix, act, 1.0f / y.a8, dst, 1, nullptr);
    else
      hipLaunchKernelGGL(conv_direct_kernel<uint16_t>, dim3(blocks), dim3(256), 0, s, src, y.w, y.b,
                         y.cin, y.cout, y.k, H, W, npix, act, 1.0f, dst, y.dil, res);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "direct conv launch: %s", hipGetErrorString(e));
    return NPG_OK;
  }
};

Src plain(const void *p, int C, float q) { return Src{SRC_PLAIN, p, nullptr, nullptr, C, 0, q, 1.0f}; }
Src pooled(const void *p, int C, float q) { return Src{SRC_POOL, p, nullptr, nullptr, C, 0, q, 1.0f}; }
Src upcat(const void *lo, int Cu, const void *skip, int Cs, float qlo, float qskip) {
  return Src{SRC_UPCAT, lo, skip, nullptr, Cu, Cs, qlo, qskip};
}

}  // namespace

namespace {

// Activation scratch of the network for one leaf.
struct NetPlan {
  size_t per_leaf = 0;              // bytes
  std::vector<size_t> skip_elems;   // U-Net skip tensors (elements per leaf)
  size_t tmp_elems = 0;             // each of the two ping-pong buffers
  bool pool = false;                // U-Net: the skip tensors' 2x2 means too (a quarter each)
};

NetPlan plan_net(const npg_model *m, int H, int W, size_t esz) {
  NetPlan p;
  const size_t HW = (size_t)H * W;
  if (m->arch == 1) {
    for (const LayerDev &y : m->layer) p.tmp_elems = std::max(p.tmp_elems, (size_t)y.cout * HW);
    p.per_leaf = 2 * npg_align(p.tmp_elems * esz, 64);
    return p;
  }
  const int D = m->levels;
  for (int d = 0; d < D; ++d) {
    const size_t e = (size_t)m->layer[2 * d].cout * (HW >> (2 * d));
    p.tmp_elems = std::max(p.tmp_elems, e);
    if (d < D - 1) p.skip_elems.push_back(e);
  }
  p.pool = m->arch == 2;
  for (size_t e : p.skip_elems) p.per_leaf += npg_align(e * esz, 64) + (p.pool ? npg_align(e / 4 * esz, 64) : 0);
  p.per_leaf += 2 * npg_align(p.tmp_elems * esz, 64);
  return p;
}

struct NetBufs {
  std::vector<char *> skip;
  std::vector<char *> pool;  // 2x2 means of each skip tensor (U-Net), or empty
  char *tA = nullptr, *tB = nullptr;
};

size_t net_bufs_bytes(const NetPlan &p, size_t chunk, size_t esz) {
  size_t b = 0;
  for (size_t e : p.skip_elems) b += npg_align(chunk * e * esz) + (p.pool ? npg_align(chunk * (e / 4) * esz) : 0);
  return b + 2 * npg_align(chunk * p.tmp_elems * esz);
}

NetBufs carve_net(Carver &cv, const NetPlan &p, size_t chunk, size_t esz) {
  NetBufs B;
  for (size_t e : p.skip_elems) B.skip.push_back(cv.take<char>(chunk * e * esz));
  if (p.pool)
    for (size_t e : p.skip_elems) B.pool.push_back(cv.take<char>(chunk * (e / 4) * esz));
  B.tA = cv.take<char>(chunk * p.tmp_elems * esz);
  B.tB = cv.take<char>(chunk * p.tmp_elems * esz);
  return B;
}

// The paper-style U-Net on one chunk (FP32 or BF16 activations): ELU after
// every 3x3 conv, residual links around the second conv of each level and
// around both dilated convs of the bottleneck, the 1x1 softplus head.
// Buffers: level outputs of the encoder in the skip buffers, everything
// else alternates between tA and tB (a conv never writes its own input or
// residual).
int paper_chunk(Runner &R, const Src &in, int Lc, int H, int W, float *dens, const NetBufs &B) {
  const npg_model *m = R.m;
  const int D = m->levels;
  int h = H, w = W, li = 0, rc;
  const void *prev = nullptr;
  int prevC = 0;
  for (int d = 0; d < D; ++d) {  // encoder
    const LayerDev &la = m->layer[li];
    Src sa = in;
    if (d > 0) {
      h /= 2;
      w /= 2;
      sa = pooled(prev, prevC, 1.0f);
    }
    rc = R.conv(la, sa, Lc, h, w, B.tA, nullptr, ACT_ELU);
    if (rc) return rc;
    if (d < D - 1) {
      const LayerDev &lb = m->layer[li + 1];
      rc = R.conv(lb, plain(B.tA, la.cout, 1.0f), Lc, h, w, B.skip[d], nullptr, ACT_ELU, B.tA);
      if (rc) return rc;
      prev = B.skip[d];
      li += 2;
    } else {  // bottleneck: dilations 2 and 4, each with its residual link
      const LayerDev &l2 = m->layer[li + 1], &l4 = m->layer[li + 2];
      rc = R.conv(l2, plain(B.tA, la.cout, 1.0f), Lc, h, w, B.tB, nullptr, ACT_ELU, B.tA);
      if (rc) return rc;
      rc = R.conv(l4, plain(B.tB, la.cout, 1.0f), Lc, h, w, B.tA, nullptr, ACT_ELU, B.tB);
      if (rc) return rc;
      prev = B.tA;
      li += 3;
    }
    prevC = la.cout;
  }
  for (int d = D - 2; d >= 0; --d) {  // decoder
    const LayerDev &la = m->layer[li], &lb = m->layer[li + 1];
    li += 2;
    h *= 2;
    w *= 2;
    const int cs = m->layer[2 * d].cout;
    char *ta = prev == B.tA ? B.tB : B.tA;
    char *tb = ta == B.tA ? B.tB : B.tA;  // held the level below, read by the first conv only
    rc = R.conv(la, upcat(prev, prevC, B.skip[d], cs, 1.0f, 1.0f), Lc, h, w, ta, nullptr, ACT_ELU);
    if (rc) return rc;
    rc = R.conv(lb, plain(ta, la.cout, 1.0f), Lc, h, w, tb, nullptr, ACT_ELU, ta);
    if (rc) return rc;
    prev = tb;
    prevC = lb.cout;
  }
  return R.conv(m->layer[li], plain(prev, prevC, 1.0f), Lc, H, W, dens, nullptr, ACT_SOFTPLUS);
}

// The network on one chunk of Lc leaves: `in` is the energy source (with
// per-leaf totals), `dens` receives the softplus densities.
int net_chunk(Runner &R, const Src &in, int Lc, int H, int W, float *dens, const NetBufs &B) {
  const npg_model *m = R.m;
  int rc;
  R.call = 0;
  // FP8: value of one stored unit of a layer's output
  auto dq = [&](const LayerDev &y) { return R.prec == NPG_FP8 ? y.a8 : 1.0f; };
  if (m->arch == 1) {
    const int n = (int)m->layer.size();
    Src cur = in;
    char *bufs[2] = {B.tA, B.tB};
    int i0 = 0;
    Tiling tf;
    if (n > 2 && R.first_fusable(m->layer[0], m->layer[1], H, W, &tf)) {
      rc = R.conv_first_fused(m->layer[0], m->layer[1], in, Lc, H, W, bufs[1]);
      if (rc) return rc;
      cur = plain(bufs[1], 16, dq(m->layer[1]));
      i0 = 2;
    }
    for (int i = i0; i < n; ++i) {
      const LayerDev &y = m->layer[i];
      const bool last = i == n - 1;
      void *dst = last ? (void *)dens : (void *)bufs[i & 1];
      rc = R.conv(y, cur, Lc, H, W, dst, nullptr, last ? ACT_SOFTPLUS : ACT_RELU);
      if (rc) return rc;
      cur = plain(dst, y.cout, dq(y));
    }
    return NPG_OK;
  }
  if (m->arch == 3) return paper_chunk(R, in, Lc, H, W, dens, B);
  const int D = m->levels;
  int h = H, w = W;
  const void *prev = nullptr;
  int prevC = 0;
  float prevQ = 1.0f;
  bool have_pool = false;  // the level above stored its output's 2x2 means
  for (int d = 0; d < D; ++d) {  // encoder
    const LayerDev &la = m->layer[2 * d], &lb = m->layer[2 * d + 1];
    Src sa = in;
    if (d > 0) {
      h /= 2;
      w /= 2;
      sa = have_pool ? plain(B.pool[d - 1], prevC, prevQ) : pooled(prev, prevC, prevQ);
    }
    void *ob = d < D - 1 ? (void *)B.skip[d] : (void *)B.tB;
    // the level's output tile also stores its 2x2 means, the next level's input
    void *po = d < D - 1 && R.pool_outputs && !B.pool.empty() ? (void *)B.pool[d] : nullptr;
    Tiling tf;
    if (d == 0 && R.first_fusable(la, lb, h, w, &tf)) {
      rc = R.conv_first_fused(la, lb, sa, Lc, h, w, ob, po);
      if (rc) return rc;
    } else {
      rc = R.conv(la, sa, Lc, h, w, B.tA, nullptr, ACT_RELU);
      if (rc) return rc;
      rc = R.conv(lb, plain(B.tA, la.cout, dq(la)), Lc, h, w, ob, nullptr, ACT_RELU, nullptr, po);
      if (rc) return rc;
    }
    have_pool = po && R.pooled;
    prev = ob;
    prevC = lb.cout;
    prevQ = dq(lb);
  }
  int li = 2 * D;
  for (int d = D - 2; d >= 0; --d) {  // decoder
    const LayerDev &la = m->layer[li], &lb = m->layer[li + 1];
    li += 2;
    h *= 2;
    w *= 2;
    const int cs = m->layer[2 * d].cout;
    rc = R.conv(la, upcat(prev, prevC, B.skip[d], cs, prevQ, dq(m->layer[2 * d + 1])), Lc, h, w, B.tA, nullptr,
                ACT_RELU);
    if (rc) return rc;
    const Src sb = plain(B.tA, la.cout, dq(la));
    if (d == 0) {
      const LayerDev &hd = m->layer[li];
      Tiling t;
      const bool fuse = !R.amax && lb.cout == 16 && R.mfma_fits(lb, sb, h, w, &t, 4);
      if (fuse) {
        rc = R.conv(lb, sb, Lc, h, w, dens, &hd, ACT_RELU);
        if (rc) return rc;
      } else {
        rc = R.conv(lb, sb, Lc, h, w, B.tB, nullptr, ACT_RELU);
        if (rc) return rc;
        rc = R.conv(hd, plain(B.tB, lb.cout, dq(lb)), Lc, h, w, dens, nullptr, ACT_SOFTPLUS);
        if (rc) return rc;
      }
    } else {
      rc = R.conv(lb, sb, Lc, h, w, B.tB, nullptr, ACT_RELU);
      if (rc) return rc;
      prev = B.tB;
      prevC = lb.cout;
      prevQ = dq(lb);
    }
  }
  if (D == 1) {
    const LayerDev &hd = m->layer[2];
    rc = R.conv(hd, plain(prev, prevC, prevQ), Lc, H, W, dens, nullptr, ACT_SOFTPLUS);
    if (rc) return rc;
  }
  return NPG_OK;
}

int check_net_args(npg_ctx *ctx, const npg_model *m, int H, int W, npg_precision precision, int in_ch = 1) {
  if (!m) return npg_fail(ctx, NPG_E_ARG, "reconstruct: null model");
  if (m->in_ch != in_ch)
    return npg_fail(ctx, NPG_E_ARG, in_ch == 1 ? "reconstruct: a five-channel model needs npg_reconstruct_density5"
                                               : "reconstruct: npg_reconstruct_density5 needs a five-channel U-Net");
  if (!pow2_in(H, 4, 1024) || !pow2_in(W, 4, 1024))
    return npg_fail(ctx, NPG_E_ARG, "reconstruct: bad H=%d W=%d", H, W);
  if (precision != NPG_FP32 && precision != NPG_BF16 && precision != NPG_FP8)
    return npg_fail(ctx, NPG_E_ARG, "reconstruct: bad precision %d", (int)precision);
  if (precision == NPG_FP8 && !m->fp8_ready)
    return npg_fail(ctx, NPG_E_ARG, "reconstruct: FP8 needs npg_model_calibrate_fp8 first");
  if (m->arch == 2 || m->arch == 3) {
    const int f = 1 << (m->levels - 1);
    if (H % f || W % f) return npg_fail(ctx, NPG_E_ARG, "reconstruct: %dx%d not divisible by 2^%d", H, W, m->levels - 1);
  }
  return NPG_OK;
}

std::string tune_key(const npg_model *m, npg_precision p, int H, int W) {
  char b[96];
  snprintf(b, sizeof(b), "%p:%d:%d:%d", (const void *)m, (int)p, H, W);
  return b;
}

Runner make_runner(npg_ctx *ctx, const npg_model *m, npg_precision prec, hipStream_t s) {
  Runner R{ctx, m, prec, s, prec == NPG_FP32 ? sizeof(double) : prec == NPG_FP8 ? (size_t)1 : (size_t)2};
  R.force_direct = (int)ctx->opt("force_direct", 0);
  R.upsample_taps9 = (int)ctx->opt("upsample_taps9", 0);
  R.fuse_first = ctx->opt("fuse_first", 1) ? 1 : 0;
  R.pool_outputs = ctx->opt("pool_outputs", 1) ? 1 : 0;
  const long long cap = ctx->opt("tile_cap", 4);  // testing: pixel tiles of at most 64 * cap
  R.mw_all = cap >= 8 ? 8 : cap >= 4 ? 4 : cap >= 2 ? 2 : 1;
  return R;
}

// Leaves per chunk: tuned value, else the context option, else 1024; then
// bounded by the budget.  per_extra = other per-leaf scratch bytes.
int chunk_for(npg_ctx *ctx, const npg_model *m, npg_precision prec, int H, int W, uint32_t L, size_t per_leaf,
              size_t fixed, size_t *chunk_out) {
  size_t chunk = 1024;
  auto it = ctx->tune.find(tune_key(m, prec, H, W));
  if (it != ctx->tune.end() && !it->second.empty() && it->second[0] > 0) chunk = (size_t)it->second[0];
  const long long o = ctx->opt("chunk_leaves", 0);
  if (o > 0) chunk = (size_t)o;
  chunk = std::min<size_t>(chunk, L);
  if (ctx->budget) {
    const uint64_t others = ctx->held - ctx->scratch_bytes;
    const uint64_t avail = ctx->budget > others ? ctx->budget - others : 0;
    if (avail < fixed + per_leaf) return npg_fail(ctx, NPG_E_BUDGET, "reconstruct: budget too small for one leaf");
    chunk = std::min<size_t>(chunk, (avail - fixed) / per_leaf);
  }
  *chunk_out = std::max<size_t>(1, chunk);
  return NPG_OK;
}

void apply_tune(npg_ctx *ctx, Runner &R, int H, int W, std::vector<int> *hold) {
  auto it = ctx->tune.find(tune_key(R.m, R.prec, H, W));
  if (it != ctx->tune.end() && it->second.size() > 1) {
    hold->assign(it->second.begin() + 1, it->second.end());
    R.mw_cap = hold;
    R.mw_all = 8;  // the table's picks (up to 8, as probed) cap each call
  }
}

}  // namespace

// The network over L energy maps, chunk by chunk.  `amax` (calibration):
// per-layer output maxima are recorded, with the head left unfused.
static int run_density(npg_ctx *ctx, const npg_model *m, npg_precision precision, const uint64_t *energy_dev,
                       uint32_t L, int H, int W, float *density_dev, hipStream_t s, unsigned *amax) {
  Runner R = make_runner(ctx, m, precision, s);
  R.amax = amax;
  std::vector<int> caps;
  apply_tune(ctx, R, H, W, &caps);
  const size_t HW = (size_t)H * W;
  const NetPlan plan = plan_net(m, H, W, R.esz);
  const size_t fixed = npg_align(sizeof(double) * L) + (16u << 20);
  size_t chunk = 0;
  int rc = chunk_for(ctx, m, precision, H, W, L, plan.per_leaf, fixed, &chunk);
  if (rc) return rc;
  void *scr = nullptr;
  rc = npg_scratch(ctx, fixed + net_bufs_bytes(plan, chunk, R.esz), s, &scr);
  if (rc) return rc;
  Carver cv(scr);
  double *tot = cv.take<double>(L);
  const NetBufs B = carve_net(cv, plan, chunk, R.esz);
  NPG_HIP_CHECK(ctx, launch_leaf_scale(energy_dev, L, (int)HW, tot, s));
  for (size_t l0 = 0; l0 < L; l0 += chunk) {
    const int Lc = (int)std::min<size_t>(chunk, L - l0);
    const Src in{SRC_ENERGY, energy_dev + l0 * HW, nullptr, tot + l0, 0, 0};
    rc = net_chunk(R, in, Lc, H, W, density_dev + l0 * HW, B);
    if (rc) return rc;
  }
  return NPG_OK;
}

extern "C" int npg_reconstruct_density(npg_ctx *ctx, const npg_model *m, const uint64_t *energy_dev,
                                       const uint32_t *count_dev, uint32_t L, int H, int W,
                                       npg_precision precision, float *density_dev, void *stream) {
  (void)count_dev;
  if (!ctx) return NPG_E_ARG;
  int rc = check_net_args(ctx, m, H, W, precision);
  if (rc) return rc;
  if (L == 0) return NPG_OK;
  if (!energy_dev || !density_dev) return npg_fail(ctx, NPG_E_ARG, "reconstruct: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  return run_density(ctx, m, precision, energy_dev, L, H, W, density_dev, static_cast<hipStream_t>(stream),
                     nullptr);
}

// ---------------------------------------------------------------------------
// The network without allocation (npg_reconstruct_density_noalloc): the same
// chunked network over a file-scope device array instead of the context's
// scratch arena.  Each GPU the library runs on holds its own copy of the
// array from the library's load until the process ends.  The host-side name
// `scratch` is a stand-in, not a device address: host code uses only the
// address hipGetSymbolAddress returns on each device.
constexpr size_t NPG_NOALLOC_BYTES = (size_t)256 << 20;
static __device__ __align__(256) char scratch[NPG_NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};
}  // namespace

int npg_noalloc_setup(npg_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= NOALLOC_MAX_DEVICES)
    return npg_fail(ctx, NPG_E_ARG, "device %d: at most %d devices", ctx->device, NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[ctx->device]) {
    int rc = npg_set_device(ctx);
    if (rc) return rc;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return npg_fail(ctx, NPG_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_noalloc_ptr[ctx->device] = p;
  }
  ctx->noalloc_scratch = g_noalloc_ptr[ctx->device];
  return NPG_OK;
}

extern "C" int npg_reconstruct_density_noalloc(npg_ctx *ctx, const npg_model *m, const uint64_t *energy_dev,
                                               uint32_t L, int H, int W, npg_precision precision,
                                               float *density_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  int rc = check_net_args(ctx, m, H, W, precision);
  if (rc) return rc;
  if (L == 0) return NPG_OK;
  if (!energy_dev || !density_dev) return npg_fail(ctx, NPG_E_ARG, "reconstruct_noalloc: null pointer");
  if (!ctx->noalloc_scratch) return npg_fail(ctx, NPG_E_HIP, "reconstruct_noalloc: scratch address not set up");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Runner R = make_runner(ctx, m, precision, s);
  std::vector<int> caps;
  apply_tune(ctx, R, H, W, &caps);
  const size_t HW = (size_t)H * W;
  const NetPlan plan = plan_net(m, H, W, R.esz);
  // per chunk: the leaves' totals, then the activation buffers
  // (the last MiB of the array stays unused, as the arena keeps a margin
  // after its buffers)
  constexpr size_t usable = NPG_NOALLOC_BYTES - ((size_t)1 << 20);
  auto bytes_for = [&](size_t c) { return npg_align(c * sizeof(double)) + net_bufs_bytes(plan, c, R.esz); };
  if (bytes_for(1) > usable)
    return npg_fail(ctx, NPG_E_BUDGET,
                    "reconstruct_noalloc: one %dx%d leaf needs %zu bytes of scratch, the static array offers %zu",
                    H, W, bytes_for(1), usable);
  size_t chunk = 1024;
  auto it = ctx->tune.find(tune_key(m, precision, H, W));
  if (it != ctx->tune.end() && !it->second.empty() && it->second[0] > 0) chunk = (size_t)it->second[0];
  const long long o = ctx->opt("chunk_leaves", 0);
  if (o > 0) chunk = (size_t)o;
  chunk = std::min<size_t>(chunk, L);
  chunk = std::min<size_t>(chunk, usable / bytes_for(1) + 1);
  while (chunk > 1 && bytes_for(chunk) > usable) --chunk;
  Carver cv(ctx->noalloc_scratch);
  double *tot = cv.take<double>(chunk);
  const NetBufs B = carve_net(cv, plan, chunk, R.esz);
  for (size_t l0 = 0; l0 < L; l0 += chunk) {
    const int Lc = (int)std::min<size_t>(chunk, L - l0);
    NPG_HIP_CHECK(ctx, launch_leaf_scale(energy_dev + l0 * HW, (uint32_t)Lc, (int)HW, tot, s));
    const Src in{SRC_ENERGY, energy_dev + l0 * HW, nullptr, tot, 0, 0};
    rc = net_chunk(R, in, Lc, H, W, density_dev + l0 * HW, B);
    if (rc) return rc;
  }
  return NPG_OK;
}

extern "C" int npg_reconstruct_density5(npg_ctx *ctx, const npg_model *m, const uint64_t *energy_dev,
                                        const uint32_t *count_dev, const uint64_t *energy_prev_dev,
                                        const uint32_t *count_prev_dev, uint32_t L, int H, int W,
                                        npg_precision precision, float *density_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  int rc = check_net_args(ctx, m, H, W, precision, 5);
  if (rc) return rc;
  if (precision == NPG_FP8) return npg_fail(ctx, NPG_E_ARG, "reconstruct5: FP32 or BF16 only");
  if (L == 0) return NPG_OK;
  if (!energy_dev || !count_dev || !energy_prev_dev || !count_prev_dev || !density_dev)
    return npg_fail(ctx, NPG_E_ARG, "reconstruct5: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Runner R = make_runner(ctx, m, precision, s);
  std::vector<int> caps;
  apply_tune(ctx, R, H, W, &caps);
  const size_t HW = (size_t)H * W;
  const NetPlan plan = plan_net(m, H, W, R.esz);
  const size_t fixed = npg_align(4 * sizeof(double) * L) + (16u << 20);
  size_t chunk = 0;
  rc = chunk_for(ctx, m, precision, H, W, L, plan.per_leaf, fixed, &chunk);
  if (rc) return rc;
  void *scr = nullptr;
  rc = npg_scratch(ctx, fixed + net_bufs_bytes(plan, chunk, R.esz), s, &scr);
  if (rc) return rc;
  Carver cv(scr);
  double *tot = cv.take<double>(4 * (size_t)L);
  const NetBufs B = carve_net(cv, plan, chunk, R.esz);
  hipLaunchKernelGGL(leaf_totals5_kernel, dim3(L), dim3(256), 0, s, energy_dev, energy_prev_dev, count_dev,
                     count_prev_dev, (int)HW, tot);
  NPG_HIP_CHECK(ctx, hipGetLastError());
  for (size_t l0 = 0; l0 < L; l0 += chunk) {
    const int Lc = (int)std::min<size_t>(chunk, L - l0);
    Src in{SRC_FIVE, energy_dev + l0 * HW, energy_prev_dev + l0 * HW, tot + 4 * l0, 5, 0};
    in.s2 = count_dev + l0 * HW;
    in.s3 = count_prev_dev + l0 * HW;
    rc = net_chunk(R, in, Lc, H, W, density_dev + l0 * HW, B);
    if (rc) return rc;
  }
  return NPG_OK;
}

// ----------------------------------------------------------- fused path
// splat -> normalise -> network -> CDF, chunk by chunk: the energy maps and
// densities of a chunk live in scratch only, never at full batch size.
static int fused_enqueue(npg_ctx *ctx, const npg_model *m, const float *dir, const uint32_t *w,
                         const uint32_t *perm, const uint32_t *off, uint32_t L, int H, int W, npg_precision prec,
                         float *pdf, float *marg, float *cond, double *total, hipStream_t s) {
  Runner R = make_runner(ctx, m, prec, s);
  std::vector<int> caps;
  apply_tune(ctx, R, H, W, &caps);
  const size_t HW = (size_t)H * W;
  const NetPlan plan = plan_net(m, H, W, R.esz);
  const size_t per_leaf = plan.per_leaf + HW * (sizeof(uint64_t) + sizeof(float)) + sizeof(double) + 3 * 256;
  size_t chunk = 0;
  int rc = chunk_for(ctx, m, prec, H, W, L, per_leaf, 16u << 20, &chunk);
  if (rc) return rc;
  const size_t bytes = npg_align(chunk * HW * sizeof(uint64_t)) + npg_align(chunk * HW * sizeof(float)) +
                       npg_align(chunk * sizeof(double)) + net_bufs_bytes(plan, chunk, R.esz);
  void *scr = nullptr;
  rc = npg_scratch(ctx, bytes, s, &scr);
  if (rc) return rc;
  Carver cv(scr);
  uint64_t *energy = cv.take<uint64_t>(chunk * HW);
  float *dens = cv.take<float>(chunk * HW);
  double *tot = cv.take<double>(chunk);
  const NetBufs B = carve_net(cv, plan, chunk, R.esz);
  for (size_t l0 = 0; l0 < L; l0 += chunk) {
    const uint32_t Lc = (uint32_t)std::min<size_t>(chunk, L - l0);
    NPG_HIP_CHECK(ctx, launch_splat(ctx->bnd_dev, dir, w, perm, off + l0, Lc, H, W, energy, nullptr, 0, ctx->err_dev, s));
    NPG_HIP_CHECK(ctx, launch_leaf_scale(energy, Lc, (int)HW, tot, s));
    const Src in{SRC_ENERGY, energy, nullptr, tot, 0, 0};
    rc = net_chunk(R, in, (int)Lc, H, W, dens, B);
    if (rc) return rc;
    NPG_HIP_CHECK(ctx, launch_build_cdf(dens, Lc, H, W, pdf + l0 * HW, marg + l0 * (H + 1),
                                        cond + l0 * H * (size_t)(W + 1), total ? total + l0 : nullptr,
                                        ctx->err_dev, s));
  }
  return NPG_OK;
}

extern "C" int npg_reconstruct_fused(npg_ctx *ctx, const npg_model *m, const float *dir_dev, const uint32_t *w_dev,
                                     const uint32_t *perm_dev, const uint32_t *leaf_off_dev, uint32_t L, int H,
                                     int W, npg_precision precision, float *pdf_dev, float *marg_dev,
                                     float *cond_dev, double *total_dev, void *stream) {
  if (!ctx) return NPG_E_ARG;
  int rc = check_net_args(ctx, m, H, W, precision);
  if (rc) return rc;
  if (L == 0) return NPG_OK;
  if (!dir_dev || !w_dev || !leaf_off_dev || !pdf_dev || !marg_dev || !cond_dev)
    return npg_fail(ctx, NPG_E_ARG, "reconstruct_fused: null pointer");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!ctx->opt("graphs", 0) || s == nullptr)
    return fused_enqueue(ctx, m, dir_dev, w_dev, perm_dev, leaf_off_dev, L, H, W, precision, pdf_dev, marg_dev,
                         cond_dev, total_dev, s);
  // Graph replay: the first call with a given argument tuple runs eagerly
  // (allocating scratch and setting kernel attributes), the second is
  // captured, later ones replay the captured graph.
  char key[512];
  snprintf(key, sizeof(key), "fused:%p:%p:%p:%p:%p:%u:%d:%d:%d:%p:%p:%p:%p:%p:%p:%zu:%lld", (const void *)m,
           (const void *)dir_dev, (const void *)w_dev, (const void *)perm_dev, (const void *)leaf_off_dev, L, H, W,
           (int)precision, (void *)pdf_dev, (void *)marg_dev, (void *)cond_dev, (void *)total_dev, (void *)s,
           ctx->scratch, ctx->scratch_bytes, ctx->opt("chunk_leaves", 0));
  for (auto &g : ctx->graphs)
    if (g.key == key) {
      NPG_HIP_CHECK(ctx, hipGraphLaunch(g.exec, s));
      return NPG_OK;
    }
  if (!ctx->graph_seen.count(key)) {
    ctx->graph_seen.insert(key);
    return fused_enqueue(ctx, m, dir_dev, w_dev, perm_dev, leaf_off_dev, L, H, W, precision, pdf_dev, marg_dev,
                         cond_dev, total_dev, s);
  }
  NPG_HIP_CHECK(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  rc = fused_enqueue(ctx, m, dir_dev, w_dev, perm_dev, leaf_off_dev, L, H, W, precision, pdf_dev, marg_dev,
                     cond_dev, total_dev, s);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(s, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "graph capture: %s", hipGetErrorString(ec));
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) return npg_fail(ctx, NPG_E_HIP, "graph instantiate: %s", hipGetErrorString(ei));
  if (ctx->graphs.size() >= 32) {
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  ctx->graphs.push_back({key, exec});
  NPG_HIP_CHECK(ctx, hipGraphLaunch(exec, s));
  return NPG_OK;
}

bool npg_model_fp8_ready(const npg_model *m) { return m && m->fp8_ready; }
int npg_model_in_channels(const npg_model *m) { return m ? m->in_ch : 0; }

bool npg_model_fits(const npg_model *m, int H, int W) {
  if (m->arch != 2 && m->arch != 3) return true;
  const int f = 1 << (m->levels - 1);
  return H % f == 0 && W % f == 0;
}

// One serving batch: leaves described by per-leaf descriptors (photon
// windows of several requests, output table pointers), chunked like the
// fused path.
int npg_run_desc_batch(npg_ctx *ctx, const npg_model *m, npg_precision prec, const npg_leaf_desc *d_dev,
                       uint32_t L, int H, int W, hipStream_t s) {
  int rc = check_net_args(ctx, m, H, W, prec);
  if (rc) return rc;
  rc = npg_set_device(ctx);
  if (rc) return rc;
  Runner R = make_runner(ctx, m, prec, s);
  std::vector<int> caps;
  apply_tune(ctx, R, H, W, &caps);
  const size_t HW = (size_t)H * W;
  const NetPlan plan = plan_net(m, H, W, R.esz);
  const size_t per_leaf = plan.per_leaf + HW * (sizeof(uint64_t) + sizeof(float)) + sizeof(double) + 3 * 256;
  size_t chunk = 0;
  rc = chunk_for(ctx, m, prec, H, W, L, per_leaf, 16u << 20, &chunk);
  if (rc) return rc;
  const size_t bytes = npg_align(chunk * HW * sizeof(uint64_t)) + npg_align(chunk * HW * sizeof(float)) +
                       npg_align(chunk * sizeof(double)) + net_bufs_bytes(plan, chunk, R.esz);
  void *scr = nullptr;
  rc = npg_scratch(ctx, bytes, s, &scr);
  if (rc) return rc;
  Carver cv(scr);
  uint64_t *energy = cv.take<uint64_t>(chunk * HW);
  float *dens = cv.take<float>(chunk * HW);
  double *tot = cv.take<double>(chunk);
  const NetBufs B = carve_net(cv, plan, chunk, R.esz);
  for (size_t l0 = 0; l0 < L; l0 += chunk) {
    const uint32_t Lc = (uint32_t)std::min<size_t>(chunk, L - l0);
    NPG_HIP_CHECK(ctx, launch_splat_desc(ctx->bnd_dev, d_dev + l0, Lc, H, W, energy, ctx->err_dev, s));
    NPG_HIP_CHECK(ctx, launch_leaf_scale(energy, Lc, (int)HW, tot, s));
    const Src in{SRC_ENERGY, energy, nullptr, tot, 0, 0};
    rc = net_chunk(R, in, (int)Lc, H, W, dens, B);
    if (rc) return rc;
    NPG_HIP_CHECK(ctx, launch_build_cdf_desc(dens, d_dev + l0, Lc, H, W, ctx->err_dev, s));
  }
  return NPG_OK;
}

// -------------------------------------------------------------- autotune
// Times every convolution of the network under each tile cap (64, 128, 256, 512
// pixels per workgroup) on `probe` zero-energy leaves and keeps the fastest
// per call, then times leaf-chunk sizes with those tiles.  Tile and chunk
// choices do not change any result: each output sums its terms in the same
// order whatever the tiling.
extern "C" int npg_autotune(npg_ctx *ctx, const npg_model *m, int H, int W, npg_precision precision,
                            uint32_t probe, void *stream) {
  if (!ctx) return NPG_E_ARG;
  const int in_ch = m ? m->in_ch : 1;
  int rc = check_net_args(ctx, m, H, W, precision, in_ch);
  if (rc) return rc;
  if (in_ch == 5 && precision == NPG_FP8) return npg_fail(ctx, NPG_E_ARG, "autotune: five-channel models run FP32 or BF16");
  if (probe == 0) return npg_fail(ctx, NPG_E_ARG, "autotune: probe_leaves = 0");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Runner R = make_runner(ctx, m, precision, s);
  const size_t HW = (size_t)H * W;
  const NetPlan plan = plan_net(m, H, W, R.esz);
  const size_t bytes = npg_align(probe * HW * sizeof(uint64_t)) + npg_align(probe * HW * sizeof(float)) +
                       npg_align(4 * probe * sizeof(double)) + net_bufs_bytes(plan, probe, R.esz);
  void *scr = nullptr;
  rc = npg_scratch(ctx, bytes, s, &scr);
  if (rc) return rc;
  Carver cv(scr);
  uint64_t *energy = cv.take<uint64_t>(probe * HW);
  float *dens = cv.take<float>(probe * HW);
  double *tot = cv.take<double>(4 * (size_t)probe);
  const NetBufs B = carve_net(cv, plan, probe, R.esz);
  NPG_HIP_CHECK(ctx, hipMemsetAsync(energy, 0, probe * HW * sizeof(uint64_t), s));
  // zero maps; a five-channel model reads them as all four of its maps (the
  // zero words serve as uint32 counts too)
  const uint32_t *zc = reinterpret_cast<const uint32_t *>(energy);
  if (in_ch == 5) {
    hipLaunchKernelGGL(leaf_totals5_kernel, dim3(probe), dim3(256), 0, s, energy, energy, zc, zc, (int)HW, tot);
    NPG_HIP_CHECK(ctx, hipGetLastError());
  } else {
    NPG_HIP_CHECK(ctx, launch_leaf_scale(energy, probe, (int)HW, tot, s));
  }
  auto src_at = [&](uint32_t l0) {
    if (in_ch == 1) return Src{SRC_ENERGY, energy + l0 * HW, nullptr, tot + l0, 0, 0};
    Src f{SRC_FIVE, energy + l0 * HW, energy + l0 * HW, tot + 4 * (size_t)l0, 5, 0};
    f.s2 = zc + l0 * HW;
    f.s3 = zc + l0 * HW;
    return f;
  };
  const Src in = src_at(0);
  // count the calls of one chunk
  rc = net_chunk(R, in, 1, H, W, dens, B);
  if (rc) return rc;
  const int ncall = R.call;
  std::vector<hipEvent_t> ev(2 * ncall);
  for (auto &e : ev) NPG_HIP_CHECK(ctx, hipEventCreate(&e));
  const int caps[4] = {8, 4, 2, 1};
  std::vector<float> best(ncall, 1e30f);
  std::vector<int> pick(ncall, 4);
  int err = NPG_OK;
  for (int ci = 0; ci < 4 && !err; ++ci) {
    R.mw_all = caps[ci];
    R.ev = nullptr;
    err = net_chunk(R, in, (int)probe, H, W, dens, B);  // warm-up
    for (int rep = 0; rep < 3 && !err; ++rep) {
      R.ev = &ev;
      err = net_chunk(R, in, (int)probe, H, W, dens, B);
      if (err) break;
      if (hipStreamSynchronize(s) != hipSuccess) { err = npg_fail(ctx, NPG_E_HIP, "autotune sync"); break; }
      for (int c = 0; c < ncall; ++c) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev[2 * c], ev[2 * c + 1]) == hipSuccess && ms < best[c]) {
          best[c] = ms;
          pick[c] = caps[ci];
        }
      }
    }
  }
  R.ev = nullptr;
  R.mw_all = 4;
  R.mw_cap = &pick;
  // chunk size
  int best_chunk = (int)probe;
  float best_t = 1e30f;
  hipEvent_t e0 = ev[0], e1 = ev[1];
  const uint32_t cands[6] = {64, 128, 256, 512, 1024, 2048};
  for (int k = 0; k < 6 && !err; ++k) {
    const uint32_t c = std::min(cands[k], probe);
    if (k > 0 && c == std::min(cands[k - 1], probe)) continue;
    for (int rep = 0; rep < 2 && !err; ++rep) {
      (void)hipEventRecord(e0, s);
      for (uint32_t l0 = 0; l0 < probe && !err; l0 += c) {
        const uint32_t Lc = std::min(c, probe - l0);
        err = net_chunk(R, src_at(l0), (int)Lc, H, W, dens + l0 * HW, B);
      }
      (void)hipEventRecord(e1, s);
      if (hipStreamSynchronize(s) != hipSuccess) { err = npg_fail(ctx, NPG_E_HIP, "autotune sync"); break; }
      float ms = 0;
      if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess && rep == 1 && ms < best_t) {
        best_t = ms;
        best_chunk = (int)c;
      }
    }
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  if (err) return err;
  std::vector<int> entry;
  entry.push_back(best_chunk);
  entry.insert(entry.end(), pick.begin(), pick.end());
  ctx->tune[tune_key(m, precision, H, W)] = entry;
  return NPG_OK;
}

extern "C" int npg_tune_table(const npg_ctx *ctx, const npg_model *m, int H, int W, npg_precision precision,
                              int32_t *out, int capacity) {
  if (!ctx) return NPG_E_ARG;
  auto it = ctx->tune.find(tune_key(m, precision, H, W));
  if (it == ctx->tune.end()) return 0;
  const int n = (int)it->second.size();
  for (int i = 0; i < n && i < capacity; ++i) out[i] = it->second[i];
  return n;
}

// Layer whose output feeds each input channel of layer i (-1: the energy
// map), following the CNN chain and the U-Net schedule of net_chunk.
static std::vector<int> channel_producers(const npg_model *m, int i) {
  const int cin = m->layer[i].cin;
  std::vector<int> p(cin, i - 1);
  if (i == 0) {
    p.assign(cin, -1);
    return p;
  }
  if (m->arch != 2) return p;
  const int D = m->levels, j = i - 2 * D;  // j: index among decoder layers and head
  if (j < 0 || j == 2 * (D - 1) || j % 2 == 1) return p;
  // first conv of decoder level d: [upsampled previous output, skip of level d]
  const int d = D - 2 - j / 2;
  const int cu = m->layer[i - 1].cout;
  for (int c = cu; c < cin; ++c) p[c] = 2 * d + 1;
  return p;
}

extern "C" int npg_model_calibrate_fp8(npg_ctx *ctx, npg_model *m, const uint64_t *energy_dev, uint32_t L, int H,
                                       int W, void *stream) {
  if (!ctx) return NPG_E_ARG;
  int rc = check_net_args(ctx, m, H, W, NPG_FP32);
  if (rc) return rc;
  if (L == 0 || !energy_dev) return npg_fail(ctx, NPG_E_ARG, "calibrate_fp8: empty calibration batch");
  rc = npg_set_device(ctx);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = (int)m->layer.size();
  // 1. FP32 forward pass recording the largest stored value of every layer
  void *tmp = nullptr;
  const size_t dens_bytes = npg_align((size_t)L * H * W * sizeof(float));
  const size_t tmp_bytes = dens_bytes + npg_align(sizeof(unsigned) * n);
  rc = npg_device_alloc(ctx, tmp_bytes, &tmp);
  if (rc) return rc;
  float *dens = static_cast<float *>(tmp);
  unsigned *amax_dev = reinterpret_cast<unsigned *>(static_cast<char *>(tmp) + dens_bytes);
  std::vector<unsigned> amax(n, 0u);
  rc = hipMemsetAsync(amax_dev, 0, sizeof(unsigned) * n, s) == hipSuccess ? NPG_OK
                                                                          : npg_fail(ctx, NPG_E_HIP, "memset");
  if (!rc) rc = run_density(ctx, m, NPG_FP32, energy_dev, L, H, W, dens, s, amax_dev);
  if (!rc && (hipMemcpyAsync(amax.data(), amax_dev, sizeof(unsigned) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess))
    rc = npg_fail(ctx, NPG_E_HIP, "calibrate_fp8: readback failed");
  npg_device_free(ctx, tmp, tmp_bytes);
  if (rc) return rc;
  // 2. activation scales: the largest stored value maps to the largest e4m3
  std::vector<float> a8(n, 1.0f);
  for (int i = 0; i < n; ++i) {
    float v;
    memcpy(&v, &amax[i], 4);
    if (v > 0.0f && std::isfinite(v)) a8[i] = v / E4M3_MAX;
  }
  // 3. weights of every 3x3 layer fed by stored activations: fold the input
  // channels' scales in, one scale per output channel, pack as the BF16 tiles
  std::vector<char> blob;
  struct Off { size_t p8, p8s, sc; };
  std::vector<Off> offs(n, Off{(size_t)-1, (size_t)-1, (size_t)-1});
  auto put = [&](const void *src, size_t bytes) {
    size_t at = npg_align(blob.size());
    blob.resize(at + npg_align(bytes));
    memcpy(blob.data() + at, src, bytes);
    return at;
  };
  for (int i = 1; i < n; ++i) {
    const LayerDev &y = m->layer[i];
    if (y.k != 3) continue;
    const std::vector<int> prod = channel_producers(m, i);
    const std::vector<float> &w = m->host_w[i];
    std::vector<float> wf(w.size()), sc(y.cout, 1.0f);
    for (int co = 0; co < y.cout; ++co) {
      float mx = 0.0f;
      for (int ci = 0; ci < y.cin; ++ci)
        for (int t = 0; t < 9; ++t) {
          const size_t k = ((size_t)co * y.cin + ci) * 9 + t;
          wf[k] = w[k] * (prod[ci] >= 0 ? a8[prod[ci]] : 1.0f);
          mx = std::max(mx, std::fabs(wf[k]));
        }
      if (mx > 0.0f) sc[co] = mx / E4M3_MAX;
    }
    const int nch = (y.cin + KC8 - 1) / KC8, nchs = (y.cin + KC8S - 1) / KC8S;
    std::vector<uint8_t> p8((size_t)nch * 9 * y.cout * KC8, 0), p8s((size_t)nchs * 9 * y.cout * KC8S, 0);
    for (int co = 0; co < y.cout; ++co)
      for (int ci = 0; ci < y.cin; ++ci)
        for (int t = 0; t < 9; ++t) {
          const uint8_t q = e4m3_enc(wf[((size_t)co * y.cin + ci) * 9 + t] / sc[co]);
          p8[(((size_t)(ci / KC8) * 9 + t) * y.cout + co) * KC8 + ci % KC8] = q;
          p8s[(((size_t)(ci / KC8S) * 9 + t) * y.cout + co) * KC8S + ci % KC8S] = q;
        }
    offs[i].p8 = put(p8.data(), p8.size());
    offs[i].p8s = put(p8s.data(), p8s.size());
    offs[i].sc = put(sc.data(), 4 * sc.size());
  }
  void *dev = nullptr;
  if (!blob.empty()) {
    rc = npg_device_alloc(ctx, blob.size(), &dev);
    if (rc) return rc;
    if (hipMemcpy(dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
      npg_device_free(ctx, dev, blob.size());
      return npg_fail(ctx, NPG_E_HIP, "calibrate_fp8: upload failed");
    }
  }
  if (m->blob8) npg_device_free(ctx, m->blob8, m->blob8_bytes);
  m->blob8 = dev;
  m->blob8_bytes = blob.size();
  char *base = static_cast<char *>(dev);
  for (int i = 0; i < n; ++i) {
    LayerDev &y = m->layer[i];
    y.a8 = a8[i];
    y.pk8 = offs[i].p8 == (size_t)-1 ? nullptr : reinterpret_cast<uint8_t *>(base + offs[i].p8);
    y.pk8s = offs[i].p8s == (size_t)-1 ? nullptr : reinterpret_cast<uint8_t *>(base + offs[i].p8s);
    y.wsc8 = offs[i].sc == (size_t)-1 ? nullptr : reinterpret_cast<float *>(base + offs[i].sc);
  }
  m->fp8_ready = true;
  return NPG_OK;
}
