// Learned warm start: BF16 matrix-core (MFMA) convolution kernels with FP32
// accumulation, training (backward, Adam) and inference, behind the C ABI of
// include/adrnn.h.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x16_bf16: M = pixels,
// N = 32 output channels (two 16x16 tiles), K = (tap, input channel).  The
// 32 -> 32 layers run tiled (k_conv32t: a 16 x 16-pixel tile and its dilated
// halo staged in LDS), the 4 -> 32 first layer directly from global memory
// (k_conv_in), the 32 -> 1 last layer on the vector ALUs.  Operand layout of the instruction: lane l supplies
// A[l%16][4(l/16) .. 4(l/16)+3] and B[4(l/16) .. +3][l%16]; it receives
// D[4(l/16) + v][l%16], v = 0..3.  NHWC activations make a lane's four K
// values (four consecutive channels of one pixel) one 8-byte load.
// Layer l's taps are dilated by kDil[l]: tap (dy, dx) reads the pixel
// (y + d dy, x + d dx), zero outside the image.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/adrnn.h"

namespace {

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));
typedef unsigned short bf16_t;

constexpr int kCh = 32;
constexpr int kThreads = 256;
constexpr int kW1 = 32 * 9 * 4, kW2 = 32 * 9 * 32, kW4 = 9 * 32;
// offsets in the parameter vector
constexpr int oW1 = 0, ob1 = oW1 + kW1, oW2 = ob1 + 32, ob2 = oW2 + kW2, oW3 = ob2 + 32, ob3 = oW3 + kW2,
              oW4 = ob3 + 32, ob4 = oW4 + kW4, kParams = ob4 + 1;
constexpr int kChunk = 256;  // pixels per weight-gradient chunk
constexpr int kDil[4] = {1, 2, 4, 8};

__device__ __forceinline__ bf16_t f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                      // round to nearest even
    return static_cast<bf16_t>(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(static_cast<unsigned>(h) << 16); }
__device__ __forceinline__ bool bf_pos(bf16_t h) { return h != 0 && (h & 0x8000) == 0 && h <= 0x7f80; }

__device__ __forceinline__ v4f32 mfma(v4i16 a, v4i16 b, v4f32 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ conv, 4 -> 32 (first layer)
// y = bf16(relu(conv(x0) + bias)); x0: [NP][4] BF16, Wg: [32][9][4].  A wavefront
// computes 16 pixels x 32 channels; K = 12 taps (9, padded) x 4 channels, one
// tap per lane group, so a lane's 4 K values are one pixel's 4 channels.
__global__ __launch_bounds__(kThreads) void k_conv_in(const bf16_t *__restrict__ x, const bf16_t *__restrict__ Wg,
                                                      const float *__restrict__ bias, bf16_t *__restrict__ y,
                                                      int NP, int H, int W, int d) {
    constexpr int CIN = 4, KT = 12;
    __shared__ __align__(16) bf16_t Ws[kCh * KT * CIN];
    for (int e = threadIdx.x; e < kCh * KT * CIN; e += kThreads) {
        const int n = e / (KT * CIN), r = e % (KT * CIN), tap = r / CIN, c = r % CIN;
        Ws[e] = tap < 9 ? Wg[(n * 9 + tap) * CIN + c] : bf16_t(0);
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    const int HW = H * W;
    const int ntiles = (NP + 15) / 16;
    const v4i16 zero = {0, 0, 0, 0};
    const float bias0 = bias[i], bias1 = bias[i + 16];
    for (int t = blockIdx.x * 4 + wave; t < ntiles; t += gridDim.x * 4) {
        const int gp = t * 16 + i;  // pixel of this lane's A row
        const bool pv = gp < NP;
        const int b = gp / HW, p = gp - b * HW, py = p / W, px = p - py * W;
        v4f32 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
        // every A fragment is loaded before the first product: a tap outside
        // the image reads a valid pixel (the tile's own, or pixel 0 past the
        // end) and is replaced by zeros, so no load sits behind a branch
        const ptrdiff_t self = pv ? gp : 0;
        v4i16 av[3];
#pragma unroll
        for (int kc = 0; kc < 3; ++kc) {
            const int tap = kc * 4 + g;  // this lane group's tap
            const int dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
            const bool ok = tap < 9 && pv && py + dy >= 0 && py + dy < H && px + dx >= 0 && px + dx < W;
            const v4i16 v = *reinterpret_cast<const v4i16 *>(
                x + (ok ? static_cast<ptrdiff_t>(gp + dy * W + dx) : self) * CIN);
            av[kc] = ok ? v : zero;
        }
#pragma unroll
        for (int kc = 0; kc < 3; ++kc) {
            const int tap = kc * 4 + g;
            const v4i16 b0 = *reinterpret_cast<const v4i16 *>(&Ws[(i * KT + tap) * CIN]);
            const v4i16 b1 = *reinterpret_cast<const v4i16 *>(&Ws[((i + 16) * KT + tap) * CIN]);
            acc0 = mfma(av[kc], b0, acc0);
            acc1 = mfma(av[kc], b1, acc1);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int po = t * 16 + 4 * g + v;
            if (po >= NP) continue;
            y[static_cast<size_t>(po) * kCh + i] = f2bf(fmaxf(acc0[v] + bias0, 0.f));
            y[static_cast<size_t>(po) * kCh + i + 16] = f2bf(fmaxf(acc1[v] + bias1, 0.f));
        }
    }
}

// ------------------------------------------------------------------ conv, 32 -> 32, tiled
// A workgroup computes a 16 x 16-pixel output tile of one image for all 32
// output channels.  The input patch ((16 + 2d)^2 pixels x 32 channels, zeros
// outside the image) and the weights are staged in LDS once; pixel rows are
// padded to kCP channels and weight rows to kWS entries so that the fragment
// reads of a wavefront spread over the LDS banks.  Wavefront w computes tile
// rows 4w .. 4w+3 (4 M-tiles of 16 pixels) x 32 channels (2 N-tiles).
// EPI 0: y = bf16(relu(acc + bias)).  EPI 1: y = bf16(acc * (ymask > 0)) (back-
// propagation through the ReLU of the layer input, with flipped taps).
constexpr int kTile = 16;
constexpr int kCP = 36;            // staged channels per pixel (32 + pad)
constexpr int kWS = 9 * kCh + 4;   // staged weight row (one output channel: 9 taps x 32 inputs + pad)
constexpr int kMaxDilT = 4;        // largest dilation the tiled kernel stages (patch (16 + 2*4)^2)
constexpr int kWStage = (kCh * 36 + kThreads - 1) / kThreads;
constexpr int kXStage = ((kTile + 2 * kMaxDilT) * (kTile + 2 * kMaxDilT) * 4 + kThreads - 1) / kThreads;

__host__ __device__ inline int conv_tiles(int H, int W) { return ((H + kTile - 1) / kTile) * ((W + kTile - 1) / kTile); }
__host__ __device__ inline size_t conv_tiled_lds(int d) {
    const int P = kTile + 2 * d;
    return sizeof(bf16_t) * (static_cast<size_t>(kCh) * kWS + static_cast<size_t>(P) * P * kCP);
}

template <int EPI>
__global__ __launch_bounds__(kThreads) void k_conv32t(const bf16_t *__restrict__ x, const bf16_t *__restrict__ Wg,
                                                      const float *__restrict__ bias,
                                                      const bf16_t *__restrict__ ymask, bf16_t *__restrict__ y,
                                                      int H, int W, int d) {
    extern __shared__ __align__(16) unsigned char sm[];
    bf16_t *Ws = reinterpret_cast<bf16_t *>(sm);  // [32][kWS]
    bf16_t *Xs = Ws + kCh * kWS;                  // [P*P][kCP]
    const int P = kTile + 2 * d;
    const int tw = (W + kTile - 1) / kTile, tpi = conv_tiles(H, W);
    const int b = blockIdx.x / tpi, t = blockIdx.x - b * tpi;
    const int ty = t / tw, tx = t - ty * tw;
    const int y0 = ty * kTile, x0 = tx * kTile;
    // staging, 16 bytes (8 channels) per load, every load issued before the
    // first LDS store: the weights (32 rows of 288 entries), then the input
    // patch (a pixel outside the image reads the tile's first in-image pixel
    // and stores zeros)
    const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
    uint4 wv[kWStage];
#pragma unroll
    for (int u = 0; u < kWStage; ++u) {
        const int e = threadIdx.x + u * kThreads;
        wv[u] = reinterpret_cast<const uint4 *>(Wg)[e < kCh * 36 ? e : 0];
    }
    const bf16_t *xb = x + static_cast<size_t>(b) * H * W * kCh;
    const uint4 *x00 = reinterpret_cast<const uint4 *>(xb + (static_cast<size_t>(y0) * W + x0) * kCh);
    uint4 xv[kXStage];
    bool in[kXStage];
#pragma unroll
    for (int u = 0; u < kXStage; ++u) {
        const int e = threadIdx.x + u * kThreads;
        const int pix = e >> 2, q = e & 3;
        const int py = pix / P, px = pix - py * P;
        const int gy = y0 - d + py, gx = x0 - d + px;
        in[u] = e < P * P * 4 && gy >= 0 && gy < H && gx >= 0 && gx < W;
        const uint4 *src = in[u] ? reinterpret_cast<const uint4 *>(xb + (static_cast<size_t>(gy) * W + gx) * kCh) + q
                                 : x00;
        xv[u] = *src;
    }
#pragma unroll
    for (int u = 0; u < kWStage; ++u) {
        const int e = threadIdx.x + u * kThreads;
        if (e < kCh * 36) {
            const int n = e / 36, q = e - n * 36;
            uint2 *dst = reinterpret_cast<uint2 *>(Ws + n * kWS + q * 8);
            dst[0] = make_uint2(wv[u].x, wv[u].y);
            dst[1] = make_uint2(wv[u].z, wv[u].w);
        }
    }
#pragma unroll
    for (int u = 0; u < kXStage; ++u) {
        const int e = threadIdx.x + u * kThreads;
        if (e < P * P * 4) {
            const uint4 v = in[u] ? xv[u] : z4;
            uint2 *dst = reinterpret_cast<uint2 *>(Xs + (e >> 2) * kCP + (e & 3) * 8);
            dst[0] = make_uint2(v.x, v.y);
            dst[1] = make_uint2(v.z, v.w);
        }
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    v4f32 acc[4][2];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) acc[mt][0] = acc[mt][1] = v4f32{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int oy = d + d * (tap / 3 - 1), ox = d + d * (tap % 3 - 1);
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
            const v4i16 b0 = *reinterpret_cast<const v4i16 *>(&Ws[i * kWS + tap * kCh + cc * 16 + g * 4]);
            const v4i16 b1 = *reinterpret_cast<const v4i16 *>(&Ws[(i + 16) * kWS + tap * kCh + cc * 16 + g * 4]);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int r = wave * 4 + mt;
                const v4i16 a =
                    *reinterpret_cast<const v4i16 *>(&Xs[((r + oy) * P + i + ox) * kCP + cc * 16 + g * 4]);
                acc[mt][0] = mfma(a, b0, acc[mt][0]);
                acc[mt][1] = mfma(a, b1, acc[mt][1]);
            }
        }
    }
    const float bias0 = EPI == 0 ? bias[i] : 0.f, bias1 = EPI == 0 ? bias[i + 16] : 0.f;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const int gy = y0 + wave * 4 + mt;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int gx = x0 + 4 * g + v;
            if (gy >= H || gx >= W) continue;
            const size_t po = (static_cast<size_t>(b) * H + gy) * W + gx;
            float z0 = acc[mt][0][v], z1 = acc[mt][1][v];
            if constexpr (EPI == 0) {
                z0 = fmaxf(z0 + bias0, 0.f);
                z1 = fmaxf(z1 + bias1, 0.f);
            } else {
                z0 = bf_pos(ymask[po * kCh + i]) ? z0 : 0.f;
                z1 = bf_pos(ymask[po * kCh + i + 16]) ? z1 : 0.f;
            }
            y[po * kCh + i] = f2bf(z0);
            y[po * kCh + i + 16] = f2bf(z1);
        }
    }
}

// ------------------------------------------------------------------ weight gradient (MFMA)
// part[blk][ (n*9 + tap)*CIN + c ] = sum over the block's pixels of g[p][n] x[p + d off(tap)][c]
// and part[blk][32*9*CIN + n] = sum g[p][n].  g: [NP][32], x: [NP][CIN] BF16.
// A chunk of kChunk consecutive pixels reads x in three bands (tap rows
// dy = -1, 0, 1), each kChunk + 2d pixels long, staged channel-major in LDS.
template <int CIN>
__global__ __launch_bounds__(kThreads) void k_wgrad32(const bf16_t *__restrict__ gsrc, const bf16_t *__restrict__ x,
                                                      float *__restrict__ part, int NP, int H, int W, int d) {
    constexpr int NCOL = 9 * CIN;                 // (tap, c) columns
    constexpr int NJT = (NCOL + 15) / 16;         // column tiles
    constexpr int NT = 2 * NJT;                   // output tiles (2 row tiles of 16 channels)
    constexpr int TPW = (NT + 3) / 4;             // tiles per wave
    const int bspan = (kChunk + 2 * d + 3) & ~3;  // one band (a multiple of 4: aligned fragments)
    const int span = 3 * bspan;
    extern __shared__ __align__(16) unsigned char sm[];
    constexpr int GS = kChunk + 4;                              // gT row stride (8-byte aligned, 2-way banks)
    bf16_t *gT = reinterpret_cast<bf16_t *>(sm);                // [32][GS]
    bf16_t *xT = gT + kCh * GS;                                 // [CIN][3][bspan]
    unsigned short *vm = reinterpret_cast<unsigned short *>(xT + CIN * span);  // [kChunk] valid taps (bit tap)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    const int HW = H * W;
    v4f32 acc[TPW];
#pragma unroll
    for (int q = 0; q < TPW; ++q) acc[q] = v4f32{0.f, 0.f, 0.f, 0.f};
    float dbias = 0.f;
    const int nchunks = (NP + kChunk - 1) / kChunk;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int c0 = ch * kChunk;
        __syncthreads();
        for (int e = threadIdx.x; e < kCh * kChunk; e += kThreads) {
            const int pl = e / kCh, n = e % kCh;  // coalesced read of g
            const int gp = c0 + pl;
            const bf16_t gv = gp < NP ? gsrc[static_cast<size_t>(gp) * kCh + n] : bf16_t(0);
            gT[n * GS + pl] = gv;
            dbias += bf2f(gv);  // this thread always stages channel n = threadIdx.x % 32
        }
        for (int e = threadIdx.x; e < span * CIN; e += kThreads) {
            const int sl = e / CIN, c = e % CIN;  // coalesced read of x
            const int band = sl / bspan, bl = sl - band * bspan;
            const int gp = c0 + (band - 1) * d * W - d + bl;
            xT[c * span + sl] = (gp >= 0 && gp < NP) ? x[static_cast<size_t>(gp) * CIN + c] : bf16_t(0);
        }
        for (int pl = threadIdx.x; pl < kChunk; pl += kThreads) {
            const int gp = c0 + pl;
            unsigned mask = 0;
            if (gp < NP) {
                const int p = gp % HW, yy = p / W, xx = p % W;
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) {
                    const int dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
                    if (yy + dy >= 0 && yy + dy < H && xx + dx >= 0 && xx + dx < W) mask |= 1u << tap;
                }
            }
            vm[pl] = static_cast<unsigned short>(mask);
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < TPW; ++q) {
            const int tile = wave * TPW + q;
            if (tile >= NT) continue;
            const int rt = tile / NJT, jt = tile % NJT;
            const int n = rt * 16 + i;                 // A row (output channel)
            const int col = jt * 16 + i;               // B column (tap, c)
            const bool colok = col < NCOL;
            const int tap = colok ? col / CIN : 0, c = colok ? col % CIN : 0;
            const int dx = d * (tap % 3 - 1);
            const int off = (tap / 3) * bspan + d + dx;  // band of the tap row, then the shift in the band
            const unsigned tbit = colok ? 1u << tap : 0u;
            const int base = c * span + off;
            for (int k0 = 0; k0 < kChunk; k0 += 16) {
                const v4i16 a = *reinterpret_cast<const v4i16 *>(&gT[n * GS + k0 + 4 * g]);
                const int pl0 = k0 + 4 * g;
                // the valid-tap masks of the 4 pixels, one 8-byte read
                const uint2 mw = *reinterpret_cast<const uint2 *>(&vm[pl0]);
                const unsigned m4[4] = {mw.x & 0xffffu, mw.x >> 16, mw.y & 0xffffu, mw.y >> 16};
                // 4 consecutive pixels of channel c shifted by the tap: with 32 input
                // channels all lanes of a column tile share the tap, so the alignment
                // (and the read width) is uniform across the wavefront
                v4i16 raw;
                if (CIN == 32 && (off & 3) == 0) {
                    raw = *reinterpret_cast<const v4i16 *>(&xT[base + pl0]);
                } else if (CIN == 32 && (off & 1) == 0) {
                    const unsigned lo = *reinterpret_cast<const unsigned *>(&xT[base + pl0]);
                    const unsigned hi = *reinterpret_cast<const unsigned *>(&xT[base + pl0 + 2]);
                    raw[0] = static_cast<short>(lo & 0xffffu);
                    raw[1] = static_cast<short>(lo >> 16);
                    raw[2] = static_cast<short>(hi & 0xffffu);
                    raw[3] = static_cast<short>(hi >> 16);
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) raw[v] = static_cast<short>(xT[base + pl0 + v]);
                }
                v4i16 bv;
#pragma unroll
                for (int v = 0; v < 4; ++v) bv[v] = (m4[v] & tbit) ? raw[v] : short(0);
                acc[q] = mfma(a, bv, acc[q]);
            }
        }
    }
    float *out = part + static_cast<size_t>(blockIdx.x) * (kCh * NCOL + kCh);
#pragma unroll
    for (int q = 0; q < TPW; ++q) {
        const int tile = wave * TPW + q;
        if (tile >= NT) continue;
        const int rt = tile / NJT, jt = tile % NJT;
        const int col = jt * 16 + i;
        if (col >= NCOL) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int n = rt * 16 + 4 * g + v;
            out[n * NCOL + col] = acc[q][v];
        }
    }
    // bias gradient: the 8 threads of each channel, in thread order
    __syncthreads();
    float *bred = reinterpret_cast<float *>(sm);
    bred[threadIdx.x] = dbias;
    __syncthreads();
    if (threadIdx.x < kCh) {
        float sb = 0.f;
        for (int r = 0; r < kThreads / kCh; ++r) sb += bred[threadIdx.x + r * kCh];
        out[kCh * NCOL + threadIdx.x] = sb;
    }
}

// sum of per-block partials (deterministic): a 256-thread block covers 32
// elements; thread group r (8 groups) sums the partials of blocks r, r+8, ...
// with four loads in flight, then the 8 group sums are added in group order
__global__ __launch_bounds__(kThreads) void k_reduce(const float *__restrict__ part, int nblk, int len,
                                                     float *__restrict__ out) {
    const int el = blockIdx.x * 32 + (threadIdx.x & 31), r = threadIdx.x >> 5;
    float a4[4] = {0.f, 0.f, 0.f, 0.f};
    if (el < len) {
        int b = r;
        for (; b + 24 < nblk; b += 32) {
            float p4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) p4[u] = part[static_cast<size_t>(b + 8 * u) * len + el];
#pragma unroll
            for (int u = 0; u < 4; ++u) a4[u] += p4[u];
        }
        for (; b < nblk; b += 8) a4[0] += part[static_cast<size_t>(b) * len + el];
    }
    __shared__ float red[8][32];
    red[r][threadIdx.x & 31] = (a4[0] + a4[1]) + (a4[2] + a4[3]);
    __syncthreads();
    if (r == 0 && el < len) {
        float sum = 0.f;
        for (int q = 0; q < 8; ++q) sum += red[q][threadIdx.x];
        out[el] = sum;
    }
}

// ------------------------------------------------------------------ last layer (32 -> 1), VALU
__global__ __launch_bounds__(kThreads) void k_last_fwd(const bf16_t *__restrict__ y3, const float *__restrict__ W4,
                                                       const float *__restrict__ b4, float *__restrict__ out, int NP,
                                                       int H, int W, int d) {
    __shared__ float w4s[kW4];
    for (int e = threadIdx.x; e < kW4; e += blockDim.x) w4s[e] = W4[e];
    __syncthreads();
    const int gp = blockIdx.x * blockDim.x + threadIdx.x;
    if (gp >= NP) return;
    const int HW = H * W, p = gp % HW, py = p / W, px = p % W;
    float s = b4[0];
    // taps in groups of 3: each tap's 32 channels are four 16-byte loads, all
    // issued before use; a tap outside the image reads the pixel itself and is
    // dropped
#pragma unroll
    for (int t0 = 0; t0 < 9; t0 += 3) {
        uint4 v[3][4];
        bool ok[3];
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            const int tap = t0 + u, dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
            ok[u] = py + dy >= 0 && py + dy < H && px + dx >= 0 && px + dx < W;
            const uint4 *src = reinterpret_cast<const uint4 *>(y3 + static_cast<size_t>(ok[u] ? gp + dy * W + dx : gp) * kCh);
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4) v[u][c4] = src[c4];
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) {
            if (!ok[u]) continue;
            const float *w = w4s + (t0 + u) * kCh;
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4) {
                const unsigned q[4] = {v[u][c4].x, v[u][c4].y, v[u][c4].z, v[u][c4].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int c = c4 * 8 + 2 * e;
                    s += w[c] * __uint_as_float(q[e] << 16) + w[c + 1] * __uint_as_float(q[e] & 0xffff0000u);
                }
            }
        }
    }
    out[gp] = s;
}

// g4 = 2 (out - target) mask / cnt; partial sums of mask (out - target)^2 per block
__global__ void k_loss(const float *__restrict__ out, const float *__restrict__ tgt, const uint8_t *__restrict__ mask,
                       float *__restrict__ g4, double *__restrict__ lpart, int NP, int HW, double inv_cnt) {
    const int gp = blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (gp < NP) {
        const bool m = mask[gp % HW] != 0;
        const float d = m ? out[gp] - tgt[gp] : 0.f;
        g4[gp] = static_cast<float>(2.0 * d * inv_cnt);
        e2 = static_cast<double>(d) * d;
    }
    __shared__ double red[kThreads];
    red[threadIdx.x] = e2;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// g3 = bf16( (sum_tap W4[tap][c] g4[p - d off(tap)]) * (y3 > 0) )
__global__ __launch_bounds__(kThreads) void k_last_dgrad(const float *__restrict__ g4, const float *__restrict__ W4,
                                                         const bf16_t *__restrict__ y3, bf16_t *__restrict__ g3,
                                                         int NP, int H, int W, int d) {
    __shared__ float w4s[kW4];
    for (int e = threadIdx.x; e < kW4; e += blockDim.x) w4s[e] = W4[e];
    __syncthreads();
    const int gp = blockIdx.x * blockDim.x + threadIdx.x;
    if (gp >= NP) return;
    const int HW = H * W, p = gp % HW, py = p / W, px = p % W;
    float gn[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
        // pixel gp feeds output gp - d off through tap
        const bool ok = py - dy >= 0 && py - dy < H && px - dx >= 0 && px - dx < W;
        const float gvl = g4[ok ? gp - dy * W - dx : gp];
        gn[tap] = ok ? gvl : 0.f;
    }
    // the pixel's 32 stored activations (ReLU mask) and gradients as four 16-byte words
    const uint4 *ysrc = reinterpret_cast<const uint4 *>(y3 + static_cast<size_t>(gp) * kCh);
    uint4 *gdst = reinterpret_cast<uint4 *>(g3 + static_cast<size_t>(gp) * kCh);
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
        const uint4 yv = ysrc[c4];
        const unsigned yq[4] = {yv.x, yv.y, yv.z, yv.w};
        unsigned oq[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            unsigned packed = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int c = c4 * 8 + 2 * e + h;
                float s_ = 0.f;
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) s_ += w4s[tap * kCh + c] * gn[tap];
                const bf16_t yb = static_cast<bf16_t>(h == 0 ? (yq[e] & 0xffffu) : (yq[e] >> 16));
                packed |= static_cast<unsigned>(f2bf(bf_pos(yb) ? s_ : 0.f)) << (16 * h);
            }
            oq[e] = packed;
        }
        gdst[c4] = make_uint4(oq[0], oq[1], oq[2], oq[3]);
    }
}

// part[blk][tap*32 + c] = sum over the block's pixels of g4[p] y3[p + d off][c]; part[blk][288] = sum g4.
// Thread t: channel pair cp = t % 16 (channels 2cp, 2cp+1) of the pixels p = t / 16 (mod 16) of
// every chunk: 18 accumulators (9 taps x 2 channels); the 16 pixel groups are summed in LDS
// at the end (fixed order).  A pixel row of y3 is read by 16 consecutive threads (64 bytes).
__global__ __launch_bounds__(kThreads) void k_last_wgrad(const float *__restrict__ g4, const bf16_t *__restrict__ y3,
                                                         float *__restrict__ part, int NP, int H, int W, int d) {
    const int cp = threadIdx.x & 15, pg = threadIdx.x >> 4;
    const int HW = H * W;
    float acc[9][2];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) acc[tap][0] = acc[tap][1] = 0.f;
    float gsum = 0.f;
    const int nchunks = (NP + kChunk - 1) / kChunk;
    for (int ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const int c0 = ch * kChunk;
        for (int pl = pg; pl < kChunk; pl += 16) {
            const int gp = c0 + pl;
            if (gp >= NP) break;
            const float gv = g4[gp];
            if (cp == 0) gsum += gv;
            const int p = gp % HW, py = p / W, px = p % W;
            unsigned v[9];
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
                const bool ok = py + dy >= 0 && py + dy < H && px + dx >= 0 && px + dx < W;
                const unsigned w = *reinterpret_cast<const unsigned *>(
                    y3 + static_cast<size_t>(ok ? gp + dy * W + dx : gp) * kCh + 2 * cp);
                v[tap] = ok ? w : 0u;
            }
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                acc[tap][0] += gv * __uint_as_float(v[tap] << 16);
                acc[tap][1] += gv * __uint_as_float(v[tap] & 0xffff0000u);
            }
        }
    }
    __shared__ float red[16][kW4 + 1];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        red[pg][tap * kCh + 2 * cp] = acc[tap][0];
        red[pg][tap * kCh + 2 * cp + 1] = acc[tap][1];
    }
    if (cp == 0) red[pg][kW4] = gsum;
    __syncthreads();
    for (int el = threadIdx.x; el <= kW4; el += kThreads) {
        float sum = 0.f;
        for (int q = 0; q < 16; ++q) sum += red[q][el];
        part[static_cast<size_t>(blockIdx.x) * (kW4 + 1) + el] = sum;
    }
}

// ------------------------------------------------------------------ parameters
// BF16 copies: forward layouts (= parameter layout) for W1..W3, FP32 of the BF16
// value for W4, and the flipped/transposed dgrad weights Wt[c][8-tap][n] of W2, W3.
__global__ void k_convert(const float *__restrict__ P, bf16_t *__restrict__ w1, bf16_t *__restrict__ w2,
                          bf16_t *__restrict__ w3, bf16_t *__restrict__ w2t, bf16_t *__restrict__ w3t,
                          float *__restrict__ w4) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kW1) w1[e] = f2bf(P[oW1 + e]);
    if (e < kW2) {
        const bf16_t a = f2bf(P[oW2 + e]), b = f2bf(P[oW3 + e]);
        w2[e] = a;
        w3[e] = b;
        const int n = e / (9 * kCh), r = e % (9 * kCh), tap = r / kCh, c = r % kCh;
        const int t = (c * 9 + (8 - tap)) * kCh + n;
        w2t[t] = a;
        w3t[t] = b;
    }
    if (e < kW4) w4[e] = bf2f(f2bf(P[oW4 + e]));
}

__global__ void k_adam(float *__restrict__ P, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float c1, float c2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gv = g[e];
    const float mv = 0.9f * m[e] + 0.1f * gv;
    const float vv = 0.999f * v[e] + 0.001f * gv * gv;
    m[e] = mv;
    v[e] = vv;
    P[e] -= lr * (mv / c1) / (sqrtf(vv / c2) + 1e-8f);
}

// ------------------------------------------------------------------ inputs and warm start
__global__ __launch_bounds__(kThreads) void k_norms(const double *__restrict__ f, const double *__restrict__ s,
                                                    const uint8_t *__restrict__ mask, double *__restrict__ fn,
                                                    double *__restrict__ sn, int HW) {
    const int b = blockIdx.x;
    double mf = 0.0, ms = 0.0;
    for (int p = threadIdx.x; p < HW; p += kThreads) {
        if (!mask[p]) continue;
        mf = fmax(mf, fabs(f[static_cast<size_t>(b) * HW + p]));
        ms = fmax(ms, fabs(s[static_cast<size_t>(b) * HW + p]));
    }
    __shared__ double rf[kThreads], rs[kThreads];
    rf[threadIdx.x] = mf;
    rs[threadIdx.x] = ms;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) {
            rf[threadIdx.x] = fmax(rf[threadIdx.x], rf[threadIdx.x + w]);
            rs[threadIdx.x] = fmax(rs[threadIdx.x], rs[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        fn[b] = rf[0] > 0.0 ? rf[0] : 1.0;
        sn[b] = rs[0] > 0.0 ? rs[0] : 1.0;
    }
}

__global__ void k_pack(const double *__restrict__ f, const double *__restrict__ s, const uint8_t *__restrict__ mask,
                       const double *__restrict__ lmu, const double *__restrict__ fn, const double *__restrict__ sn,
                       const double *__restrict__ ustar, bf16_t *__restrict__ x0, float *__restrict__ tgt, int NP,
                       int HW) {
    const int gp = blockIdx.x * blockDim.x + threadIdx.x;
    if (gp >= NP) return;
    const int b = gp / HW, p = gp - b * HW;
    const bool m = mask[p] != 0;
    const double sv = s[gp];
    bf16_t *o = x0 + static_cast<size_t>(gp) * 4;
    o[0] = f2bf(static_cast<float>(m ? f[gp] / fn[b] : 0.0));
    o[1] = f2bf(static_cast<float>(lmu[b] + 2.0));
    o[2] = f2bf(static_cast<float>(m ? sv / sn[b] : 0.0));
    o[3] = f2bf(m ? 1.f : 0.f);
    if (ustar) tgt[gp] = static_cast<float>(m ? (ustar[gp] - sv) / sn[b] : 0.0);
}

__global__ void k_warm(const double *__restrict__ s, const double *__restrict__ sn, const float *__restrict__ out,
                       const uint8_t *__restrict__ mask, double *__restrict__ u, int NP, int HW) {
    const int gp = blockIdx.x * blockDim.x + threadIdx.x;
    if (gp >= NP) return;
    const int b = gp / HW;
    u[gp] = mask[gp - b * HW] ? s[gp] + sn[b] * static_cast<double>(out[gp]) : 0.0;
}

__global__ void k_probe(const bf16_t *__restrict__ A, const bf16_t *__restrict__ B, float *__restrict__ D) {
    const int l = threadIdx.x, i = l & 15, g = l >> 4;
    v4i16 a, b;
    for (int v = 0; v < 4; ++v) {
        a[v] = static_cast<short>(A[i * 16 + 4 * g + v]);   // A[i][k]
        b[v] = static_cast<short>(B[(4 * g + v) * 16 + i]); // B[k][j]
    }
    v4f32 d = mfma(a, b, v4f32{0.f, 0.f, 0.f, 0.f});
    for (int v = 0; v < 4; ++v) D[(4 * g + v) * 16 + i] = d[v];
}

}  // namespace

// ================================================================== context
struct adrnn_ctx {
    int H = 0, W = 0, maxB = 0;
    hipStream_t st = nullptr;
    std::vector<void *> owned;
    float *P = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    bf16_t *w1 = nullptr, *w2 = nullptr, *w3 = nullptr, *w2t = nullptr, *w3t = nullptr;
    float *w4 = nullptr;
    bf16_t *y1 = nullptr, *y2 = nullptr, *y3 = nullptr, *ga = nullptr, *gb = nullptr;
    float *out = nullptr, *g4 = nullptr, *part = nullptr, *lmu = nullptr;
    double *lpart = nullptr, *fn = nullptr, *dlmu = nullptr;
    int wblocks = 512;
    int64_t step = 0;
    std::string err;
};

namespace {

struct NNError {
    adr_status code;
    std::string msg;
};

#define NNCHK(x)                                                                                           \
    do {                                                                                                   \
        hipError_t e_ = (x);                                                                               \
        if (e_ != hipSuccess) throw NNError{ADR_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

template <typename T>
T *nn_alloc(adrnn_ctx *c, size_t n) {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) throw NNError{ADR_ENOMEM, "hipMalloc"};
    c->owned.push_back(p);
    return static_cast<T *>(p);
}

size_t wgrad_lds(int cin, int d) {
    const int span = 3 * ((kChunk + 2 * d + 3) & ~3);
    return sizeof(bf16_t) * (kCh * (kChunk + 4) + static_cast<size_t>(cin) * span) + sizeof(short) * 2 * kChunk;
}

void convert(adrnn_ctx *c) {
    hipLaunchKernelGGL(k_convert, dim3((kW2 + 255) / 256), dim3(256), 0, c->st, c->P, c->w1, c->w2, c->w3, c->w2t,
                       c->w3t, c->w4);
    NNCHK(hipGetLastError());
}

int conv_grid(int NP) { return std::min(4096, std::max(1, (NP + 16 * 4 * 8 - 1) / (16 * 4 * 8))); }

// 32 -> 32 convolution of B images (tiled kernel)
template <int EPI>
void conv32t(adrnn_ctx *c, int B, const bf16_t *x, const bf16_t *w, const float *bias, const bf16_t *ymask, bf16_t *y,
             int d) {
    if (d < 1 || d > kMaxDilT) throw NNError{ADR_EINVAL, "tiled convolution: dilation out of range"};
    const size_t lds = conv_tiled_lds(d);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_conv32t<EPI>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    hipLaunchKernelGGL((k_conv32t<EPI>), dim3(B * conv_tiles(c->H, c->W)), dim3(kThreads), lds, c->st, x, w, bias,
                       ymask, y, c->H, c->W, d);
    NNCHK(hipGetLastError());
}

void forward(adrnn_ctx *c, int B, const bf16_t *x0, float *out) {
    const int NP = B * c->H * c->W, gridc = conv_grid(NP);
    hipLaunchKernelGGL(k_conv_in, dim3(gridc), dim3(kThreads), 0, c->st, x0, c->w1, c->P + ob1, c->y1, NP, c->H,
                       c->W, kDil[0]);
    conv32t<0>(c, B, c->y1, c->w2, c->P + ob2, nullptr, c->y2, kDil[1]);
    conv32t<0>(c, B, c->y2, c->w3, c->P + ob3, nullptr, c->y3, kDil[2]);
    NNCHK(hipGetLastError());
    hipLaunchKernelGGL(k_last_fwd, dim3((NP + 255) / 256), dim3(256), 0, c->st, c->y3, c->w4, c->P + ob4, out, NP,
                       c->H, c->W, kDil[3]);
    NNCHK(hipGetLastError());
}

template <int CIN>
void wgrad(adrnn_ctx *c, const bf16_t *g, const bf16_t *x, int NP, int d, float *dst) {
    const size_t lds = wgrad_lds(CIN, d);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wgrad32<CIN>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    const int nchunks = (NP + kChunk - 1) / kChunk;
    const int nb = std::min(c->wblocks, nchunks);
    hipLaunchKernelGGL((k_wgrad32<CIN>), dim3(nb), dim3(kThreads), lds, c->st, g, x, c->part, NP, c->H, c->W, d);
    NNCHK(hipGetLastError());
    const int len = kCh * 9 * CIN + kCh;
    hipLaunchKernelGGL(k_reduce, dim3((len + 31) / 32), dim3(kThreads), 0, c->st, c->part, nb, len, dst);
    NNCHK(hipGetLastError());
}

double grads(adrnn_ctx *c, int B, const bf16_t *x0, const float *tgt, const uint8_t *mask, float *G) {
    const int HW = c->H * c->W, NP = B * HW;
    forward(c, B, x0, c->out);
    // interior pixel count (mask shared by the images)
    std::vector<uint8_t> hm(HW);
    NNCHK(hipMemcpyAsync(hm.data(), mask, HW, hipMemcpyDeviceToHost, c->st));
    NNCHK(hipStreamSynchronize(c->st));
    int64_t cnt = 0;
    for (uint8_t b : hm) cnt += b != 0;
    const double inv_cnt = 1.0 / (static_cast<double>(B) * std::max<int64_t>(cnt, 1));
    const int lb = (NP + 255) / 256;
    hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, c->st, c->out, tgt, mask, c->g4, c->lpart, NP, HW, inv_cnt);
    // layer 4
    const int nchunks = (NP + kChunk - 1) / kChunk, nb = std::min(c->wblocks, nchunks);
    hipLaunchKernelGGL(k_last_wgrad, dim3(nb), dim3(kThreads), 0, c->st, c->g4, c->y3, c->part, NP, c->H, c->W,
                       kDil[3]);
    hipLaunchKernelGGL(k_reduce, dim3((kW4 + 1 + 31) / 32), dim3(kThreads), 0, c->st, c->part, nb, kW4 + 1, G + oW4);
    hipLaunchKernelGGL(k_last_dgrad, dim3(lb), dim3(256), 0, c->st, c->g4, c->w4, c->y3, c->ga, NP, c->H, c->W,
                       kDil[3]);
    NNCHK(hipGetLastError());
    // layer 3: g3 = ga
    wgrad<32>(c, c->ga, c->y2, NP, kDil[2], G + oW3);  // writes W3 then b3 (contiguous in the layout)
    // the transposed convolution is the convolution with flipped taps at the same dilation
    conv32t<1>(c, B, c->ga, c->w3t, nullptr, c->y2, c->gb, kDil[2]);
    // layer 2: g2 = gb
    wgrad<32>(c, c->gb, c->y1, NP, kDil[1], G + oW2);
    conv32t<1>(c, B, c->gb, c->w2t, nullptr, c->y1, c->ga, kDil[1]);
    // layer 1: g1 = ga
    wgrad<4>(c, c->ga, x0, NP, kDil[0], G + oW1);
    NNCHK(hipGetLastError());
    std::vector<double> lp(lb);
    NNCHK(hipMemcpyAsync(lp.data(), c->lpart, sizeof(double) * lb, hipMemcpyDeviceToHost, c->st));
    NNCHK(hipStreamSynchronize(c->st));
    double L = 0.0;
    for (double v : lp) L += v;
    return L * inv_cnt;
}

adr_status fail(adrnn_ctx *c, const NNError &e) {
    if (c) c->err = e.msg;
    return e.code;
}

}  // namespace

extern "C" {

int64_t adrnn_param_count(void) { return kParams; }

adr_status adrnn_create(int32_t H, int32_t W, int32_t max_batch, void *stream, adrnn_ctx **out) {
    if (!out || H < 3 || W < 3 || max_batch < 1) return ADR_EINVAL;
    *out = nullptr;
    adrnn_ctx *c = new adrnn_ctx;
    try {
        c->H = H;
        c->W = W;
        c->maxB = max_batch;
        c->st = static_cast<hipStream_t>(stream);
        const size_t NP = static_cast<size_t>(max_batch) * H * W;
        if (NP * kCh > (size_t(1) << 31)) throw NNError{ADR_EINVAL, "batch too large"};
        c->P = nn_alloc<float>(c, kParams);
        c->m = nn_alloc<float>(c, kParams);
        c->v = nn_alloc<float>(c, kParams);
        c->grad = nn_alloc<float>(c, kParams);
        c->w1 = nn_alloc<bf16_t>(c, kW1);
        c->w2 = nn_alloc<bf16_t>(c, kW2);
        c->w3 = nn_alloc<bf16_t>(c, kW2);
        c->w2t = nn_alloc<bf16_t>(c, kW2);
        c->w3t = nn_alloc<bf16_t>(c, kW2);
        c->w4 = nn_alloc<float>(c, kW4);
        c->y1 = nn_alloc<bf16_t>(c, NP * kCh);
        c->y2 = nn_alloc<bf16_t>(c, NP * kCh);
        c->y3 = nn_alloc<bf16_t>(c, NP * kCh);
        c->ga = nn_alloc<bf16_t>(c, NP * kCh);
        c->gb = nn_alloc<bf16_t>(c, NP * kCh);
        c->out = nn_alloc<float>(c, NP);
        c->g4 = nn_alloc<float>(c, NP);
        c->part = nn_alloc<float>(c, static_cast<size_t>(c->wblocks) * (kCh * 9 * kCh + kCh));
        c->lpart = nn_alloc<double>(c, (NP + 255) / 256);
        c->fn = nn_alloc<double>(c, 2 * static_cast<size_t>(max_batch));
        c->dlmu = nn_alloc<double>(c, max_batch);
        std::vector<float> zero(kParams, 0.f);
        NNCHK(hipMemcpy(c->P, zero.data(), sizeof(float) * kParams, hipMemcpyHostToDevice));
        NNCHK(hipMemset(c->m, 0, sizeof(float) * kParams));
        NNCHK(hipMemset(c->v, 0, sizeof(float) * kParams));
        convert(c);
        NNCHK(hipStreamSynchronize(c->st));
    } catch (const NNError &e) {
        for (void *p : c->owned) (void)hipFree(p);
        delete c;
        return e.code;
    }
    *out = c;
    return ADR_OK;
}

adr_status adrnn_destroy(adrnn_ctx *c) {
    if (!c) return ADR_OK;
    (void)hipStreamSynchronize(c->st);
    for (void *p : c->owned) (void)hipFree(p);
    delete c;
    return ADR_OK;
}

adr_status adrnn_set_params(adrnn_ctx *c, const float *params) {
    if (!c || !params) return ADR_EINVAL;
    try {
        NNCHK(hipMemcpy(c->P, params, sizeof(float) * kParams, hipMemcpyHostToDevice));
        NNCHK(hipMemset(c->m, 0, sizeof(float) * kParams));
        NNCHK(hipMemset(c->v, 0, sizeof(float) * kParams));
        c->step = 0;
        convert(c);
        return ADR_OK;
    } catch (const NNError &e) {
        return fail(c, e);
    }
}

adr_status adrnn_get_params(adrnn_ctx *c, float *params) {
    if (!c || !params) return ADR_EINVAL;
    try {
        NNCHK(hipMemcpyAsync(params, c->P, sizeof(float) * kParams, hipMemcpyDeviceToHost, c->st));
        NNCHK(hipStreamSynchronize(c->st));
        return ADR_OK;
    } catch (const NNError &e) {
        return fail(c, e);
    }
}

adr_status adrnn_pack(adrnn_ctx *c, int32_t B, const double *f, const double *s, const uint8_t *mask,
                      const double *mu, const double *u_star, void *x0, float *target, double *s_norm) {
    if (!c || B < 1 || B > c->maxB || !f || !s || !mask || !mu || !x0 || (u_star && !target)) return ADR_EINVAL;
    try {
        const int HW = c->H * c->W, NP = B * HW;
        std::vector<double> lm(B);
        for (int b = 0; b < B; ++b) {
            if (!(mu[b] > 0)) throw NNError{ADR_EINVAL, "mu must be > 0"};
            lm[b] = std::log10(mu[b]);
        }
        NNCHK(hipMemcpy(c->dlmu, lm.data(), sizeof(double) * B, hipMemcpyHostToDevice));
        double *fn = c->fn, *sn = s_norm ? s_norm : c->fn + c->maxB;
        hipLaunchKernelGGL(k_norms, dim3(B), dim3(kThreads), 0, c->st, f, s, mask, fn, sn, HW);
        hipLaunchKernelGGL(k_pack, dim3((NP + 255) / 256), dim3(256), 0, c->st, f, s, mask, c->dlmu, fn, sn, u_star,
                           static_cast<bf16_t *>(x0), target, NP, HW);
        NNCHK(hipGetLastError());
        return ADR_OK;
    } catch (const NNError &e) {
        return fail(c, e);
    }
}

adr_status adrnn_forward(adrnn_ctx *c, int32_t B, const void *x0, float *out) {
    if (!c || B < 1 || B > c->maxB || !x0 || !out) return ADR_EINVAL;
    try {
        forward(c, B, static_cast<const bf16_t *>(x0), out);
        return ADR_OK;
    } catch (const NNError &e) {
        return fail(c, e);
    }
}

adr_status adrnn_grads(adrnn_ctx *c, int32_t B, const void *x0, const float *target, const uint8_t *mask,
                       float *G, double *loss) {
    if (!c || B < 1 || B > c->maxB || !x0 || !target || !mask || !G) return ADR_EINVAL;
    try {
        const double L = grads(c, B, static_cast<const bf16_t *>(x0), target, mask, G);
        if (loss) *loss = L;
        return ADR_OK;
    } catch (const NNError &e) {
        return fail(c, e);
    }
}

adr_status adrnn_adam(adrnn_ctx *c, const float *G, float lr) {
    if (!c || !G) return ADR_EINVAL;
    try {
        c->step += 1;
        const float c1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(c->step)));
        const float c2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(c->step)));
        hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, c->st, c->P, c->m, c->v, G, kParams, lr,
                           c1, c2);
        NNCHK(hipGetLastError());
        convert(c);
        return ADR_OK;
    } catch (const NNError &e) {
        return fail(c, e);
    }
}

adr_status adrnn_train_step(adrnn_ctx *c, int32_t B, const void *x0, const float *target, const uint8_t *mask,
                            float lr, double *loss) {
    adr_status s = adrnn_grads(c, B, x0, target, mask, c ? c->grad : nullptr, loss);
    if (s != ADR_OK) return s;
    return adrnn_adam(c, c->grad, lr);
}

adr_status adrnn_warm_start(adrnn_ctx *c, int32_t B, const double *s, const double *s_norm, const float *out,
                            const uint8_t *mask, double *u) {
    if (!c || B < 1 || B > c->maxB || !s || !s_norm || !out || !mask || !u) return ADR_EINVAL;
    try {
        const int HW = c->H * c->W, NP = B * HW;
        hipLaunchKernelGGL(k_warm, dim3((NP + 255) / 256), dim3(256), 0, c->st, s, s_norm, out, mask, u, NP, HW);
        NNCHK(hipGetLastError());
        return ADR_OK;
    } catch (const NNError &e) {
        return fail(c, e);
    }
}

adr_status adrnn_mfma_probe(const void *A, const void *B, float *D, void *stream) {
    if (!A || !B || !D) return ADR_EINVAL;
    hipLaunchKernelGGL(k_probe, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                       static_cast<const bf16_t *>(A), static_cast<const bf16_t *>(B), D);
    return hipGetLastError() == hipSuccess ? ADR_OK : ADR_EDEVICE;
}

const char *adrnn_last_error(const adrnn_ctx *c) { return c ? c->err.c_str() : ""; }

}  // extern "C"
