// Learned warm start: BF16 matrix-core (MFMA) convolution kernels with FP32
// accumulation, training (backward, Adam) and inference, behind the C ABI of
// include/adrnn.h.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x16_bf16: M = pixels,
// N = 32 output channels (two 16x16 tiles), K = (tap, input channel).  The
// 32 -> 32 layers run tiled and persistent (k_conv32t: 16 x 16-pixel tiles
// with their dilated halo staged in LDS, the next tile prefetched), the
// 4 -> 32 first layer directly from global memory (k_conv_in), the 32 -> 1
// last layer on the vector ALUs.  Weight gradients are GEMMs with K = pixels
// (k_wgradt: tiles transposed to channel-major LDS).  Operand layout of the
// instruction: lane l supplies A[l%16][4(l/16) .. 4(l/16)+3] and
// B[4(l/16) .. +3][l%16]; it receives D[4(l/16) + v][l%16], v = 0..3.  NHWC
// activations make a lane's four K values (four consecutive channels of one
// pixel) one 8-byte load.
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
constexpr int kDil[4] = {1, 2, 4, 8};
// widest fine grid of adrnn_restrict (one FP64 row of column sums in 64 KB of LDS)
constexpr int kMaxRestrictWidth = 8192;

// FP32 -> BF16, round to nearest even: the gfx950 conversion instruction
// (v_cvt_pk_bf16_f32), one value or a packed pair (low half: a)
typedef __bf16 v2bf16 __attribute__((ext_vector_type(2)));
typedef float v2f32 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16_t f2bf(float f) { return __builtin_bit_cast(bf16_t, static_cast<__bf16>(f)); }
__device__ __forceinline__ unsigned f2bf2(float a, float b) {
    return __builtin_bit_cast(unsigned, __builtin_convertvector(v2f32{a, b}, v2bf16));
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(static_cast<unsigned>(h) << 16); }
__device__ __forceinline__ bool bf_pos(bf16_t h) { return h != 0 && (h & 0x8000) == 0 && h <= 0x7f80; }

__device__ __forceinline__ v4f32 mfma(v4i16 a, v4i16 b, v4f32 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ conv, 4 -> 32 (first layer)
// y = bf16(relu(conv(x0) + bias)); x0: [NP][4] BF16, Wg: [32][9][4].  A wavefront
// computes 16 pixels x 32 channels; K = 12 taps (9, padded) x 4 channels, one
// tap per lane group, so a lane's 4 K values are one pixel's 4 channels.  N-tile
// 0 holds the even output channels and N-tile 1 the odd ones: a lane stores its
// two results of a pixel as one 4-byte pair.
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
    const float bias0 = bias[2 * i], bias1 = bias[2 * i + 1];
    unsigned *yw = reinterpret_cast<unsigned *>(y);
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
            const v4i16 b0 = *reinterpret_cast<const v4i16 *>(&Ws[((2 * i) * KT + tap) * CIN]);
            const v4i16 b1 = *reinterpret_cast<const v4i16 *>(&Ws[((2 * i + 1) * KT + tap) * CIN]);
            acc0 = mfma(av[kc], b0, acc0);
            acc1 = mfma(av[kc], b1, acc1);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int po = t * 16 + 4 * g + v;
            if (po >= NP) continue;
            yw[static_cast<unsigned>(po) * (kCh / 2) + i] = f2bf2(fmaxf(acc0[v] + bias0, 0.f), fmaxf(acc1[v] + bias1, 0.f));
        }
    }
}

// ------------------------------------------------------------------ conv, 32 -> 32, tiled
// A workgroup computes 16 x 16-pixel output tiles (all 32 output channels) in
// turn.  The weights are staged in LDS once; per tile the input patch
// ((16 + 2d)^2 pixels x 32 channels, zeros outside the image) is staged, and
// the next tile's patch loads are issued before the current tile's products.
// Pixel rows are padded to kCP channels and weight rows to kWS entries so that
// the fragment reads of a wavefront spread over the LDS banks.  Wavefront w
// computes tile rows 4w .. 4w+3 (4 M-tiles of 16 pixels) x 32 channels: N-tile
// 0 holds the even output channels and N-tile 1 the odd ones, so that a lane's
// two results of a pixel are adjacent channels (one 4-byte store).
// EPI 0: y = bf16(relu(acc + bias)).  EPI 1: y = bf16(acc * (ymask > 0)) (back-
// propagation through the ReLU of the layer input, with flipped taps).
constexpr int kTile = 16;
constexpr int kCP = 36;            // staged channels per pixel (32 + pad)
constexpr int kWS = 9 * kCh + 4;   // staged weight row (one output channel: 9 taps x 32 inputs + pad)
constexpr int kMaxDilT = 4;        // largest dilation the tiled kernels stage (patch (16 + 2*4)^2)
constexpr int kWStage = (kCh * 36 + kThreads - 1) / kThreads;

__host__ __device__ inline int conv_tiles(int H, int W) { return ((H + kTile - 1) / kTile) * ((W + kTile - 1) / kTile); }
__host__ __device__ inline size_t conv_tiled_lds(int d) {
    const int P = kTile + 2 * d;
    return sizeof(bf16_t) * (static_cast<size_t>(kCh) * kWS + static_cast<size_t>(P) * P * kCP);
}

// the patch loads of tile t (16 bytes each, issued without waiting): a pixel
// outside the image reads the image's first pixel; bit u of *inm marks load u
// as inside (the LDS store writes zeros for the others)
template <int D, int XS>
__device__ __forceinline__ void conv_patch_load(const bf16_t *__restrict__ x, int t, int tpi, int tw, int H, int W,
                                                uint4 (&xv)[XS], unsigned &inm) {
    constexpr int d = D, P = kTile + 2 * D;
    const int b = t / tpi, tt = t - b * tpi;
    const int ty = tt / tw, tx = tt - ty * tw;
    const int y0 = ty * kTile, x0 = tx * kTile;
    const unsigned ib = static_cast<unsigned>(b) * static_cast<unsigned>(H * W);
    const uint4 *xq = reinterpret_cast<const uint4 *>(x);
    unsigned m = 0;
#pragma unroll
    for (int u = 0; u < XS; ++u) {
        const int e = threadIdx.x + u * kThreads;
        const int pix = e >> 2, q = e & 3;
        const int py = pix / P, px = pix - py * P;
        const int gy = y0 - d + py, gx = x0 - d + px;
        const bool ok = e < P * P * 4 && gy >= 0 && gy < H && gx >= 0 && gx < W;
        const unsigned gp = ib + (ok ? static_cast<unsigned>(gy * W + gx) : 0u);
        xv[u] = xq[gp * (kCh / 8) + q];
        m |= ok ? 1u << u : 0u;
    }
    inm = m;
}

// the ReLU mask pairs (channels 2i, 2i+1) of a lane's 16 outputs in tile t of
// the transposed pass: rows 4 wave + mt, columns 4 g + v (outside the image:
// the image's first pixel, not used)
__device__ __forceinline__ void conv_mask_load(const bf16_t *__restrict__ ymask, int t, int tpi, int tw, int H, int W,
                                               int wave, int g, int i, unsigned (&mk)[4][4]) {
    const int b = t / tpi, tt = t - b * tpi;
    const int ty = tt / tw, tx = tt - ty * tw;
    const int y0 = ty * kTile, x0 = tx * kTile;
    const unsigned *mw = reinterpret_cast<const unsigned *>(ymask);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int gy = y0 + wave * 4 + mt, gx = x0 + 4 * g + v;
            const bool in = gy < H && gx < W;
            const unsigned po = (static_cast<unsigned>(b) * H + (in ? gy : 0)) * W + (in ? gx : 0);
            mk[mt][v] = mw[po * (kCh / 2) + i];
        }
}

// patch loads per thread at dilation d: ceil((16 + 2d)^2 * 4 / 256) (the prefetch registers)
__host__ __device__ constexpr int conv_xs(int d) { return ((kTile + 2 * d) * (kTile + 2 * d) * 4 + kThreads - 1) / kThreads; }

template <int EPI, int D>
__global__ __launch_bounds__(kThreads) void k_conv32t(const bf16_t *__restrict__ x, const bf16_t *__restrict__ Wg,
                                                      const float *__restrict__ bias,
                                                      const bf16_t *__restrict__ ymask, bf16_t *__restrict__ y,
                                                      int H, int W, int ntiles) {
    constexpr int d = D, P = kTile + 2 * D, XS = conv_xs(D);
    extern __shared__ __align__(16) unsigned char sm[];
    bf16_t *Ws = reinterpret_cast<bf16_t *>(sm);  // [32][kWS]
    bf16_t *Xs = Ws + kCh * kWS;                  // [P*P][kCP]
    const int tw = (W + kTile - 1) / kTile, tpi = conv_tiles(H, W);
    const uint4 z4 = make_uint4(0u, 0u, 0u, 0u);
    // weights, once (32 rows of 288 entries, 16 bytes per load)
    {
        uint4 wv[kWStage];
#pragma unroll
        for (int u = 0; u < kWStage; ++u) {
            const int e = threadIdx.x + u * kThreads;
            wv[u] = reinterpret_cast<const uint4 *>(Wg)[e < kCh * 36 ? e : 0];
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
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    // the bias through LDS: a global load pending at the epilogue would make the
    // epilogue wait for the next tile's patch loads as well (one counter for all)
    __shared__ float bs[kCh];
    if (threadIdx.x < kCh) bs[threadIdx.x] = EPI == 0 ? bias[threadIdx.x] : 0.f;
    uint4 xv[XS];
    unsigned inm = 0;
    // EPI 1: the ReLU mask pairs of this lane's outputs, double-buffered: the
    // next tile's are loaded with its patch, so the epilogue never waits
    unsigned mk[4][4], mkn[4][4];
    int t = blockIdx.x;
    if (t < ntiles) {
        if constexpr (EPI == 1) conv_mask_load(ymask, t, tpi, tw, H, W, wave, g, i, mkn);
        conv_patch_load<D, XS>(x, t, tpi, tw, H, W, xv, inm);
    }
    for (; t < ntiles; t += gridDim.x) {
        __syncthreads();  // the previous tile's products are done with Xs
#pragma unroll
        for (int u = 0; u < XS; ++u) {
            const int e = threadIdx.x + u * kThreads;
            if (e < P * P * 4) {
                const uint4 v = (inm >> u) & 1u ? xv[u] : z4;
                uint2 *dst = reinterpret_cast<uint2 *>(Xs + (e >> 2) * kCP + (e & 3) * 8);
                dst[0] = make_uint2(v.x, v.y);
                dst[1] = make_uint2(v.z, v.w);
            }
        }
        __syncthreads();
        const float bias0 = bs[2 * i], bias1 = bs[2 * i + 1];
        const int b = t / tpi, tt = t - b * tpi;
        const int ty = tt / tw, tx = tt - ty * tw;
        const int y0 = ty * kTile, x0 = tx * kTile;
        if constexpr (EPI == 1) {
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int v = 0; v < 4; ++v) mk[mt][v] = mkn[mt][v];
        }
        if (t + static_cast<int>(gridDim.x) < ntiles) {  // in flight during the products
            if constexpr (EPI == 1) conv_mask_load(ymask, t + gridDim.x, tpi, tw, H, W, wave, g, i, mkn);
            conv_patch_load<D, XS>(x, t + gridDim.x, tpi, tw, H, W, xv, inm);
        }
        v4f32 acc[4][2];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt][0] = acc[mt][1] = v4f32{0.f, 0.f, 0.f, 0.f};
#pragma unroll 3
        for (int tap = 0; tap < 9; ++tap) {
            const int oy = d + d * (tap / 3 - 1), ox = d + d * (tap % 3 - 1);
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) {
                const v4i16 b0 = *reinterpret_cast<const v4i16 *>(&Ws[(2 * i) * kWS + tap * kCh + cc * 16 + g * 4]);
                const v4i16 b1 = *reinterpret_cast<const v4i16 *>(&Ws[(2 * i + 1) * kWS + tap * kCh + cc * 16 + g * 4]);
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
        unsigned *yw = reinterpret_cast<unsigned *>(y);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            const int gy = y0 + wave * 4 + mt;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int gx = x0 + 4 * g + v;
                if (gy >= H || gx >= W) continue;
                const unsigned po = (static_cast<unsigned>(b) * H + gy) * W + gx;
                float z0 = acc[mt][0][v], z1 = acc[mt][1][v];
                if constexpr (EPI == 0) {
                    z0 = fmaxf(z0 + bias0, 0.f);
                    z1 = fmaxf(z1 + bias1, 0.f);
                } else {
                    z0 = bf_pos(static_cast<bf16_t>(mk[mt][v] & 0xffffu)) ? z0 : 0.f;
                    z1 = bf_pos(static_cast<bf16_t>(mk[mt][v] >> 16)) ? z1 : 0.f;
                }
                yw[po * (kCh / 2) + i] = f2bf2(z0, z1);
            }
        }
    }
}

// ------------------------------------------------------------------ weight gradient (MFMA), tiled
// part[blk][(n*9 + tap)*CIN + c] = sum over the block's pixels p of g[p][n] x[p + d off(tap)][c]
// and part[blk][32*9*CIN + n] = sum g[p][n]; g: [NP][32], x: [NP][CIN] BF16.
// A workgroup takes 16 x 16-pixel tiles of the images in turn.  Per tile it
// stages g (the tile's 256 pixels) and the input patch ((16 + 2d)^2 pixels,
// zeros outside the image) channel-major in LDS; a lane's MFMA operand is then
// 4 consecutive pixels of one channel, one 8-byte read.  The pixel quads are
// transposed in registers (4 pixels x 8 channels -> 8 channels x 4 pixels), and
// the next tile's loads are issued before the current tile's products.
// GEMM view: M = 32 output channels (2 row tiles), N = 9 CIN (tap, c)
// columns, K = the tile's pixels, one tile row (16 pixels) per MFMA.
constexpr int kGS = kTile * kTile + 4;  // gT row stride: 16 rows of one fragment read fall on distinct bank pairs
__host__ __device__ constexpr int wg_pw(int d) { return (kTile + 2 * d + 3) & ~3; }  // patch row (multiple of 4)
__host__ __device__ constexpr int wg_cs(int d) {  // patch channel stride, = 4 (mod 64) like kGS
    const int raw = (kTile + 2 * d) * wg_pw(d);
    return raw + (((4 - raw) % 64) + 64) % 64;
}
__host__ __device__ inline size_t wgrad_lds(int cin, int d) {
    return sizeof(bf16_t) * (static_cast<size_t>(kCh) * kGS + static_cast<size_t>(cin) * wg_cs(d));
}
// patch items at dilation d: CIN 32: (row, pixel quad, channel octet); CIN 4: (row, pixel quad)
__host__ __device__ constexpr int wg_nxi(int cin, int d) {
    return (kTile + 2 * d) * (wg_pw(d) / 4) * (cin == 32 ? 4 : 1);
}

__device__ __forceinline__ unsigned word_of(const uint4 &v, int w) {
    return w == 0 ? v.x : w == 1 ? v.y : w == 2 ? v.z : v.w;
}

// 4 pixels' words w of a channel octet -> the two 4-pixel rows of channels 2w, 2w+1
__device__ __forceinline__ void tr_pair(unsigned p0, unsigned p1, unsigned p2, unsigned p3, uint2 &ev, uint2 &od) {
    ev.x = (p0 & 0xffffu) | (p1 << 16);
    ev.y = (p2 & 0xffffu) | (p3 << 16);
    od.x = (p0 >> 16) | (p1 & 0xffff0000u);
    od.y = (p2 >> 16) | (p3 & 0xffff0000u);
}

// Loads of one tile (g quad and patch items of this thread), issued without
// waiting: out-of-image pixels read the image's first pixel and are marked in
// *okm (bit v: g pixel v; bit 4 + 4u + v: patch item u, pixel v), zeroed at
// the LDS store.  Offsets are 32-bit (an activation buffer holds < 2^31 entries).
template <int CIN, int D, int XI, int XU>
__device__ __forceinline__ void wg_load(const bf16_t *__restrict__ gsrc, const bf16_t *__restrict__ x, int t,
                                        int tpi, int tw, int H, int W, int tid, uint4 (&gv)[4], uint4 (&xv)[XI][XU],
                                        unsigned &okm) {
    constexpr int d = D, P = kTile + 2 * D, QW = wg_pw(D) / 4, nxi = wg_nxi(CIN, D);
    const int b = t / tpi, tt = t - b * tpi;
    const int ty = tt / tw, tx = tt - ty * tw;
    const int y0 = ty * kTile, x0 = tx * kTile;
    const unsigned ib = static_cast<unsigned>(b) * static_cast<unsigned>(H * W);
    unsigned m = 0;
    {
        const int gq = tid >> 2, go = tid & 3;
        const int gy = y0 + (gq >> 2), gx0 = x0 + 4 * (gq & 3);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const bool ok = gy < H && gx0 + v < W;
            const unsigned pix = ib + (ok ? static_cast<unsigned>(gy * W + gx0 + v) : 0u);
            gv[v] = reinterpret_cast<const uint4 *>(gsrc)[pix * (kCh / 8) + go];
            m |= ok ? 1u << v : 0u;
        }
    }
#pragma unroll
    for (int u = 0; u < XI; ++u) {
        const int e = tid + u * kThreads;
        const int it = CIN == 32 ? e >> 2 : e;
        const int py = it / QW, qx = it - py * QW;
        const int gy = y0 - d + py;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int px = 4 * qx + v, gx = x0 - d + px;
            const bool ok = e < nxi && px < P && gy >= 0 && gy < H && gx >= 0 && gx < W;
            const unsigned pix = ib + (ok ? static_cast<unsigned>(gy * W + gx) : 0u);
            if (CIN == 32) {
                xv[u][v] = reinterpret_cast<const uint4 *>(x)[pix * (kCh / 8) + (e & 3)];
            } else {
                const uint2 w2 = reinterpret_cast<const uint2 *>(x)[pix];
                // two pixels per uint4: v even -> .x .y, v odd -> .z .w
                if (v & 1) { xv[u][v >> 1].z = w2.x; xv[u][v >> 1].w = w2.y; }
                else { xv[u][v >> 1].x = w2.x; xv[u][v >> 1].y = w2.y; }
            }
            m |= ok ? 1u << (4 + 4 * u + v) : 0u;
        }
    }
    okm = m;
}

template <int CIN, int D>
__global__ __launch_bounds__(kThreads) void k_wgradt(const bf16_t *__restrict__ gsrc, const bf16_t *__restrict__ x,
                                                     float *__restrict__ part, int ntiles, int H, int W) {
    constexpr int NCOL = 9 * CIN;          // (tap, c) columns
    constexpr int NJT = (NCOL + 15) / 16;  // column tiles
    constexpr int CPW = (NJT + 3) / 4;     // column tiles per wave
    constexpr int d = D;
    constexpr int XI = (wg_nxi(CIN, D) + kThreads - 1) / kThreads;
    constexpr int XU = CIN == 32 ? 4 : 2;  // 16-byte loads per patch item
    extern __shared__ __align__(16) unsigned char sm[];
    bf16_t *gT = reinterpret_cast<bf16_t *>(sm);  // [32][kGS]
    bf16_t *xT = gT + kCh * kGS;                  // [CIN][CS]: row py at py * PW
    constexpr int PW = wg_pw(D), CS = wg_cs(D);
    constexpr int QW = PW / 4;                    // pixel quads per patch row
    constexpr int nxi = wg_nxi(CIN, D);
    const int tw = (W + kTile - 1) / kTile, tpi = conv_tiles(H, W);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i = lane & 15, g = lane >> 4;
    // this thread's g item: pixel quad gq (tile row gq / 4, pixels 4 (gq % 4) ..), channel octet go
    const int gq = tid >> 2, go = tid & 3;

    uint4 gv[4], xv[XI][XU];
    unsigned okm = 0;
    v4f32 acc[CPW][2];
#pragma unroll
    for (int q = 0; q < CPW; ++q) acc[q][0] = acc[q][1] = v4f32{0.f, 0.f, 0.f, 0.f};
    float db[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    // column tiles of this wave: jt = wave + 4 cq (cq < CPW, jt < NJT), each with
    // both row tiles, so that a B fragment feeds two products.  CIN 32: a column
    // tile is 16 channels of one tap, so its tap and offset are uniform over the
    // wavefront (scalar); the lane adds c * CS + 4 g.
    const int wv = __builtin_amdgcn_readfirstlane(wave);
    int bofs[CPW];
    bool jok[CPW], colok_q[CPW];
#pragma unroll
    for (int cq = 0; cq < CPW; ++cq) {
        const int jt = wv + 4 * cq;
        jok[cq] = jt < NJT;
        if (CIN == 32) {
            const int tap = jok[cq] ? jt >> 1 : 4, dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
            bofs[cq] = (jt & 1) * 16 * CS + (d + dy) * PW + d + dx;  // uniform
            colok_q[cq] = jok[cq];
        } else {
            const int col = jt * 16 + i;
            const bool ok = jok[cq] && col < NCOL;
            const int tap = ok ? col / CIN : 4, c = ok ? col % CIN : 0;
            const int dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
            bofs[cq] = c * CS + (d + dy) * PW + d + dx;  // per lane
            colok_q[cq] = ok;
        }
    }
    const int lbase = (CIN == 32 ? i * CS : 0) + 4 * g;

    int t = blockIdx.x;
    if (t < ntiles) wg_load<CIN, D, XI, XU>(gsrc, x, t, tpi, tw, H, W, tid, gv, xv, okm);
    for (; t < ntiles; t += gridDim.x) {
        __syncthreads();  // the previous tile's products are done with the LDS
        // g: 8 channels x 4 pixels -> 8 rows of gT (and the bias gradient)
        {
            const int pl = (gq >> 2) * kTile + 4 * (gq & 3);
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const unsigned p0 = (okm & 1u) ? word_of(gv[0], w) : 0u, p1 = (okm & 2u) ? word_of(gv[1], w) : 0u;
                const unsigned p2 = (okm & 4u) ? word_of(gv[2], w) : 0u, p3 = (okm & 8u) ? word_of(gv[3], w) : 0u;
                uint2 ev, od;
                tr_pair(p0, p1, p2, p3, ev, od);
                *reinterpret_cast<uint2 *>(&gT[(8 * go + 2 * w) * kGS + pl]) = ev;
                *reinterpret_cast<uint2 *>(&gT[(8 * go + 2 * w + 1) * kGS + pl]) = od;
                db[2 * w] += bf2f(static_cast<bf16_t>(p0 & 0xffffu)) + bf2f(static_cast<bf16_t>(p1 & 0xffffu)) +
                             bf2f(static_cast<bf16_t>(p2 & 0xffffu)) + bf2f(static_cast<bf16_t>(p3 & 0xffffu));
                db[2 * w + 1] += bf2f(static_cast<bf16_t>(p0 >> 16)) + bf2f(static_cast<bf16_t>(p1 >> 16)) +
                                 bf2f(static_cast<bf16_t>(p2 >> 16)) + bf2f(static_cast<bf16_t>(p3 >> 16));
            }
        }
        // patch: channel-major rows
#pragma unroll
        for (int u = 0; u < XI; ++u) {
            const int e = tid + u * kThreads;
            if (e >= nxi) continue;
            const int it = CIN == 32 ? e >> 2 : e;
            const int py = it / QW, qx = it - py * QW;
            const int off = py * PW + 4 * qx;
            if (CIN == 32) {
                const int c0 = 8 * (e & 3);
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    uint2 ev, od;
                    const unsigned mu = okm >> (4 + 4 * u);
                    tr_pair((mu & 1u) ? word_of(xv[u][0], w) : 0u, (mu & 2u) ? word_of(xv[u][1], w) : 0u,
                            (mu & 4u) ? word_of(xv[u][2], w) : 0u, (mu & 8u) ? word_of(xv[u][3], w) : 0u, ev, od);
                    *reinterpret_cast<uint2 *>(&xT[(c0 + 2 * w) * CS + off]) = ev;
                    *reinterpret_cast<uint2 *>(&xT[(c0 + 2 * w + 1) * CS + off]) = od;
                }
            } else {
                // pixels v = 0..3 hold words (c0 c1), (c2 c3): xv[u][v / 2] .x .y (even v) or .z .w (odd v)
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    const unsigned mu = okm >> (4 + 4 * u);
                    const unsigned p0 = (mu & 1u) ? word_of(xv[u][0], w) : 0u;
                    const unsigned p1 = (mu & 2u) ? word_of(xv[u][0], 2 + w) : 0u;
                    const unsigned p2 = (mu & 4u) ? word_of(xv[u][1], w) : 0u;
                    const unsigned p3 = (mu & 8u) ? word_of(xv[u][1], 2 + w) : 0u;
                    uint2 ev, od;
                    tr_pair(p0, p1, p2, p3, ev, od);
                    *reinterpret_cast<uint2 *>(&xT[(2 * w) * CS + off]) = ev;
                    *reinterpret_cast<uint2 *>(&xT[(2 * w + 1) * CS + off]) = od;
                }
            }
        }
        __syncthreads();
        if (t + static_cast<int>(gridDim.x) < ntiles)  // in flight during the products
            wg_load<CIN, D, XI, XU>(gsrc, x, t + gridDim.x, tpi, tw, H, W, tid, gv, xv, okm);
        // all fragment reads of a tile row are issued before its products: the
        // read form is the same for every tile (CIN 32: two 4-byte halves, the
        // tap shift d + dx being even; CIN 4: four 2-byte reads)
#pragma unroll 1
        for (int r = 0; r < kTile; ++r) {
            const v4i16 a0 = *reinterpret_cast<const v4i16 *>(&gT[i * kGS + r * kTile + 4 * g]);
            const v4i16 a1 = *reinterpret_cast<const v4i16 *>(&gT[(16 + i) * kGS + r * kTile + 4 * g]);
            v4i16 bv[CPW];
#pragma unroll
            for (int cq = 0; cq < CPW; ++cq) {
                const bf16_t *src = &xT[lbase + bofs[cq] + r * PW];
                if (CIN == 32) {
                    const unsigned lo = *reinterpret_cast<const unsigned *>(src);
                    const unsigned hi = *reinterpret_cast<const unsigned *>(src + 2);
                    bv[cq][0] = static_cast<short>(lo & 0xffffu);
                    bv[cq][1] = static_cast<short>(lo >> 16);
                    bv[cq][2] = static_cast<short>(hi & 0xffffu);
                    bv[cq][3] = static_cast<short>(hi >> 16);
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) bv[cq][v] = colok_q[cq] ? static_cast<short>(src[v]) : short(0);
                }
            }
#pragma unroll
            for (int cq = 0; cq < CPW; ++cq) {
                if (!jok[cq]) continue;  // uniform
                acc[cq][0] = mfma(a0, bv[cq], acc[cq][0]);
                acc[cq][1] = mfma(a1, bv[cq], acc[cq][1]);
            }
        }
    }
    float *out = part + static_cast<size_t>(blockIdx.x) * (kCh * NCOL + kCh);
#pragma unroll
    for (int cq = 0; cq < CPW; ++cq) {
        const int col = (wv + 4 * cq) * 16 + i;
        if (!jok[cq] || col >= NCOL) continue;
#pragma unroll
        for (int rt = 0; rt < 2; ++rt)
#pragma unroll
            for (int v = 0; v < 4; ++v) out[(rt * 16 + 4 * g + v) * NCOL + col] = acc[cq][rt][v];
    }
    // bias gradient: channel 8 o + k is summed by the 64 threads with tid % 4 = o, in thread order
    __syncthreads();
    float *bred = reinterpret_cast<float *>(sm);  // [8][256]
#pragma unroll
    for (int k = 0; k < 8; ++k) bred[k * kThreads + tid] = db[k];
    __syncthreads();
    if (tid < kCh) {
        const int o = tid >> 3, k = tid & 7;
        float sb = 0.f;
        for (int q = 0; q < kThreads / 4; ++q) sb += bred[k * kThreads + 4 * q + o];
        out[kCh * NCOL + tid] = sb;
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
// 32 -> 1 last layer (no activation): out[p] = b + sum_tap sum_c W4[tap][c] y3[p + d off(tap)][c].
// Four lanes per pixel, lane o holding channels 8o .. 8o+7 (one 16-byte load per
// tap; a wavefront's load covers 16 whole pixels), the four partial sums added
// across the lanes; a workgroup walks pixel groups of 64 with the weights in
// registers.
__global__ __launch_bounds__(kThreads) void k_last_fwd(const bf16_t *__restrict__ y3, const float *__restrict__ W4,
                                                       const float *__restrict__ b4, float *__restrict__ out, int NP,
                                                       int H, int W, int d) {
    __shared__ __align__(16) float w4s[kW4];
    for (int e = threadIdx.x; e < kW4; e += blockDim.x) w4s[e] = W4[e];
    __syncthreads();
    const int ps = threadIdx.x >> 2, o = threadIdx.x & 3;
    float wr[9][8];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const float4 lo = *reinterpret_cast<const float4 *>(&w4s[tap * kCh + 8 * o]);
        const float4 hi = *reinterpret_cast<const float4 *>(&w4s[tap * kCh + 8 * o + 4]);
        wr[tap][0] = lo.x; wr[tap][1] = lo.y; wr[tap][2] = lo.z; wr[tap][3] = lo.w;
        wr[tap][4] = hi.x; wr[tap][5] = hi.y; wr[tap][6] = hi.z; wr[tap][7] = hi.w;
    }
    const float bias = b4[0];
    const int HW = H * W;
    const uint4 *yv = reinterpret_cast<const uint4 *>(y3);
    for (int gp0 = blockIdx.x * 64; gp0 < NP; gp0 += gridDim.x * 64) {
        const int gp = gp0 + ps;
        if (gp >= NP) break;
        const int p = gp % HW, py = p / W, px = p - py * W;
        uint4 v[9];
        bool ok[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
            ok[tap] = py + dy >= 0 && py + dy < H && px + dx >= 0 && px + dx < W;
            v[tap] = yv[static_cast<unsigned>(ok[tap] ? gp + dy * W + dx : gp) * (kCh / 8) + o];
        }
        float s = 0.f;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const unsigned q[4] = {v[tap].x, v[tap].y, v[tap].z, v[tap].w};
            float t = 0.f;
#pragma unroll
            for (int e = 0; e < 4; ++e)
                t += wr[tap][2 * e] * __uint_as_float(q[e] << 16) + wr[tap][2 * e + 1] * __uint_as_float(q[e] & 0xffff0000u);
            s += ok[tap] ? t : 0.f;
        }
        s += __shfl_xor(s, 1, 4);
        s += __shfl_xor(s, 2, 4);
        if (o == 0) out[gp] = s + bias;
    }
}

// interior pixels of the mask: cnt[0] += the nonzero bytes (zeroed before).
// A thread counts 16 bytes (one 16-byte load from the first 16-byte boundary
// on); the bytes before that boundary and after the last full word are
// counted one by one by one thread.  A workgroup adds its count once (integer:
// any order gives the same sum).
__global__ __launch_bounds__(kThreads) void k_mask_count(const uint8_t *__restrict__ mask, int HW, int *__restrict__ cnt) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const int head = static_cast<int>((16u - (reinterpret_cast<uintptr_t>(mask) & 15u)) & 15u);
    const int h = head < HW ? head : HW;
    const int n16 = (HW - h) / 16;
    int c = 0;
    if (i < n16) {
        const uint4 v = reinterpret_cast<const uint4 *>(mask + h)[i];
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int bt = 0; bt < 4; ++bt) c += ((w[k] >> (8 * bt)) & 0xffu) != 0u;
    } else if (i == n16) {
        for (int p = 0; p < h; ++p) c += mask[p] != 0;
        for (int p = h + 16 * n16; p < HW; ++p) c += mask[p] != 0;
    }
    __shared__ int red[kThreads];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] != 0) atomicAdd(cnt, red[0]);
}

// g4 = 2 (out - target) mask / (B cnt); partial sums of mask (out - target)^2 per block
__global__ void k_loss(const float *__restrict__ out, const float *__restrict__ tgt, const uint8_t *__restrict__ mask,
                       float *__restrict__ g4, double *__restrict__ lpart, int NP, int HW, int B,
                       const int *__restrict__ cnt) {
    const int gp = blockIdx.x * blockDim.x + threadIdx.x;
    const double inv_cnt = 1.0 / (static_cast<double>(B) * (cnt[0] > 0 ? cnt[0] : 1));
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

// loss of the step = sum of the block partials (fixed order) / (B cnt): acc[2]
// = this step's loss, acc[0] += it, acc[1] += 1 (one workgroup)
__global__ __launch_bounds__(kThreads) void k_loss_sum(const double *__restrict__ lpart, int nb, int B,
                                                       const int *__restrict__ cnt, double *__restrict__ acc) {
    double sum = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) sum += lpart[b];
    __shared__ double red[kThreads];
    red[threadIdx.x] = sum;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double L = red[0] / (static_cast<double>(B) * (cnt[0] > 0 ? cnt[0] : 1));
        acc[2] = L;
        acc[0] += L;
        acc[1] += 1.0;
    }
}

// g3 = bf16( (sum_tap W4[tap][c] g4[p - d off(tap)]) * (y3 > 0) ).  Four lanes per
// pixel (lane o: channels 8o .. 8o+7, one 16-byte mask load and one 16-byte store),
// weights in registers, a workgroup walks pixel groups of 64.
// (at most 4 waves per SIMD: with the 72 weights in registers, a tighter
// register budget makes the compiler wait for each tap's load in turn)
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_last_dgrad(const float *__restrict__ g4, const float *__restrict__ W4,
                                                         const bf16_t *__restrict__ y3, bf16_t *__restrict__ g3,
                                                         int NP, int H, int W, int d) {
    __shared__ __align__(16) float w4s[kW4];
    for (int e = threadIdx.x; e < kW4; e += blockDim.x) w4s[e] = W4[e];
    __syncthreads();
    const int ps = threadIdx.x >> 2, o = threadIdx.x & 3;
    float wr[9][8];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const float4 lo = *reinterpret_cast<const float4 *>(&w4s[tap * kCh + 8 * o]);
        const float4 hi = *reinterpret_cast<const float4 *>(&w4s[tap * kCh + 8 * o + 4]);
        wr[tap][0] = lo.x; wr[tap][1] = lo.y; wr[tap][2] = lo.z; wr[tap][3] = lo.w;
        wr[tap][4] = hi.x; wr[tap][5] = hi.y; wr[tap][6] = hi.z; wr[tap][7] = hi.w;
    }
    const int HW = H * W;
    const uint4 *ysrc = reinterpret_cast<const uint4 *>(y3);
    uint4 *gdst = reinterpret_cast<uint4 *>(g3);
    for (int gp0 = blockIdx.x * 64; gp0 < NP; gp0 += gridDim.x * 64) {
        const int gp = gp0 + ps;
        if (gp >= NP) break;
        const int p = gp % HW, py = p / W, px = p - py * W;
        float gn[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
            // pixel gp feeds output gp - d off through tap
            const bool ok = py - dy >= 0 && py - dy < H && px - dx >= 0 && px - dx < W;
            const float gvl = g4[ok ? gp - dy * W - dx : gp];
            gn[tap] = ok ? gvl : 0.f;
        }
        const uint4 yv = ysrc[static_cast<unsigned>(gp) * (kCh / 8) + o];

        const unsigned yq[4] = {yv.x, yv.y, yv.z, yv.w};
        unsigned oq[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            unsigned packed = 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                float s_ = 0.f;
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) s_ += wr[tap][2 * e + h] * gn[tap];
                const bf16_t yb = static_cast<bf16_t>(h == 0 ? (yq[e] & 0xffffu) : (yq[e] >> 16));
                packed |= static_cast<unsigned>(f2bf(bf_pos(yb) ? s_ : 0.f)) << (16 * h);
            }
            oq[e] = packed;
        }
        gdst[static_cast<unsigned>(gp) * (kCh / 8) + o] = make_uint4(oq[0], oq[1], oq[2], oq[3]);
    }
}

// part[blk][tap*32 + c] = sum over the block's pixels of g4[p] y3[p + d off][c]; part[blk][288] = sum g4.
// Four lanes per activation pixel (lane o: channels 8o .. 8o+7, one 16-byte
// load), 72 accumulators per lane; a workgroup walks pixel groups of 64.  At the end
// the 16 pixel lanes of a wavefront are summed by a butterfly, then the four
// wavefronts in LDS (fixed order).
__global__ __launch_bounds__(kThreads) void k_last_wgrad(const float *__restrict__ g4, const bf16_t *__restrict__ y3,
                                                         float *__restrict__ part, int NP, int H, int W, int d) {
    const int ps = threadIdx.x >> 2, o = threadIdx.x & 3;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int HW = H * W;
    const uint4 *yv = reinterpret_cast<const uint4 *>(y3);
    float acc[9][8];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[tap][k] = 0.f;
    float gsum = 0.f;
    // summed over the activation pixel q = p + d off(tap): each activation is
    // loaded and converted once, and the nine taps take the output gradient at
    // q - d off(tap) (a scalar shared by the pixel's four lanes); the pairs
    // (p, q) are those with both pixels in the image, as in the definition
    for (int q0 = blockIdx.x * 64; q0 < NP; q0 += gridDim.x * 64) {
        const int gq = q0 + ps;
        if (gq >= NP) break;
        const int pq = gq % HW, qy = pq / W, qx = pq - qy * W;
        const uint4 yv4 = yv[static_cast<unsigned>(gq) * (kCh / 8) + o];
        float gt[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = d * (tap / 3 - 1), dx = d * (tap % 3 - 1);
            const bool ok = qy - dy >= 0 && qy - dy < H && qx - dx >= 0 && qx - dx < W;
            const float gvl = g4[ok ? gq - dy * W - dx : gq];
            gt[tap] = ok ? gvl : 0.f;
        }
        gsum += gt[4];  // the centre tap: every pixel's own gradient once
        const unsigned w4[4] = {yv4.x, yv4.y, yv4.z, yv4.w};
        float yf[8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            yf[2 * e] = __uint_as_float(w4[e] << 16);
            yf[2 * e + 1] = __uint_as_float(w4[e] & 0xffff0000u);
        }
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[tap][k] += gt[tap] * yf[k];
    }
    // butterfly over the 16 pixel lanes of each octet (lane bits 2..5)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            float a = acc[tap][k];
            a += __shfl_xor(a, 4);
            a += __shfl_xor(a, 8);
            a += __shfl_xor(a, 16);
            a += __shfl_xor(a, 32);
            acc[tap][k] = a;
        }
    gsum += __shfl_xor(gsum, 4);
    gsum += __shfl_xor(gsum, 8);
    gsum += __shfl_xor(gsum, 16);
    gsum += __shfl_xor(gsum, 32);
    __shared__ float red[4][kW4 + 1];
    if (lane < 4) {
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int k = 0; k < 8; ++k) red[wave][tap * kCh + 8 * lane + k] = acc[tap][k];
        if (lane == 0) red[wave][kW4] = gsum;
    }
    __syncthreads();
    for (int el = threadIdx.x; el <= kW4; el += kThreads)
        part[static_cast<size_t>(blockIdx.x) * (kW4 + 1) + el] = ((red[0][el] + red[1][el]) + red[2][el]) + red[3][el];
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
// per-image max |f| and max |s| over the interior pixels: workgroup (b, sl)
// takes slice sl of image b (loads issued unconditionally, the mask applied by
// a select) and folds its maxima into bits[2b], bits[2b+1] (zeroed before) by
// an integer max of the FP64 bit patterns, whose order is that of the values
// for non-negative numbers (exact, and the same in any order)
constexpr int kNormSlices = 16;
__global__ __launch_bounds__(kThreads) void k_norms(const double *__restrict__ f, const double *__restrict__ s,
                                                    const uint8_t *__restrict__ mask,
                                                    unsigned long long *__restrict__ bits, int HW) {
    const int b = blockIdx.x / kNormSlices, sl = blockIdx.x - b * kNormSlices;
    const int p0 = static_cast<int>(static_cast<long long>(HW) * sl / kNormSlices);
    const int p1 = static_cast<int>(static_cast<long long>(HW) * (sl + 1) / kNormSlices);
    const size_t ib = static_cast<size_t>(b) * HW;
    double mf = 0.0, ms = 0.0;
    for (int p = p0 + static_cast<int>(threadIdx.x); p < p1; p += kThreads) {
        const bool m = mask[p] != 0;
        const double fv = fabs(f[ib + p]), sv = fabs(s[ib + p]);
        mf = fmax(mf, m ? fv : 0.0);
        ms = fmax(ms, m ? sv : 0.0);
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
        atomicMax(bits + 2 * b, static_cast<unsigned long long>(__double_as_longlong(rf[0])));
        atomicMax(bits + 2 * b + 1, static_cast<unsigned long long>(__double_as_longlong(rs[0])));
    }
}

// fn[b], sn[b] from the folded maxima (1 where the maximum is 0; fmax has
// dropped NaN values, as it does in the maxima above)
__global__ void k_norms_fin(const unsigned long long *__restrict__ bits, double *__restrict__ fn,
                            double *__restrict__ sn, int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double vf = __longlong_as_double(static_cast<long long>(bits[2 * b]));
    const double vs = __longlong_as_double(static_cast<long long>(bits[2 * b + 1]));
    fn[b] = vf > 0.0 ? vf : 1.0;
    sn[b] = vs > 0.0 ? vs : 1.0;
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

// Coarse grid of H x W nodes inside a fine grid of Hf = r (H - 1) + 1 by
// Wf = r (W - 1) + 1 nodes, coarse node (i, j) on fine node (r i, r j).
// Restriction: interior coarse nodes take the tent-weighted mean over the
// (2r - 1)^2 fine nodes around their fine node, weights (r - |dy|)(r - |dx|) / r^4
// (separable, each factor summing to one); boundary coarse nodes take their
// fine node's value.  One workgroup per (coarse row, image): the column
// sums of the row's fine band go to LDS with coalesced row reads, then the
// row sums are formed from LDS.
__global__ void k_restrict(const double *__restrict__ fine, double *__restrict__ coarse, int H, int W, int r) {
    extern __shared__ double colsum[];  // Wf
    const int i = blockIdx.x, b = blockIdx.y;
    const int Hf = r * (H - 1) + 1, Wf = r * (W - 1) + 1;
    const double *fb = fine + static_cast<size_t>(b) * Hf * Wf;
    double *cb = coarse + (static_cast<size_t>(b) * H + i) * W;
    const double inv = 1.0 / (static_cast<double>(r) * r);
    const bool edge = i == 0 || i == H - 1;
    if (!edge) {
        for (int x = threadIdx.x; x < Wf; x += blockDim.x) {
            const double *p = fb + static_cast<size_t>(r * i) * Wf + x;
            double acc = r * p[0];
            for (int d = 1; d < r; ++d) acc += (r - d) * (p[-static_cast<ptrdiff_t>(d) * Wf] + p[static_cast<ptrdiff_t>(d) * Wf]);
            colsum[x] = acc * inv;
        }
    }
    __syncthreads();
    for (int j = threadIdx.x; j < W; j += blockDim.x) {
        double v;
        if (edge || j == 0 || j == W - 1) {
            v = fb[static_cast<size_t>(r * i) * Wf + r * j];
        } else {
            const double *q = colsum + r * j;
            v = r * q[0];
            for (int d = 1; d < r; ++d) v += (r - d) * (q[-d] + q[d]);
            v *= inv;
        }
        cb[j] = v;
    }
}

// u = s + |s|_inf * (P out) on interior fine nodes, 0 elsewhere; P the
// bilinear interpolation of the coarse output at the fine nodes.
__global__ void k_warm_prolong(const double *__restrict__ s, const double *__restrict__ sn,
                               const float *__restrict__ out, const uint8_t *__restrict__ mask, double *__restrict__ u,
                               int H, int W, int r, int B) {
    const int Hf = r * (H - 1) + 1, Wf = r * (W - 1) + 1;
    const size_t HWf = static_cast<size_t>(Hf) * Wf;
    const size_t gp = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gp >= HWf * B) return;
    const int b = static_cast<int>(gp / HWf);
    const int p = static_cast<int>(gp - b * HWf);
    if (!mask[p]) {
        u[gp] = 0.0;
        return;
    }
    const int y = p / Wf, x = p - y * Wf;
    const int i0 = y / r, j0 = x / r, fy = y - i0 * r, fx = x - j0 * r;
    const int i1 = min(i0 + 1, H - 1), j1 = min(j0 + 1, W - 1);  // weight 0 when clamped
    const float *o = out + static_cast<size_t>(b) * H * W;
    const double v = (static_cast<double>((r - fy) * (r - fx)) * o[i0 * W + j0] +
                      static_cast<double>((r - fy) * fx) * o[i0 * W + j1] +
                      static_cast<double>(fy * (r - fx)) * o[i1 * W + j0] +
                      static_cast<double>(fy * fx) * o[i1 * W + j1]) /
                     (static_cast<double>(r) * r);
    u[gp] = s[gp] + sn[b] * v;
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
    double *lacc = nullptr;  // device: loss sum, step count, last loss
    int *cnt = nullptr;      // device: interior pixels of the last mask
    unsigned long long *nbits = nullptr;  // device: per-image maxima of |f|, |s| (FP64 bits)
    int wblocks = 512;
    int n_cu = 256;  // compute units of the device (set at creation)
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


void convert(adrnn_ctx *c) {
    hipLaunchKernelGGL(k_convert, dim3((kW2 + 255) / 256), dim3(256), 0, c->st, c->P, c->w1, c->w2, c->w3, c->w2t,
                       c->w3t, c->w4);
    NNCHK(hipGetLastError());
}

// last-layer kernels: 64 pixels per workgroup step, at most 1024 workgroups
int last_grid(int NP) { return std::min(1024, std::max(1, (NP + 63) / 64)); }
static_assert(1024 * (kW4 + 1) <= 512 * (kCh * 9 * kCh + kCh), "last-layer partials exceed the partial buffer");

int conv_grid(int NP) { return std::min(4096, std::max(1, (NP + 16 * 4 * 8 - 1) / (16 * 4 * 8))); }

// 32 -> 32 convolution of B images (tiled kernel)
template <int EPI, int D>
void conv32t_launch(adrnn_ctx *c, int B, const bf16_t *x, const bf16_t *w, const float *bias, const bf16_t *ymask,
                    bf16_t *y) {
    const size_t lds = conv_tiled_lds(D);
    const void *fn = reinterpret_cast<const void *>(&k_conv32t<EPI, D>);
    if (lds > 64 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    // one workgroup per resident slot (each walks its tiles)
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kThreads, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    const int ntiles = B * conv_tiles(c->H, c->W);
    const int nb = std::min(ntiles, per_cu * c->n_cu);
    hipLaunchKernelGGL((k_conv32t<EPI, D>), dim3(nb), dim3(kThreads), lds, c->st, x, w, bias, ymask, y, c->H, c->W,
                       ntiles);
    NNCHK(hipGetLastError());
}

// 32 -> 32 convolution of B images (tiled kernel)
template <int EPI>
void conv32t(adrnn_ctx *c, int B, const bf16_t *x, const bf16_t *w, const float *bias, const bf16_t *ymask, bf16_t *y,
             int d) {
    if (d < 1 || d > kMaxDilT) throw NNError{ADR_EINVAL, "tiled convolution: dilation out of range"};
    switch (d) {
        case 1: conv32t_launch<EPI, 1>(c, B, x, w, bias, ymask, y); break;
        case 2: conv32t_launch<EPI, 2>(c, B, x, w, bias, ymask, y); break;
        case 3: conv32t_launch<EPI, 3>(c, B, x, w, bias, ymask, y); break;
        default: conv32t_launch<EPI, 4>(c, B, x, w, bias, ymask, y); break;
    }
}

void forward(adrnn_ctx *c, int B, const bf16_t *x0, float *out) {
    const int NP = B * c->H * c->W, gridc = conv_grid(NP);
    hipLaunchKernelGGL(k_conv_in, dim3(gridc), dim3(kThreads), 0, c->st, x0, c->w1, c->P + ob1, c->y1, NP, c->H,
                       c->W, kDil[0]);
    conv32t<0>(c, B, c->y1, c->w2, c->P + ob2, nullptr, c->y2, kDil[1]);
    conv32t<0>(c, B, c->y2, c->w3, c->P + ob3, nullptr, c->y3, kDil[2]);
    NNCHK(hipGetLastError());
    hipLaunchKernelGGL(k_last_fwd, dim3(last_grid(NP)), dim3(kThreads), 0, c->st, c->y3, c->w4, c->P + ob4, out, NP,
                       c->H, c->W, kDil[3]);
    NNCHK(hipGetLastError());
}

template <int CIN, int D>
int wgrad_launch(adrnn_ctx *c, const bf16_t *g, const bf16_t *x, int NP) {
    const size_t lds = wgrad_lds(CIN, D);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_wgradt<CIN, D>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    const int ntiles = (NP / (c->H * c->W)) * conv_tiles(c->H, c->W);
    const int nb = std::min(c->wblocks, ntiles);
    hipLaunchKernelGGL((k_wgradt<CIN, D>), dim3(nb), dim3(kThreads), lds, c->st, g, x, c->part, ntiles, c->H, c->W);
    NNCHK(hipGetLastError());
    return nb;
}

template <int CIN>
void wgrad(adrnn_ctx *c, const bf16_t *g, const bf16_t *x, int NP, int d, float *dst) {
    int nb = 0;
    if constexpr (CIN == 32) {
        if (d == 2) nb = wgrad_launch<CIN, 2>(c, g, x, NP);
        else if (d == 4) nb = wgrad_launch<CIN, 4>(c, g, x, NP);
    } else {
        switch (d) {
            case 1: nb = wgrad_launch<CIN, 1>(c, g, x, NP); break;
            case 2: nb = wgrad_launch<CIN, 2>(c, g, x, NP); break;
            case 3: nb = wgrad_launch<CIN, 3>(c, g, x, NP); break;
            case 4: nb = wgrad_launch<CIN, 4>(c, g, x, NP); break;
            default: break;
        }
    }
    if (nb == 0)
        throw NNError{ADR_EINVAL, "weight gradient: dilation out of range (32 input channels: 2 or 4; 4 channels: 1..4)"};
    const int len = kCh * 9 * CIN + kCh;
    hipLaunchKernelGGL(k_reduce, dim3((len + 31) / 32), dim3(kThreads), 0, c->st, c->part, nb, len, dst);
    NNCHK(hipGetLastError());
}

// forward, loss (accumulated on the device), backward: no host synchronisation
void grads(adrnn_ctx *c, int B, const bf16_t *x0, const float *tgt, const uint8_t *mask, float *G) {
    const int HW = c->H * c->W, NP = B * HW;
    forward(c, B, x0, c->out);
    // interior pixel count (mask shared by the images), on the device
    NNCHK(hipMemsetAsync(c->cnt, 0, sizeof(int), c->st));
    hipLaunchKernelGGL(k_mask_count, dim3(HW / 16 / kThreads + 1), dim3(kThreads), 0, c->st, mask, HW, c->cnt);
    const int lb = (NP + 255) / 256;
    hipLaunchKernelGGL(k_loss, dim3(lb), dim3(256), 0, c->st, c->out, tgt, mask, c->g4, c->lpart, NP, HW, B, c->cnt);
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(kThreads), 0, c->st, c->lpart, lb, B, c->cnt, c->lacc);
    // layer 4
    // partials of up to 1024 workgroups (289 floats each) fit in the 32 -> 32 layers' buffer
    const int nb = last_grid(NP);
    hipLaunchKernelGGL(k_last_wgrad, dim3(nb), dim3(kThreads), 0, c->st, c->g4, c->y3, c->part, NP, c->H, c->W,
                       kDil[3]);
    hipLaunchKernelGGL(k_reduce, dim3((kW4 + 1 + 31) / 32), dim3(kThreads), 0, c->st, c->part, nb, kW4 + 1, G + oW4);
    hipLaunchKernelGGL(k_last_dgrad, dim3(last_grid(NP)), dim3(kThreads), 0, c->st, c->g4, c->w4, c->y3, c->ga, NP, c->H, c->W,
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
        {
            int dev = 0, ncu = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
                c->n_cu = ncu;
        }
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
        c->lacc = nn_alloc<double>(c, 3);
        c->cnt = nn_alloc<int>(c, 1);
        c->nbits = nn_alloc<unsigned long long>(c, 2 * static_cast<size_t>(max_batch));
        NNCHK(hipMemsetAsync(c->lacc, 0, 3 * sizeof(double), c->st));
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
        NNCHK(hipMemsetAsync(c->nbits, 0, sizeof(unsigned long long) * 2 * B, c->st));
        hipLaunchKernelGGL(k_norms, dim3(B * kNormSlices), dim3(kThreads), 0, c->st, f, s, mask, c->nbits, HW);
        hipLaunchKernelGGL(k_norms_fin, dim3((B + 255) / 256), dim3(256), 0, c->st, c->nbits, fn, sn, B);
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
        grads(c, B, static_cast<const bf16_t *>(x0), target, mask, G);
        if (loss) {
            NNCHK(hipMemcpyAsync(loss, c->lacc + 2, sizeof(double), hipMemcpyDeviceToHost, c->st));
            NNCHK(hipStreamSynchronize(c->st));
        }
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

adr_status adrnn_loss_sum(adrnn_ctx *c, double *sum, int64_t *steps, int32_t reset) {
    if (!c) return ADR_EINVAL;
    try {
        double h[3] = {0.0, 0.0, 0.0};
        NNCHK(hipMemcpyAsync(h, c->lacc, sizeof(h), hipMemcpyDeviceToHost, c->st));
        NNCHK(hipStreamSynchronize(c->st));
        if (sum) *sum = h[0];
        if (steps) *steps = static_cast<int64_t>(h[1]);
        if (reset) NNCHK(hipMemsetAsync(c->lacc, 0, 2 * sizeof(double), c->st));
        return ADR_OK;
    } catch (const NNError &e) {
        return fail(c, e);
    }
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

adr_status adrnn_restrict(adrnn_ctx *c, int32_t B, int32_t r, const double *fine, double *coarse) {
    if (!c || B < 1 || B > c->maxB || r < 1 || !fine || !coarse) return ADR_EINVAL;
    try {
        const int64_t Wf = static_cast<int64_t>(r) * (c->W - 1) + 1, Hf = static_cast<int64_t>(r) * (c->H - 1) + 1;
        if (Wf > kMaxRestrictWidth || Hf * Wf * B > (int64_t(1) << 31))
            throw NNError{ADR_EINVAL, "fine grid too large for adrnn_restrict"};
        hipLaunchKernelGGL(k_restrict, dim3(c->H, B), dim3(256), sizeof(double) * Wf, c->st, fine, coarse, c->H, c->W,
                           static_cast<int>(r));
        NNCHK(hipGetLastError());
        return ADR_OK;
    } catch (const NNError &e) {
        return fail(c, e);
    }
}

adr_status adrnn_warm_start_prolong(adrnn_ctx *c, int32_t B, int32_t r, const double *s, const double *s_norm,
                                    const float *out, const uint8_t *mask, double *u) {
    if (!c || B < 1 || B > c->maxB || r < 1 || !s || !s_norm || !out || !mask || !u) return ADR_EINVAL;
    try {
        const int64_t NPf = (static_cast<int64_t>(r) * (c->H - 1) + 1) * (static_cast<int64_t>(r) * (c->W - 1) + 1) * B;
        if (NPf > (int64_t(1) << 31)) throw NNError{ADR_EINVAL, "fine grid too large for adrnn_warm_start_prolong"};
        hipLaunchKernelGGL(k_warm_prolong, dim3(static_cast<unsigned>((NPf + 255) / 256)), dim3(256), 0, c->st, s,
                           s_norm, out, mask, u, c->H, c->W, static_cast<int>(r), static_cast<int>(B));
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
