// Learned smoother: a bias-free 3x3 convolutional network
//   s -> conv 1->16, ReLU -> conv 16->16, ReLU -> conv 16->16, ReLU -> conv 16->1
// applied to the scaled residual s = D^-1 (f - A u) of the finest level
// (u <- u + N(s)), and its training with the energy-norm loss.
//
// Storage: activations NHWC bfloat16 with 16 channels, element (b, y, x, c)
// at ((b H + y) W + x) 16 + c; 1-channel maps float [b][y][x].  Weights: FP32
// master copy in the order W[layer][co][ci][ky][kx] (4896 numbers) and
// derived bf16 copies: per 16->16 layer and tap t = 3 ky + kx, WF[t][co][ci]
// (forward B operand) and WD[t][ci][co] (data-gradient B operand); the
// 1-channel layers keep bf16-rounded floats W1[co][t], W4[ci][t].
// Output pixel (y, x) of a layer reads input (y + ky - 1, x + kx - 1); zero
// padding outside the map.
//
// MFMA (v_mfma_f32_16x16x16_bf16, 64 lanes): D[i][j] += sum_k A[i][k] B[k][j],
// lane l supplies A[l%16][4(l/16)+q] and B[4(l/16)+q][l%16], q = 0..3, and
// receives D[4(l/16)+q][l%16].  A 16->16 layer is an implicit GEMM: 16 pixels
// of a row (i) x 16 output channels (j), accumulated over 9 taps of 16
// input channels (k).
#include "dev_common.h"

namespace mgx {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

static constexpr int kW1 = 0, kW2 = 144, kW3 = 144 + 2304, kW4 = 144 + 2 * 2304, kNW = 4896;

__device__ __forceinline__ float bfr(float x) { return bf16_round(x); }
__device__ __forceinline__ short bfs(float x) { return (short)f32_to_bf16(x); }
// ReLU that keeps NaN (fmaxf would turn it into 0 and hide a bad network)
__device__ __forceinline__ float relu(float x) { return x < 0.f ? 0.f : x; }

// ---- weight preparation: FP32 master -> bf16 copies --------------------------
__global__ void k_lprep(const float *w, LearnedW d)
{
    // the fused step's MFMA operands, zero-padded
    constexpr int nk = 5 * 16 * 32;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < 256 + 3 * nk; q += blockDim.x * gridDim.x) {
        if (q < 256) {
            const int co = q / 16, tap = q % 16;
            d.w1m[q] = tap < 9 ? f32_to_bf16(w[kW1 + co * 9 + tap]) : (bf16_t)0;
            continue;
        }
        const int r = (q - 256) % nk, which = (q - 256) / nk;  // 0: layer 2, 1: layer 3, 2: layer 4
        const int b = r / 512, row = (r / 32) % 16, k = r % 32;
        const int tap = 2 * b + k / 16, ch = k % 16;
        float v = 0.f;
        if (tap < 9) {
            if (which == 0) v = w[kW2 + (row * 16 + ch) * 9 + tap];
            else if (which == 1) v = w[kW3 + (row * 16 + ch) * 9 + tap];
            else if (row == 0) v = w[kW4 + ch * 9 + tap];
        }
        bf16_t *dst = which == 0 ? d.w2k : which == 1 ? d.w3k : d.w4k;
        dst[r] = f32_to_bf16(v);
    }
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < kNW; q += blockDim.x * gridDim.x) {
        const float v = w[q];
        if (q < kW2) {
            d.w1[q] = bfr(v);  // [co][ci=0][t] -> [co][t]
        } else if (q < kW4) {
            const int base = q < kW3 ? kW2 : kW3;
            const int r = q - base;  // [co][ci][t]
            const int co = r / 144, ci = (r / 9) % 16, t = r % 9;
            bf16_t *wf = q < kW3 ? d.wf2 : d.wf3;
            bf16_t *wd = q < kW3 ? d.wd2 : d.wd3;
            wf[(t * 16 + co) * 16 + ci] = f32_to_bf16(v);
            wd[(t * 16 + ci) * 16 + co] = f32_to_bf16(v);
        } else {
            d.w4[q - kW4] = bfr(v);  // [co=0][ci][t] -> [ci][t]
        }
    }
}

// ---- layer 1: s (float) -> relu(conv 1->16) (bf16 NHWC16) -------------------
// `s` is read as bf16-rounded values.  One thread per pixel.
__global__ __launch_bounds__(256) void k_lconv_in(const float *s, const int *idx, int B, int H, int W,
                                                  const float *w1, bf16_t *x1)
{
    const long long npx = (long long)B * H * W;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npx;
         p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((long long)W * H));
        const long long sb = (long long)(idx ? idx[b] : b) * H * W;
        float in[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            in[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? bfr(s[sb + (long long)yy * W + xx]) : 0.f;
        }
        short o[16];
#pragma unroll
        for (int co = 0; co < 16; ++co) {
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) acc += w1[co * 9 + t] * in[t];
            o[co] = bfs(relu(acc));
        }
        uint4 v0, v1;
        __builtin_memcpy(&v0, &o[0], 16);
        __builtin_memcpy(&v1, &o[8], 16);
        uint4 *dst = (uint4 *)(x1 + p * 16);
        dst[0] = v0;
        dst[1] = v1;
    }
}

// ---- 16 -> 16 layers on MFMA --------------------------------------------------
// One wavefront computes 16 consecutive pixels of one row x 16 channels.
// mode 0 (forward):  out[p][co] = bf16(relu(sum_t sum_ci WF[t][co][ci] in[p + t][ci]))
// mode 1 (data gradient): out[p][ci] = bf16(mask(p, ci) * sum_t sum_co WD[t][ci][co] in[p - t][co]),
//   mask = act[p][ci] > 0 (the forward activation of this layer's input), so
//   the result is the gradient with respect to the previous pre-activation.
template <int MODE>
__global__ __launch_bounds__(256) void k_lconv16(const bf16_t *in, bf16_t *out, const bf16_t *wt, const bf16_t *act,
                                                  int B, int H, int W)
{
    const int lane = threadIdx.x & 63;
    const int tiles_x = (W + 15) / 16;
    const long long ntiles = (long long)B * H * tiles_x;
    const long long tile = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    const int tx = (int)(tile % tiles_x), y = (int)((tile / tiles_x) % H), b = (int)(tile / ((long long)tiles_x * H));
    const int i = lane & 15, kq = (lane >> 4) * 4;
    const int x0 = tx * 16;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int ky = t / 3, kx = t % 3;
        const int yy = MODE == 0 ? y + ky - 1 : y - ky + 1;
        const int xx = MODE == 0 ? x0 + i + kx - 1 : x0 + i - kx + 1;
        v4s a = {0, 0, 0, 0};
        if (yy >= 0 && yy < H && xx >= 0 && xx < W)
            a = *(const v4s *)(in + (((long long)b * H + yy) * W + xx) * 16 + kq);
        const v4s bw = *(const v4s *)(wt + (t * 16 + i) * 16 + kq);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bw, acc, 0, 0, 0);
    }
    // lane holds pixels x0 + kq + q, channel i
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int x = x0 + kq + q;
        if (x >= W) continue;
        const long long o = (((long long)b * H + y) * W + x) * 16 + i;
        float v = acc[q];
        if (MODE == 0) v = relu(v);
        else v = (bf16_to_f32(act[o]) > 0.f) ? v : 0.f;
        out[o] = f32_to_bf16(v);
    }
}

// ---- layer 4 (training): y[p] = sum_t sum_ci W4[ci][t] x3[p + t][ci] (float) ----
__global__ __launch_bounds__(256) void k_lconv_out(const bf16_t *x3, const float *w4, int B, int H, int W, float *y)
{
    const long long npx = (long long)B * H * W;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npx;
         p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % W), yy0 = (int)((p / W) % H), b = (int)(p / ((long long)W * H));
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = yy0 + t / 3 - 1, xx = x + t % 3 - 1;
            if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
            const bf16_t *src = x3 + (((long long)b * H + yy) * W + xx) * 16;
#pragma unroll
            for (int ci = 0; ci < 16; ++ci) acc += w4[ci * 9 + t] * bf16_to_f32(src[ci]);
        }
        y[p] = acc;
    }
}

// The solver's learned update: e[p] += N(s)[p] for the FP32 / bf16 state of
// the finest level (contiguous n x n).
template <class S>
__global__ __launch_bounds__(256) void k_lupdate(const bf16_t *x3, const float *w4, int n, S *e)
{
    using T = Traits<S>;
    const long long npx = (long long)n * n;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npx;
         p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % n), y = (int)(p / n);
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            if (yy < 0 || yy >= n || xx < 0 || xx >= n) continue;
            const bf16_t *src = x3 + ((long long)yy * n + xx) * 16;
#pragma unroll
            for (int ci = 0; ci < 16; ++ci) acc += w4[ci * 9 + t] * bf16_to_f32(src[ci]);
        }
        T::st(e + p, T::rnd(T::ld(e + p) + acc));
    }
}

// ---- scaled residual of the FP32 inner problem: s = (f - A e) / D ------------
// Diffusion 5-point operator with harmonic face means of the nodal a (float,
// (n+2)^2), h^2 cancels: s = (h^2 f - (D' e - sum w e_nbr)) / D' with D' the
// face sum.
template <class S>
__global__ __launch_bounds__(256) void k_lscaled(const S *e, const float *f, const float *a, int n, double h2,
                                                 float *s)
{
    using T = Traits<S>;
    const long long npx = (long long)n * n;
    const int an = n + 2;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npx;
         p += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(p % n) + 1, j = (int)(p / n) + 1;
        auto ev = [&](int ii, int jj) -> float {
            return (ii >= 1 && ii <= n && jj >= 1 && jj <= n) ? T::ld(e + (long long)(jj - 1) * n + (ii - 1)) : 0.f;
        };
        const float ac = a[(long long)j * an + i];
        auto hm = [&](float q) { return 2.f * ac * q / (ac + q); };
        const float ww = hm(a[(long long)j * an + i - 1]), we = hm(a[(long long)j * an + i + 1]);
        const float ws = hm(a[(long long)(j - 1) * an + i]), wn = hm(a[(long long)(j + 1) * an + i]);
        const float ec = ev(i, j);
        const float Ae = ((ww * (ec - ev(i - 1, j)) + we * (ec - ev(i + 1, j))) + ws * (ec - ev(i, j - 1))) +
                         wn * (ec - ev(i, j + 1));
        const float dsum = ((ww + we) + ws) + wn;
        s[p] = ((float)h2 * f[p] - Ae) / dsum;
    }
}

// ---- energy-norm loss and its gradient with respect to the network output ---
// Per patch b (one block each): w = e - y on the window V = [border, P-border)^2,
// E = sum_faces_in_V a_f (w_p - w_q)^2, E0 = the same for e (precomputed),
// dy = -(2 / B) (A_V w) / E0, loss_b = E / E0.
__global__ __launch_bounds__(256) void k_lloss(const float *y, const float *e, const float *a, const float *E0,
                                               const int *idx, int B, int P, int border, float *dy, float *loss_b)
{
    const int b = blockIdx.x;
    const long long pb = (long long)(idx ? idx[b] : b) * P * P;
    const float inv = -2.f / ((float)B * E0[b]);
    __shared__ float red[256];
    float part = 0.f;
    for (int p = threadIdx.x; p < P * P; p += blockDim.x) {
        const int x = p % P, yy = p / P;
        const bool in = x >= border && x < P - border && yy >= border && yy < P - border;
        float g = 0.f;
        const float wc = e[pb + p] - y[(long long)b * P * P + p];
        const float ac = a[pb + p];
        auto nb = [&](int xx, int yq) -> float {
            return e[pb + (long long)yq * P + xx] - y[(long long)b * P * P + (long long)yq * P + xx];
        };
        auto hm = [&](int xx, int yq) { const float q = a[pb + (long long)yq * P + xx]; return 2.f * ac * q / (ac + q); };
        if (in) {
            const int dxs[4] = {-1, 1, 0, 0}, dys[4] = {0, 0, -1, 1};
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const int xx = x + dxs[f], yq = yy + dys[f];
                if (xx < border || xx >= P - border || yq < border || yq >= P - border) continue;
                const float d = wc - nb(xx, yq);
                const float af = hm(xx, yq);
                g += af * d;
                if (f == 1 || f == 3) part += af * d * d;  // each face once: right and down
            }
        }
        dy[(long long)b * P * P + p] = inv * g;
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_b[b] = red[0] / E0[b];
}

// E0[b] = E_V(e) of the b-th patch of the batch
__global__ __launch_bounds__(256) void k_lenergy(const float *e, const float *a, const int *idx, int P, int border,
                                                 float *E0)
{
    const int q = blockIdx.x;
    const long long pb = (long long)(idx ? idx[q] : q) * P * P;
    __shared__ float red[256];
    float part = 0.f;
    for (int p = threadIdx.x; p < P * P; p += blockDim.x) {
        const int x = p % P, y = p / P;
        if (x < border || x >= P - border || y < border || y >= P - border) continue;
        const float ac = a[pb + p], ec = e[pb + p];
        if (x + 1 < P - border) {
            const float q2 = a[pb + p + 1], d = ec - e[pb + p + 1];
            part += 2.f * ac * q2 / (ac + q2) * d * d;
        }
        if (y + 1 < P - border) {
            const float q2 = a[pb + p + P], d = ec - e[pb + p + P];
            part += 2.f * ac * q2 / (ac + q2) * d * d;
        }
    }
    red[threadIdx.x] = part;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) E0[q] = red[0];
}

// ---- backward through layer 4 (16 -> 1) ---------------------------------------
// dz3[p][ci] = bf16( [x3[p][ci] > 0] * sum_t W4[ci][t] dy[p - t] )
__global__ __launch_bounds__(256) void k_lbwd_out(const float *dy, const bf16_t *x3, const float *w4, int B, int H,
                                                  int W, bf16_t *dz3)
{
    const long long npx = (long long)B * H * W;
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npx;
         p += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((long long)W * H));
        float d[9];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y - t / 3 + 1, xx = x - t % 3 + 1;
            d[t] = (yy >= 0 && yy < H && xx >= 0 && xx < W) ? dy[((long long)b * H + yy) * W + xx] : 0.f;
        }
        short o[16];
#pragma unroll
        for (int ci = 0; ci < 16; ++ci) {
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t < 9; ++t) acc += w4[ci * 9 + t] * d[t];
            o[ci] = bfs(bf16_to_f32(x3[p * 16 + ci]) > 0.f ? acc : 0.f);
        }
        uint4 v0, v1;
        __builtin_memcpy(&v0, &o[0], 16);
        __builtin_memcpy(&v1, &o[8], 16);
        uint4 *dst = (uint4 *)(dz3 + p * 16);
        dst[0] = v0;
        dst[1] = v1;
    }
}

// ---- weight gradients: per-block partials, reduced in block order -----------
// 16->16 layer (MFMA, K = pixels): for tap t, G_t[ci][co] = sum_p in[p + t][ci] dz[p][co].
// Each wavefront takes a run of 16-pixel row tiles; a block's 4 wavefronts add
// in a fixed order; the block writes partial[block][t][ci][co] (FP32).
__global__ __launch_bounds__(256) void k_lwgrad16(const bf16_t *in, const bf16_t *dz, int B, int H, int W,
                                                  int tiles_per_wave, float *partial)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tiles_x = (W + 15) / 16;
    const long long ntiles = (long long)B * H * tiles_x;
    const int ci = lane & 15, kq = (lane >> 4) * 4;  // A row = ci; B col = co = lane & 15
    v4f acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
    const long long first = ((long long)blockIdx.x * 4 + wv) * tiles_per_wave;
    for (int k = 0; k < tiles_per_wave; ++k) {
        const long long tile = first + k;
        if (tile >= ntiles) break;
        const int tx = (int)(tile % tiles_x), y = (int)((tile / tiles_x) % H), b = (int)(tile / ((long long)tiles_x * H));
        const int x0 = tx * 16;
        // B operand: dz at pixels x0 + kq + q, channel co = lane & 15
        v4s bz;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int x = x0 + kq + q;
            bz[q] = (x < W) ? (short)dz[(((long long)b * H + y) * W + x) * 16 + (lane & 15)] : (short)0;
        }
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1;
            v4s ax;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int x = x0 + kq + q;  // output pixel p
                const int xx = x + t % 3 - 1;
                const bool ok = x < W && yy >= 0 && yy < H && xx >= 0 && xx < W;
                ax[q] = ok ? (short)in[(((long long)b * H + yy) * W + xx) * 16 + ci] : (short)0;
            }
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ax, bz, acc[t], 0, 0, 0);
        }
    }
    // lane holds G_t[ci = kq + q][co = lane & 15]; add the 4 wavefronts in order
    __shared__ float sh[4][9][256];
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) sh[wv][t][(kq + q) * 16 + (lane & 15)] = acc[t][q];
    __syncthreads();
    for (int e = threadIdx.x; e < 9 * 256; e += blockDim.x) {
        const int t = e / 256, r = e % 256;
        const float v = ((sh[0][t][r] + sh[1][t][r]) + sh[2][t][r]) + sh[3][t][r];
        partial[(long long)blockIdx.x * 2304 + e] = v;  // [t][ci][co]
    }
}

// 1-channel layers (VALU): layer 1 G[co][t] = sum_p dz1[p][co] s[p + t];
// layer 4 G[ci][t] = sum_p dy[p] x3[p + t][ci].  Each block: a run of pixels,
// fixed-order tree reduction, partial[block][16][9].
template <int LAYER>
__global__ __launch_bounds__(256) void k_lwgrad1(const float *s, const int *idx, const bf16_t *act16,
                                                 const float *dy, int B, int H, int W, int px_per_block,
                                                 float *partial)
{
    __shared__ float red[256];
    const long long npx = (long long)B * H * W;
    const long long p0 = (long long)blockIdx.x * px_per_block;
    float acc[144];
#pragma unroll
    for (int k = 0; k < 144; ++k) acc[k] = 0.f;
    for (long long p = p0 + threadIdx.x; p < min(npx, p0 + px_per_block); p += blockDim.x) {
        const int x = (int)(p % W), y = (int)((p / W) % H), b = (int)(p / ((long long)W * H));
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
            const bool ok = yy >= 0 && yy < H && xx >= 0 && xx < W;
            if (LAYER == 1) {
                const long long sb = (long long)(idx ? idx[b] : b) * H * W;
                const float sv = ok ? bfr(s[sb + (long long)yy * W + xx]) : 0.f;
#pragma unroll
                for (int co = 0; co < 16; ++co) acc[co * 9 + t] += bf16_to_f32(act16[p * 16 + co]) * sv;
            } else {
                const float d = dy[p];
#pragma unroll
                for (int ci = 0; ci < 16; ++ci) {
                    const float xv = ok ? bf16_to_f32(act16[(((long long)b * H + yy) * W + xx) * 16 + ci]) : 0.f;
                    acc[ci * 9 + t] += d * xv;
                }
            }
        }
    }
    for (int k = 0; k < 144; ++k) {
        red[threadIdx.x] = acc[k];
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[(long long)blockIdx.x * 144 + k] = red[0];
        __syncthreads();
    }
}

// Sum partials over blocks (in block order) into the flat FP32 gradient:
// g[off + map(e)] = sum_b partial[b][e].  For 16->16 layers partial entries are
// [t][ci][co] and the flat order is [co][ci][t].
__global__ void k_lreduce(const float *partial, int nblocks, int nper, int layout16, float *g)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nper; e += blockDim.x * gridDim.x) {
        float acc = 0.f;
        for (int b = 0; b < nblocks; ++b) acc += partial[(long long)b * nper + e];
        int dst = e;
        if (layout16) {
            const int t = e / 256, ci = (e / 16) % 16, co = e % 16;
            dst = (co * 16 + ci) * 9 + t;
        }
        g[dst] = acc;
    }
}

// Number of entries of order[0..cnt) outside [0, npairs), written to *bad
// (one block; guards the pair gathers against a bad caller order).
__global__ __launch_bounds__(256) void k_lcheck(const int *order, long long cnt, int npairs, int *bad)
{
    __shared__ int red[256];
    int c = 0;
    for (long long q = threadIdx.x; q < cnt; q += blockDim.x) {
        const int v = order[q];
        c += (v < 0 || v >= npairs) ? 1 : 0;
    }
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *bad = red[0];
}

// acc[0] (+)= sum of the batch's per-patch losses, in a fixed order
__global__ void k_lacc(const float *lossb, int B, int reset, double *acc)
{
    if (threadIdx.x != 0) return;
    double t = reset ? 0.0 : acc[0];
    for (int b = 0; b < B; ++b) t += lossb[b];
    acc[0] = t;
}

// Adam on the FP32 master weights (t = step number, 1-based).
__global__ void k_ladam(float *w, const float *g, float *m, float *v, int t, float lr, float b1, float b2, float eps)
{
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < kNW; q += blockDim.x * gridDim.x) {
        const float gq = g[q];
        const float mq = b1 * m[q] + (1.f - b1) * gq;
        const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
        m[q] = mq;
        v[q] = vq;
        const float mh = mq / (1.f - powf(b1, (float)t));
        const float vh = vq / (1.f - powf(b2, (float)t));
        w[q] -= lr * mh / (sqrtf(vh) + eps);
    }
}

// Training pairs: crop P x P patches at (y0, x0) (0-based interior offsets) of
// s = D^-1 (f - A u_k) (FP64 full-grid, given), e = u_star - u_k and the nodal
// coefficient (interior nodes), as float.
__global__ void k_lcrop(const double *s, const double *ustar, const double *uk, const double *a, int n, const int *y0,
                        const int *x0, int ncrops, int P, float *S, float *E, float *A)
{
    const long long tot = (long long)ncrops * P * P;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < tot; q += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(q / ((long long)P * P));
        const int r = (int)(q % ((long long)P * P));
        const int yc = y0[c], xc = x0[c];
        if (yc < 0 || xc < 0 || yc > n - P || xc > n - P) {  // crop outside the grid: NaN, no read
            S[q] = E[q] = A[q] = __builtin_nanf("");
            continue;
        }
        const int y = yc + r / P, x = xc + r % P;
        const long long o = (long long)y * n + x;
        S[q] = (float)s[o];
        E[q] = (float)(ustar[o] - uk[o]);
        A[q] = (float)a[(long long)(y + 1) * (n + 2) + (x + 1)];
    }
}

// ---- fused learned step (the solver's finest-level smoother) ----------------
// e_out = e_in + N(s), s = D^-1 (f - A e_in), for one tile of kTX x kTY outputs
// per workgroup.  The network's receptive field is 9 x 9, so the tile needs s
// on a ring of 4 more pixels, x1 on 3, x2 on 2, x3 on 1; all of them live in
// LDS (x3 reuses x1's space).  Pixels outside the domain are 0 in every map,
// as zero padding of each layer demands.
//
// Every layer runs on MFMA with the weights as the A operand (rows = output
// channels) and the activations as B (columns = 16 pixels of a row): lane
// (i = l % 16, g = l / 16) supplies W[co = i][k = 4g .. 4g+3] and the inputs
// X[k = 4g .. 4g+3][pixel i], and receives D[co = 4g .. 4g+3][pixel i] --
// four consecutive channels of one pixel, stored as one 8-byte LDS write.
// Layer 1 puts the 9 taps of its single input channel on k; layer 4 keeps
// only output row 0.  Products of bf16 values are exact; sums are FP32.
constexpr int kTX = 64, kTY = 8;
constexpr int kSX = kTX + 8, kSY = kTY + 8;  // s: origin (-4, -4)
constexpr int k1X = kTX + 6, k1Y = kTY + 6;  // x1: origin (-3, -3)
constexpr int k2X = kTX + 4, k2Y = kTY + 4;  // x2: origin (-2, -2)
constexpr int k3X = kTX + 2, k3Y = kTY + 2;  // x3: origin (-1, -1)
constexpr int kFusedThreads = 512;
constexpr int kFusedWaves = kFusedThreads / 64;

__device__ __forceinline__ v4f mfma_wx(v4s w, v4s x, v4f acc)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(w, x, acc, 0, 0, 0);
}
// K = 32: lane (i, g) supplies W[row i][k = 8g .. 8g+7] and X[k = 8g .. 8g+7][pixel i]
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
__device__ __forceinline__ v4f mfma_wx32(bf8_t w, bf8_t x, v4f acc)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, x, acc, 0, 0, 0);
}

// relu (or 0 outside the domain) of four channels, packed as bf16 into 8 bytes
__device__ __forceinline__ uint2 pack_act(v4f acc, bool inside)
{
    const float v0 = inside ? relu(acc[0]) : 0.f, v1 = inside ? relu(acc[1]) : 0.f;
    const float v2 = inside ? relu(acc[2]) : 0.f, v3 = inside ? relu(acc[3]) : 0.f;
    return make_uint2(f32x2_to_bf16x2(v0, v1), f32x2_to_bf16x2(v2, v3));
}

// The 9 taps x 16 channels of a 16-pixel row segment as five K = 32 B
// operands: block b holds taps 2b (k 0..15) and 2b+1 (k 16..31; tap 9 reads
// tap 8's address and meets zero weights).
__device__ __forceinline__ void load_taps(const bf16_t *in, int iw, int r, int c0, int i, int g, bf8_t (&x)[5])
{
    const int hi = g >> 1, c8 = 8 * (g & 1);
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        const int t = min(2 * b + hi, 8);
        x[b] = *(const bf8_t *)(in + ((r + t / 3) * iw + c0 + i + t % 3) * 16 + c8);
    }
}

// One 16 -> 16 layer over LDS maps: out (width ow, height oh, origin one pixel
// inside in's) = relu(conv(in)), zero outside the domain.  Each wavefront
// takes row segments of 16 pixels, two at a time (independent MFMA chains);
// the last segment of a row starts at ow - 16 (it overlaps the previous one
// and writes the same values).
template <int IW, int OW, int OH>
__device__ __forceinline__ void lds_conv16(const bf16_t *in, bf16_t *out, const bf8_t *wt, int gx0, int gy0, int n)
{
    constexpr int iw = IW, ow = OW, oh = OH;  // compile-time: the job index math divides by constants
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform: scalar job math
    const int i = lane & 15, g = lane >> 4, kq = 4 * g;
    constexpr int nseg = (ow + 15) / 16;
    constexpr int njobs = oh * nseg;
    for (int job = wv; job < njobs; job += 2 * kFusedWaves) {
        const int job2 = job + kFusedWaves;
        const bool two = job2 < njobs;  // wave-uniform
        const int r1 = job / nseg, c1 = min(16 * (job % nseg), ow - 16);
        const int r2 = two ? job2 / nseg : r1, c2 = two ? min(16 * (job2 % nseg), ow - 16) : c1;
        bf8_t x1[5], x2[5];
        load_taps(in, iw, r1, c1, i, g, x1);
        load_taps(in, iw, r2, c2, i, g, x2);
        v4f a1 = {0.f, 0.f, 0.f, 0.f}, a2 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 5; ++b) {
            a1 = mfma_wx32(wt[b], x1[b], a1);
            a2 = mfma_wx32(wt[b], x2[b], a2);
        }
        {
            const int c = c1 + i, gx = gx0 + c, gy = gy0 + r1;
            *(uint2 *)(out + (r1 * ow + c) * 16 + kq) = pack_act(a1, gx >= 0 && gx < n && gy >= 0 && gy < n);
        }
        if (two) {
            const int c = c2 + i, gx = gx0 + c, gy = gy0 + r2;
            *(uint2 *)(out + (r2 * ow + c) * 16 + kq) = pack_act(a2, gx >= 0 && gx < n && gy >= 0 && gy < n);
        }
    }
}

template <class S>
__global__ __launch_bounds__(kFusedThreads) void k_lstep_fused(const S *ein, S *eout, const float *f, const float *a,
                                                               int n, double h2, LearnedW d)
{
    using T = Traits<S>;
    constexpr int NQ0 = (kSY * kSX + kFusedThreads - 1) / kFusedThreads;
    __shared__ float sl[NQ0 * kFusedThreads];                             // s (padded to whole passes)
    __shared__ float et[kTY * kTX + 1];                                   // e_in on the tile + a spare slot
    __shared__ __attribute__((aligned(16))) bf16_t bufA[k1Y * k1X * 16];  // x1, then x3
    __shared__ __attribute__((aligned(16))) bf16_t bufB[k2Y * k2X * 16];  // x2
    const int tiles_x = (n + kTX - 1) / kTX;
    const int x0 = (blockIdx.x % tiles_x) * kTX, y0 = (blockIdx.x / tiles_x) * kTY;
    const int an = n + 2;
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = lane & 15, kq = (lane >> 4) * 4;
    // s = (h^2 f - A' e) / D' on the tile + 4 (h^2 cancels), bf16-rounded;
    // the tile's own e values are kept for the update.  Branch-free: loads go
    // through buffer descriptors with 32-bit offsets, and a neighbour outside
    // the domain (or any value of a pixel outside it) uses an out-of-range
    // offset, which reads 0 -- the zero boundary values; out-of-domain pixels
    // are selected away.
    {
        const rsrc_t re = make_rsrc(ein, (uint32_t)n * (uint32_t)n * (uint32_t)sizeof(S));
        const rsrc_t rfs = make_rsrc(f, (uint32_t)n * (uint32_t)n * 4u);
        const rsrc_t ras = make_rsrc(a, (uint32_t)an * (uint32_t)an * 4u);
        constexpr uint32_t SB = sizeof(S);
#pragma unroll
        for (int it = 0; it < NQ0; ++it) {
            const int q = threadIdx.x + it * kFusedThreads;
            const bool qok = q < kSY * kSX;
            const int qc = qok ? q : 0;
            const int lx = qc % kSX, ly = qc / kSX;
            const int gx = x0 - 4 + lx, gy = y0 - 4 + ly;
            const bool inside = gx >= 0 && gx < n && gy >= 0 && gy < n;
            const uint32_t pb = (uint32_t)(gy * n + gx);
            const uint32_t o_c = inside ? pb * SB : kOOB;
            const uint32_t o_w = inside && gx >= 1 ? (pb - 1u) * SB : kOOB;
            const uint32_t o_e = inside && gx + 1 < n ? (pb + 1u) * SB : kOOB;
            const uint32_t o_s = inside && gy >= 1 ? (pb - (uint32_t)n) * SB : kOOB;
            const uint32_t o_n = inside && gy + 1 < n ? (pb + (uint32_t)n) * SB : kOOB;
            const float ec = Traits<S>::bload(re, o_c);
            const float e_w = Traits<S>::bload(re, o_w), e_e = Traits<S>::bload(re, o_e);
            const float e_s = Traits<S>::bload(re, o_s), e_n = Traits<S>::bload(re, o_n);
            const uint32_t ab = (uint32_t)((gy + 1) * an + gx + 1) * 4u;
            const uint32_t a_c = inside ? ab : kOOB, a_w = inside ? ab - 4u : kOOB, a_e = inside ? ab + 4u : kOOB;
            const uint32_t a_s = inside ? ab - 4u * (uint32_t)an : kOOB, a_n = inside ? ab + 4u * (uint32_t)an : kOOB;
            const float ac = bld<float>(ras, a_c), aw = bld<float>(ras, a_w), ae = bld<float>(ras, a_e);
            const float as = bld<float>(ras, a_s), anb = bld<float>(ras, a_n);
            const float fv = bld<float>(rfs, o_c == kOOB ? kOOB : pb * 4u);
            // hardware reciprocals (1 ulp): s is rounded to bf16 right after, and
            // IEEE division sequences would make the compiler branch around them
            auto hm = [&](float qq) { return 2.f * ac * qq * __builtin_amdgcn_rcpf(ac + qq); };
            const float ww = hm(aw), we = hm(ae), ws = hm(as), wn = hm(anb);
            const float Ae = ((ww * (ec - e_w) + we * (ec - e_e)) + ws * (ec - e_s)) + wn * (ec - e_n);
            const float dsum = ((ww + we) + ws) + wn;
            const float sv = bfr(((float)h2 * fv - Ae) * __builtin_amdgcn_rcpf(dsum));
            const float v = inside ? sv : 0.f;
            sl[q] = v;  // q past the map lands in the padding
            const int tx = lx - 4, ty = ly - 4;
            const bool own = qok && inside && tx >= 0 && tx < kTX && ty >= 0 && ty < kTY;
            et[own ? ty * kTX + tx : kTY * kTX] = ec;  // others write the spare slot
        }
    }
    // A operands: layer 1 W1[co = i][tap 4g + q]; layers 2, 3 WF[t][co = i][ci];
    // layer 4 W4[ci][t] in row 0 only
    const int g = lane >> 4;
    bf8_t w2v[5], w3v[5], w4v[5];
    const v4s w1v = *(const v4s *)(d.w1m + i * 16 + kq);
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        w2v[b] = *(const bf8_t *)(d.w2k + (b * 16 + i) * 32 + 8 * g);
        w3v[b] = *(const bf8_t *)(d.w3k + (b * 16 + i) * 32 + 8 * g);
        w4v[b] = *(const bf8_t *)(d.w4k + (b * 16 + i) * 32 + 8 * g);
    }
    __syncthreads();
    // layer 1 on the tile + 3: k = the 9 taps of s
    {
        constexpr int nseg = (k1X + 15) / 16;
        for (int job = wv; job < k1Y * nseg; job += kFusedWaves) {
            const int r = job / nseg, sg = job % nseg;
            const int c0 = min(16 * sg, k1X - 16);
            v4s sv;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int tap = min(kq + q, 8);
                const float sv_f = sl[(r + tap / 3) * kSX + c0 + i + tap % 3];
                sv[q] = (short)(kq + q < 9 ? f32_to_bf16(sv_f) : 0);
            }
            const v4f acc = mfma_wx(w1v, sv, (v4f){0.f, 0.f, 0.f, 0.f});
            const int c = c0 + i, gx = x0 - 3 + c, gy = y0 - 3 + r;
            const bool inside = gx >= 0 && gx < n && gy >= 0 && gy < n;
            *(uint2 *)(bufA + (r * k1X + c) * 16 + kq) = pack_act(acc, inside);
        }
    }
    __syncthreads();
    lds_conv16<k1X, k2X, k2Y>(bufA, bufB, w2v, x0 - 2, y0 - 2, n);  // x2 on the tile + 2
    __syncthreads();
    lds_conv16<k2X, k3X, k3Y>(bufB, bufA, w3v, x0 - 1, y0 - 1, n);  // x3 on the tile + 1
    __syncthreads();
    // layer 4 and the update on the tile: output row 0 of D
    {
        constexpr int nseg = kTX / 16;
        for (int job = wv; job < kTY * nseg; job += kFusedWaves) {
            const int r = job / nseg, c0 = 16 * (job % nseg);
            bf8_t x[5];
            load_taps(bufA, k3X, r, c0, i, g, x);
            v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int b = 0; b < 5; ++b) acc = mfma_wx32(w4v[b], x[b], acc);
            const int gx = x0 + c0 + i, gy = y0 + r;
            if (lane < 16 && gx < n && gy < n) {
                const long long p = (long long)gy * n + gx;
                T::st(eout + p, T::rnd(et[r * kTX + c0 + i] + acc[0]));
            }
        }
    }
}

hipError_t learned_step_fused(int st, const void *ein, void *eout, const float *f, const float *a, int n, double h2,
                              const LearnedW &d, hipStream_t s)
{
    const int tiles = ((n + kTX - 1) / kTX) * ((n + kTY - 1) / kTY);
    if (st == ST_F32)
        hipLaunchKernelGGL((k_lstep_fused<float>), dim3(tiles), dim3(kFusedThreads), 0, s, (const float *)ein,
                           (float *)eout, f, a, n, h2, d);
    else
        hipLaunchKernelGGL((k_lstep_fused<bf16_t>), dim3(tiles), dim3(kFusedThreads), 0, s, (const bf16_t *)ein,
                           (bf16_t *)eout, f, a, n, h2, d);
    return hipGetLastError();
}

// ---- launchers -----------------------------------------------------------------
static int lgrid(long long work, int block = 256)
{
    long long g = (work + block - 1) / block;
    return (int)std::min<long long>(std::max<long long>(g, 1), 65536);
}

hipError_t learned_prep(const float *w, const LearnedW &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_lprep, dim3(lgrid(kNW)), dim3(256), 0, s, w, d);
    return hipGetLastError();
}

// Forward of B maps of H x W: s (float, indexed through idx if given) ->
// x1, x2, x3 (bf16 NHWC16); y (float) if given.
hipError_t learned_forward(const float *s, const int *idx, int B, int H, int W, const LearnedW &d, bf16_t *x1,
                           bf16_t *x2, bf16_t *x3, float *y, hipStream_t st)
{
    const long long npx = (long long)B * H * W;
    hipLaunchKernelGGL(k_lconv_in, dim3(lgrid(npx)), dim3(256), 0, st, s, idx, B, H, W, d.w1, x1);
    const long long tiles = (long long)B * H * ((W + 15) / 16);
    const int g16 = (int)((tiles + 3) / 4);
    hipLaunchKernelGGL((k_lconv16<0>), dim3(g16), dim3(256), 0, st, x1, x2, d.wf2, (const bf16_t *)nullptr, B, H, W);
    hipLaunchKernelGGL((k_lconv16<0>), dim3(g16), dim3(256), 0, st, x2, x3, d.wf3, (const bf16_t *)nullptr, B, H, W);
    if (y) hipLaunchKernelGGL(k_lconv_out, dim3(lgrid(npx)), dim3(256), 0, st, x3, d.w4, B, H, W, y);
    return hipGetLastError();
}

// The solver's learned step on the finest inner level (FP32 or bf16 state e,
// FP32 rhs f, float nodal coefficient a): e += N(D^-1 (f - A e)).
hipError_t learned_step(int st, void *e, const float *f, const float *a, int n, double h2, const LearnedW &d,
                        float *sbuf, bf16_t *x1, bf16_t *x2, bf16_t *x3, hipStream_t s)
{
    const long long npx = (long long)n * n;
    if (st == ST_F32)
        hipLaunchKernelGGL((k_lscaled<float>), dim3(lgrid(npx)), dim3(256), 0, s, (const float *)e, f, a, n, h2, sbuf);
    else
        hipLaunchKernelGGL((k_lscaled<bf16_t>), dim3(lgrid(npx)), dim3(256), 0, s, (const bf16_t *)e, f, a, n, h2, sbuf);
    hipError_t r = learned_forward(sbuf, nullptr, 1, n, n, d, x1, x2, x3, nullptr, s);
    if (r != hipSuccess) return r;
    if (st == ST_F32) hipLaunchKernelGGL((k_lupdate<float>), dim3(lgrid(npx)), dim3(256), 0, s, x3, d.w4, n, (float *)e);
    else hipLaunchKernelGGL((k_lupdate<bf16_t>), dim3(lgrid(npx)), dim3(256), 0, s, x3, d.w4, n, (bf16_t *)e);
    return hipGetLastError();
}

size_t learned_train_scratch(int B, int P)
{
    const size_t px = (size_t)B * P * P;
    const size_t tiles = (size_t)B * P * ((P + 15) / 16);
    const size_t blk16 = (tiles + 4 * 8 - 1) / (4 * 8);
    const size_t blk1 = (px + 4095) / 4096;
    size_t b = 0;
    b += 6 * px * 16 * sizeof(bf16_t);                 // x1 x2 x3 dz3 dz2 dz1
    b += 2 * px * sizeof(float);                       // y, dy
    b += 2 * (size_t)B * sizeof(float);                // loss and E0 per patch
    b += std::max(blk16 * 2304, blk1 * 144) * sizeof(float) * 2;  // partials
    b += 3 * kNW * sizeof(float) + 256;                // g, m, v, loss accumulator
    b += 2 * 144 * sizeof(float) + 4 * 2304 * sizeof(bf16_t) + (256 + 3 * 2560) * sizeof(bf16_t);  // copies
    b += 64 * 1024;                                    // alignment slack
    return b;
}

static char *carve_up(char *&p, size_t bytes)
{
    p = (char *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
    char *r = p;
    p += bytes;
    return r;
}

TrainBufs learned_carve(void *scratch, int B, int P)
{
    const size_t px = (size_t)B * P * P;
    const size_t tiles = (size_t)B * P * ((P + 15) / 16);
    const size_t blk16 = (tiles + 4 * 8 - 1) / (4 * 8);
    const size_t blk1 = (px + 4095) / 4096;
    char *p = (char *)scratch;
    TrainBufs t;
    t.x1 = (bf16_t *)carve_up(p, px * 16 * 2);
    t.x2 = (bf16_t *)carve_up(p, px * 16 * 2);
    t.x3 = (bf16_t *)carve_up(p, px * 16 * 2);
    t.dz3 = (bf16_t *)carve_up(p, px * 16 * 2);
    t.dz2 = (bf16_t *)carve_up(p, px * 16 * 2);
    t.dz1 = (bf16_t *)carve_up(p, px * 16 * 2);
    t.y = (float *)carve_up(p, px * 4);
    t.dy = (float *)carve_up(p, px * 4);
    t.lossb = (float *)carve_up(p, (size_t)B * 4);
    t.E0 = (float *)carve_up(p, (size_t)B * 4);
    t.part = (float *)carve_up(p, std::max(blk16 * 2304, blk1 * 144) * 4 * 2);
    t.g = (float *)carve_up(p, kNW * 4);
    t.m = (float *)carve_up(p, kNW * 4);
    t.v = (float *)carve_up(p, kNW * 4);
    t.lacc = (double *)carve_up(p, 256);
    t.d.w1 = (float *)carve_up(p, 144 * 4);
    t.d.w4 = (float *)carve_up(p, 144 * 4);
    t.d.wf2 = (bf16_t *)carve_up(p, 2304 * 2);
    t.d.wd2 = (bf16_t *)carve_up(p, 2304 * 2);
    t.d.wf3 = (bf16_t *)carve_up(p, 2304 * 2);
    t.d.wd3 = (bf16_t *)carve_up(p, 2304 * 2);
    t.d.w1m = (bf16_t *)carve_up(p, 256 * 2);
    t.d.w2k = (bf16_t *)carve_up(p, 2560 * 2);
    t.d.w3k = (bf16_t *)carve_up(p, 2560 * 2);
    t.d.w4k = (bf16_t *)carve_up(p, 2560 * 2);
    return t;
}

// Loss and FP32 gradient (flat, oracle order) of B patches (idx selects them
// from the pair arrays, or null for the first B) at the weights prepared in t.d.
hipError_t learned_loss_grad(const float *S, const float *E, const float *A, const int *idx, int B, int P, int border,
                             TrainBufs &t, float *g, hipStream_t st)
{
    const long long px = (long long)B * P * P;
    hipError_t r = learned_forward(S, idx, B, P, P, t.d, t.x1, t.x2, t.x3, t.y, st);
    if (r != hipSuccess) return r;
    hipLaunchKernelGGL(k_lenergy, dim3(B), dim3(256), 0, st, E, A, idx, P, border, t.E0);
    hipLaunchKernelGGL(k_lloss, dim3(B), dim3(256), 0, st, t.y, E, A, t.E0, idx, B, P, border, t.dy, t.lossb);
    // layer 4
    const int blk1 = (int)((px + 4095) / 4096);
    hipLaunchKernelGGL((k_lwgrad1<4>), dim3(blk1), dim3(256), 0, st, (const float *)nullptr, idx, t.x3, t.dy, B, P, P,
                       4096, t.part);
    hipLaunchKernelGGL(k_lreduce, dim3(1), dim3(256), 0, st, t.part, blk1, 144, 0, g + kW4);
    hipLaunchKernelGGL(k_lbwd_out, dim3(lgrid(px)), dim3(256), 0, st, t.dy, t.x3, t.d.w4, B, P, P, t.dz3);
    const long long tiles = (long long)B * P * ((P + 15) / 16);
    const int tpw = 8;
    const int blk16 = (int)((tiles + 4 * tpw - 1) / (4 * tpw));
    const int g16 = (int)((tiles + 3) / 4);
    // layer 3: weights from (x2, dz3); data gradient dz2 = mask(x2) * conv^T(dz3)
    hipLaunchKernelGGL(k_lwgrad16, dim3(blk16), dim3(256), 0, st, t.x2, t.dz3, B, P, P, tpw, t.part);
    hipLaunchKernelGGL(k_lreduce, dim3(lgrid(2304)), dim3(256), 0, st, t.part, blk16, 2304, 1, g + kW3);
    hipLaunchKernelGGL((k_lconv16<1>), dim3(g16), dim3(256), 0, st, t.dz3, t.dz2, t.d.wd3, t.x2, B, P, P);
    // layer 2
    hipLaunchKernelGGL(k_lwgrad16, dim3(blk16), dim3(256), 0, st, t.x1, t.dz2, B, P, P, tpw, t.part);
    hipLaunchKernelGGL(k_lreduce, dim3(lgrid(2304)), dim3(256), 0, st, t.part, blk16, 2304, 1, g + kW2);
    hipLaunchKernelGGL((k_lconv16<1>), dim3(g16), dim3(256), 0, st, t.dz2, t.dz1, t.d.wd2, t.x1, B, P, P);
    // layer 1
    hipLaunchKernelGGL((k_lwgrad1<1>), dim3(blk1), dim3(256), 0, st, S, idx, t.dz1, (const float *)nullptr, B, P, P,
                       4096, t.part);
    hipLaunchKernelGGL(k_lreduce, dim3(1), dim3(256), 0, st, t.part, blk1, 144, 0, g + kW1);
    return hipGetLastError();
}

hipError_t learned_energy(const float *E, const float *A, const int *idx, int B, int P, int border, float *E0,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_lenergy, dim3(B), dim3(256), 0, st, E, A, idx, P, border, E0);
    return hipGetLastError();
}

hipError_t learned_check_order(const int *order, long long cnt, int npairs, const TrainBufs &t, hipStream_t st)
{
    hipLaunchKernelGGL(k_lcheck, dim3(1), dim3(256), 0, st, order, cnt, npairs, (int *)(t.lacc + 1));
    return hipGetLastError();
}

hipError_t learned_loss_accumulate(const TrainBufs &t, int B, bool reset, hipStream_t st)
{
    hipLaunchKernelGGL(k_lacc, dim3(1), dim3(64), 0, st, t.lossb, B, reset ? 1 : 0, t.lacc);
    return hipGetLastError();
}

hipError_t learned_adam(float *w, const float *g, float *m, float *v, int t, float lr, float b1, float b2, float eps,
                        hipStream_t st)
{
    hipLaunchKernelGGL(k_ladam, dim3(lgrid(kNW)), dim3(256), 0, st, w, g, m, v, t, lr, b1, b2, eps);
    return hipGetLastError();
}

hipError_t learned_crop(const double *s, const double *ustar, const double *uk, const double *a, int n, const int *y0,
                        const int *x0, int ncrops, int P, float *S, float *E, float *A, hipStream_t st)
{
    hipLaunchKernelGGL(k_lcrop, dim3(lgrid((long long)ncrops * P * P)), dim3(256), 0, st, s, ustar, uk, a, n, y0, x0,
                       ncrops, P, S, E, A);
    return hipGetLastError();
}

}  // namespace mgx
