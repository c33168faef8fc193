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

// ---- fused learned step, row-marching form (the default) ---------------------
// A workgroup owns a strip of kMW output columns and R output rows and marches
// down it one row per step.  Each step produces one new row of every map --
// s, x1, x2, x3 and the layer-4 tap partials P -- from rows the previous steps
// left in LDS rings, so no row of any map is computed twice and one barrier a
// step suffices: a map's row r + 1 must be complete (one step earlier) before
// the next map's row r reads it, so each of x1, x2, x3 and the output runs two
// rows behind the map it reads (s rows come in batches ahead, see below).
//
// Layer 4 (16 channels -> 1) runs as P[t][q] = sum_ci W4[ci][t] x3[ci][q]
// for the 9 taps t at every x3 pixel q (one 16 x 16 x 16 MFMA per 16 pixels,
// its B operand the x3 values still in registers), and the output sums the 9
// shifted partials.
//
// Rows are counted from the strip's first s row (rho = row - y0 + 4) and the
// x1, x2 and P rings keep row rho in slot rho & 3; steps run in groups of 4,
// so every slot a step touches is a compile-time constant and every LDS
// address is a per-lane base plus an immediate.
//
// The work of a step is spread over the 4 waves: wave w takes column segment
// w of x1, x2 and x3 and the output row on steps k = w + 2 mod 4; on steps
// k = 0 mod 4 each wave computes one of the next four s rows (its global loads
// issued on the previous such step), so no step waits for a single wave's s
// row.  s rows are thus made up to three steps early: the s ring holds 8 rows
// and copies of rows 0, 1 mod 8 in slots 8, 9, so the three rows a tap window
// needs are consecutive slots from one base.
constexpr int kMW = 56;            // output columns per strip
constexpr int kMS = kMW + 8;       // s row: 64 columns from x0 - 4, one per lane
constexpr int kM1 = kMW + 6;       // x1 row: 62 columns from x0 - 3
constexpr int kM2 = kMW + 4;       // x2 row: 60 columns from x0 - 2
constexpr int kM3 = kMW + 2;       // x3 / P row: 58 columns from x0 - 1
#ifndef MGX_LSTEP_COL
#define MGX_LSTEP_COL 32
#endif
constexpr int kMCol = MGX_LSTEP_COL;  // bytes per column in the x1 and x2 rings (32; 48 measured slower)
constexpr int kMSlot = kM1 * kMCol;   // bytes per slot of the x1 and x2 rings
constexpr int kMRing = 4 * kMSlot + kMCol;  // + one column that zero-weighted reads reach past slot 3
constexpr int kMPT = 60;           // floats per tap row of a P slot (58 used; 60 spreads the taps over the banks)
constexpr int kMSP = 80;           // floats per s ring slot (64 used; 80 spreads the rows over the banks)
constexpr int kMThreads = 256;
constexpr int kMLag = 12;          // steps from a strip's first s row to its first output row
typedef uint32_t u4 __attribute__((ext_vector_type(4)));
template <int V> struct IntC {
    static constexpr int value = V;
};

// relu of four FP32 channels as packed bf16: relu(bf16(x)) == bf16(relu(x))
// (rounding keeps the sign), done as a signed 16-bit max with 0 (a NaN stays
// NaN unless its sign bit is set)
__device__ __forceinline__ uint2 relu_pack(v4f acc)
{
    typedef short s2 __attribute__((ext_vector_type(2)));
    const s2 z = {0, 0};
    const s2 lo = __builtin_elementwise_max(__builtin_bit_cast(s2, f32x2_to_bf16x2(acc[0], acc[1])), z);
    const s2 hi = __builtin_elementwise_max(__builtin_bit_cast(s2, f32x2_to_bf16x2(acc[2], acc[3])), z);
    return make_uint2(__builtin_bit_cast(uint32_t, lo), __builtin_bit_cast(uint32_t, hi));
}

// step kinds: every job's row range checked and out-of-domain values masked
// (pipeline fill and drain), or all jobs on, with or without masking
constexpr int kStepChecked = 0, kStepMasked = 1, kStepInterior = 2;

template <class S>
__global__ __launch_bounds__(kMThreads, 4) void k_lstep_march(const S *ein, S *eout, const float *f, const float *a,
                                                              int n, double h2, LearnedW d, int R)
{
    using T = Traits<S>;
    __shared__ float sr[10 * kMSP];                               // s ring (+ copies)
    __shared__ __attribute__((aligned(16))) char x1r[kMRing];    // x1 ring
    __shared__ __attribute__((aligned(16))) char x2r[kMRing];    // x2 ring
    __shared__ float pr[4 * 9 * kMPT];                            // P ring [slot][tap][column]
    __shared__ float er[16 * kMW];                                // e_in on the output columns
    const int strips = (n + kMW - 1) / kMW;
    const int x0 = (int)(blockIdx.x % strips) * kMW;
    const int y0 = (int)(blockIdx.x / strips) * R;
    const int rows = min(R, n - y0);
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int i = lane & 15, g = lane >> 4, kq = 4 * g, hi = g >> 1;

    // The K order of the operands is chosen so that every lane reads its taps
    // at a fixed base plus immediates.  16 -> 16 layers: block b pairs tap
    // A_b (lane groups 0, 1: channels 0..7, 8..15) with tap B_b (groups 2, 3),
    // B_b one column right of A_b except in block 3 (one row down); block 4's
    // B is a zero-weighted read one column right of tap (2, 2).  Layer 1:
    // group g < 3 takes the three taps of kernel row g (k = 4g .. 4g + 2), the
    // rest of k is zero-weighted.  Taps are t = 3 dy + dx.
    constexpr int kTA[5] = {0, 3, 6, 2, 8}, kTB[5] = {1, 4, 7, 5, -1};
    bf8_t w2v[5], w3v[5];
#pragma unroll
    for (int b = 0; b < 5; ++b) {
        const int t = hi ? kTB[b] : kTA[b];
        const int o = ((t >> 1) * 16 + i) * 32 + (t & 1) * 16 + 8 * (g & 1);  // in the [b][row][k] copies
        const bf8_t z = {};
        w2v[b] = t >= 0 ? *(const bf8_t *)(d.w2k + o) : z;
        w3v[b] = t >= 0 ? *(const bf8_t *)(d.w3k + o) : z;
    }
    v4s w1v, w4t;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        w1v[q] = g < 3 && q < 3 ? (short)d.w1m[i * 16 + 3 * g + q] : (short)0;
        // the P product: row = tap i < 9, k = channel: W4[ch 4g + q][tap i]
        w4t[q] = i < 9 ? (short)d.w4k[(i >> 1) * 512 + (i & 1) * 16 + kq + q] : (short)0;
    }
    // this wave's column segments and per-lane bases: vA* for the tap blocks
    // whose B tap is one column right, vB*p / vB*m for block 3 when the next
    // row's slot is the next slot / three slots back
    const int c1 = min(16 * w, kM1 - 16), c2 = min(16 * w, kM2 - 16), c3 = min(16 * w, kM3 - 16);
    const int lo16 = (g & 1) * 16;
    const int vA2 = (c2 + i) * kMCol + lo16 + hi * kMCol, vA3 = (c3 + i) * kMCol + lo16 + hi * kMCol;
    const int vB2p = (c2 + i) * kMCol + lo16 + hi * kMSlot, vB3p = (c3 + i) * kMCol + lo16 + hi * kMSlot;
    const int vB2m = (c2 + i) * kMCol + lo16 - hi * 3 * kMSlot, vB3m = (c3 + i) * kMCol + lo16 - hi * 3 * kMSlot;
    const int vW1 = (c1 + i) * kMCol + g * 8, vW2 = (c2 + i) * kMCol + g * 8;  // ring stores
    const int vS = min(g, 2) * kMSP + c1 + i;                                    // s taps (floats)
    const int vP = kq * kMPT + c3 + i;                                           // P stores (floats)
    // ring bytes no job writes (padding, x2 columns 60, 61) are read with
    // zero weights only: make them 0, not stale bits
    for (int q = threadIdx.x; q < kMRing / 16; q += kMThreads) {
        ((u4 *)x1r)[q] = u4{0u, 0u, 0u, 0u};
        ((u4 *)x2r)[q] = u4{0u, 0u, 0u, 0u};
    }

    // s row rho = (h^2 f - A' e) / D' over the 64 columns from x0 - 4 (h^2
    // cancels), bf16-rounded, 0 outside the domain; loads through buffer
    // descriptors, out-of-domain neighbours at an out-of-range offset (0)
    const rsrc_t re = make_rsrc(ein, (uint32_t)n * (uint32_t)n * (uint32_t)sizeof(S));
    const rsrc_t rfs = make_rsrc(f, (uint32_t)n * (uint32_t)n * 4u);
    const int an = n + 2;
    const rsrc_t ras = make_rsrc(a, (uint32_t)an * (uint32_t)an * 4u);
    const int sgx = x0 - 4 + lane;
    float pe_c, pe_w, pe_e, pe_s, pe_n, pa_c, pa_w, pa_e, pa_s, pa_n, pf;
    auto sload = [&](int rho) {
        constexpr uint32_t SB = sizeof(S);
        const int gy = y0 - 4 + rho;
        const bool inside = sgx >= 0 && sgx < n && gy >= 0 && gy < n;
        const uint32_t pb = (uint32_t)(gy * n + sgx);
        pe_c = T::bload(re, inside ? pb * SB : kOOB);
        pe_w = T::bload(re, inside && sgx >= 1 ? (pb - 1u) * SB : kOOB);
        pe_e = T::bload(re, inside && sgx + 1 < n ? (pb + 1u) * SB : kOOB);
        pe_s = T::bload(re, inside && gy >= 1 ? (pb - (uint32_t)n) * SB : kOOB);
        pe_n = T::bload(re, inside && gy + 1 < n ? (pb + (uint32_t)n) * SB : kOOB);
        const uint32_t ab = (uint32_t)((gy + 1) * an + sgx + 1) * 4u;
        pa_c = bld<float>(ras, inside ? ab : kOOB);
        pa_w = bld<float>(ras, inside ? ab - 4u : kOOB);
        pa_e = bld<float>(ras, inside ? ab + 4u : kOOB);
        pa_s = bld<float>(ras, inside ? ab - 4u * (uint32_t)an : kOOB);
        pa_n = bld<float>(ras, inside ? ab + 4u * (uint32_t)an : kOOB);
        pf = bld<float>(rfs, inside ? pb * 4u : kOOB);
    };
    auto sstore = [&](int rho) {
        const int gy = y0 - 4 + rho;
        const bool inside = sgx >= 0 && sgx < n && gy >= 0 && gy < n;
        auto hm = [&](float qq) { return 2.f * pa_c * qq * __builtin_amdgcn_rcpf(pa_c + qq); };
        const float ww = hm(pa_w), we = hm(pa_e), ws = hm(pa_s), wn = hm(pa_n);
        const float Ae = ((ww * (pe_c - pe_w) + we * (pe_c - pe_e)) + ws * (pe_c - pe_s)) + wn * (pe_c - pe_n);
        const float dsum = ((ww + we) + ws) + wn;
        const float sv = bfr(((float)h2 * pf - Ae) * __builtin_amdgcn_rcpf(dsum));
        const float v = inside ? sv : 0.f;
        const int sl = rho & 7;
        sr[sl * kMSP + lane] = v;
        if (sl < 2) sr[(sl + 8) * kMSP + lane] = v;
        if (lane >= 4 && lane < 4 + kMW) er[(rho & 15) * kMW + lane - 4] = pe_c;
    };
    auto inrange = [&](int rho, int gx0) {  // wave-uniform: 16 columns from gx0 of row rho inside
        const int gy = y0 - 4 + rho;
        return gy >= 0 && gy < n && gx0 >= 0 && gx0 + 16 <= n;
    };
    auto mask = [&](uint2 v, int rho, int gx) {
        const int gy = y0 - 4 + rho;
        const bool in = gy >= 0 && gy < n && gx >= 0 && gx < n;
        return in ? v : make_uint2(0u, 0u);
    };
    // one 16 -> 16 job: 16 columns from the lane bases of one ring, rows rho - 1 .. rho + 1
    // in slots S0, S1, S2 (compile-time)
    auto taps16 = [&](const char *ring, int va, int vbp, int vbm, auto s0_, auto s1_, auto s2_, u4(&x)[5]) {
        constexpr int S0 = decltype(s0_)::value, S1 = decltype(s1_)::value, S2 = decltype(s2_)::value;
        x[0] = *(const u4 *)(ring + va + S0 * kMSlot);               // taps 0 | 1
        x[1] = *(const u4 *)(ring + va + S1 * kMSlot);               // taps 3 | 4
        x[2] = *(const u4 *)(ring + va + S2 * kMSlot);               // taps 6 | 7
        x[3] = *(const u4 *)(ring + (S1 == S0 + 1 ? vbp : vbm) + S0 * kMSlot + 2 * kMCol);  // taps 2 | 5
        x[4] = *(const u4 *)(ring + va + S2 * kMSlot + 2 * kMCol);   // tap 8 | zero weights
    };

    // step k; U = k & 3 (compile-time), K = the step kind
    auto step = [&](int k, auto u_, auto kind_) {
        constexpr int U = decltype(u_)::value, K = decltype(kind_)::value;
        constexpr bool CHK = K == kStepChecked, MSK = K != kStepInterior;
        const bool do3 = !CHK || (k >= 9 && k <= rows + 10);
        const bool do2 = !CHK || (k >= 6 && k <= rows + 9);
        const bool do1 = !CHK || (k >= 3 && k <= rows + 8);
        const int r3 = k - 6, r2 = k - 4, r1 = k - 2;  // rows rho of the jobs
        // operands as integer vectors until the MFMA (bf16 vectors carried
        // across these branches would be split into 16-bit pieces)
        u4 b3[5], b2[5];
        uint2 b1;
        if (do3) taps16(x2r, vA3, vB3p, vB3m, IntC<(U + 1) & 3>{}, IntC<(U + 2) & 3>{}, IntC<(U + 3) & 3>{}, b3);
        if (do2) taps16(x1r, vA2, vB2p, vB2m, IntC<(U + 3) & 3>{}, IntC<U>{}, IntC<(U + 1) & 3>{}, b2);
        if (do1) {
            const float *ps = sr + ((r1 - 1) & 7) * kMSP + vS;
            b1 = make_uint2(f32x2_to_bf16x2(ps[0], ps[1]), f32x2_to_bf16x2(ps[2], ps[2]));
        }
        // the x3 and x2 products as two interleaved MFMA chains when both run
        v4f acc3 = {0.f, 0.f, 0.f, 0.f}, acc2 = {0.f, 0.f, 0.f, 0.f};
        if (do3 && do2) {
#pragma unroll
            for (int b = 0; b < 5; ++b) {
                acc3 = mfma_wx32(w3v[b], __builtin_bit_cast(bf8_t, b3[b]), acc3);
                acc2 = mfma_wx32(w2v[b], __builtin_bit_cast(bf8_t, b2[b]), acc2);
            }
        } else if (do3) {
#pragma unroll
            for (int b = 0; b < 5; ++b) acc3 = mfma_wx32(w3v[b], __builtin_bit_cast(bf8_t, b3[b]), acc3);
        } else if (do2) {
#pragma unroll
            for (int b = 0; b < 5; ++b) acc2 = mfma_wx32(w2v[b], __builtin_bit_cast(bf8_t, b2[b]), acc2);
        }
        if (do3) {
            uint2 x = relu_pack(acc3);
            if (MSK && !inrange(r3, x0 - 1 + c3)) x = mask(x, r3, x0 - 1 + c3 + i);
            const v4f p = mfma_wx(w4t, __builtin_bit_cast(v4s, x), (v4f){0.f, 0.f, 0.f, 0.f});
            float *pd = pr + ((U + 2) & 3) * 9 * kMPT + vP;
            if (g < 2) {
#pragma unroll
                for (int q = 0; q < 4; ++q) pd[q * kMPT] = p[q];
            } else if (g == 2) {
                pd[0] = p[0];
            }
        }
        if (do2) {
            uint2 x = relu_pack(acc2);
            if (MSK && !inrange(r2, x0 - 2 + c2)) x = mask(x, r2, x0 - 2 + c2 + i);
            *(uint2 *)(x2r + U * kMSlot + vW2) = x;
        }
        if (do1) {
            const v4f acc = mfma_wx(w1v, __builtin_bit_cast(v4s, b1), (v4f){0.f, 0.f, 0.f, 0.f});
            uint2 x = relu_pack(acc);
            if (MSK && !inrange(r1, x0 - 3 + c1)) x = mask(x, r1, x0 - 3 + c1 + i);
            *(uint2 *)(x1r + ((U + 2) & 3) * kMSlot + vW1) = x;
        }
        // s rows k .. k + 3 (one a wave) and the loads for the next four
        if (U == 0 && (!CHK || k + w <= rows + 7)) {
            sstore(k + w);
            if (k + w + 4 <= rows + 7) sload(k + w + 4);
        }
        // the output row rho = k - 8: e_out = e_in + sum of the 9 shifted partials
        if (((U + 2) & 3) == w && (!CHK || (k >= kMLag && k <= rows + 11))) {
            const int ro = y0 - kMLag + k;
            if (lane < kMW) {
                float acc = 0.f;
#pragma unroll
                for (int t = 0; t < 9; ++t) acc += pr[((U + 3 + t / 3) & 3) * 9 * kMPT + t * kMPT + lane + t % 3];
                if (x0 + lane < n)
                    T::st(eout + (long long)ro * n + x0 + lane, T::rnd(er[((k - 8) & 15) * kMW + lane] + acc));
            }
        }
        __syncthreads();
    };
    auto group = [&](int k, auto kind_) {
        step(k, IntC<0>{}, kind_);
        step(k + 1, IntC<1>{}, kind_);
        step(k + 2, IntC<2>{}, kind_);
        step(k + 3, IntC<3>{}, kind_);
    };

    sload(w);
    // pipeline fill (steps 0 .. 11), every job active (steps up to rows + 7,
    // in whole groups), drain (to rows + 11, rounded up to a group)
    group(0, IntC<kStepChecked>{});
    group(4, IntC<kStepChecked>{});
    group(8, IntC<kStepChecked>{});
    const bool interior = y0 - 4 >= 0 && y0 + rows + 4 <= n && x0 - 4 >= 0 && x0 + kMW + 4 <= n;
    int k = kMLag;
    if (interior) {
        for (; k + 3 <= rows + 7; k += 4) group(k, IntC<kStepInterior>{});
    } else {
        for (; k + 3 <= rows + 7; k += 4) group(k, IntC<kStepMasked>{});
    }
    for (; k < rows + kMLag; k += 4) group(k, IntC<kStepChecked>{});
}

// Rows per workgroup: by default as few as keep the grid within one round of
// 4 workgroups per CU on 256 CUs (each strip of R rows pays 12 steps of
// pipeline fill); MGX_LSTEP_ROWS overrides (read at every launch, like
// MGX_LSTEP_TILED, so one process can compare forms).
static int lstep_rows(int n)
{
    const char *e = getenv("MGX_LSTEP_ROWS");
    const int v = e ? atoi(e) : 0;
    if (v >= 4 && v <= 4096) return v;
    const int strips = (n + kMW - 1) / kMW;
    const int runs = max(1, 1024 / strips);
    return max(8, (n + runs - 1) / runs);
}
static bool lstep_tiled()
{
    const char *e = getenv("MGX_LSTEP_TILED");
    return e && atoi(e) != 0;
}

hipError_t learned_step_fused(int st, const void *ein, void *eout, const float *f, const float *a, int n, double h2,
                              const LearnedW &d, hipStream_t s)
{
    if (!lstep_tiled()) {
        const int R = lstep_rows(n);
        const int blocks = ((n + kMW - 1) / kMW) * ((n + R - 1) / R);
        if (st == ST_F32)
            hipLaunchKernelGGL((k_lstep_march<float>), dim3(blocks), dim3(kMThreads), 0, s, (const float *)ein,
                               (float *)eout, f, a, n, h2, d, R);
        else
            hipLaunchKernelGGL((k_lstep_march<bf16_t>), dim3(blocks), dim3(kMThreads), 0, s, (const bf16_t *)ein,
                               (bf16_t *)eout, f, a, n, h2, d, R);
        return hipGetLastError();
    }
    // the tiled form (MGX_LSTEP_TILED=1): every map on the tile and its halo at once
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
