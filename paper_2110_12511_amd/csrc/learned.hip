// Learned range bounds for the coarse-grained phase.
//
// Section 3.1.3 picks each partition's upper bound from the current supports
// with a work estimate that overshoots (the scaling factor corrects it one
// partition late).  Here a small multilayer perceptron predicts every
// vertex's final tip number as a fraction of its initial butterfly support,
// theta_hat = r_hat * support, and the bound becomes the work-weighted
// quantile of theta_hat over the alive vertices.  Bounds only change the
// schedule; every tip number stays exact (Lemmas 3 and 4 hold for any
// increasing bounds).
//
// Network: 8 -> 64 -> 64 -> 64 (ReLU) -> 1 (sigmoid), 8961 fp32 parameters
// in one flat vector: W1[64][8], b1, W2[64][64], b2, W3[64][64], b3, w4[64],
// b4 (output index first).  Loss: weighted mean squared error.  Optimiser:
// Adam with bias correction.
//
// Kernel shape: one 64-lane wave owns a chunk of 64 samples; lane l computes
// hidden unit l of every sample of the chunk.  Activations live in LDS with
// a padded row stride of 65 floats, so both a row walk (one sample, all
// units: a broadcast) and a column walk (all samples, one unit per lane) are
// free of bank conflicts.  Weight rows (forward) or columns (backward) are
// held in registers for the chunk.  The backward pass keeps each lane's row
// of the weight gradients in registers across chunks and adds them to the
// global gradient once per wave.
#include <cmath>
#include <random>

#include "dev_common.h"
#include "pbng_internal.h"

namespace pbng {

namespace {

constexpr int MI = 8, MH = 64, HS = 65, XS = 9;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + MH * MI, OFF_W2 = OFF_B1 + MH, OFF_B2 = OFF_W2 + MH * MH,
              OFF_W3 = OFF_B2 + MH, OFF_B3 = OFF_W3 + MH * MH, OFF_W4 = OFF_B3 + MH, OFF_B4 = OFF_W4 + MH,
              NPAR = OFF_B4 + 1;
static_assert(NPAR == PBNG_MLP_NPARAM, "parameter layout");

// per vertex: w = sum of neighbour degrees, largest and smallest neighbour
// degree; maxima of support and w over the side (one wave per vertex)
__global__ void k_feat_raw(const i64 *xrow, const i32 *xadj, const i64 *yrow, i64 nx, const u64 *sup, u64 *wsum,
                           i32 *dmx, i32 *dmn, u64 *maxes) {
    const int lane = threadIdx.x & (WAVE - 1);
    const i64 wave = (blockIdx.x * (i64)blockDim.x + threadIdx.x) / WAVE;
    const i64 nwaves = (i64)gridDim.x * blockDim.x / WAVE;
    u64 smax = 0, wmax = 0;
    for (i64 x = wave; x < nx; x += nwaves) {
        u64 s = 0;
        i32 mx = 0, mn = 0x7FFFFFFF;
        for (i64 j = xrow[x] + lane; j < xrow[x + 1]; j += WAVE) {
            const i32 y = xadj[j];
            const i32 dy = (i32)(yrow[y + 1] - yrow[y]);
            s += (u64)dy;
            mx = dy > mx ? dy : mx;
            mn = dy < mn ? dy : mn;
        }
        for (int d = WAVE / 2; d > 0; d >>= 1) {
            s += __shfl_xor(s, d, WAVE);
            const i32 a = __shfl_xor(mx, d, WAVE), b = __shfl_xor(mn, d, WAVE);
            mx = a > mx ? a : mx;
            mn = b < mn ? b : mn;
        }
        if (lane == 0) {
            wsum[x] = s;
            dmx[x] = mx;
            dmn[x] = mn == 0x7FFFFFFF ? 0 : mn;
            smax = sup[x] > smax ? sup[x] : smax;
            wmax = s > wmax ? s : wmax;
        }
    }
    if (lane == 0) {
        atomicMax((unsigned long long *)&maxes[0], (unsigned long long)smax);
        atomicMax((unsigned long long *)&maxes[1], (unsigned long long)wmax);
    }
}

// the eight features (computed in double, stored as fp32)
__global__ void k_feat_final(const i64 *xrow, i64 nx, const u64 *sup, const u64 *wsum, const i32 *dmx, const i32 *dmn,
                             const u64 *maxes, double logm, float *F) {
    const double ls_max = log1p((double)maxes[0]), lw_max = log1p((double)maxes[1]);
    for (i64 x = blockIdx.x * (i64)blockDim.x + threadIdx.x; x < nx; x += (i64)gridDim.x * blockDim.x) {
        float *f = F + x * MI;
        const i64 d = xrow[x + 1] - xrow[x];
        f[7] = (float)(logm / 24.0);
        if (d == 0) {
            for (int k = 0; k < 7; ++k) f[k] = 0.f;
            continue;
        }
        const double ls = log1p((double)sup[x]), lw = log1p((double)wsum[x]);
        f[0] = (float)(log1p((double)d) / 8.0);
        f[1] = (float)(ls / 32.0);
        f[2] = (float)(lw / 16.0);
        f[3] = (float)(log1p((double)dmx[x]) / 12.0);
        f[4] = (float)(log1p((double)dmn[x]) / 12.0);
        f[5] = maxes[0] > 0 ? (float)(ls / ls_max) : 0.f;
        f[6] = maxes[1] > 0 ? (float)(lw / lw_max) : 0.f;
    }
}

struct MlpArgs {
    const float *p;
    const float *X;
    const float *Y;
    const float *Wt;
    i64 n;
    float *out;   // forward: r_hat per sample
    float *grad;  // backward: unnormalised gradient sum, [NPAR]
    float *acc;   // backward: [0] sum wt * err^2, [1] sum wt
};

template <bool TRAIN>
__global__ __launch_bounds__(64) void k_mlp(MlpArgs a) {
    __shared__ float sW1[MH * XS], sB1[MH], sW2[MH * HS], sB2[MH], sW3[MH * HS], sB3[MH], sW4[MH];
    __shared__ float sX[MH * XS], sH1[MH * HS], sH2[MH * HS], sH3[MH * HS];
    __shared__ float sD[TRAIN ? MH * HS : 1], sG[MH];
    __shared__ float sB4;
    const int l = threadIdx.x;
    for (int i = l; i < MH * MI; i += MH) sW1[(i / MI) * XS + i % MI] = a.p[OFF_W1 + i];
    for (int i = l; i < MH * MH; i += MH) {
        sW2[(i / MH) * HS + i % MH] = a.p[OFF_W2 + i];
        sW3[(i / MH) * HS + i % MH] = a.p[OFF_W3 + i];
    }
    sB1[l] = a.p[OFF_B1 + l];
    sB2[l] = a.p[OFF_B2 + l];
    sB3[l] = a.p[OFF_B3 + l];
    sW4[l] = a.p[OFF_W4 + l];
    if (l == 0) sB4 = a.p[OFF_B4];
    __syncthreads();

    float gW1[MI], gW2[MH], gW3[MH];
    float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, gw4 = 0.f, gb4 = 0.f, lsum = 0.f, wsum = 0.f;
    if (TRAIN) {
#pragma unroll
        for (int k = 0; k < MI; ++k) gW1[k] = 0.f;
#pragma unroll
        for (int j = 0; j < MH; ++j) gW2[j] = gW3[j] = 0.f;
    }
    const i64 nchunks = (a.n + MH - 1) / MH;
    for (i64 ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const i64 s0 = ch * MH;
        const bool valid = s0 + l < a.n;
#pragma unroll
        for (int k = 0; k < MI; ++k) sX[l * XS + k] = valid ? a.X[(s0 + l) * MI + k] : 0.f;
        __syncthreads();
        // layer 1: lane l is unit l
        {
            float w[MI];
#pragma unroll
            for (int k = 0; k < MI; ++k) w[k] = sW1[l * XS + k];
            const float b = sB1[l];
            for (int s = 0; s < MH; ++s) {
                float z = b;
#pragma unroll
                for (int k = 0; k < MI; ++k) z = fmaf(w[k], sX[s * XS + k], z);
                sH1[s * HS + l] = z > 0.f ? z : 0.f;
            }
        }
        __syncthreads();
        // layers 2 and 3
        {
            float w[MH];
#pragma unroll
            for (int j = 0; j < MH; ++j) w[j] = sW2[l * HS + j];
            const float b = sB2[l];
            for (int s = 0; s < MH; ++s) {
                float z = b;
#pragma unroll
                for (int j = 0; j < MH; ++j) z = fmaf(w[j], sH1[s * HS + j], z);
                sH2[s * HS + l] = z > 0.f ? z : 0.f;
            }
        }
        __syncthreads();
        {
            float w[MH];
#pragma unroll
            for (int j = 0; j < MH; ++j) w[j] = sW3[l * HS + j];
            const float b = sB3[l];
            for (int s = 0; s < MH; ++s) {
                float z = b;
#pragma unroll
                for (int j = 0; j < MH; ++j) z = fmaf(w[j], sH2[s * HS + j], z);
                sH3[s * HS + l] = z > 0.f ? z : 0.f;
            }
        }
        __syncthreads();
        // output: lane l is sample l
        float z4 = sB4;
#pragma unroll
        for (int j = 0; j < MH; ++j) z4 = fmaf(sW4[j], sH3[l * HS + j], z4);
        const float y = 1.f / (1.f + expf(-z4));
        if (!TRAIN) {
            if (valid) a.out[s0 + l] = y;
            __syncthreads();
            continue;
        }
        const float wt = valid ? a.Wt[s0 + l] : 0.f;
        const float e = valid ? y - a.Y[s0 + l] : 0.f;
        lsum = fmaf(wt * e, e, lsum);
        wsum += wt;
        const float g4 = 2.f * wt * e * y * (1.f - y);
        gb4 += g4;
        sG[l] = g4;
        __syncthreads();
        // output layer weights and the error of layer 3 (lane l is unit l)
        {
            const float w4 = sW4[l];
            for (int s = 0; s < MH; ++s) {
                const float h = sH3[s * HS + l];
                gw4 = fmaf(sG[s], h, gw4);
                sD[s * HS + l] = h > 0.f ? sG[s] * w4 : 0.f;
            }
        }
        __syncthreads();
        // gradient of W3 (row l), then the error of layer 2 (lane l is unit l of
        // layer 2, with column l of W3 in registers) into sH3
        for (int s = 0; s < MH; ++s) {
            const float d = sD[s * HS + l];
            gb3 += d;
#pragma unroll
            for (int j = 0; j < MH; ++j) gW3[j] = fmaf(d, sH2[s * HS + j], gW3[j]);
        }
        {
            float wc[MH];
#pragma unroll
            for (int j = 0; j < MH; ++j) wc[j] = sW3[j * HS + l];
            for (int s = 0; s < MH; ++s) {
                float t = 0.f;
#pragma unroll
                for (int j = 0; j < MH; ++j) t = fmaf(wc[j], sD[s * HS + j], t);
                sH3[s * HS + l] = sH2[s * HS + l] > 0.f ? t : 0.f;
            }
        }
        __syncthreads();
        // gradient of W2, then the error of layer 1 into sD
        for (int s = 0; s < MH; ++s) {
            const float d = sH3[s * HS + l];
            gb2 += d;
#pragma unroll
            for (int j = 0; j < MH; ++j) gW2[j] = fmaf(d, sH1[s * HS + j], gW2[j]);
        }
        {
            float wc[MH];
#pragma unroll
            for (int j = 0; j < MH; ++j) wc[j] = sW2[j * HS + l];
            for (int s = 0; s < MH; ++s) {
                float t = 0.f;
#pragma unroll
                for (int j = 0; j < MH; ++j) t = fmaf(wc[j], sH3[s * HS + j], t);
                sD[s * HS + l] = sH1[s * HS + l] > 0.f ? t : 0.f;
            }
        }
        __syncthreads();
        for (int s = 0; s < MH; ++s) {
            const float d = sD[s * HS + l];
            gb1 += d;
#pragma unroll
            for (int k = 0; k < MI; ++k) gW1[k] = fmaf(d, sX[s * XS + k], gW1[k]);
        }
        __syncthreads();
    }
    if (!TRAIN) return;
#pragma unroll
    for (int k = 0; k < MI; ++k) atomicAdd(&a.grad[OFF_W1 + l * MI + k], gW1[k]);
#pragma unroll
    for (int j = 0; j < MH; ++j) {
        atomicAdd(&a.grad[OFF_W2 + l * MH + j], gW2[j]);
        atomicAdd(&a.grad[OFF_W3 + l * MH + j], gW3[j]);
    }
    atomicAdd(&a.grad[OFF_B1 + l], gb1);
    atomicAdd(&a.grad[OFF_B2 + l], gb2);
    atomicAdd(&a.grad[OFF_B3 + l], gb3);
    atomicAdd(&a.grad[OFF_W4 + l], gw4);
    for (int d = WAVE / 2; d > 0; d >>= 1) {
        gb4 += __shfl_xor(gb4, d, WAVE);
        lsum += __shfl_xor(lsum, d, WAVE);
        wsum += __shfl_xor(wsum, d, WAVE);
    }
    if (l == 0) {
        atomicAdd(&a.grad[OFF_B4], gb4);
        atomicAdd(&a.acc[0], lsum);
        atomicAdd(&a.acc[1], wsum);
    }
}

// Adam with bias correction on the gradient sum / sum of weights
__global__ void k_adam(float *p, float *m, float *v, const float *grad, const float *acc, float lr, float c1, float c2) {
    const float ws = acc[1];
    if (!(ws > 0.f)) return;
    const float inv = 1.f / ws;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NPAR; i += gridDim.x * blockDim.x) {
        const float g = grad[i] * inv;
        const float mi = 0.9f * m[i] + 0.1f * g;
        const float vi = 0.999f * v[i] + 0.001f * g * g;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
    }
}

__global__ void k_grad_norm(const float *grad, const float *acc, float *out, float *loss) {
    const float ws = acc[1];
    const float inv = ws > 0.f ? 1.f / ws : 0.f;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < NPAR; i += gridDim.x * blockDim.x) out[i] = grad[i] * inv;
    if (blockIdx.x == 0 && threadIdx.x == 0) loss[0] = acc[0] * inv;
}

__global__ void k_acc_add(float *dst, const float *src) {
    if (threadIdx.x < 2) dst[threadIdx.x] += src[threadIdx.x];
}

// theta_hat = floor(r_hat * support)
__global__ void k_theta_hat(const float *r, const u64 *sup, i64 n, u64 *out) {
    for (i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) {
        float q = r[i];
        q = q < 0.f ? 0.f : (q > 1.f ? 1.f : q);
        const double t = (double)q * (double)sup[i];
        u64 v = (u64)t;
        out[i] = v > sup[i] ? sup[i] : v;
    }
}

int mlp_grid(const Ctx &c, i64 n) {
    const i64 ch = (n + MH - 1) / MH;
    const i64 cap = (i64)c.num_cu * 4;
    return (int)std::max<i64>(1, std::min(ch, cap));
}

}  // namespace

void mlp_state(Ctx &c) {
    if (c.mlp_p) return;
    PBNG_HIP(hipMalloc(&c.mlp_p, sizeof(float) * 4 * NPAR + sizeof(float) * 8));
    c.mlp_m = c.mlp_p + NPAR;
    c.mlp_v = c.mlp_m + NPAR;
    c.mlp_g = c.mlp_v + NPAR;
    c.mlp_acc = c.mlp_g + NPAR;
    PBNG_HIP(hipMemsetAsync(c.mlp_p, 0, sizeof(float) * 4 * NPAR + sizeof(float) * 8, c.stream));
}

void mlp_reset_adam(Ctx &c) {
    PBNG_HIP(hipMemsetAsync(c.mlp_m, 0, sizeof(float) * 2 * NPAR, c.stream));
    c.mlp_t = 0;
}

void mlp_init(Ctx &c, u64 seed) {
    mlp_state(c);
    std::vector<float> h(NPAR, 0.f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int off, int rows, int fan_in) {
        const double lim = std::sqrt(6.0 / fan_in);
        std::uniform_real_distribution<double> u(-lim, lim);
        for (int i = 0; i < rows * fan_in; ++i) h[off + i] = (float)u(rng);
    };
    fill(OFF_W1, MH, MI);
    fill(OFF_W2, MH, MH);
    fill(OFF_W3, MH, MH);
    fill(OFF_W4, 1, MH);
    PBNG_HIP(hipMemcpyAsync(c.mlp_p, h.data(), sizeof(float) * NPAR, hipMemcpyHostToDevice, c.stream));
    mlp_reset_adam(c);
    PBNG_HIP(hipStreamSynchronize(c.stream));
    c.mlp_ready = true;
}

void mlp_set(Ctx &c, const float *host) {
    mlp_state(c);
    PBNG_HIP(hipMemcpyAsync(c.mlp_p, host, sizeof(float) * NPAR, hipMemcpyHostToDevice, c.stream));
    mlp_reset_adam(c);
    PBNG_HIP(hipStreamSynchronize(c.stream));
    c.mlp_ready = true;
}

void mlp_get(Ctx &c, float *host) {
    if (!c.mlp_ready) throw Error(PBNG_E_ARG, "no predictor parameters");
    PBNG_HIP(hipMemcpyAsync(host, c.mlp_p, sizeof(float) * NPAR, hipMemcpyDeviceToHost, c.stream));
    PBNG_HIP(hipStreamSynchronize(c.stream));
}

void mlp_forward(Ctx &c, const float *X, i64 n, float *out) {
    if (!c.mlp_ready) throw Error(PBNG_E_ARG, "no predictor parameters");
    if (n <= 0) return;
    MlpArgs a{};
    a.p = c.mlp_p;
    a.X = X;
    a.n = n;
    a.out = out;
    hipLaunchKernelGGL(k_mlp<false>, dim3(mlp_grid(c, n)), dim3(MH), 0, c.stream, a);
    PBNG_LAUNCH_CHECK();
}

// unnormalised gradient and loss sums of rows [0, n) into c.mlp_g / c.mlp_acc
static void mlp_grad_sums(Ctx &c, const float *X, const float *Y, const float *Wt, i64 n) {
    PBNG_HIP(hipMemsetAsync(c.mlp_g, 0, sizeof(float) * (NPAR + 2), c.stream));
    if (n <= 0) return;
    MlpArgs a{};
    a.p = c.mlp_p;
    a.X = X;
    a.Y = Y;
    a.Wt = Wt;
    a.n = n;
    a.grad = c.mlp_g;
    a.acc = c.mlp_acc;
    hipLaunchKernelGGL(k_mlp<true>, dim3(mlp_grid(c, n)), dim3(MH), 0, c.stream, a);
    PBNG_LAUNCH_CHECK();
}

void mlp_loss_grad(Ctx &c, const float *X, const float *Y, const float *Wt, i64 n, float *grad, float *loss_host) {
    if (!c.mlp_ready) throw Error(PBNG_E_ARG, "no predictor parameters");
    mlp_grad_sums(c, X, Y, Wt, n);
    float *loss_dev = c.alloc<float>(1);
    hipLaunchKernelGGL(k_grad_norm, dim3((NPAR + 255) / 256), dim3(256), 0, c.stream, (const float *)c.mlp_g,
                       (const float *)c.mlp_acc, grad, loss_dev);
    PBNG_LAUNCH_CHECK();
    PBNG_HIP(hipMemcpyAsync(loss_host, loss_dev, sizeof(float), hipMemcpyDeviceToHost, c.stream));
    PBNG_HIP(hipStreamSynchronize(c.stream));
}

void mlp_train(Ctx &c, const float *X, const float *Y, const float *Wt, i64 n, int batch, int epochs, float lr,
               float *epoch_loss) {
    if (!c.mlp_ready) throw Error(PBNG_E_ARG, "no predictor parameters");
    float *ep = c.alloc<float>(2);
    for (int e = 0; e < epochs; ++e) {
        PBNG_HIP(hipMemsetAsync(ep, 0, sizeof(float) * 2, c.stream));
        for (i64 b0 = 0; b0 < n; b0 += batch) {
            const i64 nb = std::min<i64>(batch, n - b0);
            mlp_grad_sums(c, X + b0 * MI, Y + b0, Wt + b0, nb);
            ++c.mlp_t;
            const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, c.mlp_t)));
            const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, c.mlp_t)));
            hipLaunchKernelGGL(k_adam, dim3((NPAR + 255) / 256), dim3(256), 0, c.stream, c.mlp_p, c.mlp_m, c.mlp_v,
                               (const float *)c.mlp_g, (const float *)c.mlp_acc, lr, c1, c2);
            hipLaunchKernelGGL(k_acc_add, dim3(1), dim3(64), 0, c.stream, ep, (const float *)c.mlp_acc);
            PBNG_LAUNCH_CHECK();
        }
        float h[2];
        PBNG_HIP(hipMemcpyAsync(h, ep, sizeof(h), hipMemcpyDeviceToHost, c.stream));
        PBNG_HIP(hipStreamSynchronize(c.stream));
        if (epoch_loss) epoch_loss[e] = h[1] > 0.f ? h[0] / h[1] : 0.f;
    }
}

void tip_features(Ctx &c, const DevGraph &G, int side, const u64 *sup, float *F) {
    hipStream_t s = c.stream;
    const i64 nx = side == 0 ? G.n_u : G.n_v;
    const i64 *xrow = side == 0 ? G.urow : G.vrow;
    const i32 *xadj = side == 0 ? G.ucol : G.vadj;
    const i64 *yrow = side == 0 ? G.vrow : G.urow;
    if (nx == 0) return;
    u64 *wsum = c.alloc<u64>(nx);
    i32 *dmx = c.alloc<i32>(nx);
    i32 *dmn = c.alloc<i32>(nx);
    u64 *maxes = c.alloc<u64>(2);
    PBNG_HIP(hipMemsetAsync(maxes, 0, sizeof(u64) * 2, s));
    hipLaunchKernelGGL(k_feat_raw, dim3(grid_1d(nx * WAVE)), dim3(256), 0, s, xrow, xadj, yrow, nx, sup, wsum, dmx, dmn,
                       maxes);
    hipLaunchKernelGGL(k_feat_final, dim3(grid_1d(nx)), dim3(256), 0, s, xrow, nx, sup, (const u64 *)wsum,
                       (const i32 *)dmx, (const i32 *)dmn, (const u64 *)maxes, std::log1p((double)G.m), F);
    PBNG_LAUNCH_CHECK();
}

void learned_theta_hat(Ctx &c, const DevGraph &G, int side, const u64 *sup, u64 *theta_hat) {
    const i64 nx = side == 0 ? G.n_u : G.n_v;
    if (nx == 0) return;
    float *F = c.alloc<float>(nx * MI);
    float *r = c.alloc<float>(nx);
    tip_features(c, G, side, sup, F);
    mlp_forward(c, F, nx, r);
    hipLaunchKernelGGL(k_theta_hat, dim3(grid_1d(nx)), dim3(256), 0, c.stream, (const float *)r, sup, nx, theta_hat);
    PBNG_LAUNCH_CHECK();
}

}  // namespace pbng
