// The parameter-selector network: d_in -> 64 -> 64 -> 64 -> 3, tanh hidden
// layers, linear output, FP32.  Parameters are one flat vector, layer by
// layer, each layer as its weight matrix [fan_out][fan_in] (row-major)
// followed by its bias.
//
// Kernels: a batched forward pass (one workgroup per tile of 32 samples); the
// mean-squared-error loss and its gradient by back-propagation (one
// workgroup walks the batch tile by tile, each thread owning a fixed slice
// of the gradient, so the sum over samples has a fixed order); and one Adam
// update (Kingma & Ba: bias-corrected first and second moments).
#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int H = 64;       // hidden width
constexpr int DOUT = 3;     // outputs
constexpr int TS = 32;      // samples per tile
constexpr int MT = 256;     // threads per workgroup
constexpr int DMAX = 128;   // largest supported input width

struct Layout {
    int64_t w[4], b[4];
    int in[4], out[4];
};

__host__ __device__ inline Layout layout(int d_in) {
    Layout L;
    const int dims[5] = {d_in, H, H, H, DOUT};
    int64_t k = 0;
    for (int i = 0; i < 4; ++i) {
        L.in[i] = dims[i];
        L.out[i] = dims[i + 1];
        L.w[i] = k;
        k += (int64_t)dims[i] * dims[i + 1];
        L.b[i] = k;
        k += dims[i + 1];
    }
    return L;
}

__host__ __device__ inline int64_t nparams(int d_in) {
    return (int64_t)d_in * H + H + 2 * ((int64_t)H * H + H) + (int64_t)H * DOUT + DOUT;
}

// act[li][s][j] for the current tile: layer li's output (li = 0 is the input)
struct Acts {
    float a0[TS][DMAX];
    float a1[TS][H], a2[TS][H], a3[TS][H];
    float out[TS][DOUT];
};

__device__ inline float *act_row(Acts &A, int li, int s) {
    switch (li) {
        case 0: return A.a0[s];
        case 1: return A.a1[s];
        case 2: return A.a2[s];
        case 3: return A.a3[s];
        default: return A.out[s];
    }
}

// forward of one tile of ns samples (threads cooperate), activations in LDS
__device__ void tile_forward(const float *__restrict__ P, const Layout &L, Acts &A, int ns) {
    for (int li = 0; li < 4; ++li) {
        const int I = L.in[li], O = L.out[li];
        const float *W = P + L.w[li], *bias = P + L.b[li];
        for (int e = threadIdx.x; e < ns * O; e += MT) {
            const int s = e / O, o = e - s * O;
            const float *x = act_row(A, li, s);
            const float *wr = W + (int64_t)o * I;
            float z = bias[o];
            for (int i = 0; i < I; ++i) z += wr[i] * x[i];
            act_row(A, li + 1, s)[o] = (li < 3) ? tanhf(z) : z;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(MT) k_mlp_forward(const float *__restrict__ P, const float *__restrict__ X,
                                                    int64_t batch, int d_in, float *__restrict__ Y) {
    __shared__ Acts A;
    const Layout L = layout(d_in);
    const int64_t s0 = (int64_t)blockIdx.x * TS;
    const int ns = (batch - s0) < TS ? (int)(batch - s0) : TS;
    for (int e = threadIdx.x; e < ns * d_in; e += MT) A.a0[e / d_in][e % d_in] = X[s0 * d_in + e];
    __syncthreads();
    tile_forward(P, L, A, ns);
    for (int e = threadIdx.x; e < ns * DOUT; e += MT) Y[s0 * DOUT + e] = A.out[e / DOUT][e % DOUT];
}

// Loss and gradient over the whole batch; one workgroup.  grad and loss are
// device outputs; grad must hold nparams floats.
__global__ void __launch_bounds__(MT) k_mlp_grad(const float *__restrict__ P, const float *__restrict__ X,
                                                 const float *__restrict__ Yt, int64_t batch, int d_in,
                                                 float *__restrict__ grad, float *__restrict__ loss) {
    __shared__ Acts A;
    __shared__ float d3[TS][H], dcur[TS][H], dout[TS][DOUT];
    __shared__ float red[MT];
    const Layout L = layout(d_in);
    const int64_t np = nparams(d_in);
    for (int64_t k = threadIdx.x; k < np; k += MT) grad[k] = 0.f;
    __syncthreads();
    float lsum = 0.f;
    const float scale = 2.0f / (float)(batch * DOUT);
    for (int64_t s0 = 0; s0 < batch; s0 += TS) {
        const int ns = (batch - s0) < TS ? (int)(batch - s0) : TS;
        for (int e = threadIdx.x; e < ns * d_in; e += MT) A.a0[e / d_in][e % d_in] = X[s0 * d_in + e];
        __syncthreads();
        tile_forward(P, L, A, ns);
        // output error
        for (int e = threadIdx.x; e < ns * DOUT; e += MT) {
            const int s = e / DOUT, o = e % DOUT;
            const float diff = A.out[s][o] - Yt[(s0 + s) * DOUT + o];
            lsum += diff * diff;
            dout[s][o] = scale * diff;
        }
        __syncthreads();
        // layers 3 .. 0: gradient of W, b, then delta of the layer below
        for (int li = 3; li >= 0; --li) {
            const int I = L.in[li], O = L.out[li];
            float(*delta)[H] = (li == 3) ? nullptr : ((li & 1) ? d3 : dcur);
            // delta of layer li's output: dout for li == 3, else in d3/dcur
            // weight and bias gradients: each thread owns fixed (o, i) pairs
            for (int e = threadIdx.x; e < O * (I + 1); e += MT) {
                const int o = e / (I + 1), i = e - o * (I + 1);
                float g = 0.f;
                for (int s = 0; s < ns; ++s) {
                    const float dl = (li == 3) ? dout[s][o] : delta[s][o];
                    g += dl * (i < I ? act_row(A, li, s)[i] : 1.0f);
                }
                if (i < I) grad[L.w[li] + (int64_t)o * I + i] += g;
                else grad[L.b[li] + o] += g;
            }
            if (li > 0) {
                float(*below)[H] = ((li - 1) & 1) ? d3 : dcur;
                const float *W = P + L.w[li];
                // compute into registers first: `below` may alias `delta`'s buffer
                float tmp[(TS * H + MT - 1) / MT];
                int cnt = 0;
                for (int e = threadIdx.x; e < ns * I; e += MT) {
                    const int s = e / I, i = e - s * I;
                    float acc = 0.f;
                    for (int o = 0; o < O; ++o) acc += ((li == 3) ? dout[s][o] : delta[s][o]) * W[(int64_t)o * I + i];
                    const float h = act_row(A, li, s)[i];
                    tmp[cnt++] = acc * (1.0f - h * h);
                }
                __syncthreads();
                cnt = 0;
                for (int e = threadIdx.x; e < ns * I; e += MT) below[e / I][e % I] = tmp[cnt++];
            }
            __syncthreads();
        }
    }
    red[threadIdx.x] = lsum;
    __syncthreads();
    for (int w = MT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)(batch * DOUT);
}

__global__ void k_adam(float *__restrict__ P, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t np, float lr, float wd, float b1, float b2, float eps,
                       float c1, float c2) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    const float gk = g[k] + wd * P[k];  // L2 penalty (wd / 2) |P|^2 folded into the gradient
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    P[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

}  // namespace

int64_t mlp_nparams(int d_in) { return nparams(d_in); }

hipError_t mlp_forward(fmm2d_ctx *c, const float *P, const float *X, int64_t batch, int d_in, float *Y,
                       hipStream_t st) {
    const unsigned grid = (unsigned)((batch + TS - 1) / TS);
    hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(MT), 0, st ? st : c->stream, P, X, batch, d_in, Y);
    return hipGetLastError();
}

hipError_t mlp_grad(fmm2d_ctx *c, const float *P, const float *X, const float *Y, int64_t batch, int d_in,
                    float *grad, float *loss) {
    hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(MT), 0, c->stream, P, X, Y, batch, d_in, grad, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(fmm2d_ctx *c, float *P, float *m, float *v, const float *g, int64_t np, int step, float lr,
                    float wd) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(np, 256)), dim3(256), 0, c->stream, P, m, v, g, np, lr, wd, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace fmm2d
