// nn.hip -- training and inference kernels of the learned preconditioner
// (3x3x3 convolutions with zero padding, ReLU, mean squared error, Adam) and
// their C-ABI entry points.  All reductions run in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "iga_nn.h"
#include "plan.hpp"

using namespace igasg;

#define NN_OK(call)                                                                         \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess) {                                                             \
            set_error("%s failed: %s", #call, hipGetErrorString(e_));                      \
            return IGA_ERR_DEVICE;                                                          \
        }                                                                                   \
    } while (0)

namespace {

constexpr int kNnBlock = 256;

inline unsigned nblocks(int64_t work) {
    int64_t b = (work + kNnBlock - 1) / kNnBlock;
    return static_cast<unsigned>(b < 1 ? 1 : (b > 65535 * 8 ? 65535 * 8 : b));
}

// y[b][co][i] = bias[co] + sum_ci sum_t w[co][ci][t] x[b][ci](i + t - 1), optional ReLU.
__global__ void __launch_bounds__(kNnBlock) k_conv_fwd(const float* __restrict__ x, const float* __restrict__ w,
                                                       const float* __restrict__ bias, float* __restrict__ y,
                                                       int nb, int cin, int cout, int n1, int n2, int n3,
                                                       int relu) {
    const int64_t n = static_cast<int64_t>(n1) * n2 * n3;
    const int64_t total = static_cast<int64_t>(nb) * cout * n;
    for (int64_t o = blockIdx.x * static_cast<int64_t>(kNnBlock) + threadIdx.x; o < total;
         o += static_cast<int64_t>(gridDim.x) * kNnBlock) {
        const int64_t i = o % n;
        const int64_t bc = o / n;
        const int co = static_cast<int>(bc % cout), b = static_cast<int>(bc / cout);
        const int i1 = static_cast<int>(i % n1), i2 = static_cast<int>((i / n1) % n2), i3 = static_cast<int>(i / (static_cast<int64_t>(n1) * n2));
        float s = bias[co];
        for (int ci = 0; ci < cin; ++ci) {
            const float* xc = x + (static_cast<int64_t>(b) * cin + ci) * n;
            const float* wc = w + (static_cast<int64_t>(co) * cin + ci) * 27;
            for (int t3 = 0; t3 < 3; ++t3) {
                const int j3 = i3 + t3 - 1;
                if (j3 < 0 || j3 >= n3) continue;
                for (int t2 = 0; t2 < 3; ++t2) {
                    const int j2 = i2 + t2 - 1;
                    if (j2 < 0 || j2 >= n2) continue;
                    for (int t1 = 0; t1 < 3; ++t1) {
                        const int j1 = i1 + t1 - 1;
                        if (j1 < 0 || j1 >= n1) continue;
                        s += wc[(t3 * 3 + t2) * 3 + t1] * xc[(static_cast<int64_t>(j3) * n2 + j2) * n1 + j1];
                    }
                }
            }
        }
        y[o] = relu && s < 0.0f ? 0.0f : s;
    }
}

// dx[b][ci][i] = sum_co sum_t w[co][ci][t] dy[b][co](i - t + 1), times the
// ReLU mask of the layer input (mask != NULL: mask > 0).
__global__ void __launch_bounds__(kNnBlock) k_conv_bwd_data(const float* __restrict__ dy, const float* __restrict__ w,
                                                            const float* __restrict__ mask, float* __restrict__ dx,
                                                            int nb, int cin, int cout, int n1, int n2, int n3) {
    const int64_t n = static_cast<int64_t>(n1) * n2 * n3;
    const int64_t total = static_cast<int64_t>(nb) * cin * n;
    for (int64_t o = blockIdx.x * static_cast<int64_t>(kNnBlock) + threadIdx.x; o < total;
         o += static_cast<int64_t>(gridDim.x) * kNnBlock) {
        const int64_t i = o % n;
        const int64_t bc = o / n;
        const int ci = static_cast<int>(bc % cin), b = static_cast<int>(bc / cin);
        const int i1 = static_cast<int>(i % n1), i2 = static_cast<int>((i / n1) % n2), i3 = static_cast<int>(i / (static_cast<int64_t>(n1) * n2));
        float s = 0.0f;
        if (!mask || mask[o] > 0.0f) {
            for (int co = 0; co < cout; ++co) {
                const float* dc = dy + (static_cast<int64_t>(b) * cout + co) * n;
                const float* wc = w + (static_cast<int64_t>(co) * cin + ci) * 27;
                for (int t3 = 0; t3 < 3; ++t3) {
                    const int j3 = i3 - t3 + 1;
                    if (j3 < 0 || j3 >= n3) continue;
                    for (int t2 = 0; t2 < 3; ++t2) {
                        const int j2 = i2 - t2 + 1;
                        if (j2 < 0 || j2 >= n2) continue;
                        for (int t1 = 0; t1 < 3; ++t1) {
                            const int j1 = i1 - t1 + 1;
                            if (j1 < 0 || j1 >= n1) continue;
                            s += wc[(t3 * 3 + t2) * 3 + t1] * dc[(static_cast<int64_t>(j3) * n2 + j2) * n1 + j1];
                        }
                    }
                }
            }
        }
        dx[o] = s;
    }
}

// One workgroup per (co, ci) pair (ci == cin: the bias of co): the 27 weight
// gradients sum_b sum_i dy[b][co](i) x[b][ci](i + t - 1), summed per thread
// over a fixed stride of (b, i) and then by a fixed tree.
__global__ void __launch_bounds__(kNnBlock) k_conv_bwd_weight(const float* __restrict__ x, const float* __restrict__ dy,
                                                              float* __restrict__ gw, float* __restrict__ gb, int nb,
                                                              int cin, int cout, int n1, int n2, int n3) {
    __shared__ float red[27][kNnBlock];
    const int co = blockIdx.x / (cin + 1), ci = blockIdx.x % (cin + 1);
    const int64_t n = static_cast<int64_t>(n1) * n2 * n3;
    float acc[27];
    for (int t = 0; t < 27; ++t) acc[t] = 0.0f;
    for (int64_t o = threadIdx.x; o < static_cast<int64_t>(nb) * n; o += kNnBlock) {
        const int64_t i = o % n;
        const int b = static_cast<int>(o / n);
        const float d = dy[(static_cast<int64_t>(b) * cout + co) * n + i];
        if (ci == cin) {
            acc[0] += d;
            continue;
        }
        const int i1 = static_cast<int>(i % n1), i2 = static_cast<int>((i / n1) % n2), i3 = static_cast<int>(i / (static_cast<int64_t>(n1) * n2));
        const float* xc = x + (static_cast<int64_t>(b) * cin + ci) * n;
        for (int t3 = 0; t3 < 3; ++t3) {
            const int j3 = i3 + t3 - 1;
            for (int t2 = 0; t2 < 3; ++t2) {
                const int j2 = i2 + t2 - 1;
                for (int t1 = 0; t1 < 3; ++t1) {
                    const int j1 = i1 + t1 - 1;
                    if (j3 < 0 || j3 >= n3 || j2 < 0 || j2 >= n2 || j1 < 0 || j1 >= n1) continue;
                    acc[(t3 * 3 + t2) * 3 + t1] += d * xc[(static_cast<int64_t>(j3) * n2 + j2) * n1 + j1];
                }
            }
        }
    }
    for (int t = 0; t < 27; ++t) red[t][threadIdx.x] = acc[t];
    __syncthreads();
    for (int h = kNnBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int t = 0; t < 27; ++t) red[t][threadIdx.x] += red[t][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 27) {
        if (ci == cin) {
            if (threadIdx.x == 0) gb[co] = red[0][0];
        } else {
            gw[(static_cast<int64_t>(co) * cin + ci) * 27 + threadIdx.x] = red[threadIdx.x][0];
        }
    }
}

// Loss gradient and per-block partial sums of the squared error (fixed tree).
// head 0: prediction y; head 1: prediction zf exp(y) with zf = channel 1 of
// the network input x (the scaled fast-diagonalisation output).
__global__ void __launch_bounds__(kNnBlock) k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                                  const float* __restrict__ x, int cin, int64_t n, int head,
                                                  float* __restrict__ dy, int64_t total, double count,
                                                  double* __restrict__ part) {
    __shared__ double red[kNnBlock];
    double s = 0.0;
    for (int64_t o = blockIdx.x * static_cast<int64_t>(kNnBlock) + threadIdx.x; o < total;
         o += static_cast<int64_t>(gridDim.x) * kNnBlock) {
        double pred = static_cast<double>(y[o]), dpred = 1.0;
        if (head == 1) {
            const int64_t b = o / n, i = o % n;  // one output channel
            const double zf = static_cast<double>(x[(b * cin + 1) * n + i]);
            pred = zf * exp(static_cast<double>(y[o]));
            dpred = pred;
        }
        const double d = pred - static_cast<double>(t[o]);
        dy[o] = static_cast<float>(d * dpred / count);
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kNnBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_sum_partials(const double* __restrict__ part, int np, double scale, double* __restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < np; ++i) s += part[i];
        *out = s * scale;
    }
}

__global__ void __launch_bounds__(kNnBlock) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v, int64_t count,
                                                   float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kNnBlock) + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * kNnBlock) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// Training pair of one component (one workgroup): x = (r / ||r||, zfd / s,
// loga - mean loga), t = (e - zfd) / s (head 0) or e / s (head 1) with
// s = ||zfd|| and e = xs - xk.
__global__ void __launch_bounds__(kNnBlock) k_pair(const double* __restrict__ r, const double* __restrict__ zfd,
                                                   const double* __restrict__ la, const double* __restrict__ xs,
                                                   const double* __restrict__ xk, int64_t n, int head,
                                                   float* __restrict__ x, float* __restrict__ t) {
    __shared__ double red[3][kNnBlock];
    double r2 = 0.0, z2 = 0.0, sa = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += kNnBlock) {
        r2 += r[i] * r[i];
        z2 += zfd[i] * zfd[i];
        sa += la[i];
    }
    red[0][threadIdx.x] = r2;
    red[1][threadIdx.x] = z2;
    red[2][threadIdx.x] = sa;
    __syncthreads();
    for (int h = kNnBlock / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
        __syncthreads();
    }
    const double sr = red[0][0] > 0.0 ? sqrt(red[0][0]) : 1.0;
    const double s = red[1][0] > 0.0 ? sqrt(red[1][0]) : 1.0;
    const double mean = red[2][0] / static_cast<double>(n);
    for (int64_t i = threadIdx.x; i < n; i += kNnBlock) {
        x[i] = static_cast<float>(r[i] / sr);
        x[n + i] = static_cast<float>(zfd[i] / s);
        x[2 * n + i] = static_cast<float>(la[i] - mean);
        if (xs && t) {
            const double e = xs[i] - (xk ? xk[i] : 0.0);
            t[i] = static_cast<float>((head == 1 ? e : e - zfd[i]) / s);
        }
    }
}

bool valid_net(const int* ch, int nl) {
    if (!ch || nl < 1 || nl > 8) return false;
    for (int l = 0; l <= nl; ++l)
        if (ch[l] < 1 || ch[l] > 256) return false;
    return true;
}

}  // namespace

extern "C" {

int64_t iga_nn_param_count(const int* channels, int nlayers) {
    if (!valid_net(channels, nlayers)) return -1;
    int64_t c = 0;
    for (int l = 0; l < nlayers; ++l) c += static_cast<int64_t>(channels[l + 1]) * (channels[l] * 27 + 1);
    return c;
}

iga_status iga_nn_forward(const int* channels, int nlayers, const float* params_dev, int nb, const int* n,
                          const float* x_dev, float* acts_dev, float* y_dev, void* stream) {
    if (!valid_net(channels, nlayers) || !params_dev || nb < 1 || !n || n[0] < 1 || n[1] < 1 || n[2] < 1 ||
        !x_dev || !y_dev) {
        set_error("iga_nn_forward: invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    if (nlayers > 1 && !acts_dev) {
        set_error("iga_nn_forward: hidden activations need acts_dev");
        return IGA_ERR_INVALID_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nv = static_cast<int64_t>(n[0]) * n[1] * n[2];
    const float* in = x_dev;
    const float* p = params_dev;
    float* act = acts_dev;
    for (int l = 0; l < nlayers; ++l) {
        const int cin = channels[l], cout = channels[l + 1];
        const bool last = l + 1 == nlayers;
        float* out = last ? y_dev : act;
        hipLaunchKernelGGL(k_conv_fwd, dim3(nblocks(nb * cout * nv)), dim3(kNnBlock), 0, st, in, p,
                           p + static_cast<int64_t>(cout) * cin * 27, out, nb, cin, cout, n[0], n[1], n[2],
                           last ? 0 : 1);
        NN_OK(hipGetLastError());
        p += static_cast<int64_t>(cout) * (cin * 27 + 1);
        if (!last) {
            in = act;
            act += static_cast<int64_t>(nb) * cout * nv;
        }
    }
    return IGA_OK;
}

iga_status iga_nn_backward(const int* channels, int nlayers, const float* params_dev, int nb, const int* n,
                           const float* x_dev, const float* acts_dev, const float* y_dev, const float* t_dev,
                           int head, double count, float* grads_dev, double* loss_dev, float* scratch_dev,
                           void* stream) {
    if (!valid_net(channels, nlayers) || !params_dev || nb < 1 || !n || n[0] < 1 || n[1] < 1 || n[2] < 1 ||
        !x_dev || !y_dev || !t_dev || !grads_dev || !scratch_dev || !(count > 0) ||
        (nlayers > 1 && !acts_dev) || head < 0 || head > 1 ||
        (head == 1 && (channels[0] < 2 || channels[nlayers] != 1))) {
        set_error("iga_nn_backward: invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nv = static_cast<int64_t>(n[0]) * n[1] * n[2];
    int cmax = 1;
    for (int l = 0; l <= nlayers; ++l) cmax = channels[l] > cmax ? channels[l] : cmax;
    float* dcur = scratch_dev;                                   // gradient w.r.t. the current layer output
    float* dnext = scratch_dev + static_cast<int64_t>(nb) * cmax * nv;
    // parameter and activation offsets per layer
    int64_t poff[9], aoff[9];
    poff[0] = 0;
    aoff[0] = 0;
    for (int l = 0; l < nlayers; ++l) {
        poff[l + 1] = poff[l] + static_cast<int64_t>(channels[l + 1]) * (channels[l] * 27 + 1);
        aoff[l + 1] = aoff[l] + (l + 1 < nlayers ? static_cast<int64_t>(nb) * channels[l + 1] * nv : 0);
    }
    // loss and dL/dy
    const int64_t ny = static_cast<int64_t>(nb) * channels[nlayers] * nv;
    const unsigned nbk = nblocks(ny) > 1024 ? 1024 : nblocks(ny);
    // block partials of the loss after the two gradient buffers (8-byte aligned: even float count)
    double* parts = reinterpret_cast<double*>(scratch_dev + 2 * static_cast<int64_t>(nb) * cmax * nv);
    hipLaunchKernelGGL(k_mse, dim3(nbk), dim3(kNnBlock), 0, st, y_dev, t_dev, x_dev, channels[0], nv, head, dcur,
                       ny, count, parts);
    NN_OK(hipGetLastError());
    if (loss_dev) {
        hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1), 0, st, parts, static_cast<int>(nbk), 0.5 / count,
                           loss_dev);
        NN_OK(hipGetLastError());
    }
    for (int l = nlayers - 1; l >= 0; --l) {
        const int cin = channels[l], cout = channels[l + 1];
        const float* xin = l == 0 ? x_dev : acts_dev + aoff[l - 1];
        const float* w = params_dev + poff[l];
        float* gw = grads_dev + poff[l];
        float* gb = gw + static_cast<int64_t>(cout) * cin * 27;
        hipLaunchKernelGGL(k_conv_bwd_weight, dim3(cout * (cin + 1)), dim3(kNnBlock), 0, st, xin, dcur, gw, gb, nb,
                           cin, cout, n[0], n[1], n[2]);
        NN_OK(hipGetLastError());
        if (l > 0) {
            hipLaunchKernelGGL(k_conv_bwd_data, dim3(nblocks(nb * cin * nv)), dim3(kNnBlock), 0, st, dcur, w, xin,
                               dnext, nb, cin, cout, n[0], n[1], n[2]);
            NN_OK(hipGetLastError());
            float* tmp = dcur;
            dcur = dnext;
            dnext = tmp;
        }
    }
    return IGA_OK;
}

iga_status iga_nn_adam(float* params_dev, const float* grads_dev, float* m_dev, float* v_dev, int64_t count,
                       float lr, float beta1, float beta2, float eps, int step, void* stream) {
    if (!params_dev || !grads_dev || !m_dev || !v_dev || count < 1 || step < 1) {
        set_error("iga_nn_adam: invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    const float c1 = 1.0f - powf(beta1, static_cast<float>(step));
    const float c2 = 1.0f - powf(beta2, static_cast<float>(step));
    hipLaunchKernelGGL(k_adam, dim3(nblocks(count)), dim3(kNnBlock), 0, static_cast<hipStream_t>(stream), params_dev,
                       grads_dev, m_dev, v_dev, count, lr, beta1, beta2, eps, c1, c2);
    NN_OK(hipGetLastError());
    return IGA_OK;
}

iga_status iga_nn_pair(const double* r_dev, const double* zfd_dev, const double* loga_dev, const double* xs_dev,
                       const double* xk_dev, int64_t n, int head, float* x_dev, float* t_dev, void* stream) {
    if (!r_dev || !zfd_dev || !loga_dev || !x_dev || n < 1 || n > 65536 || (xs_dev && !t_dev) || head < 0 ||
        head > 1) {
        set_error("iga_nn_pair: invalid arguments");
        return IGA_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_pair, dim3(1), dim3(kNnBlock), 0, static_cast<hipStream_t>(stream), r_dev, zfd_dev, loga_dev,
                       xs_dev, xk_dev, n, head, x_dev, t_dev);
    NN_OK(hipGetLastError());
    return IGA_OK;
}

}  // extern "C"
