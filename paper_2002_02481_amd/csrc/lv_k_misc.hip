// lv_k_misc.hip -- the fixed-order merge of block records, bump-and-reprice helpers,
// test-support kernels, LDS sizes for the host planner, and the allocation-free
// entry point's per-GPU workspace.
#include <mutex>

#include "lv_device.h"

namespace lvk {

size_t lds_bytes(int variant, int precision, int I, int J, int n_opt, int block, int W, int WH, int K,
                 int CH) {
    const int rb = precision == 64 ? 8 : 4;
    return lds_layout(variant, rb, rb, I, J, n_opt, block / 64, W, WH, K, CH).total;
}

// --------------------------------------------------------------------------
// Fixed-order merge of the block records: one wavefront per output; lane l takes
// the compensated sum of records l, l + 64, l + 128, ... in order, then a fixed
// butterfly combines the lanes.  The association is the same on every run,
// whatever order the blocks finished in.
// --------------------------------------------------------------------------
__device__ __forceinline__ void neumaier(double &sum, double &comp, double x) {
    const double t = sum + x;
    if (fabs(sum) >= fabs(x))
        comp += (sum - t) + x;
    else
        comp += (x - t) + sum;
    sum = t;
}

__device__ __forceinline__ double record_sum(const double *part, int Q, int q, int B, int lane) {
    double sum = 0.0, comp = 0.0;
    int b = lane;
    for (; b + 64 * 7 < B; b += 64 * 8) {   // eight loads in flight per lane
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = part[(size_t)(b + 64 * k) * Q + q];
#pragma unroll
        for (int k = 0; k < 8; ++k) neumaier(sum, comp, v[k]);
    }
    for (; b < B; b += 64) neumaier(sum, comp, part[(size_t)b * Q + q]);
    return wave_sum(sum + comp);
}

// Output t (one per wavefront): option t's price and standard error (t < n_opt),
// delta (t = n_opt), grid node t - n_opt - 1.  Payoff entries sum the first B_pay
// records, the others the first B_grad.
__global__ void k_merge(const double *part, int B_pay, int B_grad, int Q, int n_opt, int G,
                        const int *opt_orig, long long P, double spot, double *price,
                        double *stderr_, double *grad, double *delta) {
    const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const double Pd = (double)P;
    if (t < n_opt) {
        const double s1 = record_sum(part, Q, 2 * t, B_pay, lane);
        const double s2 = record_sum(part, Q, 2 * t + 1, B_pay, lane);
        if (lane == 0) {
            const int o = opt_orig[t];
            price[o] = s1 / Pd;
            const double var = (s2 - s1 * s1 / Pd) / (Pd - 1.0);
            stderr_[o] = sqrt(fmax(var, 0.0) / Pd);
        }
    } else if (t == n_opt) {
        if (delta) {
            const double s = record_sum(part, Q, 2 * n_opt, B_grad, lane);
            if (lane == 0) *delta = s / Pd / spot;
        }
    } else if (grad && t < n_opt + 1 + G) {
        const int q = t - n_opt - 1;
        const double s = record_sum(part, Q, 2 * n_opt + 1 + q, B_grad, lane);
        if (lane == 0) grad[q] = s / Pd;
    }
}

// --------------------------------------------------------------------------
// Test-support kernels
// --------------------------------------------------------------------------
// --------------------------------------------------------------------------
// Bump-and-reprice (the finite-difference estimator the adjoint replaces, Sec. III):
// surfaces 2s and 2s+1 of a batch are sigma with node m0 + s moved by +eps/2 and
// -eps/2; after they are priced on the same paths, the node's derivative is the
// weighted price difference over eps.
// --------------------------------------------------------------------------
__global__ void k_bump(const double *sigma, int G, int m0, int mc, double eps, double *out) {
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= 2LL * mc * G) return;
    const int s = (int)(e / G), g = (int)(e - (long long)s * G);
    const double v = sigma[g];
    out[e] = g == m0 + s / 2 ? v + ((s & 1) ? -0.5 * eps : 0.5 * eps) : v;
}

__global__ void k_fd(const double *prices, int n_opt, const double *weight, int m0, int mc, double eps,
                     double *grad) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= mc) return;
    const double *up = prices + (size_t)(2 * s) * n_opt, *dn = up + n_opt;
    double acc = 0.0;
    for (int k = 0; k < n_opt; ++k) acc += weight[k] * (up[k] - dn[k]);
    grad[m0 + s] = acc / eps;
}

__global__ void k_debug_philox(unsigned long long seed, unsigned long long m0, int n_m,
                               unsigned long long p0, long long n_paths, uint32_t *out) {
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= n_paths) return;
    const unsigned long long p = p0 + (unsigned long long)q;
    for (int mi = 0; mi < n_m; ++mi) {
        const unsigned long long m = m0 + (unsigned long long)mi;
        const Words w = philox10((uint32_t)m, (uint32_t)(m >> 32), (uint32_t)p, (uint32_t)(p >> 32),
                                 (uint32_t)seed, (uint32_t)(seed >> 32));
        uint32_t *o = out + ((size_t)q * n_m + mi) * 4;
        o[0] = w.x;
        o[1] = w.y;
        o[2] = w.z;
        o[3] = w.w;
    }
}

template <typename R>
__global__ void k_debug_normals(unsigned long long seed, unsigned long long p0, long long n_paths,
                                int N, R *out) {
    const long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (q >= n_paths) return;
    const unsigned long long p = p0 + (unsigned long long)q;
    for (int g = 0; 4 * g < N; ++g) {
        const Words w = philox10((uint32_t)g, 0u, (uint32_t)p, (uint32_t)(p >> 32), (uint32_t)seed,
                                 (uint32_t)(seed >> 32));
        R z[4];
        Math<R>::box_muller(w.x, w.y, (R)1, z[0], z[1]);
        Math<R>::box_muller(w.z, w.w, (R)1, z[2], z[3]);
        for (int r = 0; r < 4 && 4 * g + r < N; ++r) out[(size_t)q * N + 4 * g + r] = z[r];
    }
}

hipError_t launch_fused_ckpt(const Args &a, int precision, int blocks, int block, hipStream_t st, Ev ev) {
    if (precision == 64) {
        if (a.seg == 8) return launch_fused_p64_s8(a, blocks, block, st, ev);
        if (a.seg == 16) return launch_fused_p64_s16(a, blocks, block, st, ev);
        return launch_fused_p64_s32(a, blocks, block, st, ev);
    }
    if (a.seg == 8) return launch_fused_p32_s8(a, blocks, block, st, ev);
    if (a.seg == 16) return launch_fused_p32_s16(a, blocks, block, st, ev);
    return launch_fused_p32_s32(a, blocks, block, st, ev);
}

hipError_t launch_merge(const double *part, int B_pay, int B_grad, int Q, int n_opt, int G,
                        const int *opt_orig, long long P, double spot, double *price, double *stderr_,
                        double *grad, double *delta, hipStream_t st, Ev ev) {
    const int T = n_opt + 1 + (grad ? G : 0);   // outputs, one wavefront each
    const dim3 g((T + 3) / 4), b(256);
    if (ev.start || ev.stop)
        hipExtLaunchKernelGGL(k_merge, g, b, 0, st, ev.start, ev.stop, 0, part, B_pay, B_grad, Q, n_opt, G,
                              opt_orig, P, spot, price, stderr_, grad, delta);
    else
        hipLaunchKernelGGL(k_merge, g, b, 0, st, part, B_pay, B_grad, Q, n_opt, G, opt_orig, P, spot, price,
                           stderr_, grad, delta);
    return hipGetLastError();
}

hipError_t launch_bump(const double *sigma, int G, int m0, int mc, double eps, double *out, hipStream_t st) {
    const long long n = 2LL * mc * G;
    hipLaunchKernelGGL(k_bump, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sigma, G, m0, mc, eps, out);
    return hipGetLastError();
}

hipError_t launch_fd(const double *prices, int n_opt, const double *weight, int m0, int mc, double eps,
                     double *grad, hipStream_t st) {
    hipLaunchKernelGGL(k_fd, dim3((mc + 255) / 256), dim3(256), 0, st, prices, n_opt, weight, m0, mc, eps, grad);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Workspace of the allocation-free entry point: one array per GPU, held from the
// module's load until the process ends and shared by every such call on that GPU.
// Host code never names the array itself (its host-side name is a stand-in, not a
// device address): the address is read once per device with hipGetSymbolAddress and
// passed to the kernels like any other buffer.
// --------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(int device, void **out) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[device] = p;
    }
    *out = addr[device];
    return hipSuccess;
}

hipError_t launch_debug_philox(unsigned long long seed, unsigned long long m0, int n_m,
                               unsigned long long p0, long long n_paths, uint32_t *out,
                               hipStream_t st) {
    const int blocks = (int)((n_paths + 255) / 256);
    hipLaunchKernelGGL(k_debug_philox, dim3(blocks), dim3(256), 0, st, seed, m0, n_m, p0, n_paths, out);
    return hipGetLastError();
}

hipError_t launch_debug_normals(int precision, unsigned long long seed, unsigned long long p0,
                                long long n_paths, int n_steps, double, void *out, hipStream_t st) {
    const int blocks = (int)((n_paths + 255) / 256);
    if (precision == 64)
        hipLaunchKernelGGL((k_debug_normals<double>), dim3(blocks), dim3(256), 0, st, seed, p0, n_paths,
                           n_steps, (double *)out);
    else
        hipLaunchKernelGGL((k_debug_normals<float>), dim3(blocks), dim3(256), 0, st, seed, p0, n_paths,
                           n_steps, (float *)out);
    return hipGetLastError();
}

}  // namespace lvk
