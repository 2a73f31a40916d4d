// Time-stepping glue around the evaluation: the two Heun stages of the
// convection (eq. 7) and stretching (eq. 8) ODEs, and the FP64 energy /
// enstrophy reductions.  All bandwidth-bound, one thread per particle.
#include "kernels.h"

#include <mutex>

namespace vmfmm {

namespace {

__global__ void __launch_bounds__(256) k_rk_stage1(int n, double *__restrict__ x, double *__restrict__ a,
                                                   const double *__restrict__ u, const double *__restrict__ s,
                                                   double dt, double *__restrict__ xs, double *__restrict__ as) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < 3; ++d) {
        const size_t k = size_t(d) * n + i;
        const double xv = x[k], av = a[k], uv = u[k], sv = s[k];
        xs[k] = xv + dt * uv;              // predictor
        as[k] = av + dt * sv;
        x[k] = xv + 0.5 * dt * uv;         // first half of the trapezoid
        a[k] = av + 0.5 * dt * sv;
    }
}

__global__ void __launch_bounds__(256) k_rk_stage2(int n, double *__restrict__ x, double *__restrict__ a,
                                                   const double *__restrict__ u, const double *__restrict__ s,
                                                   double dt, TreeGeom g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int d = 0; d < 3; ++d) {
        const size_t k = size_t(d) * n + i;
        double xv = x[k] + 0.5 * dt * u[k];
        if (g.periodic) {
#pragma clang fp contract(off)
            const double sh = floor((xv - g.lo[d]) * g.inv_len);
            const double t = sh * g.box_len;
            xv = xv - t;
        }
        x[k] = xv;
        a[k] = a[k] + 0.5 * dt * s[k];
    }
}

// Per-block partial sums of |u|^2, |curl u|^2, |alpha|^2 (fixed order).
constexpr int kDiagThreads = 256;
constexpr int kDiagMaxBlocks = 1024;

// The partial sums of the allocation-free diagnostics entry point: one slot
// of three doubles per block of the partial-sum pass, at most kDiagMaxBlocks
// blocks, 24 KiB on every device the library runs on, held until the process
// ends.  Host code never passes this name to a kernel (on the host it is only
// a stand-in for the symbol): it passes the device address that
// diag_scratch() looked up on the device concerned.
static __device__ __align__(256) double scratch[3 * kDiagMaxBlocks];

__global__ void __launch_bounds__(kDiagThreads) k_diag_partial(int n, const double *__restrict__ u,
                                                               const double *__restrict__ J,
                                                               const double *__restrict__ a,
                                                               double *__restrict__ part) {
    __shared__ double sh[3][kDiagThreads];
    double e = 0.0, w = 0.0, q = 0.0;
    for (int i = blockIdx.x * kDiagThreads + threadIdx.x; i < n; i += gridDim.x * kDiagThreads) {
        for (int d = 0; d < 3; ++d) {
            const double uv = u[size_t(d) * n + i];
            e += uv * uv;
            if (a) {
                const double av = a[size_t(d) * n + i];
                q += av * av;
            }
        }
        if (J) {
            // curl u: (J[1][2] - J[2][1], J[2][0] - J[0][2], J[0][1] - J[1][0]), J[a][b] at 3a+b
            const double w0 = J[size_t(5) * n + i] - J[size_t(7) * n + i];
            const double w1 = J[size_t(6) * n + i] - J[size_t(2) * n + i];
            const double w2 = J[size_t(1) * n + i] - J[size_t(3) * n + i];
            w += w0 * w0 + w1 * w1 + w2 * w2;
        }
    }
    sh[0][threadIdx.x] = e;
    sh[1][threadIdx.x] = w;
    sh[2][threadIdx.x] = q;
    __syncthreads();
    for (int off = kDiagThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < 3; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[size_t(blockIdx.x) * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(64) k_diag_final(int nblk, const double *__restrict__ part, double h3,
                                                   double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < nblk; ++b)
        for (int k = 0; k < 3; ++k) s[k] += part[size_t(b) * 3 + k];
    out[0] = 0.5 * h3 * s[0];
    out[1] = 0.5 * h3 * s[1];
    out[2] = 0.5 * s[2] / h3;
}

inline int blocks(int n, int t) { return (n + t - 1) / t; }

}  // namespace

hipError_t launch_rk_stage1(hipStream_t s, int n, double *x, double *a, const double *u, const double *sv,
                            double dt, double *xs, double *as) {
    hipLaunchKernelGGL(k_rk_stage1, dim3(blocks(n, 256)), dim3(256), 0, s, n, x, a, u, sv, dt, xs, as);
    return hipGetLastError();
}

hipError_t launch_rk_stage2(hipStream_t s, int n, double *x, double *a, const double *u, const double *sv,
                            double dt, const TreeGeom &g) {
    hipLaunchKernelGGL(k_rk_stage2, dim3(blocks(n, 256)), dim3(256), 0, s, n, x, a, u, sv, dt, g);
    return hipGetLastError();
}

int diag_blocks(int n) { return std::min(kDiagMaxBlocks, std::max(1, blocks(n, kDiagThreads))); }

hipError_t launch_diagnostics(hipStream_t s, int n, const double *u, const double *J, const double *a,
                              double h3, double *part, double *out) {
    const int nblk = diag_blocks(n);
    hipLaunchKernelGGL(k_diag_partial, dim3(nblk), dim3(kDiagThreads), 0, s, n, u, J, a, part);
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, s, nblk, (const double *)part, h3, out);
    return hipGetLastError();
}

constexpr int kMaxDevices = 64;

hipError_t diag_scratch(int device, double **ptr) {
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        // the caller has made `device` current; each device holds its own copy
        // of the array at its own address
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = static_cast<double *>(p);
    }
    *ptr = addr[device];
    return hipSuccess;
}

size_t diag_scratch_bytes() { return sizeof(double) * 3 * kDiagMaxBlocks; }

}  // namespace vmfmm
