// Shell energy spectrum of a lattice velocity: the power of the half-spectrum
// a real-to-complex FFT returns, then one fixed-order sum per wavenumber shell
// over a host-built list of the shell's entries (deterministic, no atomics).
#include "kernels.h"

namespace vmfmm {

namespace {

// power[e] (+)= w_e |U_e|^2 / (2 ng^6) for entry e = (ix ng + iy) nzc + kz of the
// half spectrum, nzc = ng/2 + 1; w_e = 2 where the conjugate partner is not
// stored (0 < kz and, for even ng, kz < ng/2), else 1.
__global__ void __launch_bounds__(256) k_spec_power(int ng, int64_t total, const double2 *__restrict__ U,
                                                    double scale, int first, double *__restrict__ power) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= total) return;
    const int nzc = ng / 2 + 1;
    const int kz = int(e % nzc);
    const bool paired = kz > 0 && !(ng % 2 == 0 && kz == ng / 2);
    const double2 v = U[e];
    const double pw = (paired ? 2.0 : 1.0) * scale * (v.x * v.x + v.y * v.y);
    power[e] = first ? pw : power[e] + pw;
}

// E[s] = sum over the entries of shell s (list[start[s] .. start[s+1])) of power,
// one workgroup per shell: strided in a fixed order, then a fixed tree.
__global__ void __launch_bounds__(256) k_shell_sum(const int32_t *__restrict__ start,
                                                   const int32_t *__restrict__ list,
                                                   const double *__restrict__ power, double *__restrict__ E) {
    __shared__ double red[4];
    const int s = blockIdx.x, tid = threadIdx.x;
    double acc = 0.0;
    for (int i = start[s] + tid; i < start[s + 1]; i += 256) acc += power[list[i]];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) E[s] = (red[0] + red[1]) + (red[2] + red[3]);
}

}  // namespace

hipError_t launch_spec_power(hipStream_t s, int ng, const void *U, double scale, int first, double *power) {
    const int64_t total = int64_t(ng) * ng * (ng / 2 + 1);
    hipLaunchKernelGGL(k_spec_power, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, ng, total,
                       static_cast<const double2 *>(U), scale, first, power);
    return hipGetLastError();
}

hipError_t launch_shell_sum(hipStream_t s, int nshell, const int32_t *start, const int32_t *list,
                            const double *power, double *E) {
    hipLaunchKernelGGL(k_shell_sum, dim3(unsigned(nshell)), dim3(256), 0, s, start, list, power, E);
    return hipGetLastError();
}

}  // namespace vmfmm
