// The exact operator y = A x by direct summation, and BLAS-1 kernels for GMRES.
//
// A_ii = diag, A_ij = w K(x_i - x_j) (Section 1, eq. discbie).  Each workgroup owns 256
// targets and streams the sources through LDS in tiles of 256 points.
#include "rss_internal.h"

namespace rss {

__global__ void __launch_bounds__(256) k_matvec_direct(const double* __restrict__ pts, int64_t n, double coef,
                                                       double diag, const double* __restrict__ x,
                                                       double* __restrict__ y) {
    __shared__ double sx[256], sy[256], sv[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double xi = 0.0, yi = 0.0;
    if (i < n) { xi = pts[2 * i]; yi = pts[2 * i + 1]; }
    double acc = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += 256) {
        int64_t j = j0 + threadIdx.x;
        __syncthreads();
        if (j < n) { sx[threadIdx.x] = pts[2 * j]; sy[threadIdx.x] = pts[2 * j + 1]; sv[threadIdx.x] = x[j]; }
        else { sx[threadIdx.x] = 0.0; sy[threadIdx.x] = 0.0; sv[threadIdx.x] = 0.0; }
        __syncthreads();
        const int lim = (int)min<int64_t>(256, n - j0);
        for (int jj = 0; jj < lim; ++jj) {
            double dx = xi - sx[jj], dy = yi - sy[jj];
            double r2 = dx * dx + dy * dy;
            if (j0 + jj != i) acc += log(r2) * sv[jj];
        }
    }
    if (i < n) y[i] = diag * x[i] + coef * acc;
}

void launch_matvec_direct(const double* pts, int64_t n, const KernelParams& kp, const double* x, double* y,
                          hipStream_t s) {
    k_matvec_direct<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(pts, n, kp.coef, kp.diag, x, y);
}

constexpr int kDotBlocks = 1024;

__global__ void __launch_bounds__(256) k_dot_partial(const double* __restrict__ x, const double* __restrict__ y,
                                                     int64_t n, double* __restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) s += x[i] * y[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

int dot_partial_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)(b < kDotBlocks ? (b < 1 ? 1 : b) : kDotBlocks);
}

void launch_dot_partial(const double* x, const double* y, int64_t n, double* part, hipStream_t s) {
    k_dot_partial<<<dim3(dot_partial_blocks(n)), dim3(256), 0, s>>>(x, y, n, part);
}

__global__ void k_axpy(double a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

void launch_axpy(double a, const double* x, double* y, int64_t n, hipStream_t s) {
    k_axpy<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(a, x, y, n);
}

__global__ void k_scal_copy(double a, const double* __restrict__ x, double* __restrict__ y, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

void launch_scal_copy(double a, const double* x, double* y, int64_t n, hipStream_t s) {
    k_scal_copy<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(a, x, y, n);
}

__global__ void k_fill(double* __restrict__ y, double v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

void launch_fill(double* y, double v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    k_fill<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(y, v, n);
}

}  // namespace rss
