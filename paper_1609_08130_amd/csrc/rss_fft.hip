// Exact operator y = A x for points on a uniform grid, by FFT convolution.
//
// When point g = i + n j sits at (x0 + i h, y0 + j h), the off-diagonal part of A is
// block Toeplitz with Toeplitz blocks: (A - diag I)_{gg'} = w K(h (i - i', j - j')).  Its
// generator is embedded in an L x L circulant (L = power of two >= 2n - 1, zero at the
// origin and in the wrap-around gap), so A x = diag x + IFFT2(FFT2(c) .* FFT2(pad(x)))
// restricted to the n x n block (the paper applies K by FFT in its experiments, Section 4).
//
// 1D transforms of length L run in LDS, one workgroup per row or column: radix-2
// decimation in time after a bit-reversed load, twiddles from a table built on the host.
#include <cmath>
#include <vector>

#include "rss_internal.h"

namespace rss {

struct cplx {
    double re, im;
};

__device__ inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

// One length-L transform per workgroup on a[base + k * es], base = blockIdx.x * rs.
__global__ void __launch_bounds__(256) k_fft_lines(cplx* __restrict__ a, int L, int logL, int64_t rs, int64_t es,
                                                   const cplx* __restrict__ tw, int inverse) {
    extern __shared__ cplx sl[];
    const int tid = threadIdx.x;
    // workgroups go to the 8 XCDs round-robin: give each XCD a run of adjacent lines, so
    // that the lines sharing a cache line (strided passes) meet in one L2
    const int nl = gridDim.x, b = blockIdx.x;
    const int li = (nl % 8 == 0) ? (b & 7) * (nl >> 3) + (b >> 3) : b;
    cplx* line = a + (int64_t)li * rs;
    for (int k = tid; k < L; k += 256) {
        unsigned r = __brev((unsigned)k) >> (32 - logL);
        sl[r] = line[(int64_t)k * es];
    }
    __syncthreads();
    for (int len = 2, step = L >> 1; len <= L; len <<= 1, step >>= 1) {
        const int half = len >> 1;
        for (int b = tid; b < (L >> 1); b += 256) {
            int grp = b / half, pos = b - grp * half;
            int i = grp * len + pos, j = i + half;
            cplx w = tw[pos * step];
            if (inverse) w.im = -w.im;
            cplx t = cmul(w, sl[j]);
            cplx u = sl[i];
            sl[i] = {u.re + t.re, u.im + t.im};
            sl[j] = {u.re - t.re, u.im - t.im};
        }
        __syncthreads();
    }
    for (int k = tid; k < L; k += 256) line[(int64_t)k * es] = sl[k];
}

__global__ void k_fft_pad(const double* __restrict__ x, int n, int L, cplx* __restrict__ a) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)L * L) return;
    int64_t j = e / L, i = e % L;
    a[e] = {(i < n && j < n) ? x[i + (int64_t)n * j] : 0.0, 0.0};
}

__global__ void k_fft_mul(cplx* __restrict__ a, const cplx* __restrict__ c, int64_t tot) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < tot) a[e] = cmul(a[e], c[e]);
}

__global__ void k_fft_extract(const cplx* __restrict__ a, const double* __restrict__ x, int n, int L, double scale,
                              double diag, double* __restrict__ y) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * n) return;
    int64_t i = e % n, j = e / n;
    y[e] = diag * x[e] + scale * a[j * L + i].re;
}

// circulant generator c[q][p] (row q: y offset, column p: x offset)
__global__ void k_fft_generator(int n, int L, double h, double coef, cplx* __restrict__ c) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)L * L) return;
    int q = (int)(e / L), p = (int)(e % L);
    int dx = p < n ? p : (p > L - n ? p - L : 0x7fffffff);
    int dy = q < n ? q : (q > L - n ? q - L : 0x7fffffff);
    double v = 0.0;
    if (dx != 0x7fffffff && dy != 0x7fffffff && (dx != 0 || dy != 0)) {
        double ddx = dx * h, ddy = dy * h;
        v = coef * log(ddx * ddx + ddy * ddy);
    }
    c[e] = {v, 0.0};
}

// flag |= 1 unless every point g = i + n j equals (x0 + i h, y0 + j h) to 1e-12 h
__global__ void k_grid_check(const double* __restrict__ pts, int64_t N, int n, double x0, double y0, double h,
                             int* flag) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    int64_t i = g % n, j = g / n;
    double ex = x0 + (double)i * h, ey = y0 + (double)j * h;
    if (!(fabs(pts[2 * g] - ex) <= 1e-12 * h && fabs(pts[2 * g + 1] - ey) <= 1e-12 * h)) atomicOr(flag, 1);
}

static void fft2(const FFTPlan& P, cplx* a, int rows_first_n, int inverse, hipStream_t s) {
    const size_t lds = sizeof(cplx) * P.L;
    if (!inverse) {
        // rows (only the first rows_first_n rows can be nonzero), then all columns
        k_fft_lines<<<dim3(rows_first_n), dim3(256), lds, s>>>(a, P.L, P.logL, P.L, 1, (const cplx*)P.tw, 0);
        k_fft_lines<<<dim3(P.L), dim3(256), lds, s>>>(a, P.L, P.logL, 1, P.L, (const cplx*)P.tw, 0);
    } else {
        // all columns, then only the rows that are read back
        k_fft_lines<<<dim3(P.L), dim3(256), lds, s>>>(a, P.L, P.logL, 1, P.L, (const cplx*)P.tw, 1);
        k_fft_lines<<<dim3(rows_first_n), dim3(256), lds, s>>>(a, P.L, P.logL, P.L, 1, (const cplx*)P.tw, 1);
    }
}

// Grid detection: fills P.n, P.L, P.logL, P.h and returns true when the points form a
// uniform n x n grid in DOF order g = i + n j and one line of length L fits in LDS.
bool fft_grid_detect(FFTPlan& P, const double* pts, int64_t N, int* dflag, hipStream_t s) {
    int n = (int)llround(std::sqrt((double)N));
    if ((int64_t)n * n != N || n < 2) return false;
    double p0[2], p1[2], pn[2];
    if (hipMemcpyAsync(p0, pts, sizeof(p0), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (hipMemcpyAsync(p1, pts + 2, sizeof(p1), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (hipMemcpyAsync(pn, pts + 2 * (int64_t)n, sizeof(pn), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (hipMemsetAsync(dflag, 0, sizeof(int), s) != hipSuccess) return false;
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    double h = p1[0] - p0[0];
    if (!(h > 0) || std::fabs((pn[1] - p0[1]) - h) > 1e-12 * h) return false;
    k_grid_check<<<dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s>>>(pts, N, n, p0[0], p0[1], h, dflag);
    int flag = 1;
    if (hipMemcpyAsync(&flag, dflag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return false;
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    if (flag) return false;
    int L = 1, logL = 0;
    while (L < 2 * n - 1) { L <<= 1; ++logL; }
    if (L > 8192) return false;   // one line must fit in LDS
    P.n = n; P.L = L; P.logL = logL; P.h = h;
    return true;
}

// P.chat, P.work (L^2 complex each) and P.tw (L/2 complex) are allocated by the caller.
bool fft_plan_init(FFTPlan& P, const KernelParams& kp, hipStream_t s) {
    const int L = P.L;
    const int64_t LL = (int64_t)L * L;
    std::vector<cplx> tw(L / 2);
    for (int k = 0; k < L / 2; ++k) {
        long double th = -2.0L * 3.141592653589793238462643383279502884L * (long double)k / (long double)L;
        tw[k] = {(double)std::cos(th), (double)std::sin(th)};
    }
    if (hipMemcpyAsync(P.tw, tw.data(), sizeof(cplx) * (L / 2), hipMemcpyHostToDevice, s) != hipSuccess) return false;
    k_fft_generator<<<dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, s>>>(P.n, L, P.h, kp.coef, (cplx*)P.chat);
    fft2(P, (cplx*)P.chat, L, 0, s);
    if (hipStreamSynchronize(s) != hipSuccess) return false;
    P.ready = true;
    return true;
}

void launch_matvec_fft(const FFTPlan& P, const KernelParams& kp, const double* x, double* y, hipStream_t s) {
    const int64_t LL = (int64_t)P.L * P.L;
    cplx* a = (cplx*)P.work;
    k_fft_pad<<<dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, s>>>(x, P.n, P.L, a);
    fft2(P, a, P.n, 0, s);
    k_fft_mul<<<dim3((unsigned)((LL + 255) / 256)), dim3(256), 0, s>>>(a, (const cplx*)P.chat, LL);
    fft2(P, a, P.n, 1, s);
    const int64_t nn = (int64_t)P.n * P.n;
    k_fft_extract<<<dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s>>>(a, x, P.n, P.L, 1.0 / (double)LL, kp.diag,
                                                                         y);
}

}  // namespace rss
