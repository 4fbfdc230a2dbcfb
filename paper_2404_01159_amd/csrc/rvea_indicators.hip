// rvea_indicators.hip -- quality indicators of a population on the device:
// the hypervolume of App. C.2 (reference point ones on normalised
// objectives, m = 2 or 3) and the expected utility over a weight set (the
// neuroevolution appendix's EU).  Kernels and their C entry points.
//
// Hypervolume without a sequential sweep.  Order the counted points by their
// last objective z (ties by row).  The dominated volume is the integral over
// z of the area dominated in the first two objectives by the points at or
// below z, and that area grows by D_t, the part of point t's rectangle
// [x_t,1] x [y_t,1] not already covered by the rectangles of the points
// ordered before it, when t is reached.  Hence
//     HV = sum_t (1 - z_t) D_t,
// and every D_t is independent of the others:
//     D_t = integral over x in [x_t, 1] of max(0, Y_t(x) - y_t),
// with Y_t(x) the lowest y among the points before t whose x is at most x
// (1 if none).  With the points sorted once by x, Y_t at each point is a
// running minimum, so one wavefront per t integrates D_t in one pass over the
// sorted points: O(n^2) work in all, spread over n wavefronts, every term a
// product of non-negative differences.  For m = 2 every z is 0 and the order
// is the row order, so HV = sum_t D_t.  The x order is found by counting, for
// each point, the points before it in (x, row) order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "rvea.h"
#include "rvea_internal.h"

namespace {

constexpr int kMaxObj = 8;
constexpr int64_t kMaxRows = (int64_t)1 << 24;   // rows and weights of the expected utility
constexpr int64_t kMaxHvRows = (int64_t)1 << 18;  // rows of the hypervolume (O(n^2) work)
constexpr int kRankChunk = 512;  // k-range counted by one workgroup of k_hv_rank

struct Norm {
    double lo[kMaxObj], inv[kMaxObj];  // f' = (f - lo) / (hi - lo), scale given as hi - lo
    int m;
};

// Workspace of the hypervolume for n rows: the normalised points by row
// (x, y, z), their x-rank, the points in x order (x, y, z, row) and each
// row's term; 256-byte aligned pieces.
struct HvSpace {
    double *px, *py, *pz;
    int32_t *rank;
    double *sx, *sy, *sz;
    int32_t *sk;
    double *term;
};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

size_t hv_bytes(int64_t n)
{
    const size_t nn = (size_t)(n > 0 ? n : 1);
    return 7 * up256(nn * 8) + 2 * up256(nn * 4);
}

HvSpace hv_space(void *ws, int64_t n)
{
    const size_t nn = (size_t)(n > 0 ? n : 1);
    char *p = (char *)ws;
    HvSpace S;
    auto take = [&](size_t b) {
        char *q = p;
        p += up256(b);
        return q;
    };
    S.px = (double *)take(nn * 8);
    S.py = (double *)take(nn * 8);
    S.pz = (double *)take(nn * 8);
    S.rank = (int32_t *)take(nn * 4);
    S.sx = (double *)take(nn * 8);
    S.sy = (double *)take(nn * 8);
    S.sz = (double *)take(nn * 8);
    S.sk = (int32_t *)take(nn * 4);
    S.term = (double *)take(nn * 8);
    return S;
}

// A row counts when it is marked valid (or no marks are given) and every
// objective is finite.
__device__ __forceinline__ bool row_counts(const float *F, const uint8_t *valid, int m,
                                           int64_t i)
{
    if (valid && !valid[i]) return false;
    for (int k = 0; k < m; ++k)
        if (!isfinite(F[i * m + k])) return false;
    return true;
}

// Normalised point of each row; a row that does not count, or that does not
// lie strictly inside the reference box, becomes (1, 1, 1), which neither
// adds volume nor covers any.  Also clears the x-ranks.
__global__ void k_hv_points(const float *F, const uint8_t *valid, int64_t n, Norm nm, HvSpace S)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double p[3] = {1.0, 1.0, 0.0};
    bool in = row_counts(F, valid, nm.m, i);
    if (in) {
        for (int k = 0; k < nm.m; ++k) {
            p[k] = ((double)F[i * nm.m + k] - nm.lo[k]) / nm.inv[k];
            in = in && p[k] < 1.0;
        }
    }
    if (!in) p[0] = p[1] = p[2] = 1.0;
    S.px[i] = p[0];
    S.py[i] = p[1];
    S.pz[i] = p[2];
    S.rank[i] = 0;
}

// x-rank of each row: the rows before it in (x, row) order, counted over one
// chunk of kRankChunk rows per workgroup (blockIdx.y) and added atomically
// (integer sums: the result does not depend on the order).
__global__ __launch_bounds__(256) void k_hv_rank(int64_t n, HvSpace S)
{
    __shared__ double sxk[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double xi = i < n ? S.px[i] : 0.0;
    const int64_t k0 = (int64_t)blockIdx.y * kRankChunk;
    const int64_t k1 = k0 + kRankChunk < n ? k0 + kRankChunk : n;
    int32_t cnt = 0;
    for (int64_t kb = k0; kb < k1; kb += 256) {
        __syncthreads();
        const int64_t k = kb + threadIdx.x;
        sxk[threadIdx.x] = k < k1 ? S.px[k] : INFINITY;
        __syncthreads();
        const int lim = k1 - kb < 256 ? (int)(k1 - kb) : 256;
        for (int q = 0; q < lim; ++q) {
            const double xk = sxk[q];
            cnt += (xk < xi || (xk == xi && kb + q < i)) ? 1 : 0;
        }
    }
    if (i < n && cnt) atomicAdd(&S.rank[i], cnt);
}

__global__ void k_hv_scatter(int64_t n, HvSpace S)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t r = S.rank[i];
    S.sx[r] = S.px[i];
    S.sy[r] = S.py[i];
    S.sz[r] = S.pz[i];
    S.sk[r] = (int32_t)i;
}

// Running minimum over the lanes of a wavefront (lane l: min of lanes 0..l).
__device__ __forceinline__ double wave_prefix_min(double v, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(v, off, 64);
        if (lane >= off) v = v < y ? v : y;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Term of row t, (1 - z_t) D_t, by one wavefront per row (four per block).
__global__ __launch_bounds__(256) void k_hv_terms(int64_t n, HvSpace S)
{
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= n) return;  // uniform per wavefront
    const double xt = S.px[t], yt = S.py[t], zt = S.pz[t];
    double carry = 1.0, acc = 0.0;
    for (int64_t base = 0; base < n; base += 64) {
        const int64_t p = base + lane;
        double x = 1.0, y = 1.0, z = 1.0, xn = 1.0;
        int64_t k = n;
        if (p < n) {
            x = S.sx[p];
            y = S.sy[p];
            z = S.sz[p];
            k = S.sk[p];
            if (p + 1 < n) xn = S.sx[p + 1];
        }
        const bool before = p < n && (z < zt || (z == zt && k < t));
        double Y = wave_prefix_min(before ? y : 1.0, lane);
        Y = Y < carry ? Y : carry;
        carry = __shfl(Y, 63, 64);
        const double lo = x > xt ? x : xt;
        const double w = xn > lo ? xn - lo : 0.0;
        const double h = Y > yt ? Y - yt : 0.0;
        acc = fma(w, h, acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) S.term[t] = (1.0 - zt) * acc;
}

// out = (sum of v[0..n)) / div in a fixed order: one workgroup, strided
// partial sums per thread, then a tree in LDS.  n = 0 writes `empty`.
__global__ __launch_bounds__(1024) void k_sum_fixed(const double *v, int64_t n, double div,
                                                    double empty, double *out)
{
    __shared__ double s[1024];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) a += v[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = n > 0 ? s[0] / div : empty;
}

// Best utility -w.f' of each weight row over the counted rows, one
// wavefront per weight (the dot product as an fma chain in objective order).
__global__ __launch_bounds__(256) void k_eu_best(const float *F, const uint8_t *valid,
                                                 int64_t n, Norm nm, const double *W,
                                                 int64_t nw, double *best)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= nw) return;  // uniform per wavefront
    double wk[kMaxObj];
    for (int k = 0; k < nm.m; ++k) wk[k] = W[w * nm.m + k];
    double b = -INFINITY;
    for (int64_t i = lane; i < n; i += 64) {
        if (!row_counts(F, valid, nm.m, i)) continue;
        double u = 0.0;
        for (int k = 0; k < nm.m; ++k)
            u = fma(wk[k], ((double)F[i * nm.m + k] - nm.lo[k]) / nm.inv[k], u);
        b = -u > b ? -u : b;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(b, off, 64);
        b = o > b ? o : b;
    }
    if (lane == 0) best[w] = b;
}

// Scratch of rvea_hypervolume_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends; room for kNoAllocRows rows.  Host
// code must never pass `scratch` itself to a kernel (in host code the name
// stands for a host-side symbol, not a device address): its device address
// is looked up once per device and kept in g_scratch.
constexpr int64_t kNoAllocRows = (int64_t)1 << 17;
constexpr size_t kScratchBytes = 7 * ((size_t)kNoAllocRows * 8) + 2 * ((size_t)kNoAllocRows * 4);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// device address of the current device's scratch (looked up on the first
// call on that device, with that device current)
hipError_t scratch_of_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

rvea_status norm_of(int m, const double *lo, const double *hi, Norm *nm)
{
    if (!lo || !hi) return RVEA_EINVAL;
    nm->m = m;
    for (int k = 0; k < m; ++k) {
        if (!std::isfinite(lo[k]) || !std::isfinite(hi[k]) || !(hi[k] > lo[k]))
            return RVEA_EINVAL;
        nm->lo[k] = lo[k];
        nm->inv[k] = hi[k] - lo[k];
    }
    return RVEA_OK;
}

rvea_status device_error(const char *what, hipError_t e)
{
    rvea::note_thread_error(what, e);
    return RVEA_EDEVICE;
}

// the hypervolume's launches on workspace ws (at least hv_bytes(n))
hipError_t enqueue_hv(const float *F, const uint8_t *valid, int64_t n, const Norm &nm,
                      double *out, void *ws, hipStream_t s)
{
    const HvSpace S = hv_space(ws, n);
    if (n > 0) {
        const unsigned nb = (unsigned)((n + 255) / 256);
        hipLaunchKernelGGL(k_hv_points, dim3(nb), dim3(256), 0, s, F, valid, n, nm, S);
        const unsigned nc = (unsigned)((n + kRankChunk - 1) / kRankChunk);
        hipLaunchKernelGGL(k_hv_rank, dim3(nb, nc), dim3(256), 0, s, n, S);
        hipLaunchKernelGGL(k_hv_scatter, dim3(nb), dim3(256), 0, s, n, S);
        hipLaunchKernelGGL(k_hv_terms, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, S);
    }
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(1024), 0, s, S.term, n, 1.0, 0.0, out);
    return hipGetLastError();
}

}  // namespace

extern "C" {

rvea_status rvea_indicator_footprint(int m, int64_t n, int64_t nw, size_t *bytes)
{
    if (!bytes || m < 2 || m > kMaxObj || n < 0 || n > kMaxRows || nw < 0 || nw > kMaxRows)
        return RVEA_EINVAL;
    const size_t hv = m <= 3 && n <= kMaxHvRows ? hv_bytes(n) : 0;
    const size_t eu = up256((size_t)(nw > 0 ? nw : 1) * 8);
    *bytes = hv > eu ? hv : eu;
    return RVEA_OK;
}

rvea_status rvea_hypervolume(int m, int64_t n, const float *F, const uint8_t *valid,
                             const double *lo, const double *hi, double *out, void *workspace,
                             size_t workspace_bytes, void *hip_stream)
{
    if (m < 2 || m > 3 || n < 0 || n > kMaxHvRows || !out || (n > 0 && !F)) return RVEA_EINVAL;
    if (!workspace || ((uintptr_t)workspace & 255u)) return RVEA_EINVAL;
    Norm nm;
    rvea_status st = norm_of(m, lo, hi, &nm);
    if (st != RVEA_OK) return st;
    if (workspace_bytes < hv_bytes(n)) return RVEA_ENOMEM;
    const hipError_t e = enqueue_hv(F, valid, n, nm, out, workspace, (hipStream_t)hip_stream);
    return e == hipSuccess ? RVEA_OK : device_error("hypervolume launch", e);
}

rvea_status rvea_expected_utility(int m, int64_t n, const float *F, const uint8_t *valid,
                                  const double *lo, const double *hi, int64_t nw,
                                  const double *W, double *out, void *workspace,
                                  size_t workspace_bytes, void *hip_stream)
{
    if (m < 2 || m > kMaxObj || n < 0 || n > kMaxRows || nw < 1 || nw > kMaxRows || !W ||
        !out || (n > 0 && !F))
        return RVEA_EINVAL;
    if (!workspace || ((uintptr_t)workspace & 255u)) return RVEA_EINVAL;
    Norm nm;
    rvea_status st = norm_of(m, lo, hi, &nm);
    if (st != RVEA_OK) return st;
    if (workspace_bytes < (size_t)nw * 8) return RVEA_ENOMEM;
    hipStream_t s = (hipStream_t)hip_stream;
    double *best = (double *)workspace;
    hipLaunchKernelGGL(k_eu_best, dim3((unsigned)((nw + 3) / 4)), dim3(256), 0, s, F, valid, n,
                       nm, W, nw, best);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(1024), 0, s, best, nw, (double)nw, -INFINITY,
                       out);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RVEA_OK : device_error("expected-utility launch", e);
}

rvea_status rvea_hypervolume_noalloc(int m, int64_t n, const float *F, const uint8_t *valid,
                                     const double *lo, const double *hi, double *out,
                                     void *hip_stream)
{
    if (m < 2 || m > 3 || n < 0 || !out || (n > 0 && !F)) return RVEA_EINVAL;
    if (n > kNoAllocRows) {
        rvea::note_thread_message("rvea_hypervolume_noalloc: more rows than its static "
                                  "scratch holds (at most 131072)");
        return RVEA_ENOMEM;
    }
    Norm nm;
    rvea_status st = norm_of(m, lo, hi, &nm);
    if (st != RVEA_OK) return st;
    void *ws = nullptr;
    hipError_t e = scratch_of_current_device(&ws);
    if (e != hipSuccess) return device_error("hipGetSymbolAddress(scratch)", e);
    if (hv_bytes(n) > kScratchBytes) return RVEA_ENOMEM;
    e = enqueue_hv(F, valid, n, nm, out, ws, (hipStream_t)hip_stream);
    return e == hipSuccess ? RVEA_OK : device_error("hypervolume launch", e);
}

}  // extern "C"
