// mpdata_reduce.hip -- gfx950 kernels of the mass check and of the input
// validation of libmpdata.  Compiled with full IEEE semantics (NaN and Inf
// are detected here), unlike the step kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "mpdata_kernels.h"

namespace mpd {

// ============================================================ mass reduction
// Double-double accumulation (TwoProduct by FMA, Knuth TwoSum), a wave64
// butterfly with double-double adds, a block combine in LDS, one partial per
// block; the final pass sums the partials in a fixed order.

struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD two_sum(double a, double b)
{
#pragma clang fp contract(off)
    double s = a + b;
    double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
#pragma clang fp contract(off)
    DD s = two_sum(a.hi, b.hi);
    double lo = s.lo + (a.lo + b.lo);
    double hi = s.hi + lo;
    return {hi, lo - (hi - s.hi)};
}

__device__ __forceinline__ DD dd_add_prod(DD acc, double x, double y)
{
#pragma clang fp contract(off)
    double p = x * y;
    double e = fma(x, y, -p);
    DD s = two_sum(acc.hi, p);
    return {s.hi, acc.lo + (s.lo + e)};
}

__device__ __forceinline__ DD wave_reduce(DD v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        DD o{__shfl_xor(v.hi, m, 64), __shfl_xor(v.lo, m, 64)};
        v = dd_add(v, o);
    }
    return v;
}

__device__ __forceinline__ DD block_reduce(DD v)
{
    __shared__ double s_hi[16], s_lo[16];
    v = wave_reduce(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        s_hi[w] = v.hi;
        s_lo[w] = v.lo;
    }
    __syncthreads();
    DD r{0.0, 0.0};
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) r = dd_add(r, DD{s_hi[i], s_lo[i]});
    }
    return r;
}

template <typename T>
__global__ __launch_bounds__(256) void mass_partials(const T *__restrict__ psi,
                                                     const T *__restrict__ h, size_t n,
                                                     double *__restrict__ partials)
{
    DD acc{0.0, 0.0};
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (size_t)gridDim.x * blockDim.x)
        acc = dd_add_prod(acc, double(h[c]), double(psi[c]));
    DD r = block_reduce(acc);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = r.hi;
        partials[2 * blockIdx.x + 1] = r.lo;
    }
}

__global__ __launch_bounds__(256) void mass_final(const double *__restrict__ partials, int nparts,
                                                  double *__restrict__ result)
{
    DD acc{0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += blockDim.x)
        acc = dd_add(acc, DD{partials[2 * i], partials[2 * i + 1]});
    DD r = block_reduce(acc);
    if (threadIdx.x == 0) {
        result[0] = r.hi + r.lo;
        result[1] = r.lo;
    }
}

// ================================================================ validation

__device__ __forceinline__ bool same_bits(double a, double b)
{
    return __double_as_longlong(a) == __double_as_longlong(b);
}

__device__ __forceinline__ bool same_bits(float a, float b)
{
    return __float_as_int(a) == __float_as_int(b);
}

// flags[0]: count of h <= 0 or non-finite; flags[1]: count of periodic face
// pairs (face n vs face 0) that differ bitwise.

template <typename T>
__global__ __launch_bounds__(256) void validate(const T *__restrict__ h, const T *__restrict__ u1,
                                                const T *__restrict__ u2, const T *__restrict__ u3,
                                                int nx, int ny, int nz, int periodic,
                                                unsigned int *__restrict__ flags)
{
    const size_t n = (size_t)nx * ny * nz;
    unsigned int bad_h = 0, bad_f = 0;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (size_t)gridDim.x * blockDim.x) {
        const T v = h[c];
        if (!(v > T(0)) || !isfinite(v)) ++bad_h;
        if (periodic) {
            const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
            if (i == 0) {
                const size_t r = ((size_t)k * ny + j) * (nx + 1);
                if (!same_bits(u1[r], u1[r + nx])) ++bad_f;
            }
            if (j == 0) {
                const size_t r0 = ((size_t)k * (ny + 1)) * nx + i;
                if (!same_bits(u2[r0], u2[r0 + (size_t)ny * nx])) ++bad_f;
            }
            if (k == 0) {
                const size_t r0 = (size_t)j * nx + i;
                if (!same_bits(u3[r0], u3[r0 + (size_t)nz * ny * nx])) ++bad_f;
            }
        }
    }
    if (bad_h) atomicAdd(&flags[0], bad_h);
    if (bad_f) atomicAdd(&flags[1], bad_f);
}

// Periodic face pairs of a further time level of the Courant numbers:
// thread r of the grid-stride loop takes pair r of the ny*nz x-pairs, then
// the nz*nx y-pairs, then the ny*nx z-pairs.
template <typename T>
__global__ __launch_bounds__(256) void periodic_faces(const T *__restrict__ u1, const T *__restrict__ u2,
                                                      const T *__restrict__ u3, int nx, int ny, int nz,
                                                      unsigned int *__restrict__ flags)
{
    const size_t n1 = (size_t)ny * nz, n2 = (size_t)nz * nx, n3 = (size_t)ny * nx;
    unsigned int bad = 0;
    for (size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x; r < n1 + n2 + n3;
         r += (size_t)gridDim.x * blockDim.x) {
        if (r < n1) {
            const size_t o = r * (nx + 1);
            bad += !same_bits(u1[o], u1[o + nx]);
        } else if (r < n1 + n2) {
            const size_t k = (r - n1) / nx, i = (r - n1) % nx;
            const size_t o = k * (ny + 1) * nx + i;
            bad += !same_bits(u2[o], u2[o + (size_t)ny * nx]);
        } else {
            const size_t o = r - n1 - n2;
            bad += !same_bits(u3[o], u3[o + (size_t)nz * ny * nx]);
        }
    }
    if (bad) atomicAdd(flags, bad);
}

// ================================================================ copy back
// psi[1] -> psi[0] for every grid of a launch (ends an odd number of steps);
// one workgroup row per grid.

template <typename T>
__global__ __launch_bounds__(256) void copy_back(const GridDesc<T> *__restrict__ grids)
{
    const GridDesc<T> g = grids[blockIdx.y];
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (size_t)gridDim.x * blockDim.x)
        g.psi[0][c] = g.psi[1][c];
}

// ===================================================================== launch

template <typename T> const void *copy_back_kernel_ptr() { return (const void *)copy_back<T>; }

template <typename T> hipError_t launch_copy_back(const GridDesc<T> *grids, int ngrids, hipStream_t s)
{
    copy_back<T><<<dim3(1024, ngrids), 256, 0, s>>>(grids);
    return hipGetLastError();
}

template const void *copy_back_kernel_ptr<double>();
template const void *copy_back_kernel_ptr<float>();
template hipError_t launch_copy_back<double>(const GridDesc<double> *, int, hipStream_t);
template hipError_t launch_copy_back<float>(const GridDesc<float> *, int, hipStream_t);

template <typename T>
hipError_t launch_mass(const T *psi, const T *h, size_t n, double *partials, int nparts,
                       double *result, hipStream_t s)
{
    mass_partials<T><<<nparts, 256, 0, s>>>(psi, h, n, partials);
    mass_final<<<1, 256, 0, s>>>(partials, nparts, result);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_validate(const T *h, const T *u1, const T *u2, const T *u3, int nx, int ny,
                           int nz, int periodic, unsigned int *flags, hipStream_t s)
{
    const size_t n = (size_t)nx * ny * nz;
    const int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    validate<T><<<blocks, 256, 0, s>>>(h, u1, u2, u3, nx, ny, nz, periodic, flags);
    return hipGetLastError();
}

// ============================================ mass without any allocation
// The scratch of mpdata_mass_noalloc: the block partials (double-double) and
// the result of one reduction, in a file-scope device array of fixed size
// that every GPU the library runs on holds until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address comes from
// hipGetSymbolAddress, once per device with that device current, and is
// kept per device.
static __device__ __align__(256) double scratch[2 * kScratchParts + 2];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_address(double **out)
{
    int dev = -1;
    hipError_t r = hipGetDevice(&dev);
    if (r != hipSuccess) return r;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        r = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (r != hipSuccess) return r;
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

template <typename T>
hipError_t launch_mass_noalloc(const T *psi, const T *h, size_t n, int nparts, double *out,
                               hipStream_t s)
{
    if (nparts < 1 || nparts > kScratchParts) return hipErrorInvalidValue;
    double *sp = nullptr;
    hipError_t r = scratch_address(&sp);
    if (r != hipSuccess) return r;
    // every block writes its partial, so nothing needs clearing first
    double *partials = sp, *result = sp + 2 * kScratchParts;
    mass_partials<T><<<nparts, 256, 0, s>>>(psi, h, n, partials);
    mass_final<<<1, 256, 0, s>>>(partials, nparts, result);
    r = hipGetLastError();
    if (r != hipSuccess) return r;
    return hipMemcpyAsync(out, result, sizeof(double), hipMemcpyDeviceToDevice, s);
}

template hipError_t launch_mass_noalloc<double>(const double *, const double *, size_t, int,
                                                double *, hipStream_t);
template hipError_t launch_mass_noalloc<float>(const float *, const float *, size_t, int, double *,
                                               hipStream_t);

template <typename T>
hipError_t launch_check_periodic_faces(const T *u1, const T *u2, const T *u3, int nx, int ny,
                                       int nz, unsigned int *flags, hipStream_t s)
{
    const size_t n = (size_t)ny * nz + (size_t)nz * nx + (size_t)ny * nx;
    const int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
    periodic_faces<T><<<blocks, 256, 0, s>>>(u1, u2, u3, nx, ny, nz, flags);
    return hipGetLastError();
}

template hipError_t launch_check_periodic_faces<double>(const double *, const double *,
                                                        const double *, int, int, int,
                                                        unsigned int *, hipStream_t);
template hipError_t launch_check_periodic_faces<float>(const float *, const float *, const float *,
                                                       int, int, int, unsigned int *, hipStream_t);
template hipError_t launch_mass<double>(const double *, const double *, size_t, double *, int,
                                        double *, hipStream_t);
template hipError_t launch_mass<float>(const float *, const float *, size_t, double *, int,
                                       double *, hipStream_t);
template hipError_t launch_validate<double>(const double *, const double *, const double *,
                                            const double *, int, int, int, int, unsigned int *,
                                            hipStream_t);
template hipError_t launch_validate<float>(const float *, const float *, const float *,
                                           const float *, int, int, int, int, unsigned int *,
                                           hipStream_t);

}  // namespace mpd
