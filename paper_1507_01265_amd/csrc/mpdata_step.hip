// mpdata_step.hip -- the persistent fused step kernels (one MPDATA time
// step per launch; the march they run is in mpdata_march.h) and the
// donor-cell kernel of iord 1, with their launchers.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mpdata_march.h"

namespace mpd {

// Persistent step kernel: workgroup b walks the segments [wg_begin[b],
// wg_begin[b+1]) of the plan -- (grid, tile, z-range) pieces balanced over
// the workgroups and grouped so that neighbouring tiles share an XCD -- and
// advances each one time step.  With seg_ticks non-null the wall-clock
// duration of every segment is recorded (the per-block speeds a plan tuner
// measures while all workgroups run together).  TVEL: one grid whose
// Courant numbers change in time; tv holds both time levels of the step
// (the grid descriptor's own Courant pointers are not used).
template <typename T, int RX, int RY, bool OPEN, bool NONOS, bool VSIGN, bool DIV, bool TVEL>
__global__ __launch_bounds__(RX * RY) void step_kernel(const GridDesc<T> *__restrict__ grids,
                                                      const Segment *__restrict__ segs,
                                                      const int *__restrict__ wg_begin, int flip,
                                                      double eps, long long *__restrict__ seg_ticks,
                                                      TvArgs<T> tv)
{
    __shared__ Smem<T, RX, RY, kModeStep, DIV> sm;
    smem_clear(sm);
    const int b = wg_begin[blockIdx.x], e = wg_begin[blockIdx.x + 1];
    for (int s = b; s < e; ++s) {
        const Segment sg = segs[s];
        const long long t_start = seg_ticks ? (long long)wall_clock64() : 0;
        auto run = [&](const GridDesc<T> &g) {
            if constexpr (OPEN) {
                // open grid: interior tiles take the periodic x-y addressing
                if (xy_interior<RX, RY>(sg.tx, sg.ty, g.nx, g.ny))
                    march<T, RX, RY, false, true, NONOS, VSIGN, DIV, kModeStep, TVEL>(
                        g, PassIO<T>{}, flip, sg.tx, sg.ty, sg.z0, sg.z1, eps, sm, tv);
                else
                    march<T, RX, RY, true, true, NONOS, VSIGN, DIV, kModeStep, TVEL>(
                        g, PassIO<T>{}, flip, sg.tx, sg.ty, sg.z0, sg.z1, eps, sm, tv);
            } else {
                march<T, RX, RY, false, false, NONOS, VSIGN, DIV, kModeStep, TVEL>(
                    g, PassIO<T>{}, flip, sg.tx, sg.ty, sg.z0, sg.z1, eps, sm, tv);
            }
        };
        if constexpr (TVEL) {
            GridDesc<T> g = grids[sg.grid];
            g.u1 = tv.u1;
            g.u2 = tv.u2;
            g.u3 = tv.u3;
            run(g);
        } else {
            run(grids[sg.grid]);
        }
        __syncthreads();
        // optional per-segment duration (workgroup-uniform; one lane stores)
        if (seg_ticks && threadIdx.x == 0) seg_ticks[s] = (long long)wall_clock64() - t_start;
    }
}

// Persistent step kernel of a launch that mixes region shapes: segment s
// marches a 32x24 region (shape 0) or a 24x32 one (shape 1), both 768
// threads; the two LDS layouts share one allocation.  FP32 periodic grids.
template <bool NONOS>
__global__ __launch_bounds__(768) void step_kernel_mixed(const GridDesc<float> *__restrict__ grids,
                                                       const Segment *__restrict__ segs,
                                                       const int *__restrict__ wg_begin, int flip,
                                                       double eps, long long *__restrict__ seg_ticks,
                                                       TvArgs<float> tv)
{
    (void)tv;
    __shared__ union {
        Smem<float, 32, 24, kModeStep, false> a;
        Smem<float, 24, 32, kModeStep, false> b;
    } sm;
    // values a march reads before its own planes are written are finite:
    // both layouts start cleared, and later hold only finite results
    smem_clear(sm.a);
    smem_clear(sm.b);
    const int b = wg_begin[blockIdx.x], e = wg_begin[blockIdx.x + 1];
    for (int s = b; s < e; ++s) {
        const Segment sg = segs[s];
        const long long t_start = seg_ticks ? (long long)wall_clock64() : 0;
        const GridDesc<float> &g = grids[sg.grid];
        if (sg.shape == 1)
            march<float, 24, 32, false, false, NONOS, false, false, kModeStep>(
                g, PassIO<float>{}, flip, sg.tx, sg.ty, sg.z0, sg.z1, eps, sm.b);
        else
            march<float, 32, 24, false, false, NONOS, false, false, kModeStep>(
                g, PassIO<float>{}, flip, sg.tx, sg.ty, sg.z0, sg.z1, eps, sm.a);
        __syncthreads();
        if (seg_ticks && threadIdx.x == 0) seg_ticks[s] = (long long)wall_clock64() - t_start;
    }
}

// ======================================================= donor cell (iord 1)

template <typename T, bool OPEN>
__global__ __launch_bounds__(256) void step_donor(DonorArgs<T> a)
{
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t n = (size_t)nx * ny * nz;
    for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((size_t)nx * ny));
        auto at = [&](int ii, int jj, int kk) {
            return a.psi_in[((size_t)cell_of<OPEN>(kk, nz) * ny + cell_of<OPEN>(jj, ny)) * nx +
                            cell_of<OPEN>(ii, nx)];
        };
        const T vc = a.psi_in[c];
        const T f1lo = donor(at(i - 1, j, k), vc, a.u1[((size_t)k * ny + j) * (nx + 1) + i]);
        const T f1hi = donor(vc, at(i + 1, j, k), a.u1[((size_t)k * ny + j) * (nx + 1) + i + 1]);
        const T f2lo = donor(at(i, j - 1, k), vc, a.u2[((size_t)k * (ny + 1) + j) * nx + i]);
        const T f2hi = donor(vc, at(i, j + 1, k), a.u2[((size_t)k * (ny + 1) + j + 1) * nx + i]);
        const T f3lo = donor(at(i, j, k - 1), vc, a.u3[((size_t)k * ny + j) * nx + i]);
        const T f3hi = donor(vc, at(i, j, k + 1), a.u3[((size_t)(k + 1) * ny + j) * nx + i]);
        a.psi_out[c] = vc - (((f1hi - f1lo) + (f2hi - f2lo)) + (f3hi - f3lo)) * rcp_nr(a.h[c]);
    }
}

// ===================================================================== launch

const TileShape *tile_shapes(int *count)
{
    // 24x32 (tile 7): FP32 only -- FP64 takes x-neighbours from the adjacent
    // lanes, which needs rows that tile a wave of 64
    static const TileShape shapes[] = {
        {64, 16}, {32, 32}, {64, 8}, {32, 16}, {32, 24}, {16, 16}, {24, 32},
    };
    *count = (int)(sizeof(shapes) / sizeof(shapes[0]));
    return shapes;
}

template <typename T, int RX, int RY, bool VSIGN, bool DIV, bool TVEL = false>
static const void *pick4(bool open, bool nonos)
{
    if (open)
        return nonos ? (const void *)step_kernel<T, RX, RY, true, true, VSIGN, DIV, TVEL>
                     : (const void *)step_kernel<T, RX, RY, true, false, VSIGN, DIV, TVEL>;
    return nonos ? (const void *)step_kernel<T, RX, RY, false, true, VSIGN, DIV, TVEL>
                 : (const void *)step_kernel<T, RX, RY, false, false, VSIGN, DIV, TVEL>;
}

template <typename T, int RX, int RY, bool OPEN, bool DIV>
static const void *pick_tvel(bool nonos)
{
    return nonos ? (const void *)step_kernel<T, RX, RY, OPEN, true, false, DIV, true>
                 : (const void *)step_kernel<T, RX, RY, OPEN, false, false, DIV, true>;
}

// Courant numbers that change in time: built for the default launch shape
// of each precision and boundary mode (32x24 regions; 32x32 for FP32 with
// open boundaries), without the variable-sign option.
template <typename T, int RX, int RY> static const void *pick_tv(bool open, bool nonos, bool div)
{
    if constexpr (RX == 32 && RY == 24) {
        if (!open) return div ? pick_tvel<T, RX, RY, false, true>(nonos) : pick_tvel<T, RX, RY, false, false>(nonos);
        if constexpr (sizeof(T) == 8)
            return div ? pick_tvel<T, RX, RY, true, true>(nonos) : pick_tvel<T, RX, RY, true, false>(nonos);
    }
    if constexpr (RX == 32 && RY == 32 && sizeof(T) == 4) {
        if (open) return div ? pick_tvel<T, RX, RY, true, true>(nonos) : pick_tvel<T, RX, RY, true, false>(nonos);
    }
    return nullptr;
}

// The variable-sign option and the divergent-flow term are built for the
// default launch shapes only (32x24 and 32x32 regions).
template <typename T, int RX, int RY> static const void *pick(int variant)
{
    const bool open = variant & kVariantOpen, nonos = variant & kVariantNonos;
    const bool vsign = variant & kVariantVsign, div = variant & kVariantDiv;
    if (variant & kVariantTvel) return vsign ? nullptr : pick_tv<T, RX, RY>(open, nonos, div);
    if (vsign || div) {
        if constexpr (RX == 32 && (RY == 24 || RY == 32)) {
            if (vsign && div) return pick4<T, RX, RY, true, true>(open, nonos);
            if (vsign) return pick4<T, RX, RY, true, false>(open, nonos);
            return pick4<T, RX, RY, false, true>(open, nonos);
        }
        return nullptr;
    }
    return pick4<T, RX, RY, false, false>(open, nonos);
}

template <typename T> const void *step_kernel_ptr(int tile, int variant)
{
    if (variant & kVariantMixed) {
        // the mixed launch family: FP32, periodic, plain options
        if constexpr (sizeof(T) == 4) {
            if ((tile == kMixedTiles[0] || tile == kMixedTiles[1]) &&
                !(variant & (kVariantOpen | kVariantVsign | kVariantDiv | kVariantTvel)))
                return (variant & kVariantNonos) ? (const void *)step_kernel_mixed<true>
                                                 : (const void *)step_kernel_mixed<false>;
        }
        return nullptr;
    }
    switch (tile) {
    case 1: return pick<T, 64, 16>(variant);
    case 2: return pick<T, 32, 32>(variant);
    case 3: return pick<T, 64, 8>(variant);
    case 4: return pick<T, 32, 16>(variant);
    case 5: return pick<T, 32, 24>(variant);
    case 6: return pick<T, 16, 16>(variant);
    case 7:
        if constexpr (sizeof(T) == 4) {
            if (!(variant & (kVariantVsign | kVariantDiv | kVariantTvel))) return pick<T, 24, 32>(variant);
        }
        return nullptr;
    default: return nullptr;
    }
}

template <typename T>
hipError_t launch_persistent(const GridDesc<T> *grids, const Segment *segs, const int *wg_begin,
                             int nwg, int tile, int variant, int flip, double eps,
                             long long *seg_ticks, const TvArgs<T> &tv, hipStream_t s)
{
    int count = 0;
    const TileShape *sh = tile_shapes(&count);
    const void *k = step_kernel_ptr<T>(tile, variant);
    if (!k || nwg < 1) return hipErrorInvalidValue;
    TvArgs<T> tva = tv;
    void *args[] = {(void *)&grids, (void *)&segs, (void *)&wg_begin, (void *)&flip, (void *)&eps,
                    (void *)&seg_ticks, (void *)&tva};
    return hipLaunchKernel(k, dim3(nwg), dim3(sh[tile - 1].rx * sh[tile - 1].ry), args, 0, s);
}

template <typename T> const void *donor_kernel_ptr(bool open)
{
    return open ? (const void *)step_donor<T, true> : (const void *)step_donor<T, false>;
}

template <typename T> hipError_t launch_donor(const DonorArgs<T> &a, bool open, hipStream_t s)
{
    const size_t n = (size_t)a.nx * a.ny * a.nz;
    const int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    if (open) step_donor<T, true><<<blocks, 256, 0, s>>>(a);
    else step_donor<T, false><<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

template const void *step_kernel_ptr<double>(int, int);
template const void *step_kernel_ptr<float>(int, int);
template hipError_t launch_persistent<double>(const GridDesc<double> *, const Segment *,
                                              const int *, int, int, int, int, double,
                                              long long *, const TvArgs<double> &, hipStream_t);
template hipError_t launch_persistent<float>(const GridDesc<float> *, const Segment *, const int *,
                                             int, int, int, int, double, long long *,
                                             const TvArgs<float> &, hipStream_t);
template const void *donor_kernel_ptr<double>(bool);
template const void *donor_kernel_ptr<float>(bool);
template hipError_t launch_donor<double>(const DonorArgs<double> &, bool, hipStream_t);
template hipError_t launch_donor<float>(const DonorArgs<float> &, bool, hipStream_t);

}  // namespace mpd
