// mpdata_pass.hip -- the launches of a time step with more than one
// corrective pass (iord > 2).
//
// MPDATA may repeat its corrective pass (Smolarkiewicz 1984): pass k runs
// the pseudo-velocity, limiter and corrective donor-cell stages again on the
// result of pass k-1, with the limited antidiffusive velocity of pass k-1 in
// the place of the Courant numbers.  The limiter bounds of a pass run over
// psi^n and every iterate of the step so far.  A step of iord = k + 1 is a
// chain of k launches of the fused march (mpdata_march.h):
//   head  psi^n -> psi^(2), the ordinary fused step, which also writes its
//         limited velocity (face arrays) and psi1;
//   mid   psi^(j) -> psi^(j+1), one further pass that reads the iterate and
//         two bound arrays in place of the donor-cell pass and writes its
//         velocity and the running bounds max/min(bounds, psi^(j)) on;
//   last  the final pass, which writes psi^(n+1) only.
// The bounds of a pass are the cell-by-cell max(bx, bn, iterate) and
// min(bx, bn, iterate) of two arrays and the iterate: psi1 and psi^n after
// the head launch (psi^n is still the step's input), the running maximum and
// minimum after a middle one.  They are what makes one march per pass
// enough: the 7-point max/min over several fields equals the 7-point max/min
// of their cell-by-cell max/min.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mpdata_march.h"

namespace mpd {

static_assert(kPassHead == kModeHead && kPassMid == kModeMid && kPassLast == kModeLast,
              "pass modes are march modes");

// Persistent kernel of one pass: workgroup b walks the segments
// [wg_begin[b], wg_begin[b+1]) of the plan, as the step kernel does;
// grids[g].psi[0] is the input iterate and grids[g].psi[1] the output.
template <typename T, int RX, int RY, bool OPEN, bool NONOS, bool VSIGN, bool DIV, int MODE>
__global__ __launch_bounds__(RX * RY) void pass_kernel(const GridDesc<T> *__restrict__ grids,
                                                      const PassIO<T> *__restrict__ io,
                                                      const Segment *__restrict__ segs,
                                                      const int *__restrict__ wg_begin, double eps)
{
    __shared__ Smem<T, RX, RY, MODE, DIV> sm;
    smem_clear(sm);
    const int b = wg_begin[blockIdx.x], e = wg_begin[blockIdx.x + 1];
    for (int s = b; s < e; ++s) {
        const Segment sg = segs[s];
        const GridDesc<T> &g = grids[sg.grid];
        if constexpr (OPEN) {
            // open grid: interior tiles take the periodic x-y addressing
            if (xy_interior<RX, RY>(sg.tx, sg.ty, g.nx, g.ny))
                march<T, RX, RY, false, true, NONOS, VSIGN, DIV, MODE>(
                    g, io[sg.grid], 0, sg.tx, sg.ty, sg.z0, sg.z1, eps, sm);
            else
                march<T, RX, RY, true, true, NONOS, VSIGN, DIV, MODE>(
                    g, io[sg.grid], 0, sg.tx, sg.ty, sg.z0, sg.z1, eps, sm);
        } else {
            march<T, RX, RY, false, false, NONOS, VSIGN, DIV, MODE>(
                g, io[sg.grid], 0, sg.tx, sg.ty, sg.z0, sg.z1, eps, sm);
        }
        __syncthreads();
    }
}

template <typename T, int RX, int RY, bool OPEN, bool DIV, int MODE>
static const void *pick_options(bool nonos, bool vsign)
{
    if (vsign)
        return nonos ? (const void *)pass_kernel<T, RX, RY, OPEN, true, true, DIV, MODE>
                     : (const void *)pass_kernel<T, RX, RY, OPEN, false, true, DIV, MODE>;
    return nonos ? (const void *)pass_kernel<T, RX, RY, OPEN, true, false, DIV, MODE>
                 : (const void *)pass_kernel<T, RX, RY, OPEN, false, false, DIV, MODE>;
}

template <typename T, int RX, int RY, bool OPEN, int MODE>
static const void *pick_div(bool nonos, bool vsign, bool div)
{
    return div ? pick_options<T, RX, RY, OPEN, true, MODE>(nonos, vsign)
               : pick_options<T, RX, RY, OPEN, false, MODE>(nonos, vsign);
}

template <typename T, int RX, int RY, bool OPEN>
static const void *pick_mode(int mode, bool nonos, bool vsign, bool div)
{
    switch (mode) {
    case kModeHead: return pick_div<T, RX, RY, OPEN, kModeHead>(nonos, vsign, div);
    case kModeMid: return pick_div<T, RX, RY, OPEN, kModeMid>(nonos, vsign, div);
    case kModeLast: return pick_div<T, RX, RY, OPEN, kModeLast>(nonos, vsign, div);
    default: return nullptr;
    }
}

// The chain is built for the default launch shape of each precision and
// boundary mode: 32x24 regions (tile 5), and 32x32 (tile 2) for FP32 with
// open boundaries.
template <typename T> const void *pass_kernel_ptr(int tile, int variant, int mode)
{
    const bool open = variant & kVariantOpen, nonos = variant & kVariantNonos;
    const bool vsign = variant & kVariantVsign, div = variant & kVariantDiv;
    if constexpr (sizeof(T) == 4) {
        if (open) return tile == 2 ? pick_mode<T, 32, 32, true>(mode, nonos, vsign, div) : nullptr;
        return tile == 5 ? pick_mode<T, 32, 24, false>(mode, nonos, vsign, div) : nullptr;
    } else {
        if (tile != 5) return nullptr;
        return open ? pick_mode<T, 32, 24, true>(mode, nonos, vsign, div)
                    : pick_mode<T, 32, 24, false>(mode, nonos, vsign, div);
    }
}

template <typename T>
hipError_t launch_pass(const GridDesc<T> *grids, const PassIO<T> *io, const Segment *segs,
                       const int *wg_begin, int nwg, int tile, int variant, int mode, double eps,
                       hipStream_t s)
{
    int count = 0;
    const TileShape *sh = tile_shapes(&count);
    const void *k = pass_kernel_ptr<T>(tile, variant, mode);
    if (!k || nwg < 1) return hipErrorInvalidValue;
    void *args[] = {(void *)&grids, (void *)&io, (void *)&segs, (void *)&wg_begin, (void *)&eps};
    return hipLaunchKernel(k, dim3(nwg), dim3(sh[tile - 1].rx * sh[tile - 1].ry), args, 0, s);
}

template const void *pass_kernel_ptr<double>(int, int, int);
template const void *pass_kernel_ptr<float>(int, int, int);
template hipError_t launch_pass<double>(const GridDesc<double> *, const PassIO<double> *,
                                        const Segment *, const int *, int, int, int, int, double,
                                        hipStream_t);
template hipError_t launch_pass<float>(const GridDesc<float> *, const PassIO<float> *,
                                       const Segment *, const int *, int, int, int, int, double,
                                       hipStream_t);

}  // namespace mpd
