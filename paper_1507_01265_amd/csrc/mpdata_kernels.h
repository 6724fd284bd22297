// mpdata_kernels.h -- internal interface between the host ABI and the
// gfx950 kernels of libmpdata (not installed, not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace mpd {

// Arguments of one step launch: psi_in -> psi_out over an nx*ny*nz grid.
template <typename T> struct StepArgs {
    const T *psi_in;
    T *psi_out;
    const T *u1, *u2, *u3, *h;
    int nx, ny, nz;
    int zlen;    // planes per z-chunk (one workgroup marches one chunk)
    double eps;
};

// x-y region of one workgroup (output tile = region minus a 2-cell halo)
struct TileShape {
    int rx, ry;
};

const TileShape *tile_shapes(int *count);

template <typename T>
hipError_t launch_step(const StepArgs<T> &a, int tile, int iord, bool open, bool nonos,
                       hipStream_t s);

template <typename T>
hipError_t launch_mass(const T *psi, const T *h, size_t n, double *partials, int nparts,
                       double *result, hipStream_t s);

template <typename T>
hipError_t launch_validate(const T *h, const T *u1, const T *u2, const T *u3, int nx, int ny,
                           int nz, int periodic, unsigned int *flags, hipStream_t s);

}  // namespace mpd
