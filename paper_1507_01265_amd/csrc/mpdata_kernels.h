// mpdata_kernels.h -- internal interface between the host ABI and the
// gfx950 kernels of libmpdata (not installed, not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace mpd {

// One grid of a launch: its read-only inputs and the two psi buffers of the
// time loop (a step reads psi[flip] and writes psi[1 - flip]).
template <typename T> struct GridDesc {
    const T *u1, *u2, *u3, *h;
    T *psi[2];
    int nx, ny, nz, pad;
};

// The extra arrays of one launch in a chain of corrective passes (a step
// with iord > 2): bmx, bmn are two cell arrays whose cell-by-cell max and
// min with the iterate bound a further pass (psi1 and psi^n after the head
// launch, the running bounds after a middle one); w1, w2, w3 the limited
// antidiffusive velocity of the launch (face arrays) and mx, mn its running
// bounds (cell arrays; the head launch writes psi1 to mx and nothing to mn),
// both written for the next pass.
template <typename T> struct PassIO {
    const T *bmx, *bmn;
    T *w1, *w2, *w3, *mx, *mn;
};

// A piece of work of the persistent step kernel: output tile (tx, ty) of a
// grid over the planes [z0, z1); in a launch that mixes region shapes,
// shape = the index of the segment's region in that launch family (0 or 1),
// else 0.
struct Segment {
    int grid, tx, ty, z0, z1, shape, pad1, pad2;
};

// x-y region of one workgroup (output tile = region minus a 2-cell halo)
struct TileShape {
    int rx, ry;
};

const TileShape *tile_shapes(int *count);

// Kernel variants: open boundaries, limiter on, variable-sign option,
// divergent-flow term, Courant numbers that change in time.
enum { kVariantOpen = 1, kVariantNonos = 2, kVariantVsign = 4, kVariantDiv = 8, kVariantTvel = 16,
       kVariantMixed = 32 };

// The launch family of kVariantMixed: one persistent launch in which every
// segment names one of two regions of 768 threads (Segment::shape 0 and 1),
// so that each grid of a batch can take the shape that suits its size.
// Built for FP32 periodic grids without the variable-sign option or the
// divergent-flow term.
constexpr int kMixedTiles[2] = {5, 7};  // tile ids: 32x24 and 24x32 regions

// The two time levels of the Courant numbers of one step of a single grid
// whose velocity changes in time (variant kVariantTvel): u at the start of
// the step (level n, used by every stage) and w at its end (level n+1, used
// only by the time-variation term of the pseudo-velocity).  Passed by value;
// the other variants ignore it.
template <typename T> struct TvArgs {
    const T *u1, *u2, *u3, *w1, *w2, *w3;
};

// The persistent fused step kernel for (T, tile id, variant), as a function
// pointer (for graph nodes and occupancy queries); nullptr if that variant is
// not built for that shape.
template <typename T> const void *step_kernel_ptr(int tile, int variant);

template <typename T>
hipError_t launch_persistent(const GridDesc<T> *grids, const Segment *segs, const int *wg_begin,
                             int nwg, int tile, int variant, int flip, double eps,
                             long long *seg_ticks, const TvArgs<T> &tv, hipStream_t s);

// Launches of a chain of corrective passes (iord > 2), one grid each:
// grids[0].psi[0] -> grids[0].psi[1] with the arrays of io[0].  mode is
// the march mode (head: the time step plus velocity and bounds out; mid: a
// further pass with velocity and bounds out; last: the final pass).  Built
// for the default launch shape of each precision and boundary mode; the
// pointer is nullptr for other shapes.
enum { kPassHead = 1, kPassMid = 2, kPassLast = 3 };
template <typename T> const void *pass_kernel_ptr(int tile, int variant, int mode);
template <typename T>
hipError_t launch_pass(const GridDesc<T> *grids, const PassIO<T> *io, const Segment *segs,
                       const int *wg_begin, int nwg, int tile, int variant, int mode, double eps,
                       hipStream_t s);

// Donor-cell pass only (iord 1), one grid: psi[flip] -> psi[1 - flip].
template <typename T> struct DonorArgs {
    const T *psi_in;
    T *psi_out;
    const T *u1, *u2, *u3, *h;
    int nx, ny, nz;
};
template <typename T> hipError_t launch_donor(const DonorArgs<T> &a, bool open, hipStream_t s);
template <typename T> const void *donor_kernel_ptr(bool open);

// psi of every grid of a launch copied from psi[1] back to psi[0].
template <typename T> const void *copy_back_kernel_ptr();
template <typename T>
hipError_t launch_copy_back(const GridDesc<T> *grids, int ngrids, hipStream_t s);

template <typename T>
hipError_t launch_mass(const T *psi, const T *h, size_t n, double *partials, int nparts,
                       double *result, hipStream_t s);

// The mass reduction of mpdata_mass_noalloc: the same kernels as
// launch_mass with nparts <= kScratchParts blocks, the partials and the
// result in the library's fixed device scratch (no allocation), the result
// copied to out (device).  Calls that overlap on one GPU share the scratch
// and race.
constexpr int kScratchParts = 1024;
template <typename T>
hipError_t launch_mass_noalloc(const T *psi, const T *h, size_t n, int nparts, double *out,
                               hipStream_t s);

// Counts (atomically, into *flags) the periodic face pairs (face n vs face
// 0 along every axis) of u1, u2, u3 that differ bit for bit.
template <typename T>
hipError_t launch_check_periodic_faces(const T *u1, const T *u2, const T *u3, int nx, int ny,
                                       int nz, unsigned int *flags, hipStream_t s);

template <typename T>
hipError_t launch_validate(const T *h, const T *u1, const T *u2, const T *u3, int nx, int ny,
                           int nz, int periodic, unsigned int *flags, hipStream_t s);

}  // namespace mpd
