// mpdata_march.h -- the fused MPDATA march of one output tile (gfx950),
// shared by the step kernels and the kernels of further corrective passes
// (internal to libmpdata).
//
// One time step (paper, section 5.2: a chain of dependent stencil stages
// turning five input matrices into one output; the equations are those of
// the MPDATA literature the paper cites: donor-cell pass and antidiffusive
// pseudo-velocities of Smolarkiewicz 1984, non-oscillatory limiter of
// Smolarkiewicz & Grabowski 1990, density weighting of Smolarkiewicz &
// Margolin 1998):
//   S1+S2  psi1 = psi - sum_d dF_d / h,  F = donor(psi_lo, psi_hi, U)
//   S3     V on every face from psi1, U, h (A ratio, cross terms B, G)
//   S4     mx, mn = max/min of psi and psi1 over the 7-point neighbourhood
//   S5     beta_up = (mx - psi1) h / (IN + eps), beta_dn = (psi1 - mn) h / (OUT + eps)
//   S6     Vt = min(1, bdn_lo, bup_hi) pos(V) + min(1, bup_lo, bdn_hi) neg(V)
//   S7     psi_out = psi1 - sum_d dFC_d / h,  FC = donor(psi1_lo, psi1_hi, Vt)
//
// Fusion (the paper's (3+1)D decomposition, section 5.3: tile the domain
// and fuse the stage loop so intermediates stay on chip, paying with halo
// recompute), recast for CDNA:
//  * a workgroup owns an RX x RY region of x-y columns (its output tile plus
//    a 2-cell halo) and marches along z through a chunk of planes;
//  * a thread owns one column and keeps its z-history in registers;
//    in-plane neighbours are exchanged through LDS planes padded by one
//    cell on every side, so neighbour offsets are compile-time constants;
//  * the stage pipeline is skewed in z: iteration t computes psi1 at plane
//    t, V, the bounds and the limiter factors at plane t-1 (and V3 on face
//    t), the limited corrective fluxes at plane t-2 and the output at plane
//    t-3, with three workgroup barriers per iteration (each LDS buffer is
//    written in the phase after its last read); the march is unrolled by
//    three so the three psi1 planes sit in fixed LDS slots;
//  * psi^n and u3 of plane t+2 and the other inputs of plane t+1 are
//    prefetched into registers.
// Only psi^{n+1} is written to HBM: 5 array reads + 1 write per cell-step.
//
// The translation units that include this file are compiled without NaN
// semantics (finite inputs are a precondition of the step; mpdata_mass
// reports NaN/Inf in psi).
//
// Boundaries: periodic wraps cell indices (face n == face 0); open is
// zero-gradient (ghost cells equal the nearest interior cell; reads of
// cell-centred neighbours at the domain edge are redirected to the cell
// itself) with zero antidiffusive velocity on boundary-normal faces.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mpdata_kernels.h"

namespace mpd {

// ------------------------------------------------------------ index helpers

__device__ __forceinline__ int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

__device__ __forceinline__ int clampi(int i, int lo, int hi)
{
    return i < lo ? lo : (i > hi ? hi : i);
}

template <bool OPEN> __device__ __forceinline__ int cell_of(int i, int n)
{
    return OPEN ? clampi(i, 0, n - 1) : wrapi(i, n);
}

// face below / above position i along an axis of n cells (face index 0..n)
template <bool OPEN> __device__ __forceinline__ int face_lo(int i, int n)
{
    return OPEN ? clampi(i, 0, n) : wrapi(i, n);
}

template <bool OPEN> __device__ __forceinline__ int face_hi(int i, int n)
{
    return OPEN ? clampi(i + 1, 0, n) : wrapi(i, n) + 1;
}

// ---------------------------------------------------------------- arithmetic

// notation of the comments: pos(x) = max(x, 0), neg(x) = min(x, 0)

// donor-cell flux through a face with lower value l, upper value r:
// pos(c) l + neg(c) r, evaluated as c times the upwind value (the same
// number: one of the two products is an exact zero)
template <typename T> __device__ __forceinline__ T donor(T l, T r, T c)
{
    return c * (c > T(0) ? l : r);
}

// Reciprocal by the hardware estimate (v_rcp_f64 is good to 2^-24.4 relative,
// measured on gfx950; v_rcp_f32 to 1 ulp) refined with one Newton-Raphson step
// r <- r + r (1 - x r), which leaves FP64 within 2^-48.7 (measured) -- ample
// for the 1e-12 relative bound of a step -- and FP32 within an ulp.
__device__ __forceinline__ double rcp_nr(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ float rcp_nr(float x)
{
    float r = __builtin_amdgcn_rcpf(x);
    float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
}

// Quotient: FP64 multiplies by the refined reciprocal (relative error about
// 2^-48); FP32 takes v_rcp_f32 (within 1 ulp) and one residual correction
// q <- q + r (n - d q).
__device__ __forceinline__ double div_nr(double n, double d) { return n * rcp_nr(d); }

__device__ __forceinline__ float div_nr(float n, float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    const float q = n * r;
    return fmaf(fmaf(-d, q, n), r, q);
}

// Antidiffusive pseudo-velocity on a face between lower cell a and upper
// cell b (face-normal Courant number U, hs = h_a + h_b; us, ut = sums of the
// four transverse Courant numbers of a and b along the transverse axes s
// and t; s_hi = psi1_b,s+1 + psi1_a,s+1 and s_lo likewise one cell down, the
// same for t).  The definition
//   V = (|U| - U^2/G) A - (U/G) (Us Bs + Ut Bt),  G = hs/2,
//   A = (pb - pa)/(pb + pa + eps),  Bs = (s_hi - s_lo)/(2 (s_hi + s_lo + eps)),
//   Us = us/4 (and t likewise)
// is evaluated in FP64 over one common denominator, so a face costs one
// division:
//   V = [(|U| hs - 2U^2) nA dBs dBt - (U dA/4)(us nBs dBt + ut nBt dBs)]
//       / (hs dA dBs dBt).
// For psi1 >= 0 (or the variable-sign option) every ratio denominator is at
// least eps, so the common one is at least hs eps^3 (above 2e-90 for the
// smallest accepted eps, 1e-30), inside the normal range, and below 1.8e308
// while |psi1| stays below about 1e100.
// FP32 takes the three ratios and 1/hs separately, each from the hardware
// reciprocal (v_rcp_f32, within 1 ulp), as
//   V = (|U| - 2 U^2/hs) nA/dA - (U/(4 hs)) (us nBs/dBs + ut nBt/dBt):
// a cubic common denominator would leave the FP32 range for |psi1| near 2e12
// and below about 5e-14 (or wherever the transverse sums vanish), while each
// ratio here is bounded for any field whose denominators are positive, and
// four reciprocals cost fewer instructions than scaling the product (3.4 %
// faster FP32 step, measured, with the same errors against the oracle).
// FP32 steps stay finite for |psi1| below about 1e37.
// Only a field of both signs without the variable-sign option can zero a
// ratio denominator; V is then Inf or NaN exactly where the separate ratios
// of the definition divide by zero (mpdata_mass reports it).  A negative
// denominator (a field below zero) divides like any other.
// With DIV the divergent-flow term -(1/4)(U/G) dv joins V (dv: the centred
// divergence of the velocity field across the face, the sum of the
// divergences of cells a and b), in FP64 as -(U/2) dv dA dBs dBt in the
// numerator.
template <bool DIV = false, typename T>
__device__ __forceinline__ T pseudo_velocity(T U, T hs, T pa, T pb, T us, T s_hi, T s_lo, T ut,
                                             T t_hi, T t_lo, T eps, T dv = T(0))
{
    const T nA = pb - pa, dA = (pb + pa) + eps;
    const T nBs = s_hi - s_lo, dBs = (s_hi + s_lo) + eps;
    const T nBt = t_hi - t_lo, dBt = (t_hi + t_lo) + eps;
    if constexpr (sizeof(T) == 4) {
        const T rh = __builtin_amdgcn_rcpf(hs);
        const T A = nA * __builtin_amdgcn_rcpf(dA);
        const T Bs = nBs * __builtin_amdgcn_rcpf(dBs), Bt = nBt * __builtin_amdgcn_rcpf(dBt);
        const T Urh = U * rh;
        const T c = fabs(U) - T(2) * (U * Urh);
        T v = c * A - (T(0.25) * Urh) * (us * Bs + ut * Bt);
        if constexpr (DIV) v = v - (T(0.5) * Urh) * dv;
        return v;
    } else {
        const T P = dBs * dBt;
        const T c = fabs(U) * hs - T(2) * (U * U);
        const T cross = (us * nBs) * dBt + (ut * nBt) * dBs;
        T num = (c * nA) * P - (T(0.25) * U * dA) * cross;
        if constexpr (DIV) num = num - (T(0.5) * U * dv) * (dA * P);
        return div_nr(num, (hs * dA) * P);
    }
}

// Limiter factors as stored between the stages: computed in limiter
// precision (double) and capped at 1, then kept in double for FP64 grids and
// rounded to float for FP32 grids.  The FP32 variant multiplies V by the
// factor in FP32, and rounding is monotone, so min(float(a), float(b)) is
// float(min(a, b)) exactly: taking the minimum after the rounding changes no
// bit, and the factors travel through LDS and registers at half the size.
template <typename T> using Factor = std::conditional_t<sizeof(T) == 8, double, float>;

// Limited pseudo-velocity; the factors are already capped at 1
// (min(1, a, b) = min(min(1, a), min(1, b)) exactly).
// min(1, f_p) pos(V) + min(1, f_n) neg(V) is the factor of V's own sign
// times V (the other product is an exact zero).
template <typename T, typename F>
__device__ __forceinline__ T limited(T v, F bup_a, F bdn_a, F bup_b, F bdn_b)
{
    const F c = v > T(0) ? fmin(bdn_a, bup_b) : fmin(bup_a, bdn_b);
    return T(c) * v;
}

// Global memory is read and written through buffer descriptors: one
// descriptor per plane of an array (base = the plane's first element, size =
// the plane's bytes, built in scalar registers) and a loop-invariant 32-bit
// byte offset per lane.  No 64-bit address arithmetic per access, and an
// offset past the plane reads zero instead of leaving the array.  The host
// keeps every plane below 2 GiB.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

template <typename T> __device__ __forceinline__ Rsrc plane_rsrc(const T *base, size_t plane, unsigned plane_elems)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)(base + plane * plane_elems), 0,
                                             (int)(plane_elems * (unsigned)sizeof(T)), kRsrcWord3);
}

// byte_off: per-lane offset; s_off: workgroup-uniform offset added to it
// (their sum stays below 2^32; an offset past the plane reads zero)
template <typename T> __device__ __forceinline__ T bload(Rsrc r, unsigned byte_off, unsigned s_off = 0)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, (int)s_off, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, (int)s_off, 0));
}

template <typename T> __device__ __forceinline__ void bstore(Rsrc r, unsigned byte_off, T v)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, v),
                                              r, (int)byte_off, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)byte_off, 0, 0);
}

// A byte offset that every plane's range check rejects: the host keeps each
// plane below 2 GiB, so 2^31 lies past its end (and 2^31 plus an access
// size does not wrap).  A read there returns zero, a write is dropped.
constexpr unsigned kOobOffset = 0x80000000u;

// Store into plane `plane` of an array (when the workgroup-uniform plane_ok
// holds) for the lanes where lane_ok.  Every lane issues it, a disabled lane
// at kOobOffset (plane 0 when plane_ok fails), so that no branch makes the
// number of memory operations a wave has in flight depend on its lanes: the
// counter waits the compiler places before the use of a prefetched value
// then stop at that value's load, not at the prefetches issued after it
// (measured: periodic grids 1.5 % faster in FP64, 3 % in FP32; open grids
// 1.5 % (FP64) and 0.8 % (FP32) once their kernels stopped spilling much --
// with 36 spilled VGPRs the open FP64 kernel had run 13 % slower with it).
template <typename T>
__device__ __forceinline__ void bstore_if(T *base, int plane, bool plane_ok, unsigned plane_elems,
                                          unsigned byte_off, bool lane_ok, T v)
{
    bstore<T>(plane_rsrc<T>(base, plane_ok ? plane : 0, plane_elems),
              plane_ok && lane_ok ? byte_off : kOobOffset, v);
}

// Lane exchange along x inside a wave.  A workgroup's rows are RX lanes long
// and RX divides 64 or is 64, so the x-neighbours of a lane are the adjacent
// lanes of its wave: from_lo(v) is v of lane i-1, from_hi(v) v of lane i+1
// (DPP wave shifts).  The first and last lane of a row receive a value from
// another row (or 0); they hold the outermost halo columns of the region,
// and no output depends on what they compute from it.
//
// A DPP move reads its source from the other lanes only where those lanes
// are active, so it must run with the full exec mask: every exchange is a
// statement of its own in the uniform march (never an arm of a conditional
// expression, which runs for the selected lanes only), and its result is
// pinned there by an empty asm statement so that it is not sunk into a
// lane-masked region either.
constexpr int kDppWaveShr1 = 0x138, kDppWaveShl1 = 0x130;

template <int CTRL> __device__ __forceinline__ float dpp(float v)
{
    float r = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, true));
    asm volatile("" : "+v"(r));
    return r;
}

template <int CTRL> __device__ __forceinline__ double dpp(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, true);
    double r = __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
    asm volatile("" : "+v"(r));
    return r;
}

template <typename T> __device__ __forceinline__ T from_lo(T v) { return dpp<kDppWaveShr1>(v); }
template <typename T> __device__ __forceinline__ T from_hi(T v) { return dpp<kDppWaveShl1>(v); }

// Registers of one plane of a column: the Courant numbers of its x- and
// y-faces and h (needed one iteration ahead) ...
template <typename T> struct PlaneA {
    T u1lo, u1hi, u2lo, u2hi, h;
};
// ... and psi^n and the Courant number of its lower z-face (needed two
// iterations ahead; in a further corrective pass also the two cell arrays
// bx, bn that bound the earlier iterates).
template <typename T> struct PlaneB {
    T pn, u3lo, bx, bn;
};

// ================================================================ fused step

// What a launch of the march computes.  kModeStep: one time step (the
// donor-cell pass and one corrective pass).  A step with k > 1 corrective
// passes (iord = k + 1) runs as a chain of launches: kModeHead is the time
// step that also writes its limited antidiffusive velocity and psi1;
// kModeMid and kModeLast run one further corrective pass on the previous
// launch's result, with the previous limited velocity in the place of the
// Courant numbers.  Their limiter bounds run over the iterate and two cell
// arrays bx, bn, taken cell by cell as max(bx, bn, iterate) and
// min(bx, bn, iterate): psi1 and psi^n (the step's input) after the head
// launch, the running maximum and minimum after a middle one -- where
// bx >= bn, so the same expressions carry them on.  The max/min over a set of
// fields at each of the 7 points equals the 7-point max/min of their
// cell-by-cell max/min, so two arrays stand for every earlier iterate.
// kModeMid writes its velocity and the running bounds on.
enum { kModeStep = 0, kModeHead = 1, kModeMid = 2, kModeLast = 3 };

// Which stages an iteration of the march runs: all of them, or the reduced
// sets of a segment's first, second and last iteration.
enum { kPartFull = 0, kPartFirst = 1, kPartSecond = 2, kPartLast = 3 };

// LDS planes of one workgroup (each padded by one cell on every side).
template <typename T, int RX, int RY, int MODE, bool DIVP = false> struct Smem {
    static constexpr int PX = RX + 2, PP = PX * (RY + 2);
    // planes read only by x-neighbours go through LDS only where
    // x-neighbours are not exchanged between lanes (FP32)
    static constexpr int PX1 = sizeof(T) == 8 ? 1 : PP;
    // kModeStep/kModeHead: psi^n plane t (its ring holds real data);
    // kModeMid/kModeLast: the running upper bound of plane t, with the lower
    // bound in sPm
    T sP[PP];
    static constexpr int PM = MODE >= kModeMid ? PP : 1;
    T sPm[PM];
    T sQ[3][PP];                         // psi1, planes t-2 .. t in fixed slots
    // Courant column sums and h of plane t-1; the y-sums serve only the
    // x-neighbours, which FP64 exchanges between lanes
    T sC1[PP], sC2[PX1], sC3[PP], sH[PP];
    static constexpr int PD = DIVP ? PP : 1;
    T sD[PD];                            // cell divergence of the velocity field: plane t-1
    T sFA1[PX1], sFA2[PP];               // antidiffusive donor fluxes, lower faces
    Factor<T> sBU[PP], sBD[PP];          // limiter factors, plane t-2
    T sFC1[PX1], sFC2[PP];               // corrective fluxes, lower faces
};

// One workgroup advances the output tile (tx, ty) of grid g through planes
// [z0, z1): psi[flip] -> psi[1 - flip].  OPXY: open (zero-gradient)
// boundaries in x and y -- clamped addressing and redirected neighbours;
// OPZ: open in z.  An open grid's tiles whose region and ring lie inside the
// domain with a cell to spare (x_interior) run with OPXY false: there
// clamping and wrapping are both the identity and no lane sits on a
// boundary.  TVEL: Courant numbers that change in time; g holds those of
// the start of the step and tv.w1..w3 those of its end, and the pseudo-
// velocity of every face gains the time-variation term (w - u)/2 (holding u
// over the step leaves the first-order flux (1/2) dt (du/dt) psi, which the
// term takes back).
template <typename T, int RX, int RY, bool OPXY, bool OPZ, bool NONOS, bool VSIGN, bool DIV, int MODE,
          bool TVEL = false>
__device__ __forceinline__ void march(const GridDesc<T> &g, const PassIO<T> &io, int flip, int tx,
                                      int ty, int z0, int z1, double eps_d,
                                      Smem<T, RX, RY, MODE, DIV> &sm,
                                      const TvArgs<T> &tv = TvArgs<T>{})
{
    static_assert(!TVEL || MODE == kModeStep, "the time-variation term belongs to the fused step");
    constexpr bool kPass = MODE >= kModeMid;                      // S1 replaced by a load
    constexpr bool kOuts = MODE == kModeHead || MODE == kModeMid; // velocity + bounds out
    using L = double;  // limiter precision (both variants)
    constexpr int TX = RX - 4, TY = RY - 4;
    constexpr int PX = RX + 2;           // padded row pitch of every LDS plane
    constexpr int XM = -1, XP = 1, YM = -PX, YP = PX;
    T *__restrict__ sP = sm.sP;
    T *__restrict__ sPm = sm.sPm;
    auto &sQ = sm.sQ;
    T *__restrict__ sC1 = sm.sC1, *__restrict__ sC2 = sm.sC2, *__restrict__ sC3 = sm.sC3;
    T *__restrict__ sH = sm.sH, *__restrict__ sFA1 = sm.sFA1, *__restrict__ sFA2 = sm.sFA2;
    T *__restrict__ sD = sm.sD;
    using F = Factor<T>;
    F *__restrict__ sBU = sm.sBU, *__restrict__ sBD = sm.sBD;
    T *__restrict__ sFC1 = sm.sFC1, *__restrict__ sFC2 = sm.sFC2;

    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const T eps = T(eps_d);
    const L eps_l = eps_d;
    const T *psi_in = g.psi[flip];
    T *psi_out = g.psi[1 - flip];

    const int tid = threadIdx.x;
    const int lx = tid % RX, ly = tid / RX;
    const int gx = tx * TX - 2 + lx;
    const int gy = ty * TY - 2 + ly;
    const int q = (ly + 1) * PX + lx + 1;

    // in-plane offsets into the global arrays
    const int cx = cell_of<OPXY>(gx, nx), cy = cell_of<OPXY>(gy, ny);
    const unsigned pc_cells = (unsigned)nx * ny;
    const unsigned pc_u1 = (unsigned)(nx + 1) * ny;
    const unsigned pc_u2 = (unsigned)nx * (ny + 1);
    const unsigned o_c = cy * nx + cx;
    const unsigned o_u1lo = cy * (nx + 1) + face_lo<OPXY>(gx, nx);
    const unsigned o_u1hi = cy * (nx + 1) + face_hi<OPXY>(gx, nx);
    const unsigned o_u2lo = face_lo<OPXY>(gy, ny) * nx + cx;
    const unsigned o_u2hi = face_hi<OPXY>(gy, ny) * nx + cx;
    // The ring of the psi^n plane -- the padded LDS cells around the region,
    // 2 RY of them left and right, 2 RX below and above -- is loaded by the
    // first 2 (RX + RY) threads, one cell each (the other waves skip it).
    // A further corrective pass has no donor-cell pass and needs no ring.
    constexpr int NRX = 2 * RY, NR = 2 * (RX + RY);
    static_assert(NR <= RX * RY, "ring larger than the workgroup");
    const bool has_ring = !kPass && tid < NR;
    int rgx = gx, rgy = gy, p_ring = q;
    if (tid < NRX) {
        const int side = tid / RY, row = tid % RY;
        rgx = tx * TX - 2 + (side ? RX : -1);
        rgy = ty * TY - 2 + row;
        p_ring = (row + 1) * PX + (side ? RX + 1 : 0);
    } else if (has_ring) {
        const int side = (tid - NRX) / RX, col = (tid - NRX) % RX;
        rgx = tx * TX - 2 + col;
        rgy = ty * TY - 2 + (side ? RY : -1);
        p_ring = (side ? RY + 1 : 0) * PX + col + 1;
    }
    const unsigned o_ring = cell_of<OPXY>(rgy, ny) * nx + cell_of<OPXY>(rgx, nx);
    // byte offsets within a plane (the host keeps every plane below 2 GiB)
    const unsigned b_c = o_c * (unsigned)sizeof(T);
    const unsigned b_u1lo = o_u1lo * (unsigned)sizeof(T), b_u1hi = o_u1hi * (unsigned)sizeof(T);
    const unsigned b_u2lo = o_u2lo * (unsigned)sizeof(T), b_u2hi = o_u2hi * (unsigned)sizeof(T);
    const unsigned b_ring = o_ring * (unsigned)sizeof(T);

    // cell-centred neighbour offsets: at an open boundary a read of the cell
    // beyond it is redirected to the cell itself (zero gradient)
    const bool edge_lo = OPXY && gx <= 0, edge_hi = OPXY && gx >= nx - 1;
    const int cxm = edge_lo ? 0 : XM;
    const int cxp = edge_hi ? 0 : XP;
    const int cym = (OPXY && gy <= 0) ? 0 : YM;
    const int cyp = (OPXY && gy >= ny - 1) ? 0 : YP;

    // boundary-normal faces of an open domain carry no antidiffusive flux
    const bool zero_v1 = OPXY && (gx <= 0 || gx >= nx);
    const bool zero_v2 = OPXY && (gy <= 0 || gy >= ny);
    const bool is_out = lx >= 2 && lx < RX - 2 && ly >= 2 && ly < RY - 2 && gx < nx && gy < ny;
    // Writers of the limited velocity (kModeHead, kModeMid): the lower x- and
    // y-faces of the output cells, and face nx (ny) of a row (column) from the
    // lane just past its last cell, which lies within one cell of the tile.
    const bool w1_lane = ly >= 2 && ly < RY - 2 && gy < ny && lx >= 2 && lx <= RX - 2 &&
                         (gx == nx || (lx < RX - 2 && gx < nx));
    const bool w2_lane = lx >= 2 && lx < RX - 2 && gx < nx && ly >= 2 && ly <= RY - 2 &&
                         (gy == ny || (ly < RY - 2 && gy < ny));
    const unsigned b_w1 = ((unsigned)gy * (nx + 1) + (unsigned)gx) * (unsigned)sizeof(T);
    const unsigned b_w2 = ((unsigned)gy * nx + (unsigned)gx) * (unsigned)sizeof(T);

    // plane index of position t along z: wrapped (periodic) or clamped (open);
    // the march advances it by one per iteration without a division
    auto plane_of = [&](int t) { return cell_of<OPZ>(t, nz); };
    auto zface_of = [&](int t) { return face_lo<OPZ>(t, nz); };
    auto load_a = [&](int k, PlaneA<T> &r) {
        const Rsrc hp = plane_rsrc(g.h, k, pc_cells);
        const Rsrc u1p = plane_rsrc(g.u1, k, pc_u1);
        const Rsrc u2p = plane_rsrc(g.u2, k, pc_u2);
        r.h = bload<T>(hp, b_c);
        r.u1lo = bload<T>(u1p, b_u1lo);
        if (OPXY) {
            r.u1hi = bload<T>(u1p, b_u1hi);
            r.u2lo = bload<T>(u2p, b_u2lo);
            r.u2hi = bload<T>(u2p, b_u2hi);
        } else {
            // periodic: the upper faces are the next face along the axis and
            // the lower y-face has the cell's own index, so no offsets of
            // their own are held
            r.u1hi = bload<T>(u1p, b_u1lo + (unsigned)sizeof(T));
            r.u2lo = bload<T>(u2p, b_c);
            r.u2hi = bload<T>(u2p, b_c, (unsigned)nx * (unsigned)sizeof(T));
        }
    };
    auto load_b = [&](int k, int kf, PlaneB<T> &r) {
        const Rsrc pp = plane_rsrc(psi_in, k, pc_cells);
        const Rsrc u3p = plane_rsrc(g.u3, kf, pc_cells);
        r.pn = bload<T>(pp, b_c);
        r.u3lo = bload<T>(u3p, b_c);
        if constexpr (kPass && NONOS) {
            r.bx = bload<T>(plane_rsrc(io.bmx, k, pc_cells), b_c);
            r.bn = bload<T>(plane_rsrc(io.bmn, k, pc_cells), b_c);
        }
    };
    // The ring threads load their ring cell of a plane late in the
    // iteration before it is stored (it is not held across the heavy phase).
    // Issued by every lane (the others read at kOobOffset and get zero), so
    // that it leaves no branch around a memory operation (see bstore_if).
    auto load_ring = [&](int k) {
        if constexpr (kPass) return T(0);
        else return bload<T>(plane_rsrc(psi_in, k, pc_cells), has_ring ? b_ring : kOobOffset);
    };

    const int t0 = z0 - 2, tend = z1 + 2;
    PlaneA<T> curA, nxA;
    PlaneB<T> cur, nx1, nx2;
    int ka = plane_of(t0 + 1);                     // plane of t+1 (load_a)
    int kb = plane_of(t0 + 2);                     // plane of t+2 (load_b)
    load_a(plane_of(t0), curA);
    load_b(plane_of(t0), zface_of(t0), cur);
    load_b(ka, zface_of(t0 + 1), nx1);
    const T pn_prev = bload<T>(plane_rsrc(psi_in, plane_of(t0 - 1), pc_cells), b_c);
    // further pass: running bounds (earlier iterates and the input) of the
    // column at planes t and t-1; sP/sPm hold the planes for the neighbours
    T M_c = T(0), m_c = T(0), M_m1 = T(0), m_m1 = T(0);
    if constexpr (kPass && NONOS) {
        const int kp = plane_of(t0 - 1);
        const T bx_p = bload<T>(plane_rsrc(io.bmx, kp, pc_cells), b_c);
        const T bn_p = bload<T>(plane_rsrc(io.bmn, kp, pc_cells), b_c);
        M_m1 = fmax(fmax(bx_p, bn_p), pn_prev);
        m_m1 = fmin(fmin(bx_p, bn_p), pn_prev);
        M_c = fmax(fmax(cur.bx, cur.bn), cur.pn);
        m_c = fmin(fmin(cur.bx, cur.bn), cur.pn);
        sP[q] = M_c;
        sPm[q] = m_c;
    } else if constexpr (!kPass) {
        sP[q] = cur.pn;
        if (has_ring) sP[p_ring] = load_ring(plane_of(t0));
    }
    T rng = load_ring(ka);  // ring cell of plane t+1

    // z-history of the column
    T f3_c = donor(pn_prev, cur.pn, cur.u3lo);  // psi^n flux, face t
    T pn_m1 = pn_prev;
    // max/min of psi^n over the in-plane 5-point stencil of plane t-1 and the
    // plane below it: the bounds at t-1 add only psi^n(t) to these
    T zmx_m1 = T(0), zmn_m1 = T(0);
    T u1_m1 = T(0), u2_m1 = T(0);               // lower-face Courant, plane t-1
    // TVEL: plane of position t, for the end-of-step Courant numbers that
    // S3 of iteration t reads (loaded at the top of the iteration, not held
    // across iterations: the registers of the prefetch are all taken)
    int kt = plane_of(t0);
    T rh_m1 = T(1), rh_m2 = T(1), rh_m3 = T(1); // 1/h of planes t-1 .. t-3
    // Own-column psi1 of planes t-1 .. t-3 and the Courant sums and h of plane
    // t-1 also sit in LDS (for the neighbours); the column keeps its own copy
    // in registers.
    // x-neighbours by lane exchange (FP64, where LDS bandwidth binds) or
    // through LDS (FP32, where the exchange costs more issue than it saves)
    constexpr bool kDpp = sizeof(T) == 8;
    // FP32 grids open in z with 32x32 regions read the S3 operands of planes
    // t-1 and t-2 before (D) (below): measured faster there, slower with
    // 32x24 regions and on periodic grids
    constexpr bool kEarlyS3 = !kDpp && OPZ && RY == 32;
    constexpr bool kFenceFaces = kDpp || OPXY || OPZ;
    T r_p1_m1 = T(0), r_p1_m2 = T(0), r_p1_m3 = T(0);
    T r_c1_m1 = T(0), r_c2_m1 = T(0), r_c3_m1 = T(0), r_h_m1 = T(0);
    T r_d_m1 = T(0);  // divergence of the column's cell at plane t-1 (DIV)
    T v1_m2 = T(0), v2_m2 = T(0), v3_m1 = T(0); // V at plane t-2, V3 at face t-1
    T fa3_m1 = T(0);                            // antidiffusive flux, face t-1
    F bu_m2 = F(1), bd_m2 = F(1);               // limiter factors (capped at 1), plane t-2
    T fc3_m2 = T(0), fc3_m3 = T(0);             // corrective flux, faces t-2, t-3
    T fc1_m3 = T(0), fc2_m3 = T(0);             // corrective fluxes, lower x/y faces of plane t-3

    // zopen: the z-boundary handling of this iteration (OPZ, or false on the
    // planes away from an open top and bottom, where it is the identity)
    // FP32 runs the reduced first, second and last iterations (below); the
    // FP64 kernels, at their register limit, spilled with the first two
    // (22 VGPRs in the periodic limiter kernel) and run only the last one
    // reduced
    constexpr bool kTrimFill = sizeof(T) == 4;
    // part: which stages the iteration runs.  A segment's first iteration
    // (t = z0 - 2) needs only psi1 of its plane (later iterations read it),
    // its second (t = z0 - 1) psi1 and the pseudo-velocity on z-face t (the
    // limiter factors of plane z0 - 1 need it), its last (t = z1 + 2) only S7
    // of plane z1 - 1: every other result of those iterations belongs to a
    // plane no output of the segment depends on.
    auto iter = [&](const int t, auto slot, auto zopen, auto part) {
        constexpr int P = decltype(part)::value;
        constexpr bool OZ = decltype(zopen)::value;
        constexpr int s0 = decltype(slot)::value;           // slot of plane t (held t-3)
        constexpr int s1 = (s0 + 2) % 3, s2 = (s0 + 1) % 3; // planes t-1, t-2
        // end-of-step Courant numbers of the lower x/y faces of plane t-1 and
        // of z-face t (TVEL), issued before the prefetch so that waiting for
        // them in phase 2 does not wait for it
        T w1_m1 = T(0), w2_m1 = T(0), w3_c = T(0);
        if constexpr (TVEL && P != kPartLast) {
            const int kp = OPZ ? clampi(t - 1, 0, nz - 1) : (kt == 0 ? nz - 1 : kt - 1);
            const int kf = OPZ ? clampi(t, 0, nz) : kt;
            if constexpr (P == kPartFull) {
                w1_m1 = bload<T>(plane_rsrc(tv.w1, kp, pc_u1), b_u1lo);
                w2_m1 = bload<T>(plane_rsrc(tv.w2, kp, pc_u2), OPXY ? b_u2lo : b_c);
            }
            if constexpr (P != kPartFirst) w3_c = bload<T>(plane_rsrc(tv.w3, kf, pc_cells), b_c);
            kt = OPZ ? clampi(t + 1, 0, nz - 1) : (kt + 1 == nz ? 0 : kt + 1);
        }
        if constexpr (P != kPartLast) {
            load_a(ka, nxA);
            load_b(kb, OZ ? zface_of(t + 2) : kb, nx2);
            ka = kb;
            kb = OZ ? clampi(t + 3, 0, nz - 1) : (kb + 1 == nz ? 0 : kb + 1);
        }
        __syncthreads();  // (B) psi^n(t), sums/h of t-1, corrective y-fluxes of t-3 are visible
        // own-column values of planes t-1 .. t-3
        const T p1_m1 = r_p1_m1, p1_m2 = r_p1_m2, p1_m3 = r_p1_m3;
        const T c1_m1 = r_c1_m1, c2_m1 = r_c2_m1, c3_m1 = r_c3_m1, h_m1 = r_h_m1;
        const T d_m1 = r_d_m1;

        // limiter factors of plane t-2 (computed last iteration) for the
        // neighbours' corrective pass after (F); their previous contents were
        // last read before (B)
        if (NONOS && P == kPartFull) {
            sBU[q] = bu_m2;
            sBD[q] = bd_m2;
        }
        if constexpr (P == kPartFull || P == kPartLast) {
            // ---- S7 at plane t-3 (its corrective fluxes were stored last iteration)
            T fc1hi;
            if constexpr (kDpp) fc1hi = from_hi(fc1_m3);
            else fc1hi = sFC1[q + XP];
            const T fc2hi = sFC2[q + YP];
            const T fc2lo = fc2_m3;
            const T res = p1_m3 - (((fc1hi - fc1_m3) + (fc2hi - fc2lo)) + (fc3_m2 - fc3_m3)) * rh_m3;
            bstore_if<T>(psi_out, t - 3, t >= z0 + 3 && t <= tend, pc_cells, b_c, is_out, res);
        }
        if constexpr (P == kPartLast) return;

        const bool own_plane = t >= z0 && t < z1;  // plane t is one of the segment's
        T p1_c, zmx_c, zmn_c, rh_c, f3hi = T(0);
        if constexpr (kPass) {
            // ---- the iterate of plane t is the input; the running bounds over
            // the in-plane 5-point stencil of plane t and the plane below it
            rh_c = rcp_nr(curA.h);
            p1_c = cur.pn;
            const bool zlo = OZ && t <= 0;
            zmx_c = fmax(fmax(fmax(sP[q + cxm], sP[q + cxp]), fmax(sP[q + cym], sP[q + cyp])),
                         zlo ? M_c : fmax(M_c, M_m1));
            zmn_c = fmin(fmin(fmin(sPm[q + cxm], sPm[q + cxp]), fmin(sPm[q + cym], sPm[q + cyp])),
                         zlo ? m_c : fmin(m_c, m_m1));
            if constexpr (MODE == kModeMid && NONOS) {
                bstore_if<T>(io.mx, t, own_plane, pc_cells, b_c, is_out, M_c);
                bstore_if<T>(io.mn, t, own_plane, pc_cells, b_c, is_out, m_c);
            }
        } else {
            // ---- S1+S2 at plane t
            const T pL = sP[q + cxm], pR = sP[q + cxp];
            const T pD = sP[q + cym], pU = sP[q + cyp];
            const T f1lo = donor(pL, cur.pn, curA.u1lo), f1hi = donor(cur.pn, pR, curA.u1hi);
            const T f2lo = donor(pD, cur.pn, curA.u2lo), f2hi = donor(cur.pn, pU, curA.u2hi);
            f3hi = donor(cur.pn, nx1.pn, nx1.u3lo);
            rh_c = rcp_nr(curA.h);
            p1_c = cur.pn - (((f1hi - f1lo) + (f2hi - f2lo)) + (f3hi - f3_c)) * rh_c;
            // (at an open bottom the plane below t is t itself, already counted)
            const bool zlo = OZ && t <= 0;
            zmx_c = fmax(fmax(fmax(pL, pR), fmax(pD, pU)), zlo ? cur.pn : fmax(cur.pn, pn_m1));
            zmn_c = fmin(fmin(fmin(pL, pR), fmin(pD, pU)), zlo ? cur.pn : fmin(cur.pn, pn_m1));
            if constexpr (MODE == kModeHead && NONOS) {
                // psi1 for the next pass's bounds (psi^n stays in the input)
                bstore_if<T>(io.mx, t, own_plane, pc_cells, b_c, is_out, p1_c);
            }
        }
        sQ[s0][q] = p1_c;  // psi1(t-3) of this slot was last read before (B)
        const T c1_c = curA.u1lo + curA.u1hi;
        const T c2_c = curA.u2lo + curA.u2hi;
        const T c3_c = cur.u3lo + nx1.u3lo;
        // divergence of the velocity field in the cell of plane t (DIV)
        T d_c = T(0);
        if constexpr (DIV)
            d_c = ((curA.u1hi - curA.u1lo) + (curA.u2hi - curA.u2lo)) + (nx1.u3lo - cur.u3lo);
        // FP32, open in z, 32x32 regions: the LDS operands of S3 at plane t-1
        // that were complete at (B) -- psi1 of planes t-1 and t-2, h and the
        // Courant sums of plane t-1 -- are read in this phase, beside the S1
        // arithmetic, so that only psi1 of plane t waits for (D) (2.2 % faster
        // open FP32 step, measured, also in the iterations without the
        // z-boundary handling; 1.8 % slower with 32x24 regions and 4 % slower
        // on periodic grids).  FP64 has no registers to hold them across (D).
        struct {
            T qd, qyp, qym, qa, qxp, qxm;        // psi1(t-1), own stencil
            T xh, xc2, xc3, xqyp, xqym, xlo, xd; // cell a of the lower x-face
            T yxp, yxm, yh, yc3, yc1, ylo, yd;   // cell a of the lower y-face
        } e{};
        if constexpr (kEarlyS3 && P != kPartFirst) {
            const bool clo = OZ && t - 1 <= 0;
            const T *Qc = sQ[s1];
            const T *Qlo = clo ? sQ[s1] : sQ[s2];
            e.qd = Qc[q + YM], e.qyp = Qc[q + cyp], e.qym = Qc[q + cym];
            e.qa = Qc[q + XM], e.qxp = Qc[q + cxp], e.qxm = Qc[q + cxm];
            e.xh = sH[q + XM], e.xc2 = sC2[q + XM], e.xc3 = sC3[q + XM];
            e.xqyp = Qc[q + XM + cyp], e.xqym = Qc[q + XM + cym], e.xlo = Qlo[q + XM];
            e.yxp = Qc[q + YM + cxp], e.yxm = Qc[q + YM + cxm];
            e.yh = sH[q + YM], e.yc3 = sC3[q + YM], e.yc1 = sC1[q + YM], e.ylo = Qlo[q + YM];
            if constexpr (DIV) e.xd = sD[q + XM], e.yd = sD[q + YM];
        }
        __syncthreads();  // (D) psi1(t) and the limiter factors of t-2 are visible

        T v1 = T(0), v2 = T(0), v3 = T(0), fa1 = T(0), fa2 = T(0), fa3_c = T(0);
        // FP32: the LDS operands of S6 at plane t-2 (psi1 and the limiter
        // factors of the x- and y-neighbours), written before (D), are read
        // during the arithmetic of this phase instead of after (F) (1.6 %
        // faster FP32 step, measured; FP64, at its register limit, keeps them
        // after (F))
        T q6_y = T(0), q6_x = T(0);
        F bu6_y = F(1), bd6_y = F(1), bu6_x = F(1), bd6_x = F(1);
        T pc_xlo = T(0), p2_xm = T(0);
        T mx = T(0), mn = T(0);
        if constexpr (P != kPartFirst) {
            // ---- S3 at plane p = t-1 (lower x- and y-faces) and on face t
            const int p = t - 1;
            const bool clo = OZ && p <= 0, chi = OZ && p >= nz - 1;
            const T *Qc = sQ[s1];
            const T *Qb = sQ[s0];
            const T *Qlo = clo ? sQ[s1] : sQ[s2];
            const T *Qhi = chi ? sQ[s1] : sQ[s0];
            const T p1_lo = clo ? p1_m1 : p1_m2;
            const T p1_hi = chi ? p1_m1 : p1_c;

            // y-neighbours from LDS; x-neighbours from the adjacent lanes
            // (FP64) or from LDS (FP32); at an open x-boundary the cell
            // beyond is the cell itself
            // ratio operands: |psi1| with the variable-sign option
            auto av = [](T x) -> T {
                if constexpr (VSIGN) return fabs(x);
                else return x;
            };
            T qd, qyp_, qym_;  // qd: cell a of the lower y-face
            if constexpr (kEarlyS3) qd = e.qd, qyp_ = e.qyp, qym_ = e.qym;
            else qd = Qc[q + YM], qyp_ = Qc[q + cyp], qym_ = Qc[q + cym];
            T qa, qxp_, qxm_;  // qa: cell a of the lower x-face
            if constexpr (kDpp) {
                qa = from_lo(p1_m1);
                const T p1_xhi = from_hi(p1_m1);
                qxp_ = edge_hi ? p1_m1 : p1_xhi;
                qxm_ = edge_lo ? p1_m1 : qa;
                // psi1 of t and t-2 of the lower x-neighbour (reused below)
                pc_xlo = from_lo(p1_c);
                p2_xm = from_lo(p1_m2);
            } else if constexpr (kEarlyS3) {
                qa = e.qa, qxp_ = e.qxp, qxm_ = e.qxm;
            } else {
                qa = Qc[q + XM];
                qxp_ = Qc[q + cxp];
                qxm_ = Qc[q + cxm];
            }
            if constexpr (P == kPartFull) {
                // x-face between a = (lx-1) and b = own; transverse axes y then z
                T h_a, c2_a, c3_a, qyp_a, qym_a, phi_a, plo_a, d_a = T(0);
                if constexpr (kDpp) {
                    h_a = from_lo(h_m1), c2_a = from_lo(c2_m1), c3_a = from_lo(c3_m1);
                    qyp_a = from_lo(qyp_), qym_a = from_lo(qym_);
                    if constexpr (DIV) d_a = from_lo(d_m1);
                    phi_a = chi ? qa : pc_xlo, plo_a = clo ? qa : p2_xm;
                } else if constexpr (kEarlyS3) {
                    h_a = e.xh, c2_a = e.xc2, c3_a = e.xc3;
                    qyp_a = e.xqyp, qym_a = e.xqym;
                    phi_a = Qhi[q + XM], plo_a = e.xlo;
                    if constexpr (DIV) d_a = e.xd;
                } else {
                    h_a = sH[q + XM], c2_a = sC2[q + XM], c3_a = sC3[q + XM];
                    qyp_a = Qc[q + XM + cyp], qym_a = Qc[q + XM + cym];
                    phi_a = Qhi[q + XM], plo_a = Qlo[q + XM];
                    if constexpr (DIV) d_a = sD[q + XM];
                }
                v1 = pseudo_velocity<DIV>(u1_m1, h_a + h_m1, av(qa), av(p1_m1), c2_a + c2_m1,
                                          av(qyp_) + av(qyp_a), av(qym_) + av(qym_a), c3_a + c3_m1,
                                          av(p1_hi) + av(phi_a), av(p1_lo) + av(plo_a), eps,
                                          d_a + d_m1);
                if constexpr (TVEL) v1 = v1 + T(0.5) * (w1_m1 - u1_m1);
                if (zero_v1) v1 = T(0);
            }
            // the three faces are scheduled one after another: each face's
            // temporaries die before the next face's reads are issued (FP64,
            // at its register limit, and open FP32 grids); periodic FP32 lets
            // the compiler hoist the y-face's LDS reads (3.5 % faster step,
            // measured)
            if constexpr (kFenceFaces) __builtin_amdgcn_sched_barrier(0);
            if constexpr (P == kPartFull) {
                // y-face between a = (ly-1) and b = own; transverse axes z then x
                T d_ya = T(0);
                if constexpr (kEarlyS3) {
                    if constexpr (DIV) d_ya = e.yd;
                    v2 = pseudo_velocity<DIV>(u2_m1, e.yh + h_m1, av(qd), av(p1_m1), e.yc3 + c3_m1,
                                              av(p1_hi) + av(Qhi[q + YM]), av(p1_lo) + av(e.ylo),
                                              e.yc1 + c1_m1, av(qxp_) + av(e.yxp),
                                              av(qxm_) + av(e.yxm), eps, d_ya + d_m1);
                } else {
                    T qd_xp, qd_xm;
                    if constexpr (kDpp) {
                        const T xhi = from_hi(qd), xlo = from_lo(qd);
                        qd_xp = edge_hi ? qd : xhi;
                        qd_xm = edge_lo ? qd : xlo;
                    } else {
                        qd_xp = Qc[q + YM + cxp];
                        qd_xm = Qc[q + YM + cxm];
                    }
                    if constexpr (DIV) d_ya = sD[q + YM];
                    v2 = pseudo_velocity<DIV>(u2_m1, sH[q + YM] + h_m1, av(qd), av(p1_m1),
                                              sC3[q + YM] + c3_m1, av(p1_hi) + av(Qhi[q + YM]),
                                              av(p1_lo) + av(Qlo[q + YM]), sC1[q + YM] + c1_m1,
                                              av(qxp_) + av(qd_xp), av(qxm_) + av(qd_xm), eps,
                                              d_ya + d_m1);
                }
                if constexpr (TVEL) v2 = v2 + T(0.5) * (w2_m1 - u2_m1);
                if (zero_v2) v2 = T(0);
            }
            if constexpr (kFenceFaces) __builtin_amdgcn_sched_barrier(0);
            if constexpr (!kDpp && P == kPartFull) {
                q6_y = sQ[s2][q + YM];
                if (NONOS) {
                    bu6_y = sBU[q + YM];
                    bd6_y = sBD[q + YM];
                }
                q6_x = sQ[s2][q + XM];
                if (NONOS) {
                    bu6_x = sBU[q + XM];
                    bd6_x = sBD[q + XM];
                }
            }
            {
                // z-face t between a = plane t-1 and b = plane t; transverse x then y
                T pc_xp, pc_xm;
                if constexpr (kDpp) {
                    const T xhi = from_hi(p1_c);
                    pc_xp = edge_hi ? p1_c : xhi;
                    pc_xm = edge_lo ? p1_c : pc_xlo;
                } else {
                    pc_xp = Qb[q + cxp];
                    pc_xm = Qb[q + cxm];
                }
                v3 = pseudo_velocity<DIV>(cur.u3lo, h_m1 + curA.h, av(p1_m1), av(p1_c),
                                          c1_m1 + c1_c, av(pc_xp) + av(qxp_), av(pc_xm) + av(qxm_),
                                          c2_m1 + c2_c, av(Qb[q + cyp]) + av(qyp_),
                                          av(Qb[q + cym]) + av(qym_), eps, d_m1 + d_c);
            }
            if constexpr (TVEL) v3 = v3 + T(0.5) * (w3_c - cur.u3lo);
            if (OZ && (t <= 0 || t >= nz)) v3 = T(0);
            if (NONOS && P == kPartFull) {
                // ---- S4 bounds at plane p
                if constexpr (kPass) {
                    // the running bounds of plane t complete the 7 points (at
                    // an open top the plane above p is p itself)
                    mx = chi ? zmx_m1 : fmax(zmx_m1, M_c);
                    mn = chi ? zmn_m1 : fmin(zmn_m1, m_c);
                } else {
                    // psi^n(t) is the plane above p (at an open top, p itself)
                    const T pn_hi = chi ? pn_m1 : cur.pn;
                    mx = fmax(fmax(fmax(zmx_m1, fmax(qxm_, qxp_)), fmax(fmax(qym_, qyp_), p1_m1)),
                              fmax(pn_hi, fmax(p1_lo, p1_hi)));
                    mn = fmin(fmin(fmin(zmn_m1, fmin(qxm_, qxp_)), fmin(fmin(qym_, qyp_), p1_m1)),
                              fmin(pn_hi, fmin(p1_lo, p1_hi)));
                }
                fa1 = donor(qa, p1_m1, v1);
                fa2 = donor(qd, p1_m1, v2);
                if constexpr (!kDpp) sFA1[q] = fa1;
                sFA2[q] = fa2;
            }
            if (NONOS) fa3_c = donor(p1_m1, p1_c, v3);
        }
        // psi^n of plane t+1: every read of plane t in sP happened before (D)
        if constexpr (!kPass) {
            sP[q] = nx1.pn;
            if (has_ring) sP[p_ring] = rng;
        }
        // the first two iterations of a segment compute no limiter factors or
        // corrective fluxes, and so need no (F)
        if constexpr (P == kPartFull) __syncthreads();  // (F) antidiffusive fluxes visible

        F bu_m1 = F(1), bd_m1 = F(1);
        if (NONOS && P == kPartFull) {
            // ---- S5 limiter factors at plane t-1
            T fa1_hi;
            if constexpr (kDpp) fa1_hi = from_hi(fa1);
            else fa1_hi = sFA1[q + XP];
            const L x_lo = L(fa1), x_hi = L(fa1_hi);
            const L y_lo = L(fa2), y_hi = L(sFA2[q + YP]);
            const L z_lo = L(fa3_m1), z_hi = L(fa3_c);
            // IN and OUT (the sums of the fluxes into and out of the cell):
            // every face flux adds its magnitude to one of them, so with
            // ab = sum |F| and nt = the net inflow (lower faces minus upper),
            // IN = (ab + nt)/2 and OUT = (ab - nt)/2 -- 12 operations fewer than
            // six max/min pairs (FP32 step 2.7 % faster, measured).  Where no
            // face brings flux in, ab + nt is an exact zero (each term of nt is
            // then the exact negation of the same term of ab), as is ab - nt
            // where none takes flux out.
            const L ab = ((fabs(x_lo) + fabs(x_hi)) + (fabs(y_lo) + fabs(y_hi))) + (fabs(z_lo) + fabs(z_hi));
            const L nt = ((x_lo - x_hi) + (y_lo - y_hi)) + (z_lo - z_hi);
            // beta_up = (mx - psi1) h / (IN + eps), beta_dn = (psi1 - mn) h / (OUT + eps),
            // over the common denominator (IN + eps)(OUT + eps)
            const L din = fma(ab + nt, L(0.5), eps_l), dou = fma(ab - nt, L(0.5), eps_l);
            const L r = rcp_nr(din * dou) * L(h_m1);
            bu_m1 = F(fmin(L(1), ((L(mx) - L(p1_m1)) * dou) * r));
            bd_m1 = F(fmin(L(1), ((L(p1_m1) - L(mn)) * din) * r));
        }

        T fc1_r = T(0), fc2_r = T(0), fc3_m1 = T(0);
        if constexpr (P == kPartFull) {
            // ---- S6 + corrective fluxes at plane r = t-2 (lower faces) and on face t-1;
            // the y-fluxes of t-3 in sFC2 were read before (D)
            T vt1 = v1_m2, vt2 = v2_m2, vt3 = v3_m1;
            if (NONOS) {
                F bu_a, bd_a;
                if constexpr (kDpp) bu_a = from_lo(bu_m2), bd_a = from_lo(bd_m2);
                else bu_a = bu6_x, bd_a = bd6_x;
                vt1 = limited(v1_m2, bu_a, bd_a, bu_m2, bd_m2);
                if constexpr (kDpp) bu6_y = sBU[q + YM], bd6_y = sBD[q + YM];
                vt2 = limited(v2_m2, bu6_y, bd6_y, bu_m2, bd_m2);
                vt3 = limited(v3_m1, bu_m2, bd_m2, bu_m1, bd_m1);
            }
            if (zero_v1) vt1 = T(0);
            if (zero_v2) vt2 = T(0);
            if (OZ && (t - 1 <= 0 || t - 1 >= nz)) vt3 = T(0);
            if constexpr (kOuts) {
                // the limited velocity of the segment's planes and of its
                // z-faces (face nz from the segment that ends there)
                const int r = t - 2, f = t - 1;
                const bool r_ok = r >= z0 && r < z1;
                bstore_if<T>(io.w1, r, r_ok, pc_u1, b_w1, w1_lane, vt1);
                bstore_if<T>(io.w2, r, r_ok, pc_u2, b_w2, w2_lane, vt2);
                bstore_if<T>(io.w3, f, (f >= z0 && f < z1) || (f == nz && z1 == nz), pc_cells, b_c,
                             is_out, vt3);
            }
            if constexpr (!kDpp) p2_xm = q6_x;
            fc1_r = donor(p2_xm, p1_m2, vt1);
            if constexpr (kDpp) q6_y = sQ[s2][q + YM];
            fc2_r = donor(q6_y, p1_m2, vt2);
            if constexpr (!kDpp) sFC1[q] = fc1_r;
            sFC2[q] = fc2_r;
            fc3_m1 = donor(p1_m2, p1_m1, vt3);
        }
        // sums/h of plane t for the next iteration: the reads of plane t-1
        // happened before (F) (the first two iterations of a segment do not
        // read them)
        sC1[q] = c1_c;
        if constexpr (!kDpp) sC2[q] = c2_c;
        sC3[q] = c3_c;
        sH[q] = curA.h;
        if constexpr (DIV) sD[q] = d_c;
        rng = load_ring(ka);  // plane t+2
        if constexpr (kPass && NONOS) {
            // running bounds of plane t+1 for the next iteration's stencil;
            // every read of sP/sPm of plane t happened before (D)
            const T M_n = fmax(fmax(nx1.bx, nx1.bn), nx1.pn);
            const T m_n = fmin(fmin(nx1.bx, nx1.bn), nx1.pn);
            sP[q] = M_n;
            sPm[q] = m_n;
            M_m1 = M_c;
            m_m1 = m_c;
            M_c = M_n;
            m_c = m_n;
        }

        // ---- hand the planes to the next iteration
        pn_m1 = cur.pn;
        zmx_m1 = zmx_c;
        zmn_m1 = zmn_c;
        u1_m1 = curA.u1lo;
        u2_m1 = curA.u2lo;
        rh_m3 = rh_m2;
        rh_m2 = rh_m1;
        rh_m1 = rh_c;
        f3_c = f3hi;
        v1_m2 = v1;
        v2_m2 = v2;
        v3_m1 = v3;
        fa3_m1 = fa3_c;
        bu_m2 = bu_m1;
        bd_m2 = bd_m1;
        fc3_m3 = fc3_m2;
        fc3_m2 = fc3_m1;
        fc1_m3 = fc1_r;
        fc2_m3 = fc2_r;
        {
            r_p1_m3 = p1_m2;
            r_p1_m2 = p1_m1;
            r_p1_m1 = p1_c;
            r_c1_m1 = c1_c;
            r_c2_m1 = c2_c;
            r_c3_m1 = c3_c;
            r_h_m1 = curA.h;
            r_d_m1 = d_c;
        }
        curA = nxA;
        cur = nx1;
        nx1 = nx2;
    };

    // Unrolled by three so the psi1 planes sit in fixed slots: the slot of
    // position t is (t - t0 + shift) mod 3, with shift chosen so that the
    // last iteration takes slot 2.
    // With an open top and bottom, groups of three iterations t in
    // [2, nz - 4] take the code without the z-boundary handling: every
    // z-boundary test of such an iteration is false, and the planes it loads
    // (up to t + 3) need no clamping.
    using S0 = std::integral_constant<int, 0>;
    using S1 = std::integral_constant<int, 1>;
    using S2 = std::integral_constant<int, 2>;
    using ZO = std::bool_constant<OPZ>;
    using Full = std::integral_constant<int, kPartFull>;
    const int n_iter = tend - t0 + 1;  // z1 - z0 + 5 >= 6
    int t = t0;
    if constexpr (kTrimFill) {
        // the first two iterations and the last one run their reduced parts;
        // the iterations between them run their count modulo three first,
        // then groups of three (slots 2, 0, 1)
        using First = std::integral_constant<int, kPartFirst>;
        using Second = std::integral_constant<int, kPartSecond>;
        using Last = std::integral_constant<int, kPartLast>;
        switch (n_iter % 3) {
        case 0:  // shift 0
            iter(t, S0{}, ZO{}, First{});
            iter(t + 1, S1{}, ZO{}, Second{});
            t += 2;
            break;
        case 2:  // shift 1
            iter(t, S1{}, ZO{}, First{});
            iter(t + 1, S2{}, ZO{}, Second{});
            iter(t + 2, S0{}, ZO{}, Full{});
            iter(t + 3, S1{}, ZO{}, Full{});
            t += 4;
            break;
        default:  // 1: shift 2
            iter(t, S2{}, ZO{}, First{});
            iter(t + 1, S0{}, ZO{}, Second{});
            iter(t + 2, S1{}, ZO{}, Full{});
            t += 3;
            break;
        }
        if constexpr (OPZ) {
            for (; t < tend && t < 2; t += 3) {
                iter(t, S2{}, ZO{}, Full{});
                iter(t + 1, S0{}, ZO{}, Full{});
                iter(t + 2, S1{}, ZO{}, Full{});
            }
            for (; t < tend && t + 2 <= nz - 4; t += 3) {
                iter(t, S2{}, std::false_type{}, Full{});
                iter(t + 1, S0{}, std::false_type{}, Full{});
                iter(t + 2, S1{}, std::false_type{}, Full{});
            }
        }
        for (; t < tend; t += 3) {
            iter(t, S2{}, ZO{}, Full{});
            iter(t + 1, S0{}, ZO{}, Full{});
            iter(t + 2, S1{}, ZO{}, Full{});
        }
        iter(tend, S2{}, ZO{}, Last{});
    } else {
        // every iteration but the last runs all stages; the iteration count
        // modulo three is run first, in the last slots, and the last group
        // outside the loops (its third iteration reduced)
        switch (n_iter % 3) {
        case 2:
            iter(t++, S1{}, ZO{}, Full{});
            [[fallthrough]];
        case 1:
            iter(t++, S2{}, ZO{}, Full{});
            break;
        default:
            break;
        }
        if constexpr (OPZ) {
            for (; t + 2 < tend && t < 2; t += 3) {
                iter(t, S0{}, ZO{}, Full{});
                iter(t + 1, S1{}, ZO{}, Full{});
                iter(t + 2, S2{}, ZO{}, Full{});
            }
            for (; t + 2 < tend && t + 2 <= nz - 4; t += 3) {
                iter(t, S0{}, std::false_type{}, Full{});
                iter(t + 1, S1{}, std::false_type{}, Full{});
                iter(t + 2, S2{}, std::false_type{}, Full{});
            }
        }
        for (; t + 2 < tend; t += 3) {
            iter(t, S0{}, ZO{}, Full{});
            iter(t + 1, S1{}, ZO{}, Full{});
            iter(t + 2, S2{}, ZO{}, Full{});
        }
        iter(t, S0{}, ZO{}, Full{});
        iter(t + 1, S1{}, ZO{}, Full{});
        iter(t + 2, S2{}, ZO{}, std::integral_constant<int, kPartLast>{});
    }
}


// True when the region of tile (tx, ty) and the ring around it lie inside
// the x-y domain with a cell to spare on every side: no lane reads past an
// edge, sits on a boundary face or needs a redirected neighbour, so an open
// grid's tile can take the periodic addressing there.
template <int RX, int RY> __device__ __forceinline__ bool xy_interior(int tx, int ty, int nx, int ny)
{
    constexpr int TX = RX - 4, TY = RY - 4;
    return tx * TX >= 3 && tx * TX + RX <= nx + 1 && ty * TY >= 3 && ty * TY + RY <= ny + 1;
}

// Every LDS plane starts at zero, so values computed from not-yet-written
// slots in the first iterations of a march stay finite (they never reach an
// output).
template <typename T, int RX, int RY, int MODE, bool DIVP>
__device__ __forceinline__ void smem_clear(Smem<T, RX, RY, MODE, DIVP> &sm)
{
    using S = Smem<T, RX, RY, MODE, DIVP>;
    for (int i = threadIdx.x; i < S::PP; i += RX * RY) {
        sm.sP[i] = T(0);
        if (i < S::PM) sm.sPm[i] = T(0);
        if (i < S::PD) sm.sD[i] = T(0);
        sm.sQ[0][i] = sm.sQ[1][i] = sm.sQ[2][i] = T(0);
        sm.sC1[i] = sm.sC3[i] = sm.sH[i] = T(0);
        if (i < S::PX1) sm.sC2[i] = T(0);
        sm.sFA2[i] = sm.sFC2[i] = T(0);
        if (i < S::PX1) sm.sFA1[i] = sm.sFC1[i] = T(0);
        sm.sBU[i] = sm.sBD[i] = Factor<T>(1);
    }
    __syncthreads();
}

}  // namespace mpd
