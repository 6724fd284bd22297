// mpdata_kernels.hip -- gfx950 kernels of one MPDATA time step.
//
// The step (paper, section 5.2: dependent stencil stages, five input
// matrices -> one output; the equations are those of the MPDATA literature
// the paper cites: donor-cell pass and antidiffusive pseudo-velocities of
// Smolarkiewicz 1984, non-oscillatory limiter of Smolarkiewicz & Grabowski
// 1990, density weighting of Smolarkiewicz & Margolin 1998):
//   S1+S2  psi1 = psi - sum_d dF_d / h,  F = donor(psi_lo, psi_hi, U)
//   S3     V on every face from psi1, U, h (A ratio, cross terms B, G)
//   S4     mx, mn = max/min of psi and psi1 over the 7-point neighbourhood
//   S5     beta_up = (mx - psi1) h / (IN + eps), beta_dn = (psi1 - mn) h / (OUT + eps)
//   S6     Vt = min(1, bdn_lo, bup_hi) pos(V) + min(1, bup_lo, bdn_hi) neg(V)
//   S7     psi_out = psi1 - sum_d dFC_d / h,  FC = donor(psi1_lo, psi1_hi, Vt)
//
// Fusion (the paper's (3+1)D decomposition, section 5.3: tile the domain
// and fuse the stage loop so intermediates stay on chip, paying with halo
// recompute).  Recast for CDNA:
//  * one workgroup owns an RX x RY region of x-y columns (its output tile
//    plus a 2-cell halo) and marches along z through a chunk of planes;
//  * each thread owns one column and keeps the z-history of every stage in
//    registers; in-plane neighbours are exchanged through LDS planes;
//  * the stage pipeline is skewed in z: iteration t computes psi1 at plane
//    t, V and the limiter bounds/factors at plane t-1 (and V3 on face t),
//    the limited fluxes and the output at plane t-2;
//  * ψ^n of plane t+2 is prefetched into registers two iterations ahead.
// Only psi^{n+1} is written to HBM: 5 array reads + 1 write per cell-step.
//
// Boundaries: periodic wraps cell indices (face n == face 0); open is
// zero-gradient (ghost cells equal the nearest interior cell; reads of
// cell-centred neighbours at the domain edge are redirected to the cell
// itself) with zero antidiffusive velocity on boundary-normal faces.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

template <typename T> __device__ __forceinline__ T pos(T x) { return fmax(x, T(0)); }
template <typename T> __device__ __forceinline__ T neg(T x) { return fmin(x, T(0)); }

// donor-cell flux through a face with lower value l, upper value r
template <typename T> __device__ __forceinline__ T donor(T l, T r, T c)
{
    return pos(c) * l + neg(c) * r;
}

// Antidiffusive pseudo-velocity on a face between lower cell a and upper
// cell b, for the face-normal Courant number U, the face density G and the
// two transverse axes s and t (column sums of their Courant numbers in a
// and b, and psi1 of a and b one cell up/down along each).
template <typename T>
__device__ __forceinline__ T pseudo_velocity(T U, T G, T pa, T pb, T us_a, T us_b, T ps_a_hi,
                                             T ps_b_hi, T ps_a_lo, T ps_b_lo, T ut_a, T ut_b,
                                             T pt_a_hi, T pt_b_hi, T pt_a_lo, T pt_b_lo, T eps)
{
    T A = (pb - pa) / (pb + pa + eps);
    T Us = T(0.25) * (us_a + us_b);
    T s_hi = ps_b_hi + ps_a_hi, s_lo = ps_b_lo + ps_a_lo;
    T Bs = T(0.5) * (s_hi - s_lo) / (s_hi + s_lo + eps);
    T Ut = T(0.25) * (ut_a + ut_b);
    T t_hi = pt_b_hi + pt_a_hi, t_lo = pt_b_lo + pt_a_lo;
    T Bt = T(0.5) * (t_hi - t_lo) / (t_hi + t_lo + eps);
    return (fabs(U) - U * U / G) * A - (U / G) * (Us * Bs + Ut * Bt);
}

// Limited pseudo-velocity; the factors are in limiter precision (double).
template <typename T>
__device__ __forceinline__ T limited(T v, double bup_a, double bdn_a, double bup_b, double bdn_b)
{
    T cp = T(fmin(1.0, fmin(bdn_a, bup_b)));
    T cn = T(fmin(1.0, fmin(bup_a, bdn_b)));
    return cp * pos(v) + cn * neg(v);
}

// Registers of one plane of a column: the Courant numbers of its x- and
// y-faces and h (needed one iteration ahead) ...
template <typename T> struct PlaneA {
    T u1lo, u1hi, u2lo, u2hi, h;
};
// ... and psi^n, the Courant number of its lower z-face and the LDS ring of
// psi^n (needed two iterations ahead).
template <typename T> struct PlaneB {
    T pn, u3lo, ringx, ringy;
};

// ================================================================ fused step

template <typename T, int RX, int RY, bool OPEN, bool NONOS>
__global__ __launch_bounds__(RX * RY) void step_fused(StepArgs<T> a)
{
    using L = double;  // limiter precision (both variants)
    constexpr int NT = RX * RY;
    constexpr int TX = RX - 4, TY = RY - 4;
    constexpr int PX = RX + 2;  // row pitch of the psi^n plane with its ring

    __shared__ T sP[(RX + 2) * (RY + 2)];  // psi^n plane t, with a 1-cell ring
    __shared__ T sQ[3][NT];                // psi1, planes t-2 .. t
    __shared__ T sC1[NT], sC2[NT], sC3[NT], sH[NT];  // Courant column sums, h: plane t-1
    __shared__ T sFA1[NT], sFA2[NT];       // antidiffusive donor fluxes, lower faces
    __shared__ L sBU[NT], sBD[NT];         // limiter factors, plane t-2
    __shared__ T sFC1[NT], sFC2[NT];       // corrective fluxes, lower faces

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const T eps = T(a.eps);
    const L eps_l = a.eps;

    const int tid = threadIdx.x;
    const int lx = tid % RX, ly = tid / RX;
    const int gx = blockIdx.x * TX - 2 + lx;
    const int gy = blockIdx.y * TY - 2 + ly;
    const int z0 = blockIdx.z * a.zlen;
    const int z1 = min(nz, z0 + a.zlen);
    const int q = tid;

    // in-plane offsets into the global arrays
    const int cx = cell_of<OPEN>(gx, nx), cy = cell_of<OPEN>(gy, ny);
    const size_t pc_cells = (size_t)nx * ny;
    const size_t pc_u1 = (size_t)(nx + 1) * ny;
    const size_t pc_u2 = (size_t)nx * (ny + 1);
    const int o_c = cy * nx + cx;
    const int o_u1lo = cy * (nx + 1) + face_lo<OPEN>(gx, nx);
    const int o_u1hi = cy * (nx + 1) + face_hi<OPEN>(gx, nx);
    const int o_u2lo = face_lo<OPEN>(gy, ny) * nx + cx;
    const int o_u2hi = face_hi<OPEN>(gy, ny) * nx + cx;
    const bool has_rx = (lx == 0) || (lx == RX - 1);
    const bool has_ry = (ly == 0) || (ly == RY - 1);
    const int o_rx = cy * nx + cell_of<OPEN>(lx == 0 ? gx - 1 : gx + 1, nx);
    const int o_ry = cell_of<OPEN>(ly == 0 ? gy - 1 : gy + 1, ny) * nx + cx;
    const int p_own = (ly + 1) * PX + lx + 1;
    const int p_rx = (ly + 1) * PX + (lx == 0 ? 0 : RX + 1);
    const int p_ry = (ly == 0 ? 0 : RY + 1) * PX + lx + 1;

    // neighbour offsets in the NT planes: "face" reads are plain (region edge
    // clamped), "cell" reads are also redirected to self at an open boundary
    const int fxm = lx > 0 ? -1 : 0, fxp = lx < RX - 1 ? 1 : 0;
    const int fym = ly > 0 ? -RX : 0, fyp = ly < RY - 1 ? RX : 0;
    const int cxm = (OPEN && gx <= 0) ? 0 : fxm;
    const int cxp = (OPEN && gx >= nx - 1) ? 0 : fxp;
    const int cym = (OPEN && gy <= 0) ? 0 : fym;
    const int cyp = (OPEN && gy >= ny - 1) ? 0 : fyp;
    const int pxm = (OPEN && gx <= 0) ? 0 : -1;
    const int pxp = (OPEN && gx >= nx - 1) ? 0 : 1;
    const int pym = (OPEN && gy <= 0) ? 0 : -PX;
    const int pyp = (OPEN && gy >= ny - 1) ? 0 : PX;

    // boundary-normal faces of an open domain carry no antidiffusive flux
    const bool zero_v1 = OPEN && (gx <= 0 || gx >= nx);
    const bool zero_v2 = OPEN && (gy <= 0 || gy >= ny);
    const bool is_out = lx >= 2 && lx < RX - 2 && ly >= 2 && ly < RY - 2 && gx < nx && gy < ny;

    const T *__restrict__ psi = a.psi_in;
    auto load_a = [&](int t, PlaneA<T> &r) {
        const int k = cell_of<OPEN>(t, nz);
        r.h = a.h[(size_t)k * pc_cells + o_c];
        r.u1lo = a.u1[(size_t)k * pc_u1 + o_u1lo];
        r.u1hi = a.u1[(size_t)k * pc_u1 + o_u1hi];
        r.u2lo = a.u2[(size_t)k * pc_u2 + o_u2lo];
        r.u2hi = a.u2[(size_t)k * pc_u2 + o_u2hi];
    };
    auto load_b = [&](int t, PlaneB<T> &r) {
        const size_t bc = (size_t)cell_of<OPEN>(t, nz) * pc_cells;
        r.pn = psi[bc + o_c];
        r.u3lo = a.u3[(size_t)face_lo<OPEN>(t, nz) * pc_cells + o_c];
        r.ringx = has_rx ? psi[bc + o_rx] : T(0);
        r.ringy = has_ry ? psi[bc + o_ry] : T(0);
    };
    auto store_ring = [&](const PlaneB<T> &r) {
        sP[p_own] = r.pn;
        if (has_rx) sP[p_rx] = r.ringx;
        if (has_ry) sP[p_ry] = r.ringy;
    };

    const int t0 = z0 - 2, tend = z1 + 1;
    PlaneA<T> curA, nxA;
    PlaneB<T> cur, nx1, nx2;
    load_a(t0, curA);
    load_b(t0, cur);
    load_b(t0 + 1, nx1);
    const T pn_prev = psi[(size_t)cell_of<OPEN>(t0 - 1, nz) * pc_cells + o_c];
    store_ring(cur);

    // z-history of the column
    T f3_c = donor(pn_prev, cur.pn, cur.u3lo);  // psi^n flux, face t
    T pn_m1 = pn_prev, pn_m2 = T(0);
    T pmx_m1 = T(0), pmn_m1 = T(0);             // in-plane 5-point max/min of psi^n(t-1)
    T u1_m1 = T(0), u2_m1 = T(0);               // lower-face Courant, plane t-1
    T h_m2 = T(1);
    T v1_m2 = T(0), v2_m2 = T(0), v3_m1 = T(0); // V at plane t-2, V3 at face t-1
    T fa3_m1 = T(0);                            // antidiffusive flux, face t-1
    L bu_m2 = 1.0, bd_m2 = 1.0;                 // limiter factors, plane t-2
    T fc3_m2 = T(0);                            // corrective flux, face t-2
    T *__restrict__ out = a.psi_out;

    for (int t = t0; t <= tend; ++t) {
        const int it = t - t0;
        const int s0 = it % 3, s1 = (it + 2) % 3, s2 = (it + 1) % 3;  // slots t, t-1, t-2
        if (t + 1 <= tend) load_a(t + 1, nxA);
        if (t + 2 <= tend + 1) load_b(t + 2, nx2);
        __syncthreads();  // (B) psi^n(t) ring, sums/h of t-1 and beta of t-2 are visible
        // own-column values of planes t-1 and t-2 that already sit in LDS
        const T p1_m1 = sQ[s1][q], p1_m2 = sQ[s2][q];
        const T c1_m1 = sC1[q], c2_m1 = sC2[q], c3_m1 = sC3[q], h_m1 = sH[q];

        // ---- S1+S2 at plane t
        const T pL = sP[p_own + pxm], pR = sP[p_own + pxp];
        const T pD = sP[p_own + pym], pU = sP[p_own + pyp];
        const T f1lo = donor(pL, cur.pn, curA.u1lo), f1hi = donor(cur.pn, pR, curA.u1hi);
        const T f2lo = donor(pD, cur.pn, curA.u2lo), f2hi = donor(cur.pn, pU, curA.u2hi);
        const T f3hi = donor(cur.pn, nx1.pn, nx1.u3lo);
        const T p1_c = cur.pn - (((f1hi - f1lo) + (f2hi - f2lo)) + (f3hi - f3_c)) / curA.h;
        const T pmx_c = fmax(fmax(fmax(pL, pR), fmax(pD, pU)), cur.pn);
        const T pmn_c = fmin(fmin(fmin(pL, pR), fmin(pD, pU)), cur.pn);
        sQ[s0][q] = p1_c;
        const T c1_c = curA.u1lo + curA.u1hi;
        const T c2_c = curA.u2lo + curA.u2hi;
        const T c3_c = cur.u3lo + nx1.u3lo;
        __syncthreads();  // (D) psi1(t) visible

        T v1 = T(0), v2 = T(0), v3 = T(0), fa3_c = T(0);
        T mx = T(0), mn = T(0);
        if (t >= z0 - 1) {
            // ---- S3 at plane p = t-1 (lower x- and y-faces) and on face t
            const int p = t - 1;
            const bool clo = OPEN && p <= 0, chi = OPEN && p >= nz - 1;
            const T *Qc = sQ[s1];
            const T *Qlo = clo ? sQ[s1] : sQ[s2];
            const T *Qhi = chi ? sQ[s1] : sQ[s0];
            const T p1_lo = clo ? p1_m1 : p1_m2;
            const T p1_hi = chi ? p1_m1 : p1_c;

            const T qa = Qc[q + fxm];        // x-neighbour below (cell a of the x-face)
            const T qd = Qc[q + fym];        // y-neighbour below (cell a of the y-face)
            const T qyp_ = Qc[q + cyp], qym_ = Qc[q + cym];
            const T qxp_ = Qc[q + cxp], qxm_ = Qc[q + cxm];
            // x-face between a = (lx-1) and b = own
            {
                const T sa2 = sC2[q + fxm], sa3 = sC3[q + fxm];
                const T G = T(0.5) * (sH[q + fxm] + h_m1);
                v1 = pseudo_velocity(u1_m1, G, qa, p1_m1, sa2, c2_m1, Qc[q + fxm + cyp], qyp_,
                                     Qc[q + fxm + cym], qym_, sa3, c3_m1, Qhi[q + fxm], p1_hi,
                                     Qlo[q + fxm], p1_lo, eps);
                if (zero_v1) v1 = T(0);
            }
            // y-face between a = (ly-1) and b = own; transverse axes z then x
            {
                const T sa3 = sC3[q + fym], sa1 = sC1[q + fym];
                const T G = T(0.5) * (sH[q + fym] + h_m1);
                v2 = pseudo_velocity(u2_m1, G, qd, p1_m1, sa3, c3_m1, Qhi[q + fym], p1_hi,
                                     Qlo[q + fym], p1_lo, sa1, c1_m1, Qc[q + fym + cxp], qxp_,
                                     Qc[q + fym + cxm], qxm_, eps);
                if (zero_v2) v2 = T(0);
            }
            // z-face t between a = plane t-1 and b = plane t; transverse x then y
            {
                const T *Qb = sQ[s0];
                const T G = T(0.5) * (h_m1 + curA.h);
                v3 = pseudo_velocity(cur.u3lo, G, p1_m1, p1_c, c1_m1, c1_c, qxp_, Qb[q + cxp],
                                     qxm_, Qb[q + cxm], c2_m1, c2_c, qyp_, Qb[q + cyp], qym_,
                                     Qb[q + cym], eps);
                if (OPEN && (t <= 0 || t >= nz)) v3 = T(0);
            }
            if (NONOS) {
                // ---- S4 bounds at plane p
                const T pn_lo = clo ? pn_m1 : pn_m2, pn_hi = chi ? pn_m1 : cur.pn;
                mx = fmax(fmax(fmax(pmx_m1, fmax(qxm_, qxp_)), fmax(fmax(qym_, qyp_), p1_m1)),
                          fmax(fmax(pn_lo, pn_hi), fmax(p1_lo, p1_hi)));
                mn = fmin(fmin(fmin(pmn_m1, fmin(qxm_, qxp_)), fmin(fmin(qym_, qyp_), p1_m1)),
                          fmin(fmin(pn_lo, pn_hi), fmin(p1_lo, p1_hi)));
                sFA1[q] = donor(qa, p1_m1, v1);
                sFA2[q] = donor(qd, p1_m1, v2);
                fa3_c = donor(p1_m1, p1_c, v3);
            }
        }
        __syncthreads();  // (F) antidiffusive fluxes visible

        L bu_m1 = 1.0, bd_m1 = 1.0;
        if (NONOS && t >= z0) {
            // ---- S5 limiter factors at plane t-1
            const L x_lo = L(sFA1[q]), x_hi = L(sFA1[q + fxp]);
            const L y_lo = L(sFA2[q]), y_hi = L(sFA2[q + fyp]);
            const L z_lo = L(fa3_m1), z_hi = L(fa3_c);
            const L in = ((pos(x_lo) - neg(x_hi)) + (pos(y_lo) - neg(y_hi))) + (pos(z_lo) - neg(z_hi));
            const L ou = ((pos(x_hi) - neg(x_lo)) + (pos(y_hi) - neg(y_lo))) + (pos(z_hi) - neg(z_lo));
            bu_m1 = (L(mx) - L(p1_m1)) * L(h_m1) / (in + eps_l);
            bd_m1 = (L(p1_m1) - L(mn)) * L(h_m1) / (ou + eps_l);
        }

        T fc3_m1 = T(0);
        if (t >= z0 + 1) {
            // ---- S6 + corrective fluxes at plane r = t-2 (lower faces) and on face t-1
            const T *Qr = sQ[s2];
            T vt1 = v1_m2, vt2 = v2_m2, vt3 = v3_m1;
            if (NONOS) {
                vt1 = limited(v1_m2, sBU[q + fxm], sBD[q + fxm], bu_m2, bd_m2);
                vt2 = limited(v2_m2, sBU[q + fym], sBD[q + fym], bu_m2, bd_m2);
                vt3 = limited(v3_m1, bu_m2, bd_m2, bu_m1, bd_m1);
            }
            if (zero_v1) vt1 = T(0);
            if (zero_v2) vt2 = T(0);
            if (OPEN && (t - 1 <= 0 || t - 1 >= nz)) vt3 = T(0);
            sFC1[q] = donor(Qr[q + fxm], p1_m2, vt1);
            sFC2[q] = donor(Qr[q + fym], p1_m2, vt2);
            fc3_m1 = donor(p1_m2, p1_m1, vt3);
        }
        __syncthreads();  // (J) corrective fluxes visible

        if (t >= z0 + 2) {
            // ---- S7 at plane r = t-2
            const T fc1hi = sFC1[q + fxp], fc2hi = sFC2[q + fyp];
            const T res = p1_m2 - (((fc1hi - sFC1[q]) + (fc2hi - sFC2[q])) + (fc3_m1 - fc3_m2)) / h_m2;
            if (is_out) out[(size_t)(t - 2) * pc_cells + o_c] = res;
        }

        // ---- hand the planes to the next iteration
        if (NONOS) {
            sBU[q] = bu_m1;
            sBD[q] = bd_m1;
        }
        sC1[q] = c1_c;
        sC2[q] = c2_c;
        sC3[q] = c3_c;
        sH[q] = curA.h;
        store_ring(nx1);

        pn_m2 = pn_m1;
        pn_m1 = cur.pn;
        pmx_m1 = pmx_c;
        pmn_m1 = pmn_c;
        u1_m1 = curA.u1lo;
        u2_m1 = curA.u2lo;
        h_m2 = h_m1;
        f3_c = f3hi;
        v1_m2 = v1;
        v2_m2 = v2;
        v3_m1 = v3;
        fa3_m1 = fa3_c;
        bu_m2 = bu_m1;
        bd_m2 = bd_m1;
        fc3_m2 = fc3_m1;
        curA = nxA;
        cur = nx1;
        nx1 = nx2;
    }
}

// ======================================================= donor cell (iord 1)

template <typename T, bool OPEN> __global__ __launch_bounds__(256) void step_donor(StepArgs<T> a)
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
        a.psi_out[c] = vc - (((f1hi - f1lo) + (f2hi - f2lo)) + (f3hi - f3lo)) / a.h[c];
    }
}

// ============================================================ mass reduction
// Double-double accumulation (TwoProduct by FMA, Knuth TwoSum), a wave64
// butterfly with double-double adds, a block combine in LDS, one partial per
// block; the final pass sums the partials in a fixed order.

struct DD {
    double hi, lo;
};

__device__ __forceinline__ DD two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

__device__ __forceinline__ DD dd_add(DD a, DD b)
{
    DD s = two_sum(a.hi, b.hi);
    double lo = s.lo + (a.lo + b.lo);
    double hi = s.hi + lo;
    return {hi, lo - (hi - s.hi)};
}

__device__ __forceinline__ DD dd_add_prod(DD acc, double x, double y)
{
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

// ===================================================================== launch

template <typename T, int RX, int RY>
static hipError_t launch_fused_shape(const StepArgs<T> &a, bool open, bool nonos, hipStream_t s)
{
    constexpr int TX = RX - 4, TY = RY - 4;
    dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY, (a.nz + a.zlen - 1) / a.zlen);
    dim3 block(RX * RY);
    if (open) {
        if (nonos) step_fused<T, RX, RY, true, true><<<grid, block, 0, s>>>(a);
        else step_fused<T, RX, RY, true, false><<<grid, block, 0, s>>>(a);
    } else {
        if (nonos) step_fused<T, RX, RY, false, true><<<grid, block, 0, s>>>(a);
        else step_fused<T, RX, RY, false, false><<<grid, block, 0, s>>>(a);
    }
    return hipGetLastError();
}

const TileShape *tile_shapes(int *count)
{
    static const TileShape shapes[] = {
        {64, 16}, {32, 32}, {64, 8}, {32, 16}, {32, 24},
    };
    *count = (int)(sizeof(shapes) / sizeof(shapes[0]));
    return shapes;
}

template <typename T>
hipError_t launch_step(const StepArgs<T> &a, int tile, int iord, bool open, bool nonos,
                       hipStream_t s)
{
    if (iord == 1) {
        const size_t n = (size_t)a.nx * a.ny * a.nz;
        const int blocks = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
        if (open) step_donor<T, true><<<blocks, 256, 0, s>>>(a);
        else step_donor<T, false><<<blocks, 256, 0, s>>>(a);
        return hipGetLastError();
    }
    switch (tile) {
    case 1: return launch_fused_shape<T, 64, 16>(a, open, nonos, s);
    case 2: return launch_fused_shape<T, 32, 32>(a, open, nonos, s);
    case 3: return launch_fused_shape<T, 64, 8>(a, open, nonos, s);
    case 4: return launch_fused_shape<T, 32, 16>(a, open, nonos, s);
    case 5: return launch_fused_shape<T, 32, 24>(a, open, nonos, s);
    default: return hipErrorInvalidValue;
    }
}

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

template hipError_t launch_step<double>(const StepArgs<double> &, int, int, bool, bool, hipStream_t);
template hipError_t launch_step<float>(const StepArgs<float> &, int, int, bool, bool, hipStream_t);
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
