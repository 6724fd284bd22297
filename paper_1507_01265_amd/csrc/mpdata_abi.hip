// mpdata_abi.hip -- host side of the libmpdata C ABI (include/mpdata.h).
//
// Validation, workspace layout, the time loop (ping-pong between the
// caller's psi and the workspace copy) and the mass reduction.  No device
// memory is allocated here: the caller provides every buffer.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>

#include "../../include/mpdata.h"
#include "mpdata_kernels.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMassParts = 1024;  // blocks of the mass reduction (fixed: deterministic)

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

thread_local char g_create_err[256];

struct Layout {
    size_t psi2, partials, result, flags, total;
};

size_t cells_of(const mpdata_params *p)
{
    return (size_t)p->nx * (size_t)p->ny * (size_t)p->nz;
}

size_t word_of(const mpdata_params *p) { return p->dtype == MPDATA_FP32 ? 4 : 8; }

Layout layout_of(const mpdata_params *p)
{
    Layout l;
    size_t off = 0;
    l.psi2 = off;
    off += align_up(cells_of(p) * word_of(p));
    l.partials = off;
    off += align_up((size_t)kMassParts * 2 * sizeof(double));
    l.result = off;
    off += align_up(2 * sizeof(double));
    l.flags = off;
    off += align_up(4 * sizeof(unsigned int));
    l.total = off;
    return l;
}

// Default launch shape per precision: the largest region whose register
// footprint fits the workgroup without spilling.
int default_tile(const mpdata_params *p) { return p->dtype == MPDATA_FP32 ? 2 : 4; }

int planes_per_chunk(const mpdata_params *p) { return p->nz; }

const char *check_params(const mpdata_params *p)
{
    if (!p) return "params is NULL";
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return "nx, ny, nz must be >= 1";
    if ((double)p->nx * p->ny * p->nz > 2147483647.0) return "grid too large (> 2^31 cells)";
    if ((double)(p->nx + 1) * p->ny * p->nz > 2147483647.0 ||
        (double)p->nx * (p->ny + 1) * p->nz > 2147483647.0 ||
        (double)p->nx * p->ny * (p->nz + 1) > 2147483647.0)
        return "face arrays too large (> 2^31 elements)";
    if (p->dtype != MPDATA_FP64 && p->dtype != MPDATA_FP32) return "dtype must be FP64 or FP32";
    if (p->bc != MPDATA_BC_PERIODIC && p->bc != MPDATA_BC_OPEN) return "bc must be PERIODIC or OPEN";
    if (p->iord != 1 && p->iord != 2) return "iord must be 1 or 2";
    if (p->nonos != 0 && p->nonos != 1) return "nonos must be 0 or 1";
    if (p->nonos && p->iord != 2) return "nonos needs iord 2";
    if (!(p->eps > 0.0) || !isfinite(p->eps)) return "eps must be finite and > 0";
    int count = 0;
    mpd::tile_shapes(&count);
    if (p->tile < 0 || p->tile > count) return "tile id out of range";
    return nullptr;
}

bool misaligned(const void *ptr) { return ((uintptr_t)ptr & 15u) != 0; }

}  // namespace

struct mpdata_ctx {
    mpdata_params p;
    void *psi;
    const void *u1, *u2, *u3, *h;
    char *ws;
    Layout lay;
    hipStream_t stream;
    int tile;
    int64_t steps;
    char err[256];
};

static int fail(mpdata_ctx *c, int code, const char *fmt, ...)
{
    char *dst = c ? c->err : g_create_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 256, fmt, ap);
    va_end(ap);
    return code;
}

static int hip_fail(mpdata_ctx *c, hipError_t e, const char *what)
{
    return fail(c, MPDATA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

template <typename T> static hipError_t run_steps(mpdata_ctx *c, int32_t nsteps)
{
    const mpdata_params &p = c->p;
    T *bufs[2] = {(T *)c->psi, (T *)(c->ws + c->lay.psi2)};
    mpd::StepArgs<T> a;
    a.u1 = (const T *)c->u1;
    a.u2 = (const T *)c->u2;
    a.u3 = (const T *)c->u3;
    a.h = (const T *)c->h;
    a.nx = p.nx;
    a.ny = p.ny;
    a.nz = p.nz;
    a.zlen = planes_per_chunk(&p);
    a.eps = p.eps;
    for (int32_t s = 0; s < nsteps; ++s) {
        a.psi_in = bufs[s & 1];
        a.psi_out = bufs[(s + 1) & 1];
        hipError_t e = mpd::launch_step<T>(a, c->tile, p.iord, p.bc == MPDATA_BC_OPEN,
                                           p.nonos != 0, c->stream);
        if (e != hipSuccess) return e;
    }
    if (nsteps & 1)
        return hipMemcpyAsync(bufs[0], bufs[1], cells_of(&p) * sizeof(T), hipMemcpyDeviceToDevice,
                              c->stream);
    return hipSuccess;
}

extern "C" {

int mpdata_abi_version(void) { return MPDATA_ABI_VERSION; }

int mpdata_tile_count(void)
{
    int count = 0;
    mpd::tile_shapes(&count);
    return count;
}

int mpdata_tile_info(int32_t id, int32_t *tx, int32_t *ty, int32_t *threads)
{
    int count = 0;
    const mpd::TileShape *s = mpd::tile_shapes(&count);
    if (id < 1 || id > count) return MPDATA_EINVAL;
    if (tx) *tx = s[id - 1].rx - 4;
    if (ty) *ty = s[id - 1].ry - 4;
    if (threads) *threads = s[id - 1].rx * s[id - 1].ry;
    return MPDATA_OK;
}

size_t mpdata_workspace_bytes(const mpdata_params *p)
{
    if (check_params(p)) return 0;
    return layout_of(p).total;
}

int mpdata_create(const mpdata_params *p, void *psi, const void *u1, const void *u2,
                  const void *u3, const void *h, void *workspace, size_t ws_bytes, void *stream,
                  mpdata_ctx **out)
{
    g_create_err[0] = 0;
    if (!out) return fail(nullptr, MPDATA_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char *m = check_params(p)) return fail(nullptr, MPDATA_EINVAL, "%s", m);
    if (!psi || !u1 || !u2 || !u3 || !h || !workspace)
        return fail(nullptr, MPDATA_EINVAL, "NULL array or workspace pointer");
    if (misaligned(psi) || misaligned(u1) || misaligned(u2) || misaligned(u3) || misaligned(h))
        return fail(nullptr, MPDATA_EINVAL, "arrays must be 16-byte aligned");
    if (((uintptr_t)workspace & (kAlign - 1)) != 0)
        return fail(nullptr, MPDATA_EINVAL, "workspace must be 256-byte aligned");
    const Layout lay = layout_of(p);
    if (ws_bytes < lay.total)
        return fail(nullptr, MPDATA_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes,
                    lay.total);

    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)workspace;
    unsigned int *flags = (unsigned int *)(ws + lay.flags);
    hipError_t e = hipMemsetAsync(flags, 0, 4 * sizeof(unsigned int), s);
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipMemsetAsync");
    const int periodic = p->bc == MPDATA_BC_PERIODIC;
    if (p->dtype == MPDATA_FP64)
        e = mpd::launch_validate<double>((const double *)h, (const double *)u1,
                                         (const double *)u2, (const double *)u3, p->nx, p->ny,
                                         p->nz, periodic, flags, s);
    else
        e = mpd::launch_validate<float>((const float *)h, (const float *)u1, (const float *)u2,
                                        (const float *)u3, p->nx, p->ny, p->nz, periodic, flags, s);
    if (e != hipSuccess) return hip_fail(nullptr, e, "validate launch");
    unsigned int hflags[2] = {0, 0};
    e = hipMemcpyAsync(hflags, flags, sizeof(hflags), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(nullptr, e, "validate readback");
    if (hflags[0]) return fail(nullptr, MPDATA_EINVAL, "h must be finite and > 0 (%u bad cells)", hflags[0]);
    if (hflags[1])
        return fail(nullptr, MPDATA_EINVAL,
                    "periodic boundaries need face n == face 0 on every axis (%u differ)", hflags[1]);

    mpdata_ctx *c = new (std::nothrow) mpdata_ctx;
    if (!c) return fail(nullptr, MPDATA_ENOMEM, "host allocation failed");
    c->p = *p;
    c->psi = psi;
    c->u1 = u1;
    c->u2 = u2;
    c->u3 = u3;
    c->h = h;
    c->ws = ws;
    c->lay = lay;
    c->stream = s;
    c->tile = p->tile ? p->tile : default_tile(p);
    c->steps = 0;
    c->err[0] = 0;
    *out = c;
    return MPDATA_OK;
}

int mpdata_step(mpdata_ctx *c, int32_t nsteps)
{
    if (!c) return MPDATA_EINVAL;
    if (nsteps < 0) return fail(c, MPDATA_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return MPDATA_OK;
    hipError_t e = c->p.dtype == MPDATA_FP64 ? run_steps<double>(c, nsteps)
                                             : run_steps<float>(c, nsteps);
    if (e != hipSuccess) return hip_fail(c, e, "step launch");
    c->steps += nsteps;
    return MPDATA_OK;
}

int mpdata_mass(mpdata_ctx *c, double *out)
{
    if (!c || !out) return c ? fail(c, MPDATA_EINVAL, "out is NULL") : MPDATA_EINVAL;
    double *parts = (double *)(c->ws + c->lay.partials);
    double *res = (double *)(c->ws + c->lay.result);
    const size_t n = cells_of(&c->p);
    hipError_t e;
    if (c->p.dtype == MPDATA_FP64)
        e = mpd::launch_mass<double>((const double *)c->psi, (const double *)c->h, n, parts,
                                     kMassParts, res, c->stream);
    else
        e = mpd::launch_mass<float>((const float *)c->psi, (const float *)c->h, n, parts,
                                    kMassParts, res, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "mass launch");
    double r[2];
    e = hipMemcpyAsync(r, res, sizeof(r), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "mass readback");
    *out = r[0];
    if (!isfinite(r[0])) return fail(c, MPDATA_ENONFINITE, "psi holds NaN or Inf");
    return MPDATA_OK;
}

int mpdata_get_psi(mpdata_ctx *c, void *dst)
{
    if (!c) return MPDATA_EINVAL;
    if (!dst) return fail(c, MPDATA_EINVAL, "dst is NULL");
    hipError_t e = hipMemcpyAsync(dst, c->psi, cells_of(&c->p) * word_of(&c->p),
                                  hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? MPDATA_OK : hip_fail(c, e, "get_psi");
}

int mpdata_set_psi(mpdata_ctx *c, const void *src)
{
    if (!c) return MPDATA_EINVAL;
    if (!src) return fail(c, MPDATA_EINVAL, "src is NULL");
    hipError_t e = hipMemcpyAsync(c->psi, src, cells_of(&c->p) * word_of(&c->p),
                                  hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_psi");
    c->steps = 0;
    return MPDATA_OK;
}

int mpdata_sync(mpdata_ctx *c)
{
    if (!c) return MPDATA_EINVAL;
    hipError_t e = hipStreamSynchronize(c->stream);
    return e == hipSuccess ? MPDATA_OK : hip_fail(c, e, "hipStreamSynchronize");
}

int64_t mpdata_steps_done(const mpdata_ctx *c) { return c ? c->steps : -1; }

void mpdata_destroy(mpdata_ctx *c) { delete c; }

const char *mpdata_last_error(const mpdata_ctx *c) { return c ? c->err : g_create_err; }

}  // extern "C"
