// mpdata_abi.hip -- host side of the libmpdata C ABI (include/mpdata.h).
//
// Validation, workspace layout, launch plans (which workgroup of the
// persistent step kernel runs which (grid, tile, z-range) segment), the
// time loop (ping-pong between the caller's psi and a workspace copy, runs
// of steps replayed from a hipGraph), batches of grids and the mass
// reduction.  No device memory is allocated here: the caller provides every
// buffer, including the workspace that holds the plan.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <new>
#include <queue>
#include <vector>

#include "../../include/mpdata.h"
#include "mpdata_kernels.h"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMassParts = 1024;  // blocks of the mass reduction (fixed: deterministic)
constexpr int kGraphSteps = 8;    // steps per replayed graph (even: psi ends where it began)
constexpr int kXcds = 8;          // XCDs of an MI355X; workgroup w runs on XCD w % 8
constexpr int kMinShare = 24;     // fewest planes a workgroup's share of a plan marches
constexpr int kPipelineFill = 4;  // march iterations before a segment's first output plane
constexpr int kMaxIord = 16;      // most passes of one step (1 donor-cell + 15 corrective)
constexpr int64_t kMaxNoallocCells = 2147483647;  // mpdata_mass_noalloc: a grid's cell limit

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

thread_local char g_create_err[256];

size_t cells_of(const mpdata_params *p)
{
    return (size_t)p->nx * (size_t)p->ny * (size_t)p->nz;
}

size_t word_of(const mpdata_params *p) { return p->dtype == MPDATA_FP32 ? 4 : 8; }

const mpd::TileShape &shape_of(int tile)
{
    int count = 0;
    return mpd::tile_shapes(&count)[tile - 1];
}

// Default launch shape (measured on MI355X with the default plan): 32x24
// regions, except FP32 with open boundaries, whose boundary redirects cost
// enough registers that the 32x32 region runs faster.
int default_tile(int dtype, int bc)
{
    return (dtype == MPDATA_FP32 && bc == MPDATA_BC_OPEN) ? 2 : 5;
}

int tile_of(const mpdata_params *p) { return p->tile ? p->tile : default_tile(p->dtype, p->bc); }

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
    // the step kernel addresses one x-y plane of an array with 32-bit byte
    // offsets and masks lanes with an offset of 2^31, past every plane
    if ((double)(p->nx + 1) * (p->ny + 1) * (p->dtype == MPDATA_FP64 ? 8 : 4) >= 2147483648.0)
        return "x-y plane too large (>= 2 GiB)";
    if (p->bc != MPDATA_BC_PERIODIC && p->bc != MPDATA_BC_OPEN) return "bc must be PERIODIC or OPEN";
    if (p->iord < 1 || p->iord > kMaxIord) return "iord must be 1 .. 16";
    if (p->nonos != 0 && p->nonos != 1) return "nonos must be 0 or 1";
    if (p->nonos && p->iord < 2) return "nonos needs iord >= 2";
    // the common denominator of the FP64 pseudo-velocity is about
    // h eps^3 on a zero background and the limiter's (IN + eps)(OUT + eps)
    // about eps^2: eps >= 1e-30 keeps both normal
    if (!(p->eps >= 1e-30) || !isfinite(p->eps)) return "eps must be finite and >= 1e-30";
    if (p->flags & ~(MPDATA_FLAG_NO_GRAPH | MPDATA_FLAG_VSIGN | MPDATA_FLAG_DIV | MPDATA_FLAG_TVEL))
        return "unknown flag bits";
    if (p->reserved != 0) return "reserved must be 0";
    int count = 0;
    mpd::tile_shapes(&count);
    if (p->tile < 0 || p->tile > count) return "tile id out of range";
    if (p->tile == 7 && p->dtype != MPDATA_FP32)
        return "tile 7 (24x32 regions) is built for FP32 only (FP64 exchanges x-neighbours "
               "between the lanes of a wave, which needs rows that tile a wave)";
    if (p->iord > 2 && p->tile != 0 && p->tile != default_tile(p->dtype, p->bc))
        return "iord > 2 runs on the default launch shape (tile 0)";
    if ((p->flags & (MPDATA_FLAG_VSIGN | MPDATA_FLAG_DIV)) && p->tile != 0 &&
        (shape_of(p->tile).rx != 32 || (shape_of(p->tile).ry != 24 && shape_of(p->tile).ry != 32)))
        return "the variable-sign option and the divergent-flow term run on the 32x24 and 32x32 "
               "launch shapes (tile 0, 2 or 5)";
    if (p->flags & MPDATA_FLAG_TVEL) {
        if (p->iord != 2) return "Courant numbers that change in time (MPDATA_FLAG_TVEL) need iord 2";
        if (p->flags & MPDATA_FLAG_VSIGN)
            return "MPDATA_FLAG_TVEL does not combine with the variable-sign option";
        if (p->tile != 0 && p->tile != default_tile(p->dtype, p->bc))
            return "MPDATA_FLAG_TVEL runs on the default launch shape (tile 0)";
    }
    return nullptr;
}

bool misaligned(const void *ptr) { return ((uintptr_t)ptr & 15u) != 0; }

// ----------------------------------------------------------------- plans

int tiles_x(const mpdata_params &p, int tile) { return (p.nx + shape_of(tile).rx - 5) / (shape_of(tile).rx - 4); }
int tiles_y(const mpdata_params &p, int tile) { return (p.ny + shape_of(tile).ry - 5) / (shape_of(tile).ry - 4); }

// Whole-tile plan: tile i (listed grid by grid, row by row) marches all its
// planes on one workgroup; tiles are dealt round-robin over the workgroups.  Every workgroup starts its k-th tile at the
// same time and plane as its neighbours, so the halo lines that adjacent
// tiles share are fetched once into L2 while both use them (measured: about
// 15 % faster per march iteration than unaligned marches).
void whole_tile_plan(const std::vector<mpdata_params> &grids, int tile, int nwg,
                     std::vector<mpd::Segment> &segs, std::vector<int> &wg_begin)
{
    // logical slot l = i mod nwg; slots [x*per_xcd, (x+1)*per_xcd) run on
    // XCD x, so runs of consecutive tiles (row neighbours, and most column
    // neighbours) share an L2
    const int per_xcd = nwg % kXcds == 0 ? nwg / kXcds : 0;
    std::vector<std::vector<mpd::Segment>> per(nwg);
    int i = 0;
    for (int g = 0; g < (int)grids.size(); ++g) {
        const int ntx = tiles_x(grids[g], tile), nty = tiles_y(grids[g], tile);
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx, ++i) {
                const int l = i % nwg;
                const int w = per_xcd ? (l % per_xcd) * kXcds + l / per_xcd : l;
                per[w].push_back(mpd::Segment{g, tx, ty, 0, grids[g].nz, 0, 0, 0});
            }
    }
    segs.clear();
    wg_begin.assign(nwg + 1, 0);
    for (int w = 0; w < nwg; ++w) {
        wg_begin[w] = (int)segs.size();
        segs.insert(segs.end(), per[w].begin(), per[w].end());
    }
    wg_begin[nwg] = (int)segs.size();
}

// Longest march (in iterations) of a plan: planes of each segment plus the
// pipeline fill the march pays before its first output plane.
long long plan_makespan(const std::vector<mpd::Segment> &segs, const std::vector<int> &wg_begin)
{
    long long worst = 0;
    for (size_t w = 0; w + 1 < wg_begin.size(); ++w) {
        long long it = 0;
        for (int s = wg_begin[w]; s < wg_begin[w + 1]; ++s)
            it += segs[s].z1 - segs[s].z0 + kPipelineFill;
        worst = std::max(worst, it);
    }
    return worst;
}

// Contiguous-share plan: the work of all grids, counted in (tile, plane)
// units and listed tile by tile (grid, then tile row, then tile), is cut into
// nwg contiguous, equal shares.  Consecutive shares go to workgroups of the
// same XCD (workgroup w runs on XCD w % 8), so neighbouring tiles -- which
// re-read each other's halo -- share an L2.
void share_plan(const std::vector<mpdata_params> &grids, int tile, int nwg,
                std::vector<mpd::Segment> &segs, std::vector<int> &wg_begin)
{
    struct Tile {
        int grid, tx, ty, nz;
    };
    std::vector<Tile> tiles;
    long long work = 0;
    for (int g = 0; g < (int)grids.size(); ++g) {
        const int ntx = tiles_x(grids[g], tile), nty = tiles_y(grids[g], tile);
        for (int ty = 0; ty < nty; ++ty)
            for (int tx = 0; tx < ntx; ++tx) {
                tiles.push_back({g, tx, ty, grids[g].nz});
                work += grids[g].nz;
            }
    }
    // Each share should march at least kMinShare planes: a segment pays
    // PRIMING extra iterations before its first output, so tiny shares would
    // be mostly pipeline fill.  With little work only the first shares (one
    // per XCD first) are used.
    const int nwg_all = nwg;
    nwg = (int)std::max(1LL, std::min<long long>(nwg, work / kMinShare));
    // logical share l covers work units [l*work/nwg, (l+1)*work/nwg)
    std::vector<std::vector<mpd::Segment>> share(nwg_all);
    size_t ti = 0;
    long long tile_start = 0;  // work offset of tiles[ti]
    for (int l = 0; l < nwg; ++l) {
        const long long a = work * l / nwg, b = work * (l + 1) / nwg;
        long long pos = a;
        while (pos < b && ti < tiles.size()) {
            const Tile &t = tiles[ti];
            const long long t_end = tile_start + t.nz;
            const long long e = std::min(b, t_end);
            mpd::Segment s{};
            s.grid = t.grid;
            s.tx = t.tx;
            s.ty = t.ty;
            s.z0 = (int)(pos - tile_start);
            s.z1 = (int)(e - tile_start);
            share[l].push_back(s);
            pos = e;
            if (e == t_end) {
                tile_start = t_end;
                ++ti;
            }
        }
    }
    // physical workgroup w runs on XCD w % 8: consecutive logical shares go
    // to the same XCD; when fewer shares than workgroups are used they are
    // spread over the XCDs first
    const int per_xcd = nwg_all % kXcds == 0 ? nwg_all / kXcds : 0;
    segs.clear();
    wg_begin.assign(nwg_all + 1, 0);
    for (int w = 0; w < nwg_all; ++w) {
        int l = w;
        if (per_xcd) {
            const int x = w % kXcds, i = w / kXcds;          // XCD, index within it
            const int used_per_xcd = (nwg + kXcds - 1) / kXcds;
            l = i < used_per_xcd ? x * used_per_xcd + i : nwg;  // beyond nwg: idle
        }
        wg_begin[w] = (int)segs.size();
        if (l < nwg) segs.insert(segs.end(), share[l].begin(), share[l].end());
    }
    wg_begin[nwg_all] = (int)segs.size();
}

// Default plan: the whole-tile plan unless its makespan exceeds the
// contiguous-share plan's by more than the L2 gain of aligned marches.
// Longest-processing-time-first over `cost`, onto the workgroups `wgs`:
// each item (in order of decreasing cost, ties in list order) goes to the
// workgroup with the least load so far (ties to the lower id).  Returns the
// owner of every item.
std::vector<int> lpt_assign(const std::vector<long long> &cost, const std::vector<int> &wgs)
{
    std::vector<int> order(cost.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    using Slot = std::pair<long long, int>;  // (load, workgroup)
    std::priority_queue<Slot, std::vector<Slot>, std::greater<Slot>> heap;
    for (int w : wgs) heap.push({0, w});
    std::vector<int> owner(cost.size(), 0);
    for (int i : order) {
        Slot sl = heap.top();
        heap.pop();
        owner[i] = sl.second;
        heap.push({sl.first + cost[i], sl.second});
    }
    return owner;
}

// Whole tiles placed by LPT with every grid on one XCD (one L2): the grids
// are dealt to the XCDs by LPT of their work (planes plus pipeline fill of
// every tile), then each XCD's tiles by LPT over its workgroups (w % kXcds
// == x).  For batches of uneven grids, which the round-robin deal leaves
// unbalanced.
void lpt_xcd_plan(const std::vector<mpdata_params> &grids, int tile, int nwg,
                  std::vector<mpd::Segment> &segs, std::vector<int> &wg_begin)
{
    const int ng = (int)grids.size();
    std::vector<long long> grid_cost(ng);
    for (int g = 0; g < ng; ++g)
        grid_cost[g] = (long long)tiles_x(grids[g], tile) * tiles_y(grids[g], tile) *
                       (grids[g].nz + kPipelineFill);
    std::vector<int> xcds(kXcds);
    for (int x = 0; x < kXcds; ++x) xcds[x] = x;
    const std::vector<int> grid_xcd = lpt_assign(grid_cost, xcds);
    std::vector<std::vector<mpd::Segment>> per(nwg);
    for (int x = 0; x < kXcds; ++x) {
        std::vector<mpd::Segment> tl;
        std::vector<long long> cost;
        for (int g = 0; g < ng; ++g) {
            if (grid_xcd[g] != x) continue;
            const int ntx = tiles_x(grids[g], tile), nty = tiles_y(grids[g], tile);
            for (int ty = 0; ty < nty; ++ty)
                for (int tx = 0; tx < ntx; ++tx) {
                    tl.push_back(mpd::Segment{g, tx, ty, 0, grids[g].nz, 0, 0, 0});
                    cost.push_back(grids[g].nz + kPipelineFill);
                }
        }
        std::vector<int> wgs;
        for (int w = x; w < nwg; w += kXcds) wgs.push_back(w);
        const std::vector<int> owner = lpt_assign(cost, wgs);
        for (size_t i = 0; i < tl.size(); ++i) per[owner[i]].push_back(tl[i]);
    }
    segs.clear();
    wg_begin.assign(nwg + 1, 0);
    for (int w = 0; w < nwg; ++w) {
        wg_begin[w] = (int)segs.size();
        segs.insert(segs.end(), per[w].begin(), per[w].end());
    }
    wg_begin[nwg] = (int)segs.size();
}

// The library's plan: whole tiles (dealt round-robin, or by LPT with every
// grid on one XCD when nwg is a multiple of the XCD count and that balances
// better) unless they balance worse than 1.1x the makespan of equal shares
// of planes.
void default_plan(const std::vector<mpdata_params> &grids, int tile, int nwg,
                  std::vector<mpd::Segment> &segs, std::vector<int> &wg_begin)
{
    std::vector<mpd::Segment> s2, s3;
    std::vector<int> w2, w3;
    share_plan(grids, tile, nwg, segs, wg_begin);
    whole_tile_plan(grids, tile, nwg, s2, w2);
    if (nwg % kXcds == 0 && grids.size() > 1) {
        lpt_xcd_plan(grids, tile, nwg, s3, w3);
        if (plan_makespan(s3, w3) < plan_makespan(s2, w2)) {
            s2.swap(s3);
            w2.swap(w3);
        }
    }
    if (plan_makespan(s2, w2) * 10 <= plan_makespan(segs, wg_begin) * 11) {
        segs.swap(s2);
        wg_begin.swap(w2);
    }
}

// A plan must cover every output tile of every grid over all its planes
// exactly once.
// grid_tile: the launch shape of each grid (its segments' tiles are counted
// in that shape's tiling)
const char *check_plan(const std::vector<mpdata_params> &grids, const std::vector<int> &grid_tile,
                       const std::vector<mpd::Segment> &segs, const std::vector<int> &wg_begin)
{
    const int nwg = (int)wg_begin.size() - 1;
    if (nwg < 1 || wg_begin[0] != 0 || wg_begin[nwg] != (int)segs.size()) return "bad wg_begin";
    for (int w = 0; w < nwg; ++w)
        if (wg_begin[w + 1] < wg_begin[w]) return "wg_begin must be non-decreasing";
    std::vector<size_t> base(grids.size() + 1, 0);
    for (size_t g = 0; g < grids.size(); ++g)
        base[g + 1] = base[g] + (size_t)tiles_x(grids[g], grid_tile[g]) *
                                    tiles_y(grids[g], grid_tile[g]) * grids[g].nz;
    std::vector<unsigned char> seen(base.back(), 0);
    for (const mpd::Segment &s : segs) {
        if (s.grid < 0 || s.grid >= (int)grids.size()) return "segment grid out of range";
        const mpdata_params &p = grids[s.grid];
        const int tile = grid_tile[s.grid];
        const int ntx = tiles_x(p, tile), nty = tiles_y(p, tile);
        if (s.tx < 0 || s.tx >= ntx || s.ty < 0 || s.ty >= nty) return "segment tile out of range";
        if (s.z0 < 0 || s.z1 > p.nz || s.z0 >= s.z1) return "segment z-range out of range";
        for (int z = s.z0; z < s.z1; ++z) {
            unsigned char &c = seen[base[s.grid] + ((size_t)s.ty * ntx + s.tx) * p.nz + z];
            if (c) return "a (tile, plane) is covered twice";
            c = 1;
        }
    }
    for (unsigned char c : seen)
        if (!c) return "a (tile, plane) is not covered";
    return nullptr;
}

struct Layout {
    size_t psi2, grids, segs, wg, ticks, partials, result, flags;
    // a single grid with iord > 2: the buffers of the chain of corrective
    // passes (iterates, limited velocities, psi1 and running bounds, two sets used in
    // turn) and the descriptors of its launches for both step parities
    size_t it[2], w[2][3], bmx[2], bmn[2], pass_grids, pass_io;
    size_t total;
};

Layout layout_for(const std::vector<mpdata_params> &grids, int max_segs, int max_wg)
{
    Layout l{};
    size_t off = 0;
    l.psi2 = off;
    for (const mpdata_params &p : grids) off += align_up(cells_of(&p) * word_of(&p));
    l.grids = off;
    off += align_up(grids.size() * sizeof(mpd::GridDesc<double>));
    l.segs = off;
    off += align_up((size_t)max_segs * sizeof(mpd::Segment));
    l.wg = off;
    off += align_up(((size_t)max_wg + 1) * sizeof(int));
    l.ticks = off;
    off += align_up((size_t)max_segs * sizeof(long long));
    l.partials = off;
    off += align_up((size_t)kMassParts * 2 * sizeof(double));
    l.result = off;
    off += align_up(2 * sizeof(double));
    l.flags = off;
    off += align_up(4 * sizeof(unsigned int));
    if (grids.size() == 1 && grids[0].iord > 2) {
        const mpdata_params &p = grids[0];
        const size_t w = word_of(&p), nx = p.nx, ny = p.ny, nz = p.nz;
        const size_t faces[3] = {(nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1)};
        const int sets = p.iord > 3 ? 2 : 1;  // a second set only for a middle pass
        for (int s = 0; s < sets; ++s) {
            l.it[s] = off;
            off += align_up(cells_of(&p) * w);
            for (int d = 0; d < 3; ++d) {
                l.w[s][d] = off;
                off += align_up(faces[d] * w);
            }
            if (p.nonos) {
                // bmx[0] takes psi1 from the head launch; the running bounds
                // of middle pass j go to set j & 1 (passes 1 .. iord - 3), so
                // set 1 needs a minimum from iord 4 on, set 0 from iord 5 on
                l.bmx[s] = off;
                off += align_up(cells_of(&p) * w);
                if (p.iord >= 5 - s) {
                    l.bmn[s] = off;
                    off += align_up(cells_of(&p) * w);
                }
            }
        }
        l.pass_grids = off;
        off += align_up(2 * (size_t)(p.iord - 1) * sizeof(mpd::GridDesc<double>));
        l.pass_io = off;
        off += align_up(2 * (size_t)(p.iord - 1) * sizeof(mpd::PassIO<double>));
    }
    l.total = off;
    return l;
}

int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return cus;
}

// Kernel variant bits of a parameter set.
int variant_of(const mpdata_params &p)
{
    return (p.bc == MPDATA_BC_OPEN ? mpd::kVariantOpen : 0) | (p.nonos ? mpd::kVariantNonos : 0) |
           ((p.flags & MPDATA_FLAG_VSIGN) ? mpd::kVariantVsign : 0) |
           ((p.flags & MPDATA_FLAG_DIV) ? mpd::kVariantDiv : 0) |
           ((p.flags & MPDATA_FLAG_TVEL) ? mpd::kVariantTvel : 0);
}

int wg_per_cu(int dtype, int tile, int variant)
{
    const void *k = dtype == MPDATA_FP32 ? mpd::step_kernel_ptr<float>(tile, variant)
                                         : mpd::step_kernel_ptr<double>(tile, variant);
    if (!k) return 0;
    int per = 0;
    const mpd::TileShape &s = shape_of(tile);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, s.rx * s.ry, 0) != hipSuccess)
        return 0;
    return per;
}

// Largest plan of the default kind: one segment per tile and per workgroup
// boundary.
void default_plan_bounds(const std::vector<mpdata_params> &grids, int tile, int nwg, int *nseg)
{
    long long n = 0;
    for (const mpdata_params &p : grids) n += (long long)tiles_x(p, tile) * tiles_y(p, tile);
    *nseg = (int)(n + nwg);
}

}  // namespace

// ================================================================== engine
// What one launch of the persistent kernel needs, shared by contexts and
// batches.

struct Engine {
    int dtype, tile, nwg, nseg, ngrids, iord;
    bool open, nonos, use_graph;
    bool tvel = false;                         // Courant numbers that change in time
    mpd::TvArgs<double> tv{};                  // TVEL: the bound level as both ends of a step
    int variant;  // kernel variant bits (open, nonos, variable sign)
    double eps;
    hipStream_t stream;
    char *ws;
    Layout lay;
    std::vector<mpdata_params> params;
    std::vector<mpd::GridDesc<double>> grids;  // host copy (float grids reinterpret the pointers)
    hipGraphExec_t graph = nullptr;            // kGraphSteps steps
    hipGraph_t graph_def = nullptr;
    char err[256];
};

static int fail_to(char *dst, int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 256, fmt, ap);
    va_end(ap);
    return code;
}

// One launch of the fused step kernel over the engine's plan; tv: the time
// levels of the Courant numbers (read by the TVEL variant only).
static hipError_t launch_step(Engine &e, int flip, long long *ticks, const mpd::TvArgs<double> &tv)
{
    const mpd::Segment *segs = (const mpd::Segment *)(e.ws + e.lay.segs);
    const int *wg = (const int *)(e.ws + e.lay.wg);
    if (e.dtype == MPDATA_FP32)
        return mpd::launch_persistent<float>((const mpd::GridDesc<float> *)(e.ws + e.lay.grids),
                                             segs, wg, e.nwg, e.tile, e.variant, flip,
                                             e.eps, ticks, (const mpd::TvArgs<float> &)tv, e.stream);
    return mpd::launch_persistent<double>((const mpd::GridDesc<double> *)(e.ws + e.lay.grids),
                                          segs, wg, e.nwg, e.tile, e.variant, flip, e.eps,
                                          ticks, tv, e.stream);
}

static hipError_t launch_one(Engine &e, int flip, long long *ticks)
{
    if (e.iord == 1) {
        const mpd::GridDesc<double> &g = e.grids[0];
        if (e.dtype == MPDATA_FP32) {
            mpd::DonorArgs<float> a{(const float *)g.psi[flip], (float *)g.psi[1 - flip],
                                    (const float *)g.u1, (const float *)g.u2, (const float *)g.u3,
                                    (const float *)g.h, g.nx, g.ny, g.nz};
            return mpd::launch_donor<float>(a, e.open, e.stream);
        }
        mpd::DonorArgs<double> a{g.psi[flip], g.psi[1 - flip], g.u1, g.u2, g.u3, g.h,
                                 g.nx, g.ny, g.nz};
        return mpd::launch_donor<double>(a, e.open, e.stream);
    }
    const mpd::Segment *segs = (const mpd::Segment *)(e.ws + e.lay.segs);
    const int *wg = (const int *)(e.ws + e.lay.wg);
    if (e.iord > 2) {
        // the chain of corrective passes of one step: head, middle passes, last
        const int npass = e.iord - 1;
        for (int j = 0; j < npass; ++j) {
            const int mode = j == 0 ? mpd::kPassHead : (j == npass - 1 ? mpd::kPassLast : mpd::kPassMid);
            const size_t i = (size_t)flip * npass + j;
            const auto *gd = (const mpd::GridDesc<double> *)(e.ws + e.lay.pass_grids) + i;
            const auto *io = (const mpd::PassIO<double> *)(e.ws + e.lay.pass_io) + i;
            const hipError_t r =
                e.dtype == MPDATA_FP32
                    ? mpd::launch_pass<float>((const mpd::GridDesc<float> *)gd,
                                              (const mpd::PassIO<float> *)io, segs, wg, e.nwg,
                                              e.tile, e.variant, mode, e.eps, e.stream)
                    : mpd::launch_pass<double>(gd, io, segs, wg, e.nwg, e.tile, e.variant, mode,
                                               e.eps, e.stream);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    }
    return launch_step(e, flip, ticks, e.tv);
}

// Graph of kGraphSteps steps (each launch reading what the previous wrote):
// one step launch per step, or the chain of corrective passes of each step
// (iord > 2).
static hipError_t build_graph(Engine &e)
{
    hipError_t r = hipGraphCreate(&e.graph_def, 0);
    if (r != hipSuccess) return r;
    hipGraphNode_t prev = nullptr;
    const mpd::TileShape &sh = shape_of(e.tile);
    const void *gridp = e.ws + e.lay.grids;
    const void *segp = e.ws + e.lay.segs;
    const void *wgp = e.ws + e.lay.wg;
    long long *no_ticks = nullptr;
    if (e.iord > 2) {
        const int npass = e.iord - 1;
        std::vector<const void *> gds((size_t)kGraphSteps * npass), ios((size_t)kGraphSteps * npass);
        for (int s = 0; s < kGraphSteps; ++s)
            for (int j = 0; j < npass; ++j) {
                const int mode = j == 0 ? mpd::kPassHead : (j == npass - 1 ? mpd::kPassLast : mpd::kPassMid);
                const size_t i = (size_t)(s & 1) * npass + j, n = (size_t)s * npass + j;
                gds[n] = (const mpd::GridDesc<double> *)(e.ws + e.lay.pass_grids) + i;
                ios[n] = (const mpd::PassIO<double> *)(e.ws + e.lay.pass_io) + i;
                void *args[] = {(void *)&gds[n], (void *)&ios[n], (void *)&segp, (void *)&wgp,
                                (void *)&e.eps};
                hipKernelNodeParams kp{};
                kp.func = (void *)(e.dtype == MPDATA_FP32 ? mpd::pass_kernel_ptr<float>(e.tile, e.variant, mode)
                                                          : mpd::pass_kernel_ptr<double>(e.tile, e.variant, mode));
                kp.gridDim = dim3(e.nwg);
                kp.blockDim = dim3(sh.rx * sh.ry);
                kp.sharedMemBytes = 0;
                kp.kernelParams = args;
                kp.extra = nullptr;
                hipGraphNode_t node;
                r = hipGraphAddKernelNode(&node, e.graph_def, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
                if (r != hipSuccess) return r;
                prev = node;
            }
        return hipGraphInstantiate(&e.graph, e.graph_def, nullptr, nullptr, 0);
    }
    int flips[kGraphSteps];
    mpd::TvArgs<double> tv = e.tv;  // TVEL contexts: the bound level, held over each step
    for (int s = 0; s < kGraphSteps; ++s) {
        flips[s] = s & 1;
        void *args[] = {(void *)&gridp, (void *)&segp, (void *)&wgp, (void *)&flips[s],
                        (void *)&e.eps, (void *)&no_ticks, (void *)&tv};
        hipKernelNodeParams kp{};
        kp.func = (void *)(e.dtype == MPDATA_FP32 ? mpd::step_kernel_ptr<float>(e.tile, e.variant)
                                                  : mpd::step_kernel_ptr<double>(e.tile, e.variant));
        kp.gridDim = dim3(e.nwg);
        kp.blockDim = dim3(sh.rx * sh.ry);
        kp.sharedMemBytes = 0;
        kp.kernelParams = args;
        kp.extra = nullptr;
        hipGraphNode_t node;
        r = hipGraphAddKernelNode(&node, e.graph_def, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
        if (r != hipSuccess) return r;
        prev = node;
    }
    return hipGraphInstantiate(&e.graph, e.graph_def, nullptr, nullptr, 0);
}

static int engine_step(Engine &e, int32_t nsteps)
{
    if (nsteps < 0) return fail_to(e.err, MPDATA_EINVAL, "nsteps must be >= 0");
    hipError_t r = hipSuccess;
    int32_t done = 0;
    if (e.use_graph && e.iord >= 2 && nsteps >= kGraphSteps) {
        if (!e.graph) {
            r = build_graph(e);
            if (r != hipSuccess) {
                e.use_graph = false;  // fall back to plain launches of the same kernel
                // teardown of a failed build: errors here change nothing
                if (e.graph) (void)hipGraphExecDestroy(e.graph);
                if (e.graph_def) (void)hipGraphDestroy(e.graph_def);
                e.graph = nullptr;
                e.graph_def = nullptr;
                (void)hipGetLastError();
            }
        }
        while (e.graph && nsteps - done >= kGraphSteps) {
            r = hipGraphLaunch(e.graph, e.stream);
            if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(r));
            done += kGraphSteps;
        }
    }
    for (int32_t s = done; s < nsteps; ++s) {
        r = launch_one(e, (s - done) & 1, nullptr);
        if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "step launch: %s", hipGetErrorString(r));
    }
    if ((nsteps - done) & 1) {
        r = e.dtype == MPDATA_FP32
                ? mpd::launch_copy_back<float>((const mpd::GridDesc<float> *)(e.ws + e.lay.grids), e.ngrids, e.stream)
                : mpd::launch_copy_back<double>((const mpd::GridDesc<double> *)(e.ws + e.lay.grids), e.ngrids, e.stream);
        if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "copy back: %s", hipGetErrorString(r));
    }
    return MPDATA_OK;
}

// Builds the replay graph ahead of the first run of steps, so that a run's
// first steps do not pay for its instantiation; a failed build leaves plain
// launches of the same kernel.
static void engine_prepare_graph(Engine &e)
{
    if (!e.use_graph || e.iord < 2 || e.graph) return;
    if (build_graph(e) != hipSuccess) {
        e.use_graph = false;
        if (e.graph) (void)hipGraphExecDestroy(e.graph);
        if (e.graph_def) (void)hipGraphDestroy(e.graph_def);
        e.graph = nullptr;
        e.graph_def = nullptr;
        (void)hipGetLastError();
    }
}

// TVEL contexts: later time levels are checked on the stream (periodic face
// pairs into flags[2]); a nonzero count is reported once the stream is
// synchronised.
static int engine_tv_status(Engine &e)
{
    if (!e.tvel || e.params[0].bc != MPDATA_BC_PERIODIC) return MPDATA_OK;
    unsigned int bad = 0;
    hipError_t r = hipMemcpyAsync(&bad, (unsigned int *)(e.ws + e.lay.flags) + 2, sizeof(bad),
                                  hipMemcpyDeviceToHost, e.stream);
    if (r == hipSuccess) r = hipStreamSynchronize(e.stream);
    if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "level check readback: %s", hipGetErrorString(r));
    if (bad)
        return fail_to(e.err, MPDATA_EINVAL,
                       "a time level given to mpdata_step_tv breaks periodicity (%u face pairs with "
                       "face n != face 0); the steps that used it have run",
                       bad);
    return MPDATA_OK;
}

static int engine_mass(Engine &e, int i, double *out)
{
    double *parts = (double *)(e.ws + e.lay.partials);
    double *res = (double *)(e.ws + e.lay.result);
    const mpd::GridDesc<double> &g = e.grids[i];
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    hipError_t r = e.dtype == MPDATA_FP64
                       ? mpd::launch_mass<double>(g.psi[0], g.h, n, parts, kMassParts, res, e.stream)
                       : mpd::launch_mass<float>((const float *)g.psi[0], (const float *)g.h, n,
                                                 parts, kMassParts, res, e.stream);
    if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "mass launch: %s", hipGetErrorString(r));
    double h2[2];
    r = hipMemcpyAsync(h2, res, sizeof(h2), hipMemcpyDeviceToHost, e.stream);
    if (r == hipSuccess) r = hipStreamSynchronize(e.stream);
    if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "mass readback: %s", hipGetErrorString(r));
    *out = h2[0];
    if (!isfinite(h2[0])) return fail_to(e.err, MPDATA_ENONFINITE, "psi holds NaN or Inf");
    return engine_tv_status(e);
}

// Descriptors of the chain of corrective passes (iord > 2) for both step
// parities f: pass j reads psi[f] (j = 0) or iterate set (j-1) mod 2 and
// writes psi[1-f] (the last pass) or iterate set j mod 2; its velocity field
// is the Courant numbers (j = 0) or the limited velocity of pass j-1.  Its
// limiter bounds come from two cell arrays: psi1 (written by the head
// launch) and psi[f] itself for pass 1, the running bounds written by pass
// j-1 after that.  FP32 reinterprets the pointers.
static void pass_descriptors(const Engine &e, std::vector<mpd::GridDesc<double>> &pg,
                             std::vector<mpd::PassIO<double>> &pio)
{
    const int npass = e.iord - 1;
    const mpd::GridDesc<double> &g = e.grids[0];
    auto at = [&](size_t off) { return (double *)(e.ws + off); };
    pg.assign(2 * npass, g);
    pio.assign(2 * npass, mpd::PassIO<double>{});
    for (int f = 0; f < 2; ++f)
        for (int j = 0; j < npass; ++j) {
            mpd::GridDesc<double> &d = pg[f * npass + j];
            mpd::PassIO<double> &io = pio[f * npass + j];
            const int in = (j - 1) & 1, out = j & 1;
            if (j > 0) {
                d.u1 = at(e.lay.w[in][0]);
                d.u2 = at(e.lay.w[in][1]);
                d.u3 = at(e.lay.w[in][2]);
                if (e.nonos) {
                    // bounds over max/min(bmx, bmn, iterate): psi1 and psi^n
                    // after the head launch, the running bounds after a middle one
                    io.bmx = at(e.lay.bmx[in]);
                    io.bmn = j == 1 ? g.psi[f] : at(e.lay.bmn[in]);
                }
            }
            d.psi[0] = j == 0 ? g.psi[f] : at(e.lay.it[in]);
            d.psi[1] = j == npass - 1 ? g.psi[1 - f] : at(e.lay.it[out]);
            if (j < npass - 1) {
                io.w1 = at(e.lay.w[out][0]);
                io.w2 = at(e.lay.w[out][1]);
                io.w3 = at(e.lay.w[out][2]);
                if (e.nonos) {
                    io.mx = at(e.lay.bmx[out]);  // the head writes psi1 here
                    if (j > 0) io.mn = at(e.lay.bmn[out]);
                }
            }
        }
}

// Validates every grid's arrays on the device (h > 0 and finite; periodic
// faces n == 0), lays out the workspace, uploads descriptors and the plan.
static int engine_init(Engine &e, char *errbuf, int n, const mpdata_params *params,
                       void *const *psi, const void *const *u1, const void *const *u2,
                       const void *const *u3, const void *const *h, void *workspace,
                       size_t ws_bytes, void *stream, const mpdata_plan *plan, bool batch)
{
    if (n < 1) return fail_to(errbuf, MPDATA_EINVAL, "need at least one grid");
    if (!params) return fail_to(errbuf, MPDATA_EINVAL, "params is NULL");
    if (!psi || !u1 || !u2 || !u3 || !h) return fail_to(errbuf, MPDATA_EINVAL, "NULL array list");
    for (int i = 0; i < n; ++i) {
        if (const char *m = check_params(&params[i]))
            return fail_to(errbuf, MPDATA_EINVAL, "grid %d: %s", i, m);
        if (!psi[i] || !u1[i] || !u2[i] || !u3[i] || !h[i])
            return fail_to(errbuf, MPDATA_EINVAL, "grid %d: NULL array or workspace pointer", i);
        if (misaligned(psi[i]) || misaligned(u1[i]) || misaligned(u2[i]) || misaligned(u3[i]) ||
            misaligned(h[i]))
            return fail_to(errbuf, MPDATA_EINVAL, "grid %d: arrays must be 16-byte aligned", i);
        const mpdata_params &a = params[0], &b = params[i];
        if (a.dtype != b.dtype || a.bc != b.bc || a.iord != b.iord || a.nonos != b.nonos ||
            a.eps != b.eps || a.tile != b.tile ||
            (a.flags & (MPDATA_FLAG_VSIGN | MPDATA_FLAG_DIV)) !=
                (b.flags & (MPDATA_FLAG_VSIGN | MPDATA_FLAG_DIV)))
            return fail_to(errbuf, MPDATA_ENOTSUP,
                           "grid %d: a batch shares dtype, bc, iord, nonos, eps, tile and flags", i);
    }
    if (batch && params[0].iord != 2)
        return fail_to(errbuf, MPDATA_ENOTSUP, "batches run the full step (iord 2)");
    if (batch && (params[0].flags & MPDATA_FLAG_TVEL))
        return fail_to(errbuf, MPDATA_ENOTSUP,
                       "Courant numbers that change in time run on single-grid contexts");
    if (!workspace) return fail_to(errbuf, MPDATA_EINVAL, "NULL array or workspace pointer");
    if (((uintptr_t)workspace & (kAlign - 1)) != 0)
        return fail_to(errbuf, MPDATA_EINVAL, "workspace must be 256-byte aligned");

    e.params.assign(params, params + n);
    e.dtype = params[0].dtype;
    e.iord = params[0].iord;
    e.open = params[0].bc == MPDATA_BC_OPEN;
    e.nonos = params[0].nonos != 0;
    e.variant = variant_of(params[0]);
    e.eps = params[0].eps;
    e.use_graph = !(params[0].flags & MPDATA_FLAG_NO_GRAPH);
    e.tvel = (params[0].flags & MPDATA_FLAG_TVEL) != 0;
    e.stream = (hipStream_t)stream;
    e.ngrids = n;
    e.ws = (char *)workspace;
    e.err[0] = 0;

    std::vector<mpd::Segment> segs;
    std::vector<int> wg;
    std::vector<int> grid_tile;
    if (plan) {
        const int cols = plan->seg_cols == 0 ? 5 : plan->seg_cols;
        if (plan->tile < 1 || plan->tile > mpdata_tile_count() || plan->nwg < 1 || plan->nseg < 1 ||
            !plan->seg || !plan->wg_begin || (cols != 5 && cols != 6))
            return fail_to(errbuf, MPDATA_EINVAL, "invalid plan header");
        e.tile = plan->tile;
        grid_tile.assign(n, e.tile);
        if (cols == 6) {
            // per-grid launch shapes: one launch of the mixed family
            if (e.tile != mpd::kMixedTiles[0] && e.tile != mpd::kMixedTiles[1])
                return fail_to(errbuf, MPDATA_EINVAL, "a plan with per-grid shapes names tile 5 or 7");
            e.variant |= mpd::kVariantMixed;
            std::vector<int> seen_tile(n, 0);
            for (int s = 0; s < plan->nseg; ++s) {
                const int32_t *v = plan->seg + 6 * (size_t)s;
                if (v[0] < 0 || v[0] >= n) return fail_to(errbuf, MPDATA_EINVAL, "plan: segment grid out of range");
                if (v[5] != mpd::kMixedTiles[0] && v[5] != mpd::kMixedTiles[1])
                    return fail_to(errbuf, MPDATA_EINVAL, "plan: segment shape must be tile 5 or 7");
                if (seen_tile[v[0]] && seen_tile[v[0]] != v[5])
                    return fail_to(errbuf, MPDATA_EINVAL, "plan: the segments of a grid share one shape");
                seen_tile[v[0]] = v[5];
            }
            for (int g = 0; g < n; ++g)
                if (seen_tile[g]) grid_tile[g] = seen_tile[g];
        }
        if (!(e.dtype == MPDATA_FP32 ? mpd::step_kernel_ptr<float>(e.tile, e.variant)
                                     : mpd::step_kernel_ptr<double>(e.tile, e.variant)))
            return fail_to(errbuf, MPDATA_ENOTSUP, "no step kernel for this launch shape and variant");
        segs.resize(plan->nseg);
        for (int s = 0; s < plan->nseg; ++s) {
            const int32_t *v = plan->seg + (size_t)cols * s;
            const int shape = cols == 6 && v[5] == mpd::kMixedTiles[1] ? 1 : 0;
            segs[s] = mpd::Segment{v[0], v[1], v[2], v[3], v[4], shape, 0, 0};
        }
        wg.assign(plan->wg_begin, plan->wg_begin + plan->nwg + 1);
    } else {
        e.tile = tile_of(&params[0]);
        const int per = wg_per_cu(e.dtype, e.tile, e.variant);
        const int cus = device_cus();
        if (per < 1 || cus < 1) return fail_to(errbuf, MPDATA_EDEVICE, "occupancy query failed");
        default_plan(e.params, e.tile, per * cus, segs, wg);
        grid_tile.assign(n, e.tile);
    }
    if (const char *m = check_plan(e.params, grid_tile, segs, wg))
        return fail_to(errbuf, MPDATA_EINVAL, "plan: %s", m);
    if (e.iord > 2 && !(e.dtype == MPDATA_FP32 ? mpd::pass_kernel_ptr<float>(e.tile, e.variant, mpd::kPassHead)
                                               : mpd::pass_kernel_ptr<double>(e.tile, e.variant, mpd::kPassHead)))
        return fail_to(errbuf, MPDATA_ENOTSUP, "no kernels of further corrective passes for this launch shape");
    e.nwg = (int)wg.size() - 1;
    e.nseg = (int)segs.size();
    e.lay = layout_for(e.params, e.nseg, e.nwg);
    if (ws_bytes < e.lay.total)
        return fail_to(errbuf, MPDATA_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes,
                       e.lay.total);

    hipError_t r;
    unsigned int *flags = (unsigned int *)(e.ws + e.lay.flags);
    size_t off2 = e.lay.psi2;
    e.grids.resize(n);
    for (int i = 0; i < n; ++i) {
        const mpdata_params &p = params[i];
        mpd::GridDesc<double> &g = e.grids[i];
        g.u1 = (const double *)u1[i];
        g.u2 = (const double *)u2[i];
        g.u3 = (const double *)u3[i];
        g.h = (const double *)h[i];
        g.psi[0] = (double *)psi[i];
        g.psi[1] = (double *)(e.ws + off2);
        g.nx = p.nx;
        g.ny = p.ny;
        g.nz = p.nz;
        g.pad = 0;
        off2 += align_up(cells_of(&p) * word_of(&p));

        r = hipMemsetAsync(flags, 0, 4 * sizeof(unsigned int), e.stream);
        if (r != hipSuccess) return fail_to(errbuf, MPDATA_EDEVICE, "hipMemsetAsync: %s", hipGetErrorString(r));
        const int periodic = p.bc == MPDATA_BC_PERIODIC;
        r = e.dtype == MPDATA_FP64
                ? mpd::launch_validate<double>(g.h, g.u1, g.u2, g.u3, p.nx, p.ny, p.nz, periodic, flags, e.stream)
                : mpd::launch_validate<float>((const float *)g.h, (const float *)g.u1,
                                              (const float *)g.u2, (const float *)g.u3, p.nx, p.ny,
                                              p.nz, periodic, flags, e.stream);
        if (r != hipSuccess) return fail_to(errbuf, MPDATA_EDEVICE, "validate launch: %s", hipGetErrorString(r));
        unsigned int hf[2] = {0, 0};
        r = hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, e.stream);
        if (r == hipSuccess) r = hipStreamSynchronize(e.stream);
        if (r != hipSuccess) return fail_to(errbuf, MPDATA_EDEVICE, "validate readback: %s", hipGetErrorString(r));
        if (hf[0]) return fail_to(errbuf, MPDATA_EINVAL, "grid %d: h must be finite and > 0 (%u bad cells)", i, hf[0]);
        if (hf[1])
            return fail_to(errbuf, MPDATA_EINVAL,
                           "grid %d: periodic boundaries need face n == face 0 on every axis (%u differ)",
                           i, hf[1]);
    }
    if (e.tvel) {
        const mpd::GridDesc<double> &g = e.grids[0];
        e.tv = mpd::TvArgs<double>{g.u1, g.u2, g.u3, g.u1, g.u2, g.u3};
    }
    // descriptors and plan into the workspace (GridDesc<float> has the same layout)
    r = hipMemcpyAsync(e.ws + e.lay.grids, e.grids.data(), n * sizeof(mpd::GridDesc<double>),
                       hipMemcpyHostToDevice, e.stream);
    if (r == hipSuccess)
        r = hipMemcpyAsync(e.ws + e.lay.segs, segs.data(), segs.size() * sizeof(mpd::Segment),
                           hipMemcpyHostToDevice, e.stream);
    if (r == hipSuccess)
        r = hipMemcpyAsync(e.ws + e.lay.wg, wg.data(), wg.size() * sizeof(int),
                           hipMemcpyHostToDevice, e.stream);
    std::vector<mpd::GridDesc<double>> pg;
    std::vector<mpd::PassIO<double>> pio;
    if (e.iord > 2) {
        pass_descriptors(e, pg, pio);
        if (r == hipSuccess)
            r = hipMemcpyAsync(e.ws + e.lay.pass_grids, pg.data(), pg.size() * sizeof(pg[0]),
                               hipMemcpyHostToDevice, e.stream);
        if (r == hipSuccess)
            r = hipMemcpyAsync(e.ws + e.lay.pass_io, pio.data(), pio.size() * sizeof(pio[0]),
                               hipMemcpyHostToDevice, e.stream);
    }
    if (r == hipSuccess) r = hipStreamSynchronize(e.stream);
    if (r != hipSuccess) return fail_to(errbuf, MPDATA_EDEVICE, "plan upload: %s", hipGetErrorString(r));
    return MPDATA_OK;
}

// Destroy paths report nothing: the objects are gone either way.
static void engine_release(Engine &e)
{
    if (e.graph) (void)hipGraphExecDestroy(e.graph);
    if (e.graph_def) (void)hipGraphDestroy(e.graph_def);
    e.graph = nullptr;
    e.graph_def = nullptr;
}

struct mpdata_ctx {
    Engine e;
    int64_t steps;
};

struct mpdata_batch {
    Engine e;
};

static size_t workspace_for(int n, const mpdata_params *params, int max_segs, int max_wg)
{
    std::vector<mpdata_params> v(params, params + n);
    return layout_for(v, max_segs, max_wg).total;
}

// Upper bound of the default plan's size without touching the device: at
// most 8 resident workgroups of the largest shape per CU on 256 CUs.
static void default_bounds(int n, const mpdata_params *params, int tile, int *nseg, int *nwg)
{
    std::vector<mpdata_params> v(params, params + n);
    *nwg = 256 * 8;
    default_plan_bounds(v, tile, *nwg, nseg);
}


// -------------------------------------------------------------------- pools

struct mpdata_pool {
    Engine e;                 // dtype, tile, open, nonos, eps, stream, graph
    int max_grids, max_segs, nwg_all;
    struct Slot {
        bool used;
        mpdata_params p;
        mpd::GridDesc<double> g;
    };
    std::vector<Slot> slots;
    bool dirty;               // membership changed since the last upload
    // pinned host staging of the plan, double-buffered against in-flight copies
    struct Stage {
        char *host;
        hipEvent_t done;
        bool pending;
    } stage[2];
    int cur_stage;
    size_t stage_bytes;
};

static int pool_fail(mpdata_pool *p, int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(p ? p->e.err : g_create_err, 256, fmt, ap);
    va_end(ap);
    return code;
}

static Layout pool_layout(int max_grids, int max_segs, int max_wg)
{
    // no psi copies in the workspace: members bring their own second buffer
    Layout l;
    size_t off = 0;
    l.psi2 = 0;
    l.grids = off;
    off += align_up((size_t)max_grids * sizeof(mpd::GridDesc<double>));
    l.segs = off;
    off += align_up((size_t)max_segs * sizeof(mpd::Segment));
    l.wg = off;
    off += align_up(((size_t)max_wg + 1) * sizeof(int));
    l.ticks = off;
    l.partials = off;
    off += align_up((size_t)kMassParts * 2 * sizeof(double));
    l.result = off;
    off += align_up(2 * sizeof(double));
    l.flags = off;
    off += align_up(4 * sizeof(unsigned int));
    l.total = off;
    return l;
}

// Uploads descriptors and the default plan of the current members.
static int pool_upload(mpdata_pool *p)
{
    Engine &e = p->e;
    std::vector<mpdata_params> ps;
    std::vector<mpd::GridDesc<double>> gs;
    for (const auto &s : p->slots)
        if (s.used) {
            ps.push_back(s.p);
            gs.push_back(s.g);
        }
    e.ngrids = (int)gs.size();
    if (e.ngrids == 0) return MPDATA_OK;
    std::vector<mpd::Segment> segs;
    std::vector<int> wg;
    default_plan(ps, e.tile, p->nwg_all, segs, wg);
    if ((int)segs.size() > p->max_segs)
        return pool_fail(p, MPDATA_ENOMEM, "plan needs %zu segments > max_segments %d", segs.size(),
                         p->max_segs);
    e.nwg = (int)wg.size() - 1;
    e.nseg = (int)segs.size();
    mpdata_pool::Stage &st = p->stage[p->cur_stage];
    p->cur_stage ^= 1;
    if (st.pending) {
        hipError_t r = hipEventSynchronize(st.done);
        if (r != hipSuccess) return pool_fail(p, MPDATA_EDEVICE, "staging wait: %s", hipGetErrorString(r));
    }
    const size_t bg = gs.size() * sizeof(mpd::GridDesc<double>);
    const size_t bs = segs.size() * sizeof(mpd::Segment);
    const size_t bw = wg.size() * sizeof(int);
    memcpy(st.host, gs.data(), bg);
    memcpy(st.host + align_up(bg), segs.data(), bs);
    memcpy(st.host + align_up(bg) + align_up(bs), wg.data(), bw);
    hipError_t r = hipMemcpyAsync(e.ws + e.lay.grids, st.host, bg, hipMemcpyHostToDevice, e.stream);
    if (r == hipSuccess)
        r = hipMemcpyAsync(e.ws + e.lay.segs, st.host + align_up(bg), bs, hipMemcpyHostToDevice, e.stream);
    if (r == hipSuccess)
        r = hipMemcpyAsync(e.ws + e.lay.wg, st.host + align_up(bg) + align_up(bs), bw,
                           hipMemcpyHostToDevice, e.stream);
    if (r == hipSuccess) r = hipEventRecord(st.done, e.stream);
    if (r != hipSuccess) return pool_fail(p, MPDATA_EDEVICE, "plan upload: %s", hipGetErrorString(r));
    st.pending = true;
    p->dirty = false;
    // a replayed graph stays valid: it holds only the workspace addresses of
    // the plan (whose contents were just replaced, in stream order) and the
    // workgroup count, which the default plan keeps at nwg_all
    return MPDATA_OK;
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

int mpdata_fpm_check(const double *speed, int32_t nspeed, int32_t dx, int32_t *x_bad,
                     int32_t *y_bad)
{
    if (!speed || nspeed < 2 || dx < 1) return MPDATA_EINVAL;
    for (int32_t k = 1; k < nspeed; ++k)
        if (!(speed[k] > 0.0) || !std::isfinite(speed[k])) return MPDATA_EINVAL;
    // s(x)/x is compared for every pair x < y; the table is small
    int count = 0;
    for (int32_t a = 1; a < nspeed; ++a)
        for (int32_t b = a + 1; b < nspeed; ++b)
            if (speed[a] / (double)(a * dx) < speed[b] / (double)(b * dx)) {
                if (count == 0) {
                    if (x_bad) *x_bad = a * dx;
                    if (y_bad) *y_bad = b * dx;
                }
                ++count;
            }
    return count;
}

int mpdata_fpm_partition(const double *speed, int32_t nspeed, int32_t n, int32_t p, int32_t dx,
                         int32_t *x_lo, int32_t *x_hi, double *t_min)
{
    if (!speed || !x_lo || !x_hi || !t_min || dx < 1 || p < 2 || p % 2 || n < 1 || n % p ||
        (n / p) % dx)
        return MPDATA_EINVAL;
    const int32_t share = n / p;
    // the moves reach x_hi = 2 share - dx: granule index 2 share/dx - 1
    if (nspeed < 2 * (share / dx)) return MPDATA_EINVAL;
    for (int32_t k = 1; k < 2 * (share / dx); ++k)
        if (!(speed[k] > 0.0) || !std::isfinite(speed[k])) return MPDATA_EINVAL;
    auto time_of = [&](int32_t x) { return (double)x / speed[x / dx]; };
    int32_t lo = share, hi = share, best_lo = share, best_hi = share;
    double best = time_of(share);
    while (lo - dx >= dx) {
        hi += dx;
        lo -= dx;
        const double t = std::max(time_of(hi), time_of(lo));
        if (t < best) {
            best = t;
            best_lo = lo;
            best_hi = hi;
        }
    }
    *x_lo = best_lo;
    *x_hi = best_hi;
    *t_min = best;
    return MPDATA_OK;
}

int32_t mpdata_default_tile(int32_t dtype, int32_t bc)
{
    if (dtype != MPDATA_FP64 && dtype != MPDATA_FP32) return 0;
    if (bc != MPDATA_BC_PERIODIC && bc != MPDATA_BC_OPEN) return 0;
    return default_tile(dtype, bc);
}

int mpdata_occupancy(int32_t dtype, int32_t tile, int32_t bc, int32_t nonos, int32_t *per_cu,
                     int32_t *cus)
{
    if (dtype != MPDATA_FP64 && dtype != MPDATA_FP32) return MPDATA_EINVAL;
    if (tile == 0) tile = default_tile(dtype, bc);
    if (tile < 1 || tile > mpdata_tile_count()) return MPDATA_EINVAL;
    const int variant = (bc == MPDATA_BC_OPEN ? mpd::kVariantOpen : 0) | (nonos ? mpd::kVariantNonos : 0);
    if (!(dtype == MPDATA_FP32 ? mpd::step_kernel_ptr<float>(tile, variant)
                               : mpd::step_kernel_ptr<double>(tile, variant)))
        return MPDATA_ENOTSUP;
    const int per = wg_per_cu(dtype, tile, variant);
    const int c = device_cus();
    if (per < 1 || c < 1) return MPDATA_EDEVICE;
    if (per_cu) *per_cu = per;
    if (cus) *cus = c;
    return MPDATA_OK;
}

size_t mpdata_workspace_bytes(const mpdata_params *p)
{
    if (check_params(p)) return 0;
    int nseg = 0, nwg = 0;
    default_bounds(1, p, tile_of(p), &nseg, &nwg);
    return workspace_for(1, p, nseg, nwg);
}

int mpdata_create(const mpdata_params *p, void *psi, const void *u1, const void *u2,
                  const void *u3, const void *h, void *workspace, size_t ws_bytes, void *stream,
                  mpdata_ctx **out)
{
    g_create_err[0] = 0;
    if (!out) return fail_to(g_create_err, MPDATA_EINVAL, "out is NULL");
    *out = nullptr;
    if (const char *m = check_params(p)) return fail_to(g_create_err, MPDATA_EINVAL, "%s", m);
    if (!psi || !u1 || !u2 || !u3 || !h || !workspace)
        return fail_to(g_create_err, MPDATA_EINVAL, "NULL array or workspace pointer");
    if (misaligned(psi) || misaligned(u1) || misaligned(u2) || misaligned(u3) || misaligned(h))
        return fail_to(g_create_err, MPDATA_EINVAL, "arrays must be 16-byte aligned");
    if (ws_bytes < mpdata_workspace_bytes(p))
        return fail_to(g_create_err, MPDATA_ENOMEM, "workspace too small: %zu < %zu bytes",
                       ws_bytes, mpdata_workspace_bytes(p));
    mpdata_ctx *c = new (std::nothrow) mpdata_ctx;
    if (!c) return fail_to(g_create_err, MPDATA_ENOMEM, "host allocation failed");
    void *psis[1] = {psi};
    const void *a1[1] = {u1}, *a2[1] = {u2}, *a3[1] = {u3}, *ah[1] = {h};
    const int rc = engine_init(c->e, g_create_err, 1, p, psis, a1, a2, a3, ah, workspace, ws_bytes,
                               stream, nullptr, false);
    if (rc != MPDATA_OK) {
        delete c;
        return rc;
    }
    engine_prepare_graph(c->e);
    c->steps = 0;
    *out = c;
    return MPDATA_OK;
}

int mpdata_step(mpdata_ctx *c, int32_t nsteps)
{
    if (!c) return MPDATA_EINVAL;
    const int rc = engine_step(c->e, nsteps);
    if (rc == MPDATA_OK) c->steps += nsteps;
    return rc;
}

int mpdata_mass(mpdata_ctx *c, double *out)
{
    if (!c) return MPDATA_EINVAL;
    if (!out) return fail_to(c->e.err, MPDATA_EINVAL, "out is NULL");
    return engine_mass(c->e, 0, out);
}

int mpdata_mass_noalloc(int32_t dtype, const void *psi, const void *h, int64_t n,
                        double *out_device, void *stream)
{
    if (dtype != MPDATA_FP64 && dtype != MPDATA_FP32) return MPDATA_EINVAL;
    if (!psi || !h || !out_device) return MPDATA_EINVAL;
    if (n < 0 || n > kMaxNoallocCells) return MPDATA_EINVAL;
    static_assert(kMassParts <= mpd::kScratchParts, "the scratch holds the partials of mpdata_mass");
    const hipError_t r =
        dtype == MPDATA_FP64
            ? mpd::launch_mass_noalloc<double>((const double *)psi, (const double *)h, (size_t)n,
                                               kMassParts, out_device, (hipStream_t)stream)
            : mpd::launch_mass_noalloc<float>((const float *)psi, (const float *)h, (size_t)n,
                                              kMassParts, out_device, (hipStream_t)stream);
    return r == hipSuccess ? MPDATA_OK : MPDATA_EDEVICE;
}

int mpdata_get_psi(mpdata_ctx *c, void *dst)
{
    if (!c) return MPDATA_EINVAL;
    if (!dst) return fail_to(c->e.err, MPDATA_EINVAL, "dst is NULL");
    hipError_t r = hipMemcpyAsync(dst, c->e.grids[0].psi[0], cells_of(&c->e.params[0]) * word_of(&c->e.params[0]),
                                  hipMemcpyDeviceToDevice, c->e.stream);
    return r == hipSuccess ? MPDATA_OK
                           : fail_to(c->e.err, MPDATA_EDEVICE, "get_psi: %s", hipGetErrorString(r));
}

int mpdata_set_psi(mpdata_ctx *c, const void *src)
{
    if (!c) return MPDATA_EINVAL;
    if (!src) return fail_to(c->e.err, MPDATA_EINVAL, "src is NULL");
    hipError_t r = hipMemcpyAsync(c->e.grids[0].psi[0], src, cells_of(&c->e.params[0]) * word_of(&c->e.params[0]),
                                  hipMemcpyDeviceToDevice, c->e.stream);
    if (r != hipSuccess) return fail_to(c->e.err, MPDATA_EDEVICE, "set_psi: %s", hipGetErrorString(r));
    c->steps = 0;
    return MPDATA_OK;
}

int mpdata_step_tv(mpdata_ctx *c, int32_t nsteps, const void *const *u1, const void *const *u2,
                   const void *const *u3)
{
    if (!c) return MPDATA_EINVAL;
    Engine &e = c->e;
    if (!e.tvel)
        return fail_to(e.err, MPDATA_ENOTSUP, "the context was created without MPDATA_FLAG_TVEL");
    if (nsteps < 0) return fail_to(e.err, MPDATA_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return MPDATA_OK;
    if (!u1 || !u2 || !u3) return fail_to(e.err, MPDATA_EINVAL, "NULL level list");
    for (int32_t s = 0; s < nsteps; ++s) {
        if (!u1[s] || !u2[s] || !u3[s])
            return fail_to(e.err, MPDATA_EINVAL, "level %d: NULL array", (int)s + 1);
        if (misaligned(u1[s]) || misaligned(u2[s]) || misaligned(u3[s]))
            return fail_to(e.err, MPDATA_EINVAL, "level %d: arrays must be 16-byte aligned", (int)s + 1);
    }
    const mpdata_params &p = e.params[0];
    hipError_t r = hipSuccess;
    unsigned int *bad = (unsigned int *)(e.ws + e.lay.flags) + 2;
    if (p.bc == MPDATA_BC_PERIODIC)
        for (int32_t s = 0; s < nsteps && r == hipSuccess; ++s)
            r = e.dtype == MPDATA_FP64
                    ? mpd::launch_check_periodic_faces<double>((const double *)u1[s], (const double *)u2[s],
                                                               (const double *)u3[s], p.nx, p.ny, p.nz,
                                                               bad, e.stream)
                    : mpd::launch_check_periodic_faces<float>((const float *)u1[s], (const float *)u2[s],
                                                              (const float *)u3[s], p.nx, p.ny, p.nz,
                                                              bad, e.stream);
    if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "level check launch: %s", hipGetErrorString(r));
    // step s runs from level s (the bound level for s = 0) to level s + 1
    mpd::TvArgs<double> tv = e.tv;
    for (int32_t s = 0; s < nsteps; ++s) {
        tv.w1 = (const double *)u1[s];
        tv.w2 = (const double *)u2[s];
        tv.w3 = (const double *)u3[s];
        r = launch_step(e, s & 1, nullptr, tv);
        if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "step launch: %s", hipGetErrorString(r));
        tv.u1 = tv.w1;
        tv.u2 = tv.w2;
        tv.u3 = tv.w3;
    }
    if (nsteps & 1) {
        r = e.dtype == MPDATA_FP32
                ? mpd::launch_copy_back<float>((const mpd::GridDesc<float> *)(e.ws + e.lay.grids), 1, e.stream)
                : mpd::launch_copy_back<double>((const mpd::GridDesc<double> *)(e.ws + e.lay.grids), 1, e.stream);
        if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "copy back: %s", hipGetErrorString(r));
    }
    // the last level is now the bound one: the replay graph of plain steps
    // (which holds it over each step) is rebuilt for it
    e.tv = mpd::TvArgs<double>{tv.u1, tv.u2, tv.u3, tv.u1, tv.u2, tv.u3};
    e.grids[0].u1 = tv.u1;
    e.grids[0].u2 = tv.u2;
    e.grids[0].u3 = tv.u3;
    engine_release(e);
    engine_prepare_graph(e);
    c->steps += nsteps;
    return MPDATA_OK;
}

int mpdata_sync(mpdata_ctx *c)
{
    if (!c) return MPDATA_EINVAL;
    hipError_t r = hipStreamSynchronize(c->e.stream);
    if (r != hipSuccess)
        return fail_to(c->e.err, MPDATA_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(r));
    return engine_tv_status(c->e);
}

int64_t mpdata_steps_done(const mpdata_ctx *c) { return c ? c->steps : -1; }

void mpdata_destroy(mpdata_ctx *c)
{
    if (!c) return;
    // the caller may free the workspace once this returns: wait for the
    // work still queued on it
    (void)hipStreamSynchronize(c->e.stream);
    engine_release(c->e);
    delete c;
}

const char *mpdata_last_error(const mpdata_ctx *c) { return c ? c->e.err : g_create_err; }

// ------------------------------------------------------------------ batches

size_t mpdata_batch_workspace_bytes(int32_t n, const mpdata_params *params, int32_t max_segments,
                                    int32_t max_wg)
{
    if (n < 1 || !params || max_segments < 0 || max_wg < 0) return 0;
    for (int i = 0; i < n; ++i)
        if (check_params(&params[i]) || params[i].iord != 2) return 0;
    int nseg = 0, nwg = 0;
    default_bounds(n, params, tile_of(&params[0]), &nseg, &nwg);
    return workspace_for(n, params, std::max(nseg, (int)max_segments), std::max(nwg, (int)max_wg));
}

int mpdata_batch_default_plan_size(int32_t n, const mpdata_params *params, int32_t tile,
                                   int32_t *nseg, int32_t *nwg)
{
    if (n < 1 || !params) return MPDATA_EINVAL;
    for (int i = 0; i < n; ++i)
        if (check_params(&params[i])) return MPDATA_EINVAL;
    if (tile == 0) tile = tile_of(&params[0]);
    if (tile < 1 || tile > mpdata_tile_count()) return MPDATA_EINVAL;
    const int per = wg_per_cu(params[0].dtype, tile, variant_of(params[0]));
    const int cus = device_cus();
    if (per < 1 || cus < 1) return MPDATA_EDEVICE;
    std::vector<mpdata_params> v(params, params + n);
    std::vector<mpd::Segment> segs;
    std::vector<int> wg;
    default_plan(v, tile, per * cus, segs, wg);
    if (nseg) *nseg = (int32_t)segs.size();
    if (nwg) *nwg = (int32_t)wg.size() - 1;
    return MPDATA_OK;
}

int mpdata_batch_create(int32_t n, const mpdata_params *params, void *const *psi,
                        const void *const *u1, const void *const *u2, const void *const *u3,
                        const void *const *h, void *workspace, size_t ws_bytes, void *stream,
                        const mpdata_plan *plan, mpdata_batch **out)
{
    g_create_err[0] = 0;
    if (!out) return fail_to(g_create_err, MPDATA_EINVAL, "out is NULL");
    *out = nullptr;
    mpdata_batch *b = new (std::nothrow) mpdata_batch;
    if (!b) return fail_to(g_create_err, MPDATA_ENOMEM, "host allocation failed");
    const int rc = engine_init(b->e, g_create_err, n, params, psi, u1, u2, u3, h, workspace,
                               ws_bytes, stream, plan, true);
    if (rc != MPDATA_OK) {
        delete b;
        return rc;
    }
    engine_prepare_graph(b->e);
    *out = b;
    return MPDATA_OK;
}

int mpdata_batch_step(mpdata_batch *b, int32_t nsteps)
{
    if (!b) return MPDATA_EINVAL;
    return engine_step(b->e, nsteps);
}

int mpdata_batch_profile_step(mpdata_batch *b, int64_t *cycles_out, int32_t nseg)
{
    if (!b) return MPDATA_EINVAL;
    Engine &e = b->e;
    if (!cycles_out || nseg != e.nseg)
        return fail_to(e.err, MPDATA_EINVAL, "cycles_out must hold the plan's %d segments", e.nseg);
    long long *ticks = (long long *)(e.ws + e.lay.ticks);
    hipError_t r = launch_one(e, 0, ticks);
    if (r == hipSuccess)
        r = e.dtype == MPDATA_FP32
                ? mpd::launch_copy_back<float>((const mpd::GridDesc<float> *)(e.ws + e.lay.grids), e.ngrids, e.stream)
                : mpd::launch_copy_back<double>((const mpd::GridDesc<double> *)(e.ws + e.lay.grids), e.ngrids, e.stream);
    if (r == hipSuccess)
        r = hipMemcpyAsync(cycles_out, ticks, (size_t)nseg * sizeof(long long), hipMemcpyDeviceToHost,
                           e.stream);
    if (r == hipSuccess) r = hipStreamSynchronize(e.stream);
    if (r != hipSuccess) return fail_to(e.err, MPDATA_EDEVICE, "profile step: %s", hipGetErrorString(r));
    return MPDATA_OK;
}

int mpdata_batch_mass(mpdata_batch *b, int32_t i, double *out)
{
    if (!b) return MPDATA_EINVAL;
    if (!out || i < 0 || i >= b->e.ngrids) return fail_to(b->e.err, MPDATA_EINVAL, "bad grid index or out");
    return engine_mass(b->e, i, out);
}

int mpdata_batch_sync(mpdata_batch *b)
{
    if (!b) return MPDATA_EINVAL;
    hipError_t r = hipStreamSynchronize(b->e.stream);
    return r == hipSuccess ? MPDATA_OK
                           : fail_to(b->e.err, MPDATA_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(r));
}

void mpdata_batch_destroy(mpdata_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->e.stream);
    engine_release(b->e);
    delete b;
}

const char *mpdata_batch_last_error(const mpdata_batch *b) { return b ? b->e.err : g_create_err; }


// -------------------------------------------------------------------- pools

size_t mpdata_pool_workspace_bytes(int32_t max_grids, int32_t max_segments)
{
    if (max_grids < 1 || max_segments < 1) return 0;
    return pool_layout(max_grids, max_segments, 256 * 8).total;
}

int mpdata_pool_create(const mpdata_params *shared, int32_t max_grids, int32_t max_segments,
                       void *workspace, size_t ws_bytes, void *stream, mpdata_pool **out)
{
    g_create_err[0] = 0;
    if (!out) return pool_fail(nullptr, MPDATA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!shared) return pool_fail(nullptr, MPDATA_EINVAL, "shared params is NULL");
    mpdata_params sp = *shared;
    sp.nx = sp.ny = sp.nz = 1;
    sp.iord = 2;
    if (const char *m = check_params(&sp)) return pool_fail(nullptr, MPDATA_EINVAL, "%s", m);
    if (sp.flags & MPDATA_FLAG_TVEL)
        return pool_fail(nullptr, MPDATA_ENOTSUP,
                         "Courant numbers that change in time run on single-grid contexts");
    if (max_grids < 1 || max_segments < 1)
        return pool_fail(nullptr, MPDATA_EINVAL, "max_grids and max_segments must be >= 1");
    if (!workspace || ((uintptr_t)workspace & (kAlign - 1)) != 0)
        return pool_fail(nullptr, MPDATA_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    const size_t need = mpdata_pool_workspace_bytes(max_grids, max_segments);
    if (ws_bytes < need)
        return pool_fail(nullptr, MPDATA_ENOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    mpdata_pool *p = new (std::nothrow) mpdata_pool;
    if (!p) return pool_fail(nullptr, MPDATA_ENOMEM, "host allocation failed");
    Engine &e = p->e;
    e.dtype = sp.dtype;
    e.tile = tile_of(&sp);
    e.iord = 2;
    e.open = sp.bc == MPDATA_BC_OPEN;
    e.nonos = sp.nonos != 0;
    e.variant = variant_of(sp);
    e.eps = sp.eps;
    e.use_graph = !(sp.flags & MPDATA_FLAG_NO_GRAPH);
    e.stream = (hipStream_t)stream;
    e.ws = (char *)workspace;
    e.ngrids = 0;
    e.nwg = 0;
    e.nseg = 0;
    e.err[0] = 0;
    e.params.assign(1, sp);
    const int per = wg_per_cu(e.dtype, e.tile, e.variant);
    const int cus = device_cus();
    if (per < 1 || cus < 1) {
        delete p;
        return pool_fail(nullptr, MPDATA_EDEVICE, "occupancy query failed");
    }
    p->nwg_all = std::min(per * cus, 256 * 8);
    p->max_grids = max_grids;
    p->max_segs = max_segments;
    e.lay = pool_layout(max_grids, max_segments, 256 * 8);
    p->slots.assign(max_grids, mpdata_pool::Slot{false, sp, {}});
    p->dirty = false;
    p->cur_stage = 0;
    p->stage_bytes = align_up((size_t)max_grids * sizeof(mpd::GridDesc<double>)) +
                     align_up((size_t)max_segments * sizeof(mpd::Segment)) +
                     align_up(((size_t)p->nwg_all + 1) * sizeof(int));
    for (auto &st : p->stage) {
        st.host = nullptr;
        st.pending = false;
        st.done = nullptr;
    }
    for (auto &st : p->stage) {
        hipError_t r = hipHostMalloc((void **)&st.host, p->stage_bytes, hipHostMallocDefault);
        if (r == hipSuccess) r = hipEventCreateWithFlags(&st.done, hipEventDisableTiming);
        if (r != hipSuccess) {
            mpdata_pool_destroy(p);
            return pool_fail(nullptr, MPDATA_EDEVICE, "pinned staging: %s", hipGetErrorString(r));
        }
    }
    *out = p;
    return MPDATA_OK;
}

int mpdata_pool_add(mpdata_pool *p, int32_t nx, int32_t ny, int32_t nz, void *psi,
                    void *psi_scratch, const void *u1, const void *u2, const void *u3,
                    const void *h, void *validate_stream, int32_t *slot)
{
    if (!p) return MPDATA_EINVAL;
    if (!slot) return pool_fail(p, MPDATA_EINVAL, "slot is NULL");
    Engine &e = p->e;
    mpdata_params gp = e.params[0];
    gp.nx = nx;
    gp.ny = ny;
    gp.nz = nz;
    if (const char *m = check_params(&gp)) return pool_fail(p, MPDATA_EINVAL, "%s", m);
    if (!psi || !psi_scratch || !u1 || !u2 || !u3 || !h)
        return pool_fail(p, MPDATA_EINVAL, "NULL array pointer");
    if (misaligned(psi) || misaligned(psi_scratch) || misaligned(u1) || misaligned(u2) ||
        misaligned(u3) || misaligned(h))
        return pool_fail(p, MPDATA_EINVAL, "arrays must be 16-byte aligned");
    int free_slot = -1;
    for (int i = 0; i < p->max_grids; ++i)
        if (!p->slots[i].used) {
            free_slot = i;
            break;
        }
    if (free_slot < 0) return pool_fail(p, MPDATA_ENOMEM, "pool full (%d members)", p->max_grids);
    // the checks of mpdata_create, on the caller's stream
    hipStream_t vs = validate_stream ? (hipStream_t)validate_stream : e.stream;
    unsigned int *flags = (unsigned int *)(e.ws + e.lay.flags);
    hipError_t r = hipMemsetAsync(flags, 0, 4 * sizeof(unsigned int), vs);
    const int periodic = gp.bc == MPDATA_BC_PERIODIC;
    if (r == hipSuccess)
        r = e.dtype == MPDATA_FP64
                ? mpd::launch_validate<double>((const double *)h, (const double *)u1,
                                               (const double *)u2, (const double *)u3, nx, ny, nz,
                                               periodic, flags, vs)
                : mpd::launch_validate<float>((const float *)h, (const float *)u1,
                                              (const float *)u2, (const float *)u3, nx, ny, nz,
                                              periodic, flags, vs);
    unsigned int hf[2] = {0, 0};
    if (r == hipSuccess) r = hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, vs);
    if (r == hipSuccess) r = hipStreamSynchronize(vs);
    if (r != hipSuccess) return pool_fail(p, MPDATA_EDEVICE, "validate: %s", hipGetErrorString(r));
    if (hf[0]) return pool_fail(p, MPDATA_EINVAL, "h must be finite and > 0 (%u bad cells)", hf[0]);
    if (hf[1])
        return pool_fail(p, MPDATA_EINVAL,
                         "periodic boundaries need face n == face 0 on every axis (%u differ)", hf[1]);
    mpdata_pool::Slot &s = p->slots[free_slot];
    s.used = true;
    s.p = gp;
    s.g.u1 = (const double *)u1;
    s.g.u2 = (const double *)u2;
    s.g.u3 = (const double *)u3;
    s.g.h = (const double *)h;
    s.g.psi[0] = (double *)psi;
    s.g.psi[1] = (double *)psi_scratch;
    s.g.nx = nx;
    s.g.ny = ny;
    s.g.nz = nz;
    s.g.pad = 0;
    p->dirty = true;
    *slot = free_slot;
    return MPDATA_OK;
}

int mpdata_pool_remove(mpdata_pool *p, int32_t slot)
{
    if (!p) return MPDATA_EINVAL;
    if (slot < 0 || slot >= p->max_grids || !p->slots[slot].used)
        return pool_fail(p, MPDATA_EINVAL, "no member in slot %d", slot);
    p->slots[slot].used = false;
    p->dirty = true;
    return MPDATA_OK;
}

int mpdata_pool_step(mpdata_pool *p, int32_t nsteps)
{
    if (!p) return MPDATA_EINVAL;
    if (nsteps < 0) return pool_fail(p, MPDATA_EINVAL, "nsteps must be >= 0");
    if (p->dirty) {
        const int rc = pool_upload(p);
        if (rc != MPDATA_OK) return rc;
    }
    if (p->e.ngrids == 0 || nsteps == 0) return MPDATA_OK;
    return engine_step(p->e, nsteps);
}

int32_t mpdata_pool_size(const mpdata_pool *p)
{
    if (!p) return -1;
    int n = 0;
    for (const auto &s : p->slots) n += s.used;
    return n;
}

int mpdata_pool_sync(mpdata_pool *p)
{
    if (!p) return MPDATA_EINVAL;
    hipError_t r = hipStreamSynchronize(p->e.stream);
    return r == hipSuccess ? MPDATA_OK
                           : pool_fail(p, MPDATA_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(r));
}

void mpdata_pool_destroy(mpdata_pool *p)
{
    if (!p) return;
    (void)hipStreamSynchronize(p->e.stream);
    engine_release(p->e);
    for (auto &st : p->stage) {
        if (st.done) (void)hipEventDestroy(st.done);
        if (st.host) (void)hipHostFree(st.host);
    }
    delete p;
}

const char *mpdata_pool_last_error(const mpdata_pool *p) { return p ? p->e.err : g_create_err; }

}  // extern "C"
