// Host side of the wave lattice Boltzmann library: the C ABI declared in
// include/lb_wave.h (descriptor checks, workspace layout, compact sound-speed
// tables, surface stencils, launches and read-back).
//
// Method: Castro-Avila et al., "A lattice Boltzmann approach for acoustic
// manipulation" (arXiv 2404.02346).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <climits>
#include <limits>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/lb_wave.h"
#include "lb_kernels.hpp"

using namespace lbw;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(LB_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

constexpr size_t kAlign = 256;
inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

size_t elem_bytes(int storage)
{
    switch (storage) {
    case LB_F64: return 8;
    case LB_F32: return 4;
    default: return 2;
    }
}
size_t compute_bytes(int storage) { return storage == LB_F64 ? 8 : 4; }

inline int wrapi(long v, int n)
{
    long r = v % n;
    return (int)(r < 0 ? r + n : r);
}

// The 3-point kernel printed after eq. InterpolatedFields.
double roma3(double r)
{
    const double a = std::fabs(r);
    if (a <= 0.5) return (1.0 + std::sqrt(1.0 - 3.0 * a * a)) / 3.0;
    if (a <= 1.5) return (5.0 - 3.0 * a - std::sqrt(1.0 - 3.0 * (1.0 - a) * (1.0 - a))) / 6.0;
    return 0.0;
}

// Sound speed of eq. sound_speed_object, read with c = c_p inside.  For
// (r^2 - R^2)/d >= 20 the tanh rounds to 1 and c is exactly c0.
double object_c(const lb_wave_desc &d, double x, double y, double z)
{
    const double dx = x - d.obj_center[0], dy = y - d.obj_center[1];
    const double dz = d.dim == 3 ? z - d.obj_center[2] : 0.0;
    const double u = (dx * dx + dy * dy + dz * dz - d.obj_radius * d.obj_radius) / d.obj_d;
    return d.c0 - 0.5 * (d.c0 - d.obj_cp) * (1.0 - std::tanh(u));
}

constexpr double kTanhSaturate = 20.0;

inline bool finite(double v) { return std::isfinite(v); }

// Box of cells whose sound speed differs from c0 (inclusive lo, extent n).
struct Box {
    int lo[3] = {0, 0, 0};
    int n[3] = {0, 0, 0};
    size_t cells() const { return (size_t)n[0] * n[1] * n[2]; }
};

Box sound_speed_box(const lb_wave_desc &d)
{
    Box b;
    const int nn[3] = {d.nx, d.ny, d.dim == 3 ? d.nz : 1};
    if (d.c_field) {
        int lo[3] = {nn[0], nn[1], nn[2]}, hi[3] = {-1, -1, -1};
        for (int z = 0; z < nn[2]; ++z)
            for (int y = 0; y < nn[1]; ++y)
                for (int x = 0; x < nn[0]; ++x) {
                    const double c = d.c_field[((size_t)z * nn[1] + y) * nn[0] + x];
                    if (c != d.c0) {
                        const int p[3] = {x, y, z};
                        for (int a = 0; a < 3; ++a) {
                            lo[a] = std::min(lo[a], p[a]);
                            hi[a] = std::max(hi[a], p[a]);
                        }
                    }
                }
        if (hi[0] < 0) return b;
        for (int a = 0; a < 3; ++a) {
            b.lo[a] = lo[a];
            b.n[a] = hi[a] - lo[a] + 1;
        }
        return b;
    }
    if (d.obj_cp == d.c0) return b;  // c = c0 exactly everywhere
    const double h = std::sqrt(d.obj_radius * d.obj_radius + kTanhSaturate * d.obj_d);
    for (int a = 0; a < 3; ++a) {
        if (a == 2 && d.dim == 2) {
            b.lo[2] = 0;
            b.n[2] = 1;
            continue;
        }
        long lo = (long)std::floor(d.obj_center[a] - h);
        long hi = (long)std::ceil(d.obj_center[a] + h);
        lo = std::max(lo, 0L);
        hi = std::min(hi, (long)nn[a] - 1);
        if (hi < lo) return Box{};
        b.lo[a] = (int)lo;
        b.n[a] = (int)(hi - lo + 1);
    }
    return b;
}

// 3-point stencil of one surface point: base node by rounding half away from
// zero, nodes base-1, base, base+1 along each axis.
void stencil(const lb_wave_desc &d, const double *P, SurfPt &s, long xn[3])
{
    const int nn[3] = {d.nx, d.ny, d.dim == 3 ? d.nz : 1};
    for (int a = 0; a < 3; ++a) {
        if (a == 2 && d.dim == 2) {
            for (int o = 0; o < 3; ++o) {
                s.bz[o] = 0;
                s.w[6 + o] = (o == 0) ? 1.0 : 0.0;
            }
            continue;
        }
        const long b = std::lround(P[a]);
        for (int o = 0; o < 3; ++o) {
            const long node = b - 1 + o;
            const double w = roma3((double)node - P[a]);
            if (a == 0) {
                xn[o] = node;
                s.bx[o] = (int)node;
                s.w[o] = w;
            } else if (a == 1) {
                s.by[o] = wrapi(node, nn[1]);
                s.w[3 + o] = w;
            } else {
                s.bz[o] = wrapi(node, nn[2]);
                s.w[6 + o] = w;
            }
        }
    }
    s.pad = 0;
}

// Box of the stencil nodes of all surface points.  Along y and z a box that
// would cross the periodic boundary takes the whole extent.
Box measure_box(const lb_wave_desc &d)
{
    Box b;
    if (d.n_surf <= 0) return b;
    const int nn[3] = {d.nx, d.ny, d.dim == 3 ? d.nz : 1};
    long lo[3] = {LONG_MAX, LONG_MAX, LONG_MAX}, hi[3] = {LONG_MIN, LONG_MIN, LONG_MIN};
    for (int k = 0; k < d.n_surf; ++k)
        for (int a = 0; a < d.dim; ++a) {
            const long c = std::lround(d.surf_xyz[3 * k + a]);
            lo[a] = std::min(lo[a], c - 1);
            hi[a] = std::max(hi[a], c + 1);
        }
    for (int a = 0; a < 3; ++a) {
        if (a >= d.dim) {
            b.lo[a] = 0;
            b.n[a] = 1;
        } else if (lo[a] >= 0 && hi[a] < nn[a]) {
            b.lo[a] = (int)lo[a];
            b.n[a] = (int)(hi[a] - lo[a] + 1);
        } else {
            b.lo[a] = 0;
            b.n[a] = nn[a];
        }
    }
    return b;
}

// Stencil nodes relative to the moment box (y, z wrapped first).
void stencil_in_box(const lb_wave_desc &d, const double *P, const Box &mb, SurfPt &s)
{
    SurfPt g;
    long xn[3];
    stencil(d, P, g, xn);
    s = g;
    for (int o = 0; o < 3; ++o) {
        s.bx[o] = g.bx[o] - mb.lo[0];
        s.by[o] = g.by[o] - mb.lo[1];
        s.bz[o] = g.bz[o] - mb.lo[2];
    }
}

int check_one(const lb_wave_desc &d, const lb_wave_desc &d0, int idx)
{
    if (d.dim != 2 && d.dim != 3) return fail(LB_EINVAL, "instance %d: dim must be 2 or 3", idx);
    if (d.dim != d0.dim) return fail(LB_EINVAL, "instance %d: all instances must share dim", idx);
    if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(LB_EINVAL, "instance %d: bad shape", idx);
    if (d.dim == 2 && d.nz != 1) return fail(LB_EINVAL, "instance %d: nz must be 1 in 2D", idx);
    if (d.storage < LB_F64 || d.storage > LB_BF16)
        return fail(LB_EINVAL, "instance %d: bad storage", idx);
    if (d.storage != d0.storage)
        return fail(LB_EINVAL, "instance %d: all instances must share storage", idx);
    if (d.xbc != LB_XBC_DRIVEN && d.xbc != LB_XBC_PERIODIC)
        return fail(LB_EINVAL, "instance %d: bad xbc", idx);
    if (d.xbc == LB_XBC_DRIVEN && d.nx < 3)
        return fail(LB_EINVAL, "instance %d: driven x needs nx >= 3", idx);
    if (!(d.c0 > 0) || !finite(d.c0)) return fail(LB_EINVAL, "instance %d: c0 must be > 0", idx);
    if (!(d.rho0 > 0) || !finite(d.rho0))
        return fail(LB_EINVAL, "instance %d: rho0 must be > 0", idx);
    if (!(d.wall_phi >= 0 && d.wall_phi < 1))
        return fail(LB_EINVAL, "instance %d: wall_phi must lie in [0, 1)", idx);
    if (!finite(d.rho_a) || !finite(d.omega))
        return fail(LB_EINVAL, "instance %d: rho_a and omega must be finite", idx);
    if (d.avg_start < 0 || d.trace_steps < 0)
        return fail(LB_EINVAL, "instance %d: avg_start and trace_steps must be >= 0", idx);
    if (d.src_kind != LB_SRC_SHEET && d.src_kind != LB_SRC_POINT)
        return fail(LB_EINVAL, "instance %d: bad src_kind", idx);
    if (d.src_kind == LB_SRC_POINT) {
        if (d.xbc != LB_XBC_PERIODIC)
            return fail(LB_EINVAL, "instance %d: a point source needs periodic x", idx);
        const int32_t *s = d.src_cell;
        if (s[0] < 0 || s[0] >= d.nx || s[1] < 0 || s[1] >= d.ny || s[2] < 0 || s[2] >= d.nz)
            return fail(LB_EINVAL, "instance %d: source node (%d, %d, %d) outside the lattice",
                        idx, s[0], s[1], s[2]);
    }
    // sizes: rows and wave tasks are indexed with 32-bit integers
    const long pitch = (long)align_up((size_t)d.nx, 64);
    const long rows = (long)d.ny * d.nz;
    if (pitch * rows > (long)INT32_MAX * 8 || rows * ((pitch + 63) / 64) > INT32_MAX / 2)
        return fail(LB_EINVAL, "instance %d: lattice too large", idx);
    // stability of the tau = 1/2 scheme: every c <= 1/sqrt(dim)
    const double cmax_allowed = 1.0 / std::sqrt((double)d.dim) * (1.0 + 1e-12);
    double cmax = d.c0;
    if (d.c_field) {
        const size_t n = (size_t)d.nx * d.ny * d.nz;
        for (size_t i = 0; i < n; ++i) {
            if (!finite(d.c_field[i])) return fail(LB_EINVAL, "instance %d: c_field not finite", idx);
            cmax = std::max(cmax, std::fabs(d.c_field[i]));
        }
    } else {
        if (!finite(d.obj_cp) || !finite(d.obj_radius) || !finite(d.obj_d) ||
            !finite(d.obj_center[0]) || !finite(d.obj_center[1]) || !finite(d.obj_center[2]))
            return fail(LB_EINVAL, "instance %d: object parameters not finite", idx);
        if (d.obj_cp != d.c0 && !(d.obj_d > 0))
            return fail(LB_EINVAL, "instance %d: obj_d must be > 0", idx);
        cmax = std::max(cmax, std::fabs(d.obj_cp));
    }
    if (cmax > cmax_allowed)
        return fail(LB_EUNSTABLE, "instance %d: sound speed %.6g exceeds 1/sqrt(%d)", idx, cmax,
                    d.dim);
    if (d.n_surf < 0) return fail(LB_EINVAL, "instance %d: n_surf < 0", idx);
    if (d.n_surf > 0) {
        if (!d.surf_xyz || !d.surf_normal || !d.surf_area)
            return fail(LB_EINVAL, "instance %d: surface arrays missing", idx);
        const long xlo = d.xbc == LB_XBC_DRIVEN ? 2 : 0;
        const long xhi = d.xbc == LB_XBC_DRIVEN ? d.nx - 2 : d.nx - 1;
        for (int k = 0; k < d.n_surf; ++k) {
            for (int a = 0; a < 3; ++a)
                if (!finite(d.surf_xyz[3 * k + a]) || !finite(d.surf_normal[3 * k + a]))
                    return fail(LB_EINVAL, "instance %d: surface point %d not finite", idx, k);
            if (!finite(d.surf_area[k]))
                return fail(LB_EINVAL, "instance %d: surface area %d not finite", idx, k);
            SurfPt s;
            long xn[3];
            stencil(d, d.surf_xyz + 3 * k, s, xn);
            if (xn[0] < xlo || xn[2] > xhi)
                return fail(LB_EGEOMETRY,
                            "instance %d: stencil of surface point %d spans x = %ld..%ld, "
                            "outside %ld..%ld",
                            idx, k, xn[0], xn[2], xlo, xhi);
        }
    }
    return LB_OK;
}

int check_all(const lb_wave_desc *descs, int n)
{
    if (!descs || n < 1) return fail(LB_EINVAL, "need at least one descriptor");
    long tasks = 0;
    for (int i = 0; i < n; ++i) {
        int st = check_one(descs[i], descs[0], i);
        if (st != LB_OK) return st;
        const long xsegs = (descs[i].nx + 63) / 64;
        tasks += xsegs * descs[i].ny * descs[i].nz;
        // a one-step launch runs 64 threads per task and a 1D grid holds fewer than 2^32
        if (tasks > (long)(UINT32_MAX / 64)) return fail(LB_EINVAL, "batch too large");
    }
    return LB_OK;
}

// Population planes are skewed against each other: the plane stride is the
// plane rounded up to 8 KiB plus 3 KiB, so the seven planes start at seven
// different offsets modulo 8 KiB and their streams spread over the memory
// channels and banks (with power-of-two strides they collide; measured on
// the 16 x 256 x 128 x 128 workload: 5.43 -> 5.90 TB/s).
constexpr int64_t kPlaneRound = 8192, kPlaneSkew = 3072;
int64_t plane_stride(int64_t elems, size_t eb)
{
    const int64_t bytes = (elems * (int64_t)eb + kPlaneRound - 1) / kPlaneRound * kPlaneRound;
    return (bytes + kPlaneSkew) / (int64_t)eb;
}

struct InstPlan {
    Box box;   // sound speed differs from c0
    Box mbox;  // cells whose moments the surface reads
    int pitch;
    int64_t plane;
    int n_chunks;
    size_t off_surf, off_part, off_mom[kNumSlot], off_trace, off_box, off_buf[kNumBuf];
};

struct Layout {
    size_t off_inst, off_acc, off_sbtab, off_tdev, total;
    int n_sb_total;
    std::vector<InstPlan> p;
};

Layout plan(const lb_wave_desc *descs, int n)
{
    Layout L;
    size_t off = 0;
    L.off_inst = off;
    off = align_up(off + sizeof(InstDev) * n);
    L.off_acc = off;
    off = align_up(off + sizeof(AccDev) * n);
    L.n_sb_total = 0;
    for (int i = 0; i < n; ++i) L.n_sb_total += (descs[i].n_surf + 63) / 64;
    L.off_sbtab = off;
    off = align_up(off + sizeof(int32_t) * 2 * (size_t)L.n_sb_total);
    L.off_tdev = off;
    off = align_up(off + 2 * sizeof(int64_t));
    L.p.resize(n);
    for (int i = 0; i < n; ++i) {
        const lb_wave_desc &d = descs[i];
        InstPlan &P = L.p[i];
        const int Q = 2 * d.dim + 1;
        P.box = sound_speed_box(d);
        P.pitch = (int)align_up((size_t)d.nx, 64);
        P.plane = plane_stride((int64_t)P.pitch * d.ny * d.nz, elem_bytes(d.storage));
        P.n_chunks = (d.n_surf + 63) / 64;
        P.mbox = measure_box(d);
        for (int b = 0; b < kNumSlot; ++b) {
            P.off_mom[b] = off;
            off = align_up(off + 4 * compute_bytes(d.storage) * P.mbox.cells());
        }
        P.off_surf = off;
        off = align_up(off + sizeof(SurfPt) * d.n_surf);
        P.off_part = off;
        off = align_up(off + sizeof(double) * kNumSlot * 4 * (size_t)P.n_chunks);
        P.off_trace = off;
        off = align_up(off + sizeof(double) * 3 * (size_t)d.trace_steps);
        P.off_box = off;  // the box, then one c0^2 sentinel for reads from outside it
        off = align_up(off + compute_bytes(d.storage) * (P.box.cells() + 1));
        for (int b = 0; b < kNumBuf; ++b) {
            P.off_buf[b] = off;
            off = align_up(off + elem_bytes(d.storage) * (size_t)P.plane * Q);
        }
    }
    L.total = off;
    return L;
}

double storage_scale(const lb_wave_desc &d)
{
    if (d.storage == LB_F64 || d.storage == LB_F32) return 1.0;
    if (!(std::fabs(d.rho_a) > 0)) return 1.0;
    return std::ldexp(1.0, (int)std::lround(-std::log2(std::fabs(d.rho_a))));
}

// ---- host conversions for state read-back ----
inline float bf16_to_f(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}
inline uint16_t f_to_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
inline double load_host(const uint8_t *p, int storage)
{
    switch (storage) {
    case LB_F64: { double v; std::memcpy(&v, p, 8); return v; }
    case LB_F32: { float v; std::memcpy(&v, p, 4); return v; }
    case LB_F16: { _Float16 v; std::memcpy(&v, p, 2); return (double)(float)v; }
    default: { uint16_t v; std::memcpy(&v, p, 2); return (double)bf16_to_f(v); }
    }
}
inline void store_host(uint8_t *p, int storage, double v)
{
    switch (storage) {
    case LB_F64: std::memcpy(p, &v, 8); break;
    case LB_F32: { float f = (float)v; std::memcpy(p, &f, 4); break; }
    case LB_F16: { _Float16 h = (_Float16)(float)v; std::memcpy(p, &h, 2); break; }
    default: { uint16_t b = f_to_bf16((float)v); std::memcpy(p, &b, 2); break; }
    }
}

}  // namespace

struct lb_wave {
    int n = 0, dim = 0, storage = 0, vx = 1, xm = 0, nt = 0;
    int fused = 1;                    // lattice steps per launch (1 or 2)
    bool fused_ok = false;            // every instance fits the two-step kernel
    int zchunk = 0;                   // planes per chunk of the two-step kernel
    std::vector<int> blk0;            // internal order, size n + 1: two-step blocks
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    Layout lay;
    std::vector<lb_wave_desc> desc;   // user order (host arrays not kept)
    std::vector<int> order;           // internal -> user
    std::vector<int> pos;             // user -> internal
    std::vector<InstDev> hinst;       // internal order
    std::vector<int> task0;           // internal order, size n + 1
    std::vector<SegInfo> segs;        // runs of equal shape, internal order
    std::vector<double> scale;        // user order
    InstDev *d_inst = nullptr;
    AccDev *d_acc = nullptr;          // internal order
    int32_t *d_sb_inst = nullptr;     // surface block table (internal order)
    int32_t *d_sb_chunk = nullptr;
    std::vector<int> sb_first;        // internal order, size n + 1
    bool any_surf = false;
    bool any_point = false;           // some instance has a point source
    int64_t t = 0;                    // lattice steps done
    int64_t meas = 0;                 // steps whose chunk partials exist
    int64_t red = 0;                  // steps reduced into the accumulators
    bool nan_seen = false;
    int64_t *d_t = nullptr;           // device step counter {t, t mod 3}
    int64_t tdev = 0;                 // its value in stream order
    int graph_chunk = 0;              // replay steady steps as captured graphs of this length
    hipStream_t cap_stream = nullptr; // private stream used only for capture
    struct GraphEntry {
        int k, na, n_red, n_sb, nst;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    ~lb_wave()
    {
        for (auto &g : graphs) (void)hipGraphExecDestroy(g.exec);
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
    }
};

namespace {

int64_t steps_of(const lb_wave *h, int internal)
{
    const int64_t ms = h->hinst[internal].max_steps;
    return ms > 0 ? std::min(h->t, ms) : h->t;
}

int active_prefix(const lb_wave *h, int64_t t)
{
    int n = 0;
    while (n < h->n) {
        const int64_t ms = h->hinst[n].max_steps;
        if (ms > 0 && t >= ms) break;
        ++n;
    }
    return n;
}

int prefix_alive(const lb_wave *h, int64_t t)
{
    // instances are sorted by max_steps (longest first): those still alive at t form a prefix
    if (t < 0) return 0;
    return active_prefix(h, t);
}

template <int DIM, typename S, int CPL, int XM, int NT>
void launch_t(const StepArgs &a, int blocks, hipStream_t st)
{
    hipLaunchKernelGGL((step_kernel<DIM, S, CPL, XM, NT>), dim3(blocks), dim3(kStepThreads), 0, st,
                       a);
}

// Variants compiled per storage: 16-bit storage only shifts across lanes (its
// elements are 2 bytes, too small for the offset vector load).
template <int DIM, typename S, int CPL>
void launch_c(const lb_wave *h, const StepArgs &a, int blocks, hipStream_t st)
{
    constexpr bool wide = sizeof(typename StoreTraits<S>::R) >= 4;
    constexpr int XW = wide ? 1 : 0;
    if (h->xm == 1 && wide) {
        switch (h->nt) {
        case 1: launch_t<DIM, S, CPL, XW, 1>(a, blocks, st); break;
        case 2: launch_t<DIM, S, CPL, XW, 2>(a, blocks, st); break;
        default: launch_t<DIM, S, CPL, XW, 0>(a, blocks, st); break;
        }
    } else {
        switch (h->nt) {
        case 1: launch_t<DIM, S, CPL, 0, 1>(a, blocks, st); break;
        case 2: launch_t<DIM, S, CPL, 0, 2>(a, blocks, st); break;
        default: launch_t<DIM, S, CPL, 0, 0>(a, blocks, st); break;
        }
    }
}

template <int DIM, typename S>
void launch_s(const lb_wave *h, const StepArgs &a, int blocks, hipStream_t st)
{
    switch (h->vx) {
    case 2: launch_c<DIM, S, 2>(h, a, blocks, st); break;
    case 4: launch_c<DIM, S, 4>(h, a, blocks, st); break;
    default: launch_c<DIM, S, 1>(h, a, blocks, st); break;
    }
}

void launch(const lb_wave *h, const StepArgs &a, int blocks, hipStream_t st)
{
    if (blocks <= 0) return;
    const bool d2 = h->dim == 2;
    switch (h->storage) {
    case LB_F64: d2 ? launch_s<2, double>(h, a, blocks, st) : launch_s<3, double>(h, a, blocks, st); break;
    case LB_F32: d2 ? launch_s<2, float>(h, a, blocks, st) : launch_s<3, float>(h, a, blocks, st); break;
    case LB_F16:
        d2 ? launch_s<2, _Float16>(h, a, blocks, st) : launch_s<3, _Float16>(h, a, blocks, st);
        break;
    default: d2 ? launch_s<2, bf16>(h, a, blocks, st) : launch_s<3, bf16>(h, a, blocks, st); break;
    }
}

// The point sources of step t (the lattice launches of step t come first in
// stream order); two-step launches never run on a handle with point sources.
template <int DIM, typename S>
void launch_point_s(const lb_wave *h, const StepArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL((point_source_kernel<DIM, S>), dim3((h->n + 63) / 64), dim3(64), 0, st,
                       a.inst, h->n, a.tp, a.dt);
}
void launch_point(const lb_wave *h, const StepArgs &a, hipStream_t st)
{
    const bool d2 = h->dim == 2;
    switch (h->storage) {
    case LB_F64: d2 ? launch_point_s<2, double>(h, a, st) : launch_point_s<3, double>(h, a, st); break;
    case LB_F32: d2 ? launch_point_s<2, float>(h, a, st) : launch_point_s<3, float>(h, a, st); break;
    case LB_F16:
        d2 ? launch_point_s<2, _Float16>(h, a, st) : launch_point_s<3, _Float16>(h, a, st);
        break;
    default: d2 ? launch_point_s<2, bf16>(h, a, st) : launch_point_s<3, bf16>(h, a, st); break;
    }
}

// Rows per row group of the two-step kernel: 4 for FP32; 2 for FP64, whose values take
// twice the registers, and for FP16/BF16, whose 2-byte loads are latency-bound and gain
// more from the extra wavefronts than they lose to the re-read halo rows (measured).
int two_step_rows(int storage) { return storage == LB_F32 ? 4 : 2; }
// Planes per two-step chunk before the halving below.  Longer chunks re-read fewer halo
// planes (two per chunk) and make fewer, longer blocks.  Measured on 16 boxes of
// 256 x 128 x 128, ms per launch with 64 / 32 / 16 planes: FP32 (4-row groups) 0.761 /
// 0.796 / 0.791; FP16 (2-row groups) 0.490 / 0.484 / 0.498.
int two_step_zchunk(int storage) { return storage == LB_F32 ? 64 : 32; }
// Two-step plane chunks shrink (down to kMinZChunk) until a handle has at least as many blocks
// as the chip holds at once: 512 for FP32 (256 CUs, two wavefronts per SIMD), 1024 for the
// others (four).  One sphere of 256 x 128 x 128 in FP32: 2.25 forces/s with 512 blocks of 8
// planes, 2.08 with 1024 of 4.
int64_t two_step_min_blocks(int storage) { return storage == LB_F32 ? 512 : 1024; }
constexpr int kMinZChunk = 4;

// Prefetching the next plane's populations and sound speeds pays where the
// registers allow it (4- and 2-byte storage, two wavefronts per SIMD without
// spills); FP64 loads in place.
template <typename S, int R>
void launch2_t(const lb_wave *h, const StepArgs &a, int blocks, hipStream_t st)
{
    constexpr bool PF = sizeof(typename StoreTraits<S>::R) <= 4;
    if (h->nt == 0)
        hipLaunchKernelGGL((step2_kernel<S, R, 0, PF>), dim3(blocks), dim3(kStepThreads), 0, st, a);
    else
        hipLaunchKernelGGL((step2_kernel<S, R, 1, PF>), dim3(blocks), dim3(kStepThreads), 0, st, a);
}

void launch2(const lb_wave *h, const StepArgs &a, int blocks, hipStream_t st)
{
    if (blocks <= 0) return;
    switch (h->storage) {
    case LB_F64: launch2_t<double, 2>(h, a, blocks, st); break;
    case LB_F32: launch2_t<float, 4>(h, a, blocks, st); break;
    case LB_F16: launch2_t<_Float16, 2>(h, a, blocks, st); break;
    default: launch2_t<bf16, 2>(h, a, blocks, st); break;
    }
}

// Measurement part of the launch whose lattice part starts at t_launch:
// reduce every measured step whose partials an earlier launch wrote
// (steps red .. meas-1), and measure every step whose moments an earlier
// launch stored (steps meas .. t_launch-1).  A launch advances at most two
// steps, so both ranges hold at most two steps and the slots they use
// (step mod 4) differ from those the launch writes.
void plan_measure(lb_wave *h, StepArgs &a, int64_t t_launch)
{
    a.n_red = a.n_sb = a.n_ms = a.n_rs = 0;
    a.meas_off = a.red_off = 0;
    a.sb_inst = h->d_sb_inst;
    a.sb_chunk = h->d_sb_chunk;
    if (!h->any_surf) {
        h->meas = h->red = t_launch;
        return;
    }
    if (h->red < h->meas) {
        a.red_off = (int32_t)(t_launch - h->red);
        a.n_rs = (int32_t)(h->meas - h->red);
        a.n_red = prefix_alive(h, h->red);
        h->red = h->meas;
    }
    if (h->meas < t_launch) {
        a.meas_off = (int32_t)(t_launch - h->meas);
        a.n_ms = (int32_t)(t_launch - h->meas);
        a.n_sb = h->sb_first[prefix_alive(h, h->meas)];
        h->meas = t_launch;
    }
}

// Fill the lattice part of `a` for the steps t .. t+nst-1 (segments of the
// live prefix) and launch, one launch per kMaxSeg segments; the measurement
// blocks ride on the first launch.  nst = 1: wave tasks of step_kernel;
// nst = 2: blocks of step2_kernel (the live prefix is the same for both steps).
void emit_step(const lb_wave *h, StepArgs a, int64_t t, int32_t dt, int nst, hipStream_t st)
{
    const int na = active_prefix(h, t);
    const bool two = nst == 2;
    auto first_of = [&](const SegInfo &sg) { return two ? sg.blk0 : sg.task0; };
    const int n_active = two ? h->blk0[na] : h->task0[na];
    a.dt = dt;
    a.zchunk = h->zchunk;
    size_t s = 0;
    bool first = true;
    do {
        const int base = s < h->segs.size() ? first_of(h->segs[s]) : 0;
        int k = 0;
        for (; k < kMaxSeg && s + k < h->segs.size() && first_of(h->segs[s + k]) < n_active; ++k) {
            a.seg[k] = h->segs[s + k];
            a.seg[k].task0 -= two ? 0 : base;
            a.seg[k].blk0 -= two ? base : 0;
        }
        const int end = (s + k < h->segs.size()) ? std::min(first_of(h->segs[s + k]), n_active)
                                                 : n_active;
        a.nseg = k;
        a.ntask = k > 0 ? end - base : 0;
        if (!first) a.n_red = a.n_sb = a.n_ms = a.n_rs = 0;
        const int meas_blocks = a.n_red + a.n_ms * a.n_sb;
        if (two)
            launch2(h, a, meas_blocks + a.ntask, st);
        else
            launch(h, a, meas_blocks + (a.ntask + 3) / 4, st);
        first = false;
        s += k;
    } while (s < h->segs.size() && first_of(h->segs[s]) < n_active);
    if (h->any_point && !two) launch_point(h, a, st);
}

// Make the device counter equal `t` in stream order if dt would not fit.
void sync_counter(lb_wave *h, int64_t t)
{
    if (t - h->tdev > (1 << 30) || t < h->tdev) {
        hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, h->stream, h->d_t, t);
        h->tdev = t;
    }
}

// nst lattice steps (1 or 2) for every live instance, with the measurement
// of the previous steps folded into the same launch.
int enqueue_step(lb_wave *h, int nst)
{
    const int64_t t = h->t;
    sync_counter(h, t);
    StepArgs a;
    std::memset(&a, 0, sizeof a);
    a.inst = h->d_inst;
    a.tp = h->d_t;
    plan_measure(h, a, t);
    emit_step(h, a, t, (int32_t)(t - h->tdev), nst, h->stream);
    HIP_TRY(hipGetLastError());
    h->t += nst;
    return LB_OK;
}

// Steps t and t+1 can share a two-step launch: no instance stops after t.
bool can_fuse(const lb_wave *h)
{
    return h->fused == 2 && active_prefix(h, h->t) == active_prefix(h, h->t + 1);
}

// Finish the measurement of every completed step (two launches at most).
int flush_measure(lb_wave *h)
{
    while (h->red < h->t) {
        sync_counter(h, h->t);
        StepArgs a;
        std::memset(&a, 0, sizeof a);
        a.inst = h->d_inst;
        a.tp = h->d_t;
        a.dt = (int32_t)(h->t - h->tdev);
        plan_measure(h, a, h->t);
        launch(h, a, a.n_red + a.n_ms * a.n_sb, h->stream);
        HIP_TRY(hipGetLastError());
    }
    return LB_OK;
}

// Steps t .. t+k-1 all launch the same blocks (k / nst launches of nst
// steps): the measurement runs nst and 2 nst steps behind and no instance
// stops inside the window.
bool steady(const lb_wave *h, int64_t k)
{
    const int64_t t = h->t;
    const int nst = h->fused;
    if (k % nst) return false;
    if (h->any_surf && (t < 2 * nst || h->meas != t - nst || h->red != t - 2 * nst)) return false;
    for (const InstDev &I : h->hinst) {
        const int64_t ms = I.max_steps;
        if (ms > 0 && ms > t - 2 * nst && ms < t + k) return false;
    }
    return true;
}

// Replay k steady steps as one captured graph (captured once per launch
// shape on a private stream, launched on the handle's stream).
int replay_steps(lb_wave *h, int k)
{
    const int64_t t = h->t;
    const int nst = h->fused;
    const int na = active_prefix(h, t);
    const int n_red = h->any_surf ? prefix_alive(h, t - 2 * nst) : 0;
    const int n_sb = h->any_surf ? h->sb_first[prefix_alive(h, t - nst)] : 0;
    hipGraphExec_t exec = nullptr;
    for (auto &g : h->graphs)
        if (g.k == k && g.na == na && g.n_red == n_red && g.n_sb == n_sb && g.nst == nst)
            exec = g.exec;
    if (!exec) {
        if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
        StepArgs a;
        std::memset(&a, 0, sizeof a);
        a.inst = h->d_inst;
        a.tp = h->d_t;
        a.meas_off = nst;
        a.n_ms = h->any_surf ? nst : 0;
        a.red_off = 2 * nst;
        a.n_rs = h->any_surf ? nst : 0;
        a.n_red = n_red;
        a.n_sb = n_sb;
        a.sb_inst = h->d_sb_inst;
        a.sb_chunk = h->d_sb_chunk;
        for (int j = 0; j < k; j += nst) emit_step(h, a, t + j, j, nst, h->cap_stream);
        hipLaunchKernelGGL(advance_step_kernel, dim3(1), dim3(64), 0, h->cap_stream, h->d_t,
                           (int64_t)k);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(h->cap_stream, &graph);
        if (e != hipSuccess) return fail(LB_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(LB_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
        h->graphs.push_back({k, na, n_red, n_sb, nst, exec});
    }
    if (h->tdev != t) {
        hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, h->stream, h->d_t, t);
        h->tdev = t;
    }
    HIP_TRY(hipGraphLaunch(exec, h->stream));
    h->t += k;
    h->tdev += k;
    if (h->any_surf) {
        h->meas += k;
        h->red += k;
    } else {
        h->meas = h->red = h->t;
    }
    return LB_OK;
}

void drop_graphs(lb_wave *h)
{
    for (auto &g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    h->graphs.clear();
}

int zero_region(lb_wave *h, size_t off, size_t bytes)
{
    if (bytes == 0) return LB_OK;
    const int64_t n16 = (int64_t)((bytes + 15) / 16);
    const int blocks = (int)std::min<int64_t>((n16 + 255) / 256, 4096);
    hipLaunchKernelGGL(zero_kernel, dim3(blocks), dim3(256), 0, h->stream,
                       reinterpret_cast<uint4 *>(h->ws + off), n16);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

int zero_state(lb_wave *h)
{
    for (int i = 0; i < h->n; ++i) {
        const InstPlan &P = h->lay.p[i];
        const lb_wave_desc &d = h->desc[i];
        const size_t buf = elem_bytes(d.storage) * (size_t)P.plane * (2 * d.dim + 1);
        for (int b = 0; b < kNumBuf; ++b) {
            int st = zero_region(h, P.off_buf[b], buf);
            if (st) return st;
        }
        int st = zero_region(h, P.off_trace, sizeof(double) * 3 * (size_t)d.trace_steps);
        if (st) return st;
    }
    int st = zero_region(h, h->lay.off_acc, sizeof(AccDev) * h->n);
    if (st) return st;
    h->t = h->meas = h->red = 0;
    h->nan_seen = false;
    hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, h->stream, h->d_t, (int64_t)0);
    h->tdev = 0;
    return LB_OK;
}

}  // namespace

// error reporting shared with the MLP translation unit
int lbw_fail_msg(int code, const char *msg) { return fail(code, "%s", msg); }

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *lb_last_error(void) { return g_err.c_str(); }

int lb_wave_check(const lb_wave_desc *descs, int32_t n_inst)
{
    g_err.clear();
    return check_all(descs, n_inst);
}

size_t lb_wave_workspace_bytes(const lb_wave_desc *descs, int32_t n_inst)
{
    if (check_all(descs, n_inst) != LB_OK) return 0;
    return plan(descs, n_inst).total;
}

int lb_wave_create(const lb_wave_desc *descs, int32_t n_inst, void *dev_workspace,
                   size_t workspace_bytes, void *hip_stream, lb_wave **out)
{
    g_err.clear();
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    int st = check_all(descs, n_inst);
    if (st != LB_OK) return st;
    Layout L = plan(descs, n_inst);
    if (!dev_workspace) return fail(LB_ENOMEM, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign)
        return fail(LB_ENOMEM, "workspace must be 256-byte aligned");
    if (workspace_bytes < L.total)
        return fail(LB_ENOMEM, "workspace has %zu bytes, needs %zu", workspace_bytes, L.total);

    lb_wave *h = new lb_wave();
    h->n = n_inst;
    h->dim = descs[0].dim;
    h->storage = descs[0].storage;
    h->ws = static_cast<char *>(dev_workspace);
    h->ws_bytes = workspace_bytes;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->lay = L;
    h->desc.assign(descs, descs + n_inst);
    for (auto &d : h->desc) {  // the host arrays are not kept
        d.c_field = nullptr;
        d.surf_xyz = d.surf_normal = d.surf_area = nullptr;
    }
    h->d_inst = reinterpret_cast<InstDev *>(h->ws + L.off_inst);
    h->d_acc = reinterpret_cast<AccDev *>(h->ws + L.off_acc);
    h->d_sb_inst = reinterpret_cast<int32_t *>(h->ws + L.off_sbtab);
    h->d_sb_chunk = h->d_sb_inst + L.n_sb_total;
    h->d_t = reinterpret_cast<int64_t *>(h->ws + L.off_tdev);
    h->vx = 1;

    // internal order: longest runs first (so the active set is a prefix),
    // equal shapes adjacent (so they share one segment of the launch)
    h->order.resize(n_inst);
    std::iota(h->order.begin(), h->order.end(), 0);
    auto key_steps = [&](int i) {
        return descs[i].max_steps > 0 ? descs[i].max_steps : std::numeric_limits<int64_t>::max();
    };
    std::stable_sort(h->order.begin(), h->order.end(), [&](int a, int b) {
        if (key_steps(a) != key_steps(b)) return key_steps(a) > key_steps(b);
        if (descs[a].nx != descs[b].nx) return descs[a].nx > descs[b].nx;
        if (descs[a].ny != descs[b].ny) return descs[a].ny > descs[b].ny;
        return descs[a].nz > descs[b].nz;
    });
    h->pos.resize(n_inst);
    for (int i = 0; i < n_inst; ++i) h->pos[h->order[i]] = i;

    // per-instance device records, surface stencils, sound-speed boxes
    std::vector<std::vector<uint8_t>> host_blobs;
    std::vector<size_t> blob_off;
    h->hinst.resize(n_inst);
    h->scale.resize(n_inst);
    h->task0.assign(n_inst + 1, 0);
    for (int ii = 0; ii < n_inst; ++ii) {
        const int u = h->order[ii];
        const lb_wave_desc &d = descs[u];
        const InstPlan &P = L.p[u];
        InstDev &I = h->hinst[ii];
        std::memset(&I, 0, sizeof I);
        I.dim = d.dim;
        I.nx = d.nx;
        I.ny = d.ny;
        I.nz = d.nz;
        I.pitch = P.pitch;
        I.xbc = d.xbc;
        I.plane = P.plane;
        for (int b = 0; b < kNumBuf; ++b) I.buf[b] = h->ws + P.off_buf[b];
        I.c0sq = d.c0 * d.c0;
        for (int a = 0; a < 3; ++a) {
            I.bb_lo[a] = P.box.lo[a];
            I.bb_n[a] = P.box.n[a];
        }
        I.c2box = h->ws + P.off_box;
        const double sc = storage_scale(d);
        h->scale[u] = sc;
        I.src_amp = d.rho_a * sc;
        I.omega = d.omega;
        I.wall_phi = d.wall_phi;
        I.max_steps = d.max_steps;
        I.src_point = d.src_kind == LB_SRC_POINT ? 1 : 0;
        for (int a = 0; a < 3; ++a) I.src_pt[a] = I.src_point ? d.src_cell[a] : 0;
        if (I.src_point) h->any_point = true;
        for (int a = 0; a < 3; ++a) {
            I.mb_lo[a] = P.mbox.lo[a];
            I.mb_n[a] = P.mbox.n[a];
        }
        for (int b = 0; b < kNumSlot; ++b) I.mom[b] = h->ws + P.off_mom[b];
        I.n_surf = d.n_surf;
        I.n_chunks = P.n_chunks;
        I.surf = reinterpret_cast<const SurfPt *>(h->ws + P.off_surf);
        I.part = reinterpret_cast<double *>(h->ws + P.off_part);
        I.c0sq_force = d.c0 * d.c0;
        I.force_scale = -1.0 / (d.rho0 * sc * sc);
        I.avg_start = d.avg_start;
        I.acc = h->d_acc + ii;
        I.trace = reinterpret_cast<double *>(h->ws + P.off_trace);
        I.trace_cap = d.trace_steps;
        if (d.n_surf > 0) h->any_surf = true;

        const int xsegs = (d.nx + 63) / 64;
        h->task0[ii + 1] = h->task0[ii] + xsegs * d.ny * d.nz;

        // surface stencils
        if (d.n_surf > 0) {
            std::vector<uint8_t> blob(sizeof(SurfPt) * d.n_surf);
            SurfPt *sp = reinterpret_cast<SurfPt *>(blob.data());
            for (int k = 0; k < d.n_surf; ++k) {
                stencil_in_box(d, d.surf_xyz + 3 * k, P.mbox, sp[k]);
                for (int a = 0; a < 3; ++a) sp[k].nA[a] = d.surf_normal[3 * k + a] * d.surf_area[k];
            }
            host_blobs.push_back(std::move(blob));
            blob_off.push_back(P.off_surf);
        }
        // compact c^2 table in the compute type, followed by the c0^2 sentinel
        {
            const size_t cb = compute_bytes(d.storage);
            std::vector<uint8_t> blob(cb * (P.box.cells() + 1));
            size_t q = 0;
            for (int z = 0; z < P.box.n[2]; ++z)
                for (int y = 0; y < P.box.n[1]; ++y)
                    for (int x = 0; x < P.box.n[0]; ++x, ++q) {
                        const int gx = P.box.lo[0] + x, gy = P.box.lo[1] + y, gz = P.box.lo[2] + z;
                        double c;
                        if (d.c_field)
                            c = d.c_field[((size_t)gz * d.ny + gy) * d.nx + gx];
                        else
                            c = object_c(d, gx, gy, gz);
                        const double c2 = c * c;
                        if (cb == 8) {
                            std::memcpy(blob.data() + 8 * q, &c2, 8);
                        } else {
                            const float f = (float)c2;
                            std::memcpy(blob.data() + 4 * q, &f, 4);
                        }
                    }
            const double s2 = d.c0 * d.c0;  // rounded as the kernels round c0^2
            if (cb == 8) {
                std::memcpy(blob.data() + 8 * q, &s2, 8);
            } else {
                const float f = (float)s2;
                std::memcpy(blob.data() + 4 * q, &f, 4);
            }
            host_blobs.push_back(std::move(blob));
            blob_off.push_back(P.off_box);
        }
    }
    // surface block table in internal order
    std::vector<int32_t> sbtab(2 * (size_t)L.n_sb_total);
    h->sb_first.assign(n_inst + 1, 0);
    for (int ii = 0; ii < n_inst; ++ii) {
        const int nc = L.p[h->order[ii]].n_chunks;
        h->sb_first[ii + 1] = h->sb_first[ii] + nc;
        for (int c = 0; c < nc; ++c) {
            sbtab[h->sb_first[ii] + c] = ii;
            sbtab[L.n_sb_total + h->sb_first[ii] + c] = c;
        }
    }
    if (L.n_sb_total > 0) {
        std::vector<uint8_t> blob(sizeof(int32_t) * sbtab.size());
        std::memcpy(blob.data(), sbtab.data(), blob.size());
        host_blobs.push_back(std::move(blob));
        blob_off.push_back(L.off_sbtab);
    }
    // two-step decomposition: row groups of R rows, 4 / nw groups per block,
    // chunks of zchunk planes: the longest chunk (fewest re-read halo planes)
    // that still fills the chip (two_step_min_blocks)
    {
        const int R = two_step_rows(h->storage);
        auto blocks_for = [&](int zc, std::vector<int> *b0) {
            bool ok = (h->dim == 3);
            if (b0) b0->assign(n_inst + 1, 0);
            int64_t total = 0;
            for (int ii = 0; ii < n_inst; ++ii) {
                const InstDev &I = h->hinst[ii];
                int bpi = 0;
                if (I.xbc == 0) {
                    const int nsx = two_step_strips(I.nx, I.pitch);
                    const int ng = nsx > 1 ? 1 : 4 / (I.pitch / 64);
                    if (I.ny % (R * ng) == 0)
                        bpi = (I.ny / (R * ng)) * ((I.nz + zc - 1) / zc) * nsx;
                }
                if (bpi == 0) ok = false;
                total += bpi;
                if (b0) (*b0)[ii + 1] = (*b0)[ii] + bpi;
            }
            return ok ? total : (int64_t)-1;
        };
        h->zchunk = two_step_zchunk(h->storage);
        const int64_t min_blocks = two_step_min_blocks(h->storage);
        while (h->zchunk > kMinZChunk && blocks_for(h->zchunk, nullptr) >= 0 &&
               blocks_for(h->zchunk, nullptr) < min_blocks)
            h->zchunk /= 2;
        // (blocks_for also sizes blk0, which the segments below read in every case)
        const bool fits = blocks_for(h->zchunk, &h->blk0) >= 0 &&
                          h->blk0[n_inst] < std::numeric_limits<int32_t>::max() / 2;
        h->fused_ok = fits && !h->any_point;
        if (!h->fused_ok) std::fill(h->blk0.begin(), h->blk0.end(), 0);
    }
    // segments: maximal runs of equal shape in internal order
    for (int ii = 0; ii < n_inst; ++ii) {
        const InstDev &I = h->hinst[ii];
        if (ii == 0 || I.nx != h->hinst[ii - 1].nx || I.ny != h->hinst[ii - 1].ny ||
            I.nz != h->hinst[ii - 1].nz) {
            SegInfo sg;
            std::memset(&sg, 0, sizeof sg);
            sg.task0 = h->task0[ii];
            sg.first = ii;
            sg.nx = I.nx;
            sg.ny = I.ny;
            sg.nz = I.nz;
            sg.xsegs = (I.nx + 63) / 64;
            sg.tpi = sg.xsegs * I.ny * I.nz;
            sg.blk0 = h->blk0[ii];
            sg.bpi = h->blk0[ii + 1] - h->blk0[ii];
            sg.nsx = two_step_strips(I.nx, I.pitch);
            if (h->fused_ok) {
                const int ng = sg.nsx > 1 ? 1 : 4 / (I.pitch / 64);
                sg.nyb = I.ny / (two_step_rows(h->storage) * ng);
            }
            h->segs.push_back(sg);
        }
    }

    auto cleanup = [&](int code) {
        delete h;
        return code;
    };
    hipError_t e = hipMemcpyAsync(h->ws + L.off_inst, h->hinst.data(), sizeof(InstDev) * n_inst,
                                  hipMemcpyHostToDevice, h->stream);
    for (size_t b = 0; b < host_blobs.size() && e == hipSuccess; ++b)
        e = hipMemcpyAsync(h->ws + blob_off[b], host_blobs[b].data(), host_blobs[b].size(),
                           hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) return cleanup(fail(LB_EDEVICE, "upload failed: %s", hipGetErrorString(e)));
    st = zero_state(h);
    if (st != LB_OK) return cleanup(st);
    e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess)
        return cleanup(fail(LB_EDEVICE, "create: %s", hipGetErrorString(e)));
    *out = h;
    return LB_OK;
}

int lb_wave_step_n(lb_wave *h, int64_t n_steps)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (n_steps < 0) return fail(LB_EINVAL, "n_steps < 0");
    if (h->nan_seen) return fail(LB_ENAN, "a previous force was not finite");
    int64_t left = n_steps;
    while (left > 0) {
        const int k = h->graph_chunk;
        int st;
        if (k >= 2 && left >= k && steady(h, k)) {
            st = replay_steps(h, k);
            left -= k;
        } else if (left >= 2 && can_fuse(h)) {
            st = enqueue_step(h, 2);
            left -= 2;
        } else {
            st = enqueue_step(h, 1);
            left -= 1;
        }
        if (st != LB_OK) return st;
    }
    return flush_measure(h);
}

int lb_wave_set_steps_per_launch(lb_wave *h, int32_t k)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (k != 1 && k != 2) return fail(LB_EINVAL, "steps per launch must be 1 or 2");
    if (k == 2 && !h->fused_ok)
        return fail(LB_EINVAL, "two steps per launch need 3D instances with driven x sheets "
                               "and ny a multiple of the row block");
    if (k != h->fused) drop_graphs(h);
    h->fused = k;
    return LB_OK;
}

int lb_wave_get_steps_per_launch(const lb_wave *h, int32_t *k)
{
    if (!h || !k) return fail(LB_EINVAL, "NULL argument");
    *k = h->fused;
    return LB_OK;
}

int lb_wave_set_graph(lb_wave *h, int32_t chunk)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (chunk < 0 || chunk == 1 || chunk > 4096) return fail(LB_EINVAL, "chunk must be 0 or 2..4096");
    if (chunk != h->graph_chunk) drop_graphs(h);
    h->graph_chunk = chunk;
    return LB_OK;
}

int lb_surface_force(lb_wave *h, double *F_avg, int64_t *n_accum)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (!F_avg) return fail(LB_EINVAL, "F_avg is NULL");
    std::vector<AccDev> acc(h->n);
    HIP_TRY(hipMemcpyAsync(acc.data(), h->d_acc, sizeof(AccDev) * h->n, hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    int st = LB_OK;
    for (int u = 0; u < h->n; ++u) {
        const AccDev &A = acc[h->pos[u]];
        if (n_accum) n_accum[u] = A.n;
        for (int a = 0; a < 3; ++a) F_avg[3 * u + a] = A.n > 0 ? A.sum[a] / (double)A.n : 0.0;
        if (A.nan) {
            h->nan_seen = true;
            st = fail(LB_ENAN, "instance %d: non-finite force", u);
        } else if (A.n == 0 && st == LB_OK) {
            st = fail(LB_EEMPTY, "instance %d: no step accumulated", u);
        }
    }
    return st;
}

int lb_wave_destroy(lb_wave *h)
{
    delete h;
    return LB_OK;
}

int lb_wave_steps_done(const lb_wave *h, int64_t *t)
{
    if (!h || !t) return fail(LB_EINVAL, "NULL argument");
    *t = h->t;
    return LB_OK;
}

int lb_wave_reset(lb_wave *h)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    return zero_state(h);
}

int lb_wave_state_view(const lb_wave *h, int32_t inst, lb_state_view *v)
{
    if (!h || !v) return fail(LB_EINVAL, "NULL argument");
    if (inst < 0 || inst >= h->n) return fail(LB_EINVAL, "instance out of range");
    const int ii = h->pos[inst];
    const InstPlan &P = h->lay.p[inst];
    v->offset_bytes = P.off_buf[buf_of(steps_of(h, ii))];
    v->plane_bytes = elem_bytes(h->storage) * (size_t)P.plane;
    v->pitch = P.pitch;
    v->elem_bytes = (int32_t)elem_bytes(h->storage);
    v->scale = h->scale[inst];
    return LB_OK;
}

int lb_wave_get_state(lb_wave *h, int32_t inst, double *host_fnew)
{
    if (!h || !host_fnew) return fail(LB_EINVAL, "NULL argument");
    if (inst < 0 || inst >= h->n) return fail(LB_EINVAL, "instance out of range");
    lb_state_view v;
    int st = lb_wave_state_view(h, inst, &v);
    if (st) return st;
    const lb_wave_desc &d = h->desc[inst];
    const int Q = 2 * d.dim + 1;
    std::vector<uint8_t> raw(v.plane_bytes * Q);
    HIP_TRY(hipMemcpyAsync(raw.data(), h->ws + v.offset_bytes, raw.size(), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const double inv = 1.0 / v.scale;
    size_t c = 0;
    for (int z = 0; z < d.nz; ++z)
        for (int y = 0; y < d.ny; ++y)
            for (int x = 0; x < d.nx; ++x, ++c) {
                const size_t e = ((size_t)z * d.ny + y) * v.pitch + x;
                for (int i = 0; i < Q; ++i)
                    host_fnew[c * Q + i] =
                        load_host(raw.data() + i * v.plane_bytes + e * v.elem_bytes, h->storage) * inv;
            }
    return LB_OK;
}

int lb_wave_set_state(lb_wave *h, int32_t inst, const double *host_fnew)
{
    if (!h || !host_fnew) return fail(LB_EINVAL, "NULL argument");
    if (inst < 0 || inst >= h->n) return fail(LB_EINVAL, "instance out of range");
    lb_state_view v;
    int st = lb_wave_state_view(h, inst, &v);
    if (st) return st;
    const lb_wave_desc &d = h->desc[inst];
    const int Q = 2 * d.dim + 1;
    std::vector<uint8_t> raw(v.plane_bytes * Q, 0);
    size_t c = 0;
    for (int z = 0; z < d.nz; ++z)
        for (int y = 0; y < d.ny; ++y)
            for (int x = 0; x < d.nx; ++x, ++c) {
                const size_t e = ((size_t)z * d.ny + y) * v.pitch + x;
                for (int i = 0; i < Q; ++i)
                    store_host(raw.data() + i * v.plane_bytes + e * v.elem_bytes, h->storage,
                               host_fnew[c * Q + i] * v.scale);
            }
    HIP_TRY(hipMemcpyAsync(h->ws + v.offset_bytes, raw.data(), raw.size(), hipMemcpyHostToDevice,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_wave_force_trace(lb_wave *h, int32_t inst, double *host_F, int64_t n)
{
    if (!h || !host_F) return fail(LB_EINVAL, "NULL argument");
    if (inst < 0 || inst >= h->n) return fail(LB_EINVAL, "instance out of range");
    if (n < 0 || n > h->desc[inst].trace_steps)
        return fail(LB_EINVAL, "n exceeds the trace capacity");
    if (n == 0) return LB_OK;
    HIP_TRY(hipMemcpyAsync(host_F, h->ws + h->lay.p[inst].off_trace, sizeof(double) * 3 * n,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_wave_probe_rho(lb_wave *h, int32_t inst, const int64_t *dev_cells, int32_t n_cells,
                      double *dev_out)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (inst < 0 || inst >= h->n) return fail(LB_EINVAL, "instance out of range");
    if (n_cells < 0 || (n_cells > 0 && (!dev_cells || !dev_out)))
        return fail(LB_EINVAL, "probe: bad arguments");
    if (n_cells == 0) return LB_OK;
    const int ii = h->pos[inst];
    const InstPlan &P = h->lay.p[inst];
    const lb_wave_desc &d = h->desc[inst];
    const void *buf = h->ws + P.off_buf[buf_of(steps_of(h, ii))];
    const int64_t ncell = (int64_t)d.nx * d.ny * (d.dim == 3 ? d.nz : 1);
    const int Q = 2 * d.dim + 1;
    const dim3 grid((unsigned)((n_cells + 255) / 256)), blk(256);
    switch (h->storage) {
    case LB_F64:
        hipLaunchKernelGGL(probe_rho_kernel<double>, grid, blk, 0, h->stream, buf, P.plane, Q,
                           d.nx, ncell, P.pitch, dev_cells, n_cells, h->scale[inst], dev_out);
        break;
    case LB_F32:
        hipLaunchKernelGGL(probe_rho_kernel<float>, grid, blk, 0, h->stream, buf, P.plane, Q,
                           d.nx, ncell, P.pitch, dev_cells, n_cells, h->scale[inst], dev_out);
        break;
    case LB_F16:
        hipLaunchKernelGGL(probe_rho_kernel<_Float16>, grid, blk, 0, h->stream, buf, P.plane, Q,
                           d.nx, ncell, P.pitch, dev_cells, n_cells, h->scale[inst], dev_out);
        break;
    default:
        hipLaunchKernelGGL(probe_rho_kernel<bf16>, grid, blk, 0, h->stream, buf, P.plane, Q,
                           d.nx, ncell, P.pitch, dev_cells, n_cells, h->scale[inst], dev_out);
        break;
    }
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

int lb_wave_set_variant(lb_wave *h, int32_t cells_per_lane, int32_t x_mode, int32_t nontemporal)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (cells_per_lane != 1 && cells_per_lane != 2 && cells_per_lane != 4)
        return fail(LB_EINVAL, "cells_per_lane must be 1, 2 or 4");
    if (x_mode != 0 && x_mode != 1) return fail(LB_EINVAL, "x_mode must be 0 or 1");
    if (x_mode == 1 && elem_bytes(h->storage) < 4)
        return fail(LB_EINVAL, "x_mode 1 needs 4- or 8-byte storage");
    if (nontemporal < 0 || nontemporal > 2) return fail(LB_EINVAL, "nontemporal must be 0, 1 or 2");
    // the task table and any captured sequence depend on the variant
    drop_graphs(h);
    h->vx = cells_per_lane;
    h->xm = x_mode;
    h->nt = nontemporal;
    const int w = 64 * cells_per_lane;
    for (int ii = 0; ii < h->n; ++ii) {
        const InstDev &I = h->hinst[ii];
        h->task0[ii + 1] = h->task0[ii] + ((I.nx + w - 1) / w) * I.ny * I.nz;
    }
    for (auto &sg : h->segs) {
        sg.task0 = h->task0[sg.first];
        sg.xsegs = (sg.nx + w - 1) / w;
        sg.tpi = sg.xsegs * sg.ny * sg.nz;
    }
    return LB_OK;
}

int lb_wave_get_variant(const lb_wave *h, int32_t *cells_per_lane, int32_t *x_mode,
                        int32_t *nontemporal)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (cells_per_lane) *cells_per_lane = h->vx;
    if (x_mode) *x_mode = h->xm;
    if (nontemporal) *nontemporal = h->nt;
    return LB_OK;
}

int lb_wave_set_tile(lb_wave *h, int32_t cells_per_lane)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    return lb_wave_set_variant(h, cells_per_lane, h->xm, h->nt);
}

int lb_wave_get_tile(const lb_wave *h, int32_t *cells_per_lane)
{
    if (!h || !cells_per_lane) return fail(LB_EINVAL, "NULL argument");
    *cells_per_lane = h->vx;
    return LB_OK;
}

int lb_wave_autotune(lb_wave *h, int32_t n_trial, double *best_ms)
{
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    if (n_trial < 1) return fail(LB_EINVAL, "n_trial must be >= 1");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best = 1e300;
    int bv[4] = {1, 0, 0, 1};  // cells per lane, x mode, nontemporal, steps per launch
    const int xm_max = elem_bytes(h->storage) >= 4 ? 1 : 0;
    const int trial = n_trial + (n_trial & 1);  // even, so two-step launches cover it
    auto time_it = [&](double *per) -> int {
        int st = lb_wave_step_n(h, 2);  // warm-up
        if (st) return st;
        HIP_TRY(hipEventRecord(e0, h->stream));
        st = lb_wave_step_n(h, trial);
        if (st) return st;
        HIP_TRY(hipEventRecord(e1, h->stream));
        HIP_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
        *per = ms / trial;
        return LB_OK;
    };
    std::vector<std::array<int, 4>> cand;
    for (int cpl : {1, 2, 4})
        for (int xm = 0; xm <= xm_max; ++xm)
            for (int nt = 0; nt <= 2; ++nt) cand.push_back({cpl, xm, nt, 1});
    if (h->fused_ok)
        for (int nt = 0; nt <= 1; ++nt) cand.push_back({1, xm_max, nt, 2});
    for (const auto &c : cand) {
        int st = lb_wave_set_steps_per_launch(h, c[3]);
        if (st) return st;
        st = lb_wave_set_variant(h, c[0], c[1], c[2]);
        if (st) return st;
        double per = 0.0;
        st = time_it(&per);
        if (st) return st;
        if (per < best) {
            best = per;
            for (int i = 0; i < 4; ++i) bv[i] = c[i];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int st = lb_wave_set_steps_per_launch(h, bv[3]);
    if (st) return st;
    st = lb_wave_set_variant(h, bv[0], bv[1], bv[2]);
    if (st) return st;
    if (best_ms) *best_ms = best;
    st = zero_state(h);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LB_OK;
}

int lb_stream_copy(const void *dev_src, void *dev_dst, size_t bytes, void *hip_stream)
{
    if (!dev_src || !dev_dst) return fail(LB_EINVAL, "NULL pointer");
    if (bytes % 16 || reinterpret_cast<uintptr_t>(dev_src) % 16 ||
        reinterpret_cast<uintptr_t>(dev_dst) % 16)
        return fail(LB_EINVAL, "pointers and size must be multiples of 16 bytes");
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return LB_OK;
    constexpr int UNR = 4;
    const int64_t blocks = (n16 + 256 * UNR - 1) / (256 * UNR);
    if (blocks > INT32_MAX) return fail(LB_EINVAL, "copy too large");
    // non-temporal loads and stores: the fastest plain copy measured on this chip (6.2 TB/s
    // against 5.75 with cached accesses, at 1.75 GiB each way)
    hipLaunchKernelGGL((copy_kernel<UNR, true>), dim3((unsigned)blocks), dim3(256), 0,
                       static_cast<hipStream_t>(hip_stream), static_cast<const word16 *>(dev_src),
                       static_cast<word16 *>(dev_dst), n16);
    HIP_TRY(hipGetLastError());
    return LB_OK;
}

size_t lb_cavity_workspace_bytes(int32_t nx)
{
    if (nx < 16 || nx > kCavMaxNx) return 0;
    return align_up(sizeof(double) * 2 * (size_t)nx);
}

}  // extern "C"

// The lock-in sums of lb_cavity_calibrate_noalloc live in a file-scope device array, one
// copy per GPU, held until the process ends: 2 kCavMaxNx doubles (32 KiB).  Host code uses
// the address hipGetSymbolAddress returns for the current device, never the array's name.
static __device__ __align__(256) double scratch[2 * kCavMaxNx];

namespace {

// Argument checks shared by both calibration entry points; on success m_out and k_out receive
// the fit window in steps and the lattice wavenumber, n_total_out the run length.
int cavity_check(int32_t nx, double c0, double omega, double wall_phi, int32_t n_periods,
                 int32_t n_fit, const double *out, int64_t *n_total_out, int64_t *m_out,
                 double *k_out)
{
    g_err.clear();
    if (!out) return fail(LB_EINVAL, "out is NULL");
    if (nx < 16 || nx > kCavMaxNx) return fail(LB_EINVAL, "nx must lie in [16, %d]", kCavMaxNx);
    if (!(c0 > 0) || c0 > 1.0) return fail(LB_EUNSTABLE, "c0 must lie in (0, 1]");
    if (!(omega > 0) || omega >= M_PI) return fail(LB_EINVAL, "omega must lie in (0, pi)");
    if (!(wall_phi >= 0 && wall_phi < 1)) return fail(LB_EINVAL, "wall_phi must lie in [0, 1)");
    if (n_fit < 1 || n_periods < n_fit) return fail(LB_EINVAL, "need 1 <= n_fit <= n_periods");
    const double cosk = 1.0 - (1.0 - std::cos(omega)) / (c0 * c0);
    if (!(cosk > -1.0 && cosk < 1.0)) return fail(LB_EINVAL, "omega has no lattice wavenumber");
    const double period = 2.0 * M_PI / omega;
    *n_total_out = (int64_t)std::llround(n_periods * period);
    *m_out = (int64_t)std::llround(n_fit * period);
    *k_out = std::acos(cosk);
    return LB_OK;
}

// The fit of the cavity's lock-in sums (host array of 2 nx doubles: sum rho cos wt, then
// sum rho sin wt over the last m steps), into out[0..5] and optionally host_P.
int cavity_fit(int32_t nx, int64_t m, double k, const double *lock, double *out, double *host_P)
{
    // complex amplitude P = (2/m) sum rho e^{-i w t}
    auto re = [&](int x) { return 2.0 / (double)m * lock[x]; };
    auto im = [&](int x) { return -2.0 / (double)m * lock[nx + x]; };
    if (host_P)
        for (int x = 0; x < nx; ++x) {
            host_P[2 * x] = re(x);
            host_P[2 * x + 1] = im(x);
        }
    // least squares |P|^2 = a + b cos 2kx + c sin 2kx over 2 <= x <= nx-3
    double M[3][4] = {{0}};
    for (int x = 2; x <= nx - 3; ++x) {
        const double row[3] = {1.0, std::cos(2 * k * x), std::sin(2 * k * x)};
        const double y = re(x) * re(x) + im(x) * im(x);
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) M[i][j] += row[i] * row[j];
            M[i][3] += row[i] * y;
        }
    }
    for (int c = 0; c < 3; ++c) {  // Gaussian elimination with partial pivoting
        int p = c;
        for (int r = c + 1; r < 3; ++r)
            if (std::fabs(M[r][c]) > std::fabs(M[p][c])) p = r;
        for (int j = 0; j < 4; ++j) std::swap(M[c][j], M[p][j]);
        if (M[c][c] == 0.0) return fail(LB_EINVAL, "degenerate fit");
        for (int r = 0; r < 3; ++r) {
            if (r == c) continue;
            const double f = M[r][c] / M[c][c];
            for (int j = c; j < 4; ++j) M[r][j] -= f * M[c][j];
        }
    }
    const double a = M[0][3] / M[0][0], b = M[1][3] / M[1][1], c = M[2][3] / M[2][2];
    const double A = std::sqrt(a + std::hypot(b, c));
    const double x0 = std::atan2(c, b) / (2.0 * k);
    const double spacing = M_PI / k;
    const double centre = 0.5 * (nx - 1);
    const double xm = x0 + std::floor((centre - x0) / spacing) * spacing;
    out[0] = A;
    out[1] = xm;
    out[2] = k;
    out[3] = a;
    out[4] = b;
    out[5] = c;
    return LB_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

// the scratch array of the current device (looked up on the device's first call)
int cavity_scratch(double **ptr)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LB_EDEVICE, "device index %d unsupported", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LB_EDEVICE, "scratch address: %s", hipGetErrorString(e));
        g_scratch[dev] = static_cast<double *>(p);
    }
    *ptr = g_scratch[dev];
    return LB_OK;
}

}  // namespace

extern "C" {

int lb_cavity_calibrate(int32_t nx, double c0, double omega, double rho_a, double wall_phi,
                        int32_t n_periods, int32_t n_fit, void *dev_workspace,
                        size_t workspace_bytes, void *hip_stream, double *out, double *host_P)
{
    int64_t n_total = 0, m = 0;
    double k = 0.0;
    int st = cavity_check(nx, c0, omega, wall_phi, n_periods, n_fit, out, &n_total, &m, &k);
    if (st) return st;
    if (!dev_workspace || workspace_bytes < lb_cavity_workspace_bytes(nx))
        return fail(LB_ENOMEM, "workspace too small");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    double *d_lock = static_cast<double *>(dev_workspace);
    hipLaunchKernelGGL(cavity_kernel, dim3(1), dim3(kCavThreads), 0, s, nx, c0 * c0, omega,
                       rho_a, wall_phi, n_total, m, d_lock);
    HIP_TRY(hipGetLastError());
    std::vector<double> lock(2 * (size_t)nx);
    HIP_TRY(hipMemcpyAsync(lock.data(), d_lock, sizeof(double) * 2 * nx, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return cavity_fit(nx, m, k, lock.data(), out, host_P);
}

int lb_cavity_calibrate_noalloc(int32_t nx, double c0, double omega, double rho_a,
                                double wall_phi, int32_t n_periods, int32_t n_fit,
                                void *hip_stream, double *out, double *host_P)
{
    int64_t n_total = 0, m = 0;
    double k = 0.0;
    int st = cavity_check(nx, c0, omega, wall_phi, n_periods, n_fit, out, &n_total, &m, &k);
    if (st) return st;
    double *d_lock = nullptr;
    if ((st = cavity_scratch(&d_lock))) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // the kernel writes every one of the 2 nx sums, so nothing needs clearing first
    hipLaunchKernelGGL(cavity_kernel, dim3(1), dim3(kCavThreads), 0, s, nx, c0 * c0, omega,
                       rho_a, wall_phi, n_total, m, d_lock);
    HIP_TRY(hipGetLastError());
    double lock[2 * kCavMaxNx];  // host copy on the stack (no heap allocation)
    HIP_TRY(hipMemcpyAsync(lock, d_lock, sizeof(double) * 2 * nx, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return cavity_fit(nx, m, k, lock, out, host_P);
}

}  // extern "C"
