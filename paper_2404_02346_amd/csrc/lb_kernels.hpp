// Device code of the wave lattice Boltzmann library (gfx950).
//
// Method: Castro-Avila et al., "A lattice Boltzmann approach for acoustic
// manipulation" (arXiv 2404.02346), Sec. "Lattice-Boltzmann for acoustics"
// and Sec. "Wave-particle interaction and interpolation".
//
// Population storage is structure-of-arrays: plane i (velocity i) holds the
// cells row by row, x fastest, rows `pitch` elements apart (pitch is a
// multiple of 64 elements, so every row starts on a 256-byte boundary for
// 4-byte storage).  Three state buffers rotate: the state entering step t
// (f^new of step t-1) lives in buffer t mod 3, so a launch that advances one
// step (t -> t+1) or two steps (t -> t+2) always writes a buffer it does not
// read.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbw {

constexpr int kMaxSeg = 8;          // same-shape instance runs handled by one launch
constexpr int kStepThreads = 256;   // 4 wavefronts of 64 lanes

// ---------------------------------------------------------------------------
// Storage types: raw element R, compute type C
// ---------------------------------------------------------------------------
struct bf16 {  // tag type for bfloat16 storage (raw bits in uint16_t)
};

template <typename S> struct StoreTraits;
template <> struct StoreTraits<double> {
    using R = double;
    using C = double;
    __device__ static inline C to_c(R v) { return v; }
    __device__ static inline R to_r(C v) { return v; }
};
template <> struct StoreTraits<float> {
    using R = float;
    using C = float;
    __device__ static inline C to_c(R v) { return v; }
    __device__ static inline R to_r(C v) { return v; }
};
template <> struct StoreTraits<_Float16> {
    using R = _Float16;
    using C = float;
    __device__ static inline C to_c(R v) { return (float)v; }
    __device__ static inline R to_r(C v) { return (_Float16)v; }
};
template <> struct StoreTraits<bf16> {
    using R = uint16_t;
    using C = float;
    __device__ static inline C to_c(R v) { return __uint_as_float(((uint32_t)v) << 16); }
    __device__ static inline R to_r(C v) {
        // round to nearest, ties to even
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        return (R)(u >> 16);
    }
};

template <typename R, int N> struct VecT {
    using type = R __attribute__((ext_vector_type(N)));
};
template <typename R> struct VecT<R, 1> {
    using type = R;
};

// Pointers into global memory (address space 1): loads and stores through
// them take a uniform 64-bit base in scalar registers plus a 32-bit lane
// offset, instead of flat accesses with per-lane 64-bit addresses.
template <typename T> using gptr = T __attribute__((address_space(1))) *;
template <typename T> __device__ inline gptr<T> to_global(void *p) { return (gptr<T>)p; }
template <typename T> __device__ inline gptr<const T> to_global(const void *p)
{
    return (gptr<const T>)p;
}

// base + i elements with a 32-bit byte offset (i * sizeof(T) < 2^32 for any
// row offset here), so the access can use a scalar base and a 32-bit offset.
template <typename T> __device__ inline gptr<const T> at(gptr<const T> base, uint32_t i)
{
    return (gptr<const T>)((gptr<const char>)base + i * (uint32_t)sizeof(T));
}
template <typename T> __device__ inline gptr<T> at(gptr<T> base, uint32_t i)
{
    return (gptr<T>)((gptr<char>)base + i * (uint32_t)sizeof(T));
}

// The per-instance records do not change during a launch: reading them
// through the constant address space lets them live in scalar registers.
template <typename T> using cptr = const T __attribute__((address_space(4))) *;
template <typename T> __device__ inline cptr<T> to_const(const T *p) { return (cptr<T>)p; }

template <typename V, bool NT> __device__ inline V vload(gptr<const V> p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename V, bool NT> __device__ inline void vstore(gptr<V> p, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
template <typename V, bool NT> __device__ inline V vload(const V *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <typename V, bool NT> __device__ inline void vstore(V *p, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
template <typename R, int N> __device__ inline R vget(const typename VecT<R, N>::type &v, int c)
{
    if constexpr (N == 1) return v;
    else return v[c];
}
template <typename R, int N> __device__ inline void vset(typename VecT<R, N>::type &v, int c, R x)
{
    if constexpr (N == 1) v = x;
    else v[c] = x;
}

// ---------------------------------------------------------------------------
// Per-instance data (lives in the workspace)
// ---------------------------------------------------------------------------
struct SurfPt {
    int32_t bx[3], by[3], bz[3];  // stencil nodes in moment-box coordinates
    int32_t pad;
    double w[9];                  // 1D kernel weights: wx[0..2], wy[0..2], wz[0..2]
    double nA[3];                 // outward normal times element size
};

struct AccDev {
    double sum[3];
    int64_t n;
    int32_t nan;
    int32_t pad;
};

constexpr int kNumBuf = 3;   // state buffers, indexed by step mod 3
constexpr int kNumSlot = 4;  // moment boxes and partial sums, indexed by step mod 4

__host__ __device__ inline int buf_of(int64_t t) { return (int)(t % kNumBuf); }
__host__ __device__ inline int slot_of(int64_t t) { return (int)(t & (kNumSlot - 1)); }

struct InstDev {
    int32_t dim, nx, ny, nz;
    int32_t pitch, xbc;
    int64_t plane;           // elements per population plane
    void *buf[kNumBuf];      // state buffers (plane 0)
    double c0sq;             // fluid c0^2 (outside the box)
    int32_t bb_lo[3];        // sound-speed box origin
    int32_t bb_n[3];         // sound-speed box extent (0 -> no box)
    const void *c2box;       // c^2 over the box in the compute type, x fastest, then c0^2
    double src_amp;          // rho_a times the storage scale
    double omega, wall_phi;
    int64_t max_steps;       // frozen for t >= max_steps
    int32_t src_pt[3];       // point-source node (when src_point)
    int32_t src_point;       // 1: the node src_pt is imposed after every step
    // measurement
    int32_t mb_lo[3];        // moment box origin (cells whose rho, J the surface reads)
    int32_t mb_n[3];         // moment box extent (0 -> no measurement)
    void *mom[kNumSlot];     // moment boxes (rho, Jx, Jy, Jz per cell, compute type) by step mod 4
    int32_t n_surf, n_chunks;  // surface elements, 64-element chunks
    const SurfPt *surf;
    double *part;            // 4 x n_chunks x 4 per-chunk flux sums by step mod 4
    double c0sq_force;       // c0^2 in the surface integral
    double force_scale;      // -1 / (rho0 * scale^2)
    int64_t avg_start;
    AccDev *acc;
    double *trace;           // trace_cap x 3
    int64_t trace_cap;
};

struct SegInfo {
    int32_t task0;      // first wave task of the run (one-step launch)
    int32_t first;      // first (internal) instance of the run
    int32_t nx, ny, nz; // shape shared by the run
    int32_t xsegs;      // wave tasks per row
    int32_t tpi;        // wave tasks per instance
    int32_t pad;
    int32_t blk0;       // first block of the run (two-step launch)
    int32_t bpi;        // blocks per instance (two-step launch)
    int32_t nyb;        // row blocks per instance (two-step launch)
    int32_t nsx;        // x strips per row (two-step launch; 1: the row fits one block)
};

// One launch = [reducer blocks][surface blocks][lattice blocks] (the
// two-step kernel puts its lattice blocks first), a three-stage pipeline
// over consecutive steps:
//  * lattice blocks advance steps t .. t+nst-1 (nst = 1 or 2) and store
//    rho1, J1 of each f(s) in the moment box of slot s mod 4;
//  * surface blocks interpolate F(s) for the n_ms steps s = t - meas_off ..
//    that earlier launches advanced, from their moment boxes, and write one
//    partial sum per 64 elements into slot s mod 4;
//  * reducer blocks sum the partials of the n_rs steps t - red_off .. (in
//    step order, one block per instance) in a fixed order, scale, trace and
//    accumulate.
// Every stage reads what an earlier launch wrote, and the slots written and
// read by one launch differ mod 4, so no stage waits on another inside a
// launch.  The lattice step of a launch is t = *tp + dt: the counter lives
// in device memory so that a captured sequence of launches can be replayed
// at any t.
struct StepArgs {
    const InstDev *inst;
    const int64_t *tp;        // device step counter: {t, t mod 3}
    int32_t dt;               // offset of this launch from *tp
    int32_t meas_off, n_ms;   // surface stage measures t - meas_off + j, j < n_ms
    int32_t red_off, n_rs;    // reducer stage reduces t - red_off + j, j < n_rs
    int32_t nseg;
    int32_t ntask;            // lattice tasks (one-step launch) or blocks (two-step launch)
    int32_t n_red, n_sb;      // reducer blocks; surface blocks per measured step
    int32_t zchunk;           // planes per row-group chunk (two-step launch)
    int32_t pad;
    SegInfo seg[kMaxSeg];
    const int32_t *sb_inst;   // per surface block: internal instance
    const int32_t *sb_chunk;  // per surface block: chunk of 64 elements
};

__device__ inline int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Lattice part: fused pull-advection + collision + x sheets.  One wavefront
// task covers 64*CPL consecutive cells of one row; lane l owns the CPL
// contiguous cells xl = x0 + l*CPL ... and moves them with one vector load
// and one vector store per population.  The +x / -x populations come from
// the neighbouring cell: XM = 0 shifts them across lanes (one extra scalar
// load per task end), XM = 1 loads them with a vector load offset by one
// element.  NT = 0: plain loads and stores, 1: non-temporal stores,
// 2: non-temporal loads and stores.
//
// Collision with tau = 1/2 (eq. LBM-Collision) and the equilibrium of
// eq. feq_waves reduce, for these velocity sets (w_i / c_s^2 = 1/2,
// f0^eq = rho (1 - dim c^2)), to
//   f^new_{+a} = c^2 rho - f_{-a},  f^new_{-a} = c^2 rho - f_{+a},
//   f^new_0    = 2 (1 - dim c^2) rho - f_0,
// with c = c(x) the local sound speed.
// ---------------------------------------------------------------------------
// imposed density rs with the cell's own momentum (eq. imposingfields):
// f^eq(rs, J) of the pre-collision populations f
template <int DIM, typename C>
__device__ inline void impose_rule(const C *f, C c2, C rs, C *out)
{
    constexpr int Q = 2 * DIM + 1;
    const C h = (C)0.5;
    out[0] = rs * ((C)1 - (C)DIM * c2);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
        const C Ja = f[i] - f[i + 1];
        out[i] = h * (c2 * rs + Ja);
        out[i + 1] = h * (c2 * rs - Ja);
    }
}

template <int DIM, typename C>
__device__ inline void cell_rule(const C *f, C rho, C c2, int x, int nx, bool driven, C phi, C rs,
                                 C *out)
{
    constexpr int Q = 2 * DIM + 1;
    if (driven && (x == 0 || x == nx - 1)) {
        // damped bounce-back of the pre-collision populations (eq. bounce-back)
        out[0] = phi * f[0];
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            out[i] = phi * f[i + 1];
            out[i + 1] = phi * f[i];
        }
    } else if (driven && x == 1) {
        impose_rule<DIM, C>(f, c2, rs, out);
    } else {
        const C c2rho = c2 * rho;
        out[0] = (C)2 * ((C)1 - (C)DIM * c2) * rho - f[0];
#pragma unroll
        for (int i = 1; i < Q; i += 2) {
            out[i] = c2rho - f[i + 1];
            out[i + 1] = c2rho - f[i];
        }
    }
}

template <int DIM, typename S, int CPL, int XM, int NT>
__device__ inline void lattice_task(const StepArgs &a, const int64_t t, const int bsrc, int task,
                                    int lane)
{
    using T = StoreTraits<S>;
    using R = typename T::R;
    using C = typename T::C;
    using V = typename VecT<R, CPL>::type;
    constexpr int Q = 2 * DIM + 1;

    int s = 0;
#pragma unroll
    for (int k = 1; k < kMaxSeg; ++k)
        if (k < a.nseg && task >= a.seg[k].task0) s = k;
    const SegInfo &sg = a.seg[s];
    const int local = task - sg.task0;
    const int il = local / sg.tpi;
    int r = local - il * sg.tpi;
    const int z = r / (sg.ny * sg.xsegs);
    r -= z * (sg.ny * sg.xsegs);
    const int y = r / sg.xsegs;
    const int xs = r - y * sg.xsegs;
    const auto &I = to_const(a.inst)[sg.first + il];
    if (I.max_steps > 0 && t >= I.max_steps) return;

    // per-instance constants, read once before the population loads
    const int nx = sg.nx, ny = sg.ny, nz = sg.nz;
    const int pitch = I.pitch;
    const int64_t plane = I.plane;
    const bool driven = (I.xbc == 0);
    const C c0sq = (C)I.c0sq;
    const int bb_lo0 = I.bb_lo[0], bb_lo1 = I.bb_lo[1], bb_lo2 = I.bb_lo[2];
    const int bb_n0 = I.bb_n[0], bb_n1 = I.bb_n[1], bb_n2 = I.bb_n[2];
    const int mb_lo0 = I.mb_lo[0], mb_lo1 = I.mb_lo[1], mb_lo2 = I.mb_lo[2];
    const int mb_n0 = I.mb_n[0], mb_n1 = I.mb_n[1], mb_n2 = I.mb_n[2];
    const gptr<const C> c2box = to_global<C>(I.c2box);
    const gptr<C> mom = to_global<C>(I.mom[slot_of(t)]);
    const C phi = (C)I.wall_phi;
    const double src_amp = I.src_amp, omega = I.omega;
    const gptr<const R> src = to_global<R>(static_cast<const void *>(I.buf[bsrc]));
    const gptr<R> dst = to_global<R>(I.buf[bsrc == kNumBuf - 1 ? 0 : bsrc + 1]);

    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1;
    const int zp = (z == nz - 1) ? 0 : z + 1;
    const int64_t row = ((int64_t)z * ny + y) * pitch;
    // uniform row bases of the seven pulled populations
    const gptr<const R> r0 = src + row;
    const gptr<const R> r1 = src + plane + row;
    const gptr<const R> r2 = src + 2 * plane + row;
    const gptr<const R> r3 = src + 3 * plane + ((int64_t)z * ny + ym) * pitch;
    const gptr<const R> r4 = src + 4 * plane + ((int64_t)z * ny + yp) * pitch;
    const gptr<const R> r5 = src + 5 * plane + ((int64_t)zm * ny + y) * pitch;
    const gptr<const R> r6 = src + 6 * plane + ((int64_t)zp * ny + y) * pitch;

    const int x0 = xs * 64 * CPL;
    const int xl = x0 + lane * CPL;
    const uint32_t ux = (uint32_t)xl;  // unsigned lane offset: uniform base + 32-bit offset
    // the lane owns at least one real cell (the vector then lies inside the
    // row; cells >= nx of a straddling vector are padding)
    const bool lane_in = xl < nx;

    C f[Q][CPL];
    {
        V v[Q];
        if (lane_in) {
            v[0] = vload<V, (NT == 2)>((gptr<const V>)at(r0, ux));
            if (XM == 0) {
                v[1] = vload<V, (NT == 2)>((gptr<const V>)at(r1, ux));
                v[2] = vload<V, (NT == 2)>((gptr<const V>)at(r2, ux));
            } else {
                // one element earlier / later: stays inside the buffer because the
                // +x plane follows plane 0 and the -x plane precedes plane 3
                v[1] = vload<V, (NT == 2)>((gptr<const V>)at(r1 - 1, ux));
                v[2] = vload<V, (NT == 2)>((gptr<const V>)at(r2 + 1, ux));
            }
            v[3] = vload<V, (NT == 2)>((gptr<const V>)at(r3, ux));
            v[4] = vload<V, (NT == 2)>((gptr<const V>)at(r4, ux));
            if (DIM == 3) {
                v[5] = vload<V, (NT == 2)>((gptr<const V>)at(r5, ux));
                v[6] = vload<V, (NT == 2)>((gptr<const V>)at(r6, ux));
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) v[i] = V{};
        }
#pragma unroll
        for (int i = 0; i < Q; ++i)
#pragma unroll
            for (int c = 0; c < CPL; ++c) f[i][c] = T::to_c(vget<R, CPL>(v[i], c));
    }
    if (XM == 0) {
        // +x arrives from x - 1, -x from x + 1: shift within the lane, then across lanes
        const C from_left = __shfl_up(f[1][CPL - 1], 1);
        const C from_right = __shfl_down(f[2][0], 1);
#pragma unroll
        for (int c = CPL - 1; c > 0; --c) f[1][c] = f[1][c - 1];
#pragma unroll
        for (int c = 0; c < CPL - 1; ++c) f[2][c] = f[2][c + 1];
        f[1][0] = from_left;
        f[2][CPL - 1] = from_right;
        if (lane == 0 && x0 > 0) f[1][0] = T::to_c(r1[x0 - 1]);
        if (lane == 63) {
            const int xn = x0 + 64 * CPL;
            f[2][CPL - 1] = (xn < nx) ? T::to_c(r2[xn]) : C(0);
        }
    }
    // the two ends of the row: nothing enters from outside (driven) or wrap (periodic)
    if (xl == 0) f[1][0] = driven ? C(0) : T::to_c(r1[nx - 1]);
    {
        const int cl = nx - 1 - xl;
        if (cl >= 0 && cl < CPL) {
#pragma unroll
            for (int c = 0; c < CPL; ++c)
                if (c == cl) f[2][c] = driven ? C(0) : T::to_c(r2[0]);
        }
    }

    const bool in_box_yz = (bb_n0 > 0) && (y >= bb_lo1) && (y < bb_lo1 + bb_n1) &&
                           (DIM == 2 || ((z >= bb_lo2) && (z < bb_lo2 + bb_n2)));
    const bool in_mbox_yz = (mb_n0 > 0) && (y >= mb_lo1) && (y < mb_lo1 + mb_n1) &&
                            (DIM == 2 || ((z >= mb_lo2) && (z < mb_lo2 + mb_n2)));

    V o[Q];
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int x = xl + c;
        C rho = f[0][c];
#pragma unroll
        for (int i = 1; i < Q; ++i) rho += f[i][c];
        if (in_mbox_yz) {
            // rho1, J1 of the advected populations f(t) for the surface measurement
            const int bx = x - mb_lo0;
            if (bx >= 0 && bx < mb_n0 && x < nx) {
                const int by = y - mb_lo1;
                const int bz = (DIM == 3) ? z - mb_lo2 : 0;
                using V4 = typename VecT<C, 4>::type;
                V4 mv;
                mv[0] = rho;
                mv[1] = f[1][c] - f[2][c];
                mv[2] = f[3][c] - f[4][c];
                mv[3] = (DIM == 3) ? f[5][c] - f[6][c] : C(0);
                *(gptr<V4>)(mom + 4 * (((int64_t)bz * mb_n1 + by) * mb_n0 + bx)) = mv;
            }
        }
        C c2 = c0sq;
        if (in_box_yz) {
            const int bx = x - bb_lo0;
            if (bx >= 0 && bx < bb_n0) {
                const int by = y - bb_lo1;
                const int bz = (DIM == 3) ? z - bb_lo2 : 0;
                c2 = c2box[((int64_t)bz * bb_n1 + by) * bb_n0 + bx];
            }
        }
        C out[Q];
        if (x >= nx) {
#pragma unroll
            for (int i = 0; i < Q; ++i) out[i] = C(0);  // padding stays zero
        } else {
            C fc[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) fc[i] = f[i][c];
            C rs = C(0);
            if (driven && x == 1) rs = (C)(src_amp * sin(omega * (double)t));
            cell_rule<DIM, C>(fc, rho, c2, x, nx, driven, phi, rs, out);
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) vset<R, CPL>(o[i], c, T::to_r(out[i]));
    }
    if (lane_in) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
            vstore<V, (NT >= 1)>((gptr<V>)at(dst + (i * plane + row), ux), o[i]);
    }
}

// ---------------------------------------------------------------------------
// Two steps per launch (t -> t + 2; D3Q7, driven x sheets, rows of at most
// 256 cells).  A block covers whole rows: wavefront w moves the cells
// x = 64 (w % nw) + lane of row group w / nw, with nw = pitch / 64
// wavefronts per row and 4 / nw row groups (with nw = 3 the fourth
// wavefront idles but keeps the barriers).  A row group owns R consecutive
// rows and a chunk of up to zchunk planes (chosen per handle: 64 with 4-row
// groups, 32 with 2-row groups, or less when so few blocks would leave the
// chip idle).  It marches through
// the planes: for plane p it advances step t on its rows plus one halo row
// on each side (of those only the population moving into the owned rows is
// kept) and holds the post-collision values in registers; then it finishes
// step t + 1 on plane p - 1, whose seven incoming populations are now all
// known: the +x / -x ones shifted across lanes (across wavefronts through
// LDS), +y / -y from the neighbouring rows, +z / -z from planes p - 2 and p.  Per two
// steps each plane is read about (R + 2) / R times (the halo rows, and the
// halo planes at the chunk ends, are read twice) and written once, against
// two reads and two writes for two one-step launches.
// The per-cell arithmetic is cell_rule, as in lattice_task, and 16-bit
// storage rounds the step-t values through the storage type, so the state
// is bit-identical to that of two one-step launches.  Moments of f(t) and
// f(t + 1) go to their moment boxes as in lattice_task.
// ---------------------------------------------------------------------------
constexpr int kTwoStepMaxPitch = 256;
// Rows longer than kTwoStepMaxPitch are cut into strips of kStripW owned cells.  A strip's block
// spans kStripW + 2 lanes: the columns on either side are computed for step t from the loaded
// state (as the halo rows are) and hand their values inward, so no block waits for another.
constexpr int kStripW = 4 * 64 - 2;
__host__ __device__ inline int two_step_strips(int nx, int pitch)
{
    return pitch <= kTwoStepMaxPitch ? 1 : (nx + kStripW - 1) / kStripW;
}


template <typename C>
__device__ inline void store_moments(gptr<C> mom, int mrow, int mb_lo0, int mb_n0, int x, C rho,
                                     const C *f)
{
    const int bx = x - mb_lo0;
    if (mrow >= 0 && bx >= 0 && bx < mb_n0) {
        using V4 = typename VecT<C, 4>::type;
        V4 mv;
        mv[0] = rho;
        mv[1] = f[1] - f[2];
        mv[2] = f[3] - f[4];
        mv[3] = f[5] - f[6];
        *(gptr<V4>)(mom + 4 * (int64_t)(mrow + bx)) = mv;
    }
}

template <typename S, int R, int NT, bool PF>
__device__ inline void lattice2_block(const StepArgs &a, const int64_t t, const int bsrc, int lb,
                                      typename StoreTraits<S>::C (*xe)[4][R][2])
{
    using T = StoreTraits<S>;
    using E = typename T::R;
    using C = typename T::C;
    int s = 0;
#pragma unroll
    for (int k = 1; k < kMaxSeg; ++k)
        if (k < a.nseg && lb >= a.seg[k].blk0) s = k;
    const SegInfo &sg = a.seg[s];
    const int local = lb - sg.blk0;
    const int il = local / sg.bpi;
    const int nsx = sg.nsx;
    const int rem = local - il * sg.bpi;
    const int sx = rem % nsx;  // strips of one row run side by side
    const int zc = (rem / nsx) / sg.nyb;
    const int yb = rem / nsx - zc * sg.nyb;
    const auto &I = to_const(a.inst)[sg.first + il];
    const int nx = sg.nx, ny = sg.ny, nz = sg.nz;
    const int pitch = I.pitch;
    const int64_t plane = I.plane;
    const int nw = nsx > 1 ? 4 : pitch / 64;  // wavefronts per row (strip)
    const int ng = 4 / nw;                    // row groups per block
    const int lane = threadIdx.x & 63;
    const int w = wave_uniform(threadIdx.x >> 6);
    const int g = w / nw, xs = w - g * nw;
    const bool active = g < ng;
    const int y0 = (yb * ng + (active ? g : 0)) * R;
    const int z0 = zc * a.zchunk;
    const int zlen = min(a.zchunk, nz - z0);
    // owned columns [xo, xend); in a strip the first and last lanes are its halo columns
    const int xo = nsx > 1 ? sx * kStripW : 0;
    const int xend = nsx > 1 ? min(nx, xo + kStripW) : nx;
    const int x = (nsx > 1 ? xo - 1 : 0) + xs * 64 + lane;
    const bool xin = active && x >= 0 && x < nx;  // the lane has a cell
    const bool own = xin && x >= xo && x < xend;   // ... and advances it to step t + 2
    const C c0sq = (C)I.c0sq;
    const C phi = (C)I.wall_phi;
    const gptr<const C> c2box = to_global<C>(I.c2box);
    const bool meas = I.mb_n[0] > 0;
    const int bb_lo[3] = {I.bb_lo[0], I.bb_lo[1], I.bb_lo[2]};
    const int bb_n[3] = {I.bb_n[0], I.bb_n[1], I.bb_n[2]};
    const int mb_lo[3] = {I.mb_lo[0], I.mb_lo[1], I.mb_lo[2]};
    const int mb_n[3] = {I.mb_n[0], I.mb_n[1], I.mb_n[2]};
    const gptr<C> mom_a = to_global<C>(I.mom[slot_of(t)]);
    const gptr<C> mom_b = to_global<C>(I.mom[slot_of(t + 1)]);
    C rs_a = C(0), rs_b = C(0);
    if (x == 1) {
        rs_a = (C)(I.src_amp * sin(I.omega * (double)t));
        rs_b = (C)(I.src_amp * sin(I.omega * (double)(t + 1)));
    }
    const gptr<const E> src = to_global<E>(static_cast<const void *>(I.buf[bsrc]));
    const gptr<E> dst = to_global<E>(I.buf[bsrc == 0 ? 2 : bsrc - 1]);  // buffer (t + 2) mod 3
    const uint32_t ux = (uint32_t)x;

    // step-t values of plane p - 1, pull-ready for step t + 1 (owned rows)
    C Q0[R], Qpx[R], Qmx[R], Qpy[R], Qmy[R], Qpz[R], Qpz2[R];
#pragma unroll
    for (int j = 0; j < R; ++j) Q0[j] = Qpx[j] = Qmx[j] = Qpy[j] = Qmy[j] = Qpz[j] = Qpz2[j] = C(0);

    // uniform offsets, once per block: rows y0 - 1 .. y0 + R (wrapped in y) and their -y / +y
    // neighbours within a plane, and the plane size; per plane only the z bases change
    const int64_t zstride = (int64_t)ny * pitch;
    int64_t yoff[R + 2], ymoff[R + 2], ynoff[R + 2];
    // and the y part of the moment-box and sound-speed-box row indices: a row (y, z) of a box
    // (origin lo, extent n) starts at cell (bz n1 + by) n0, bz = z - lo2, by = y - lo1, the sum
    // of a y part and a z part (-1: the row misses the box)
    int mb_y[R + 2], bb_y[R + 2];
#pragma unroll
    for (int j = -1; j <= R; ++j) {
        int y = y0 + j;
        y = (y < 0) ? y + ny : (y >= ny ? y - ny : y);
        yoff[j + 1] = (int64_t)y * pitch;
        ymoff[j + 1] = (int64_t)((y == 0) ? ny - 1 : y - 1) * pitch;
        ynoff[j + 1] = (int64_t)((y == ny - 1) ? 0 : y + 1) * pitch;
        const int mby = y - mb_lo[1], bby = y - bb_lo[1];
        mb_y[j + 1] = (mb_n[0] > 0 && mby >= 0 && mby < mb_n[1]) ? mby * mb_n[0] : -1;
        bb_y[j + 1] = (bb_n[0] > 0 && bby >= 0 && bby < bb_n[1]) ? bby * bb_n[0] : -1;
    }
    auto box_z = [&](const int *lo, const int *n, int z) {
        const int bz = z - lo[2];
        return (n[0] > 0 && bz >= 0 && bz < n[2]) ? bz * n[1] * n[0] : -1;
    };
    auto box_rowj = [&](const int *ypart, int zpart, int j) {
        return (zpart >= 0 && ypart[j + 1] >= 0) ? zpart + ypart[j + 1] : -1;
    };
    // c^2 of the lane's cell in rows y0 - 1 .. y0 + R of plane zq: every lane loads, cells
    // outside the sound-speed box read the c0^2 stored after it.  Loaded a plane ahead with the
    // populations, so that no load is waited for right after it is issued
    const int n_box = bb_n[0] * bb_n[1] * bb_n[2];
    auto load_c2 = [&](int zq, C (&c)[R + 2]) {
        const int bz = box_z(bb_lo, bb_n, zq);
        const int bx = x - bb_lo[0];
        const bool xb = bx >= 0 && bx < bb_n[0];
#pragma unroll
        for (int j = -1; j <= R; ++j) {
            const int crow = box_rowj(bb_y, bz, j);
            c[j + 1] = c2box[(crow >= 0 && xb) ? crow + bx : n_box];
        }
    };

    // the seven pulled populations (step t) of row y0 + j of plane zq; the
    // +x / -x neighbours by loads offset by one element.  Every lane loads (no branch, so no
    // wait is forced early): lanes without a cell (padding, or the idle wavefront of a
    // 3-wavefront row) read x = 0 of the same row, a line the row's first wavefront fetches
    // anyway, and their results are discarded; the -1 / +1 offsets stay inside the buffer
    // because the +x plane follows plane 0 and the -x plane precedes plane 3
    const uint32_t uxl = xin ? ux : 0u;
    auto load_row = [&](int zq, int j, E *f) {
        const int64_t zb = zq * zstride;
        const int64_t zbm = ((zq == 0) ? nz - 1 : zq - 1) * zstride;
        const int64_t zbn = ((zq == nz - 1) ? 0 : zq + 1) * zstride;
        const int64_t row = zb + yoff[j + 1];
        f[0] = *at(src + row, uxl);
        f[1] = *at(src + plane + row - 1, uxl);
        f[2] = *at(src + 2 * plane + row + 1, uxl);
        f[3] = *at(src + 3 * plane + zb + ymoff[j + 1], uxl);
        f[4] = *at(src + 4 * plane + zb + ynoff[j + 1], uxl);
        f[5] = *at(src + 5 * plane + zbm + yoff[j + 1], uxl);
        f[6] = *at(src + 6 * plane + zbn + yoff[j + 1], uxl);
    };
    auto load_plane = [&](int zq, E (&L)[R + 2][7]) {
#pragma unroll
        for (int j = -1; j <= R; ++j) load_row(zq, j, L[j + 1]);
    };
    auto wrapz = [&](int z) { return (z < 0) ? z + nz : (z >= nz ? z - nz : z); };

    // PF: the loads of plane p + 1 are in flight while plane p is computed
    E Lnext[R + 2][7];
    C C2next[R + 2];
    if (PF) {
        load_plane(wrapz(z0 - 1), Lnext);
        load_c2(wrapz(z0 - 1), C2next);
    }
    C C2prev[R];  // c^2 of the owned rows of plane p - 1 (step t + 1)
#pragma unroll
    for (int j = 0; j < R; ++j) C2prev[j] = c0sq;

    for (int p = -1; p <= zlen; ++p) {
        const int zp = wrapz(z0 + p);
        const bool own_plane = p >= 0 && p < zlen;
        const int sl = (p + 2) & 1;
        E Lcur[R + 2][7];
        C C2cur[R + 2];
        if (PF) {
#pragma unroll
            for (int j = 0; j < R + 2; ++j) {
#pragma unroll
                for (int i = 0; i < 7; ++i) Lcur[j][i] = Lnext[j][i];
                C2cur[j] = C2next[j];
            }
            if (p < zlen) {
                load_plane(wrapz(z0 + p + 1), Lnext);
                load_c2(wrapz(z0 + p + 1), C2next);
            }
        } else {
            load_c2(zp, C2cur);
        }
        C N0[R], Npx[R], Nmx[R], Npy[R], Nmy[R], Npz[R], Nmz[R];
        C prev_py = C(0);
        const int mb_z = box_z(mb_lo, mb_n, zp);
#pragma unroll
        for (int j = -1; j <= R; ++j) {
            E Lrow[7];
            if constexpr (!PF) load_row(zp, j, Lrow);
            const E *L = PF ? Lcur[j + 1] : Lrow;
            // every lane computes (padding lanes on zeros); lanes beyond the row pass on zeros
            C f[7], o[7];
#pragma unroll
            for (int i = 0; i < 7; ++i) f[i] = T::to_c(L[i]);
            if (x == 0) f[1] = C(0);       // nothing enters from outside the sheets
            if (x == nx - 1) f[2] = C(0);
            C rho = f[0];
#pragma unroll
            for (int i = 1; i < 7; ++i) rho += f[i];
            if (meas && own_plane && j >= 0 && j < R && own)
                store_moments(mom_a, box_rowj(mb_y, mb_z, j), mb_lo[0], mb_n[0], x, rho, f);
            cell_rule<3, C>(f, rho, C2cur[j + 1], x, nx, true, phi, rs_a, o);
#pragma unroll
            for (int i = 0; i < 7; ++i) o[i] = xin ? T::to_c(T::to_r(o[i])) : C(0);
            if (j >= 0 && j < R) {
                N0[j] = o[0];
                Npx[j] = __shfl_up(o[1], 1);    // +x arrives from x - 1
                Nmx[j] = __shfl_down(o[2], 1);  // -x arrives from x + 1
                if (lane == 63) xe[sl][w][j][0] = o[1];
                if (lane == 0) xe[sl][w][j][1] = o[2];
                Npy[j] = prev_py;               // +y arrives from row j - 1
                Npz[j] = o[5];
                Nmz[j] = o[6];
            }
            if (j >= 1) Nmy[j - 1] = o[4];      // -y arrives from row j + 1
            prev_py = o[3];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < R; ++j) {
            // neighbours in the same row group only (an idle wavefront reads nothing)
            if (lane == 0) Npx[j] = (active && xs > 0) ? xe[sl][w - 1][j][0] : C(0);
            if (lane == 63) Nmx[j] = (active && xs < nw - 1) ? xe[sl][w + 1][j][1] : C(0);
        }
        if (p >= 1 && own) {
            // step t + 1 on plane zq = z0 + p - 1
            const int zq = z0 + p - 1;
            const int mb_zq = box_z(mb_lo, mb_n, zq);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                C f[7], o[7];
                f[0] = Q0[j];
                f[1] = (x == 0) ? C(0) : Qpx[j];
                f[2] = (x == nx - 1) ? C(0) : Qmx[j];
                f[3] = Qpy[j];
                f[4] = Qmy[j];
                f[5] = Qpz2[j];  // +z of plane zq - 1
                f[6] = Nmz[j];   // -z of plane zq + 1
                C rho = f[0];
#pragma unroll
                for (int i = 1; i < 7; ++i) rho += f[i];
                if (meas)
                    store_moments(mom_b, box_rowj(mb_y, mb_zq, j), mb_lo[0], mb_n[0], x, rho, f);
                cell_rule<3, C>(f, rho, C2prev[j], x, nx, true, phi, rs_b, o);
                const int64_t row = zq * zstride + yoff[j + 1];
#pragma unroll
                for (int i = 0; i < 7; ++i)
                    vstore<E, (NT >= 1)>(at(dst + (i * plane + row), ux), T::to_r(o[i]));
            }
        }
#pragma unroll
        for (int j = 0; j < R; ++j) {
            C2prev[j] = C2cur[j + 1];
            Qpz2[j] = Qpz[j];
            Q0[j] = N0[j];
            Qpx[j] = Npx[j];
            Qmx[j] = Nmx[j];
            Qpy[j] = Npy[j];
            Qmy[j] = Nmy[j];
            Qpz[j] = Npz[j];
        }
    }
}

// ---------------------------------------------------------------------------
// Surface part.  A block handles 64 elements of one instance; its four
// wavefronts split the 3^DIM stencil nodes (node n goes to wavefront n % 4).
// Interpolation of eq. InterpolatedFields with the 3-point kernel as a tensor
// product from the moment box of f(t_meas), then the per-element flux of
// eq. arf_integral_LBM,
//   (-|J|^2/2 + c0^2 rho^2/2) n dS + J (J . n dS),
// summed over the 64 elements in a fixed order into one partial per chunk.
// ---------------------------------------------------------------------------
template <int DIM, typename C>
__device__ inline void surface_block(const StepArgs &a, const int64_t t_meas, int sb,
                                     double (*lds)[64][4])
{
    constexpr int NN = (DIM == 3) ? 27 : 9;
    constexpr int PER = (NN + 3) / 4;
    const int lane = threadIdx.x & 63;
    const int w = wave_uniform(threadIdx.x >> 6);
    const InstDev &I = a.inst[a.sb_inst[sb]];
    const int chunk = a.sb_chunk[sb];
    const int k = chunk * 64 + lane;
    const bool live = k < I.n_surf;
    const gptr<const C> mom = to_global<C>(static_cast<const void *>(I.mom[slot_of(t_meas)]));
    const int mbx = I.mb_n[0], mby = I.mb_n[1];

    double rI = 0.0, Jx = 0.0, Jy = 0.0, Jz = 0.0;
    if (live) {
        const SurfPt &P = I.surf[k];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int n = w + 4 * j;
            if (n < NN) {
                const int dx = n % 3, dy = (n / 3) % 3, dz = n / 9;
                const gptr<const C> m =
                    mom + 4 * (((int64_t)P.bz[dz] * mby + P.by[dy]) * mbx + P.bx[dx]);
                const double wt = P.w[dx] * P.w[3 + dy] * P.w[6 + dz];
                rI += wt * (double)m[0];
                Jx += wt * (double)m[1];
                Jy += wt * (double)m[2];
                Jz += wt * (double)m[3];
            }
        }
    }
    lds[w][lane][0] = rI;
    lds[w][lane][1] = Jx;
    lds[w][lane][2] = Jy;
    lds[w][lane][3] = Jz;
    __syncthreads();
    if (w != 0) return;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    if (live) {
        rI = lds[0][lane][0] + lds[1][lane][0] + lds[2][lane][0] + lds[3][lane][0];
        Jx = lds[0][lane][1] + lds[1][lane][1] + lds[2][lane][1] + lds[3][lane][1];
        Jy = lds[0][lane][2] + lds[1][lane][2] + lds[2][lane][2] + lds[3][lane][2];
        Jz = lds[0][lane][3] + lds[1][lane][3] + lds[2][lane][3] + lds[3][lane][3];
        const SurfPt &P = I.surf[k];
        const double iso = -0.5 * (Jx * Jx + Jy * Jy + Jz * Jz) + 0.5 * I.c0sq_force * rI * rI;
        const double Jn = Jx * P.nA[0] + Jy * P.nA[1] + Jz * P.nA[2];
        fx = iso * P.nA[0] + Jx * Jn;
        fy = iso * P.nA[1] + Jy * Jn;
        fz = iso * P.nA[2] + Jz * Jn;
    }
    // fixed-order butterfly over the 64 lanes
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        fz += __shfl_xor(fz, off);
    }
    if (lane == 0) {
        double *o = I.part + (slot_of(t_meas) * I.n_chunks + chunk) * 4;
        o[0] = fx;
        o[1] = fy;
        o[2] = fz;
    }
}

// Reducer: F(t) of one instance for the steps t0 .. t0+n-1 in order, each
// from its chunk partials (written by an earlier launch), scaled, traced and
// accumulated.  One block per instance, so the accumulation order is fixed.
__device__ inline void reduce_block(const StepArgs &a, const int64_t t0, int n, int ii)
{
    if (threadIdx.x != 0) return;
    const InstDev &I = a.inst[ii];
    if (I.n_surf == 0) return;
    for (int j = 0; j < n; ++j) {
        const int64_t t = t0 + j;
        if (I.max_steps > 0 && t >= I.max_steps) return;
        const double *p = I.part + slot_of(t) * I.n_chunks * 4;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int c = 0; c < I.n_chunks; ++c) {
            s0 += p[4 * c];
            s1 += p[4 * c + 1];
            s2 += p[4 * c + 2];
        }
        const double F[3] = {s0 * I.force_scale, s1 * I.force_scale, s2 * I.force_scale};
        if (t < I.trace_cap) {
            I.trace[3 * t + 0] = F[0];
            I.trace[3 * t + 1] = F[1];
            I.trace[3 * t + 2] = F[2];
        }
        if (t >= I.avg_start) {
            AccDev *acc = I.acc;
            acc->sum[0] += F[0];
            acc->sum[1] += F[1];
            acc->sum[2] += F[2];
            acc->n += 1;
            if (!(isfinite(F[0]) && isfinite(F[1]) && isfinite(F[2]))) acc->nan = 1;
        }
    }
}

// The measurement blocks of a launch (reducers, then the surface blocks of
// each measured step); returns false for a lattice block.
template <int DIM, typename C>
__device__ inline bool measure_part(const StepArgs &a, const int64_t t, int b, double (*lds)[64][4])
{
    if (b < a.n_red) {
        reduce_block(a, t - a.red_off, a.n_rs, b);
        return true;
    }
    b -= a.n_red;
    if (b < a.n_ms * a.n_sb) {
        const int j = b / a.n_sb;
        const int sb = b - j * a.n_sb;
        const InstDev &I = a.inst[a.sb_inst[sb]];
        const int64_t t_meas = t - a.meas_off + j;
        if (I.max_steps > 0 && t_meas >= I.max_steps) return true;
        surface_block<DIM, C>(a, t_meas, sb, lds);
        return true;
    }
    return false;
}

template <int DIM, typename S, int CPL, int XM, int NT>
__global__ void __launch_bounds__(kStepThreads) step_kernel(StepArgs a)
{
    __shared__ double lds[4][64][4];
    const int64_t t = a.tp[0] + a.dt;
    const int b = blockIdx.x;
    if (measure_part<DIM, typename StoreTraits<S>::C>(a, t, b, lds)) return;
    const int bsrc = ((int)a.tp[1] + a.dt) % kNumBuf;  // t mod 3 without 64-bit division
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int task = (b - a.n_red - a.n_ms * a.n_sb) * (kStepThreads / 64) + wave;
    if (task >= a.ntask) return;
    lattice_task<DIM, S, CPL, XM, NT>(a, t, bsrc, task, threadIdx.x & 63);
}

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2):
// physical block b runs on XCD b % 8.  Give each XCD a contiguous range of
// the n logical blocks, so that neighbouring row blocks, which read each
// other's halo rows, share an L2.  A bijection on [0, n).
constexpr int kNumXcd = 8;
__device__ inline int xcd_block(int b, int n)
{
    const int q = n / kNumXcd, r = n % kNumXcd;
    const int x = b % kNumXcd, k = b / kNumXcd;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

template <typename S, int R, int NT, bool PF>
__global__ void __launch_bounds__(kStepThreads, PF ? 2 : 4) step2_kernel(StepArgs a)
{
    using C = typename StoreTraits<S>::C;
    __shared__ double lds[4][64][4];
    __shared__ C xe[2][4][R][2];
    const int64_t t = a.tp[0] + a.dt;
    const int b = blockIdx.x;
    // the long lattice blocks first, the short measurement blocks fill the tail
    if (b < a.ntask) {
        lattice2_block<S, R, NT, PF>(a, t, ((int)a.tp[1] + a.dt) % kNumBuf, xcd_block(b, a.ntask),
                                     xe);
        return;
    }
    measure_part<3, C>(a, t, b - a.ntask, lds);
}

// Device step counter: set, or advance after a replayed sequence.
// The counter holds {t, t mod 3} (the phase saves the kernels a 64-bit division).
// Point source (the paper's oscillating point source): after the lattice
// step t, the source node of every instance that has one takes
// f^eq(rho_a sin(omega t), J1) from its own pre-collision populations, as the
// source sheet does; x, y and z are periodic.  One thread per instance, in
// stream order after the step's lattice launch and before the next one.
template <int DIM, typename S>
__global__ void point_source_kernel(const InstDev *inst, int n_inst, const int64_t *tp, int32_t dt)
{
    using T = StoreTraits<S>;
    using R = typename T::R;
    using C = typename T::C;
    constexpr int Q = 2 * DIM + 1;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_inst) return;
    const InstDev &I = inst[k];
    const int64_t t = tp[0] + dt;
    if (!I.src_point || (I.max_steps > 0 && t >= I.max_steps)) return;
    const int bsrc = ((int)tp[1] + dt) % kNumBuf;
    const R *src = static_cast<const R *>(I.buf[bsrc]);
    R *dst = static_cast<R *>(I.buf[bsrc == kNumBuf - 1 ? 0 : bsrc + 1]);
    const int x = I.src_pt[0], y = I.src_pt[1], z = I.src_pt[2];
    auto at = [&](int i, int xx, int yy, int zz) {
        xx = xx < 0 ? xx + I.nx : (xx >= I.nx ? xx - I.nx : xx);
        yy = yy < 0 ? yy + I.ny : (yy >= I.ny ? yy - I.ny : yy);
        zz = zz < 0 ? zz + I.nz : (zz >= I.nz ? zz - I.nz : zz);
        return (int64_t)i * I.plane + ((int64_t)zz * I.ny + yy) * I.pitch + xx;
    };
    // the pulled populations f_i(x) = f^new_i(x - v_i) of the previous step
    C f[Q];
    f[0] = T::to_c(src[at(0, x, y, z)]);
    f[1] = T::to_c(src[at(1, x - 1, y, z)]);
    f[2] = T::to_c(src[at(2, x + 1, y, z)]);
    f[3] = T::to_c(src[at(3, x, y - 1, z)]);
    f[4] = T::to_c(src[at(4, x, y + 1, z)]);
    if (DIM == 3) {
        f[5] = T::to_c(src[at(5, x, y, z - 1)]);
        f[6] = T::to_c(src[at(6, x, y, z + 1)]);
    }
    C c2 = (C)I.c0sq;
    const int bx = x - I.bb_lo[0], by = y - I.bb_lo[1], bz = (DIM == 3) ? z - I.bb_lo[2] : 0;
    if (I.bb_n[0] > 0 && bx >= 0 && bx < I.bb_n[0] && by >= 0 && by < I.bb_n[1] &&
        (DIM == 2 || (bz >= 0 && bz < I.bb_n[2])))
        c2 = static_cast<const C *>(I.c2box)[((int64_t)bz * I.bb_n[1] + by) * I.bb_n[0] + bx];
    const C rs = (C)(I.src_amp * sin(I.omega * (double)t));
    C out[Q];
    impose_rule<DIM, C>(f, c2, rs, out);
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[at(i, x, y, z)] = T::to_r(out[i]);
}

// rho1 = sum_i f_i (eq. MacroscopicFields) at listed cells of one state buffer, summed in
// FP64 in velocity order and divided by the storage scale; a cell index outside
// 0 .. ncell-1 gives NaN.  Cell c = (z ny + y) nx + x lives at row (z ny + y) of each plane.
template <typename S>
__global__ void probe_rho_kernel(const void *buf, int64_t plane, int Q, int nx, int64_t ncell,
                                 int pitch, const int64_t *cells, int n, double scale, double *out)
{
    using T = StoreTraits<S>;
    using R = typename T::R;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t c = cells[i];
    if (c < 0 || c >= ncell) {
        out[i] = __builtin_nan("");
        return;
    }
    const int64_t off = (c / nx) * pitch + c % nx;
    const R *f = static_cast<const R *>(buf);
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s += (double)T::to_c(f[q * plane + off]);
    out[i] = s / scale;
}

__global__ void set_step_kernel(int64_t *tp, int64_t v)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        tp[0] = v;
        tp[1] = v % kNumBuf;
    }
}
__global__ void advance_step_kernel(int64_t *tp, int64_t k)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        tp[0] = tp[0] + k;
        tp[1] = (tp[1] + k) % kNumBuf;
    }
}

// Fill with zeros (used instead of hipMemsetAsync so that every node of a
// captured sequence is a kernel).
__global__ void zero_kernel(uint4 *p, int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Plain copy (bandwidth reference for the roofline): each thread moves UNR
// independent 16-byte words, consecutive threads consecutive words.
using word16 = VecT<uint32_t, 4>::type;
template <int UNR, bool NT>
__global__ void __launch_bounds__(256) copy_kernel(const word16 *__restrict__ src,
                                                    word16 *__restrict__ dst, int64_t n16)
{
    const int64_t base = (int64_t)blockIdx.x * 256 * UNR + threadIdx.x;
    word16 v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n16) v[u] = vload<word16, NT>(src + i);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n16) vstore<word16, NT>(dst + i, v[u]);
    }
}

// ---------------------------------------------------------------------------
// Empty driven cavity: the x-only field of the empty box is the 3-population
// 1D lattice (rest weight 1 - c0^2, moving weights c0^2/2), here run by one
// workgroup with the lattice in registers and the +/- populations exchanged
// through LDS.  Accumulates sum rho cos(w t) and sum rho sin(w t) per cell
// over the last n_fit steps.
// ---------------------------------------------------------------------------
constexpr int kCavThreads = 1024;
constexpr int kCavMaxNx = 2048;
constexpr int kCavPer = kCavMaxNx / kCavThreads;

__global__ void __launch_bounds__(kCavThreads)
cavity_kernel(int nx, double c0sq, double omega, double rho_a, double phi, int64_t n_total,
              int64_t n_fit, double *lockin /* 2*nx: cos sums, sin sums */)
{
    __shared__ double gp[kCavMaxNx];
    __shared__ double gm[kCavMaxNx];
    double g0[kCavPer], sc[kCavPer], ss[kCavPer];
    double np_[kCavPer], nm_[kCavPer];
#pragma unroll
    for (int j = 0; j < kCavPer; ++j) {
        g0[j] = 0.0;
        sc[j] = 0.0;
        ss[j] = 0.0;
        np_[j] = 0.0;  // post-collision +x population of the cell
        nm_[j] = 0.0;  // post-collision -x population of the cell
    }
    for (int64_t t = 0; t < n_total; ++t) {
        // publish last step's post-collision moving populations
#pragma unroll
        for (int j = 0; j < kCavPer; ++j) {
            const int x = threadIdx.x + j * kCavThreads;
            if (x < nx) {
                gp[x] = np_[j];
                gm[x] = nm_[j];
            }
        }
        __syncthreads();
        double ap[kCavPer], am[kCavPer];
#pragma unroll
        for (int j = 0; j < kCavPer; ++j) {
            const int x = threadIdx.x + j * kCavThreads;
            ap[j] = (x < nx && x > 0) ? gp[x - 1] : 0.0;
            am[j] = (x < nx - 1) ? gm[x + 1] : 0.0;
        }
        __syncthreads();
        const bool fit = t >= n_total - n_fit;
        double cw = 0.0, sw = 0.0;
        if (fit) sincos(omega * (double)t, &sw, &cw);
        const double rs = rho_a * sin(omega * (double)t);
#pragma unroll
        for (int j = 0; j < kCavPer; ++j) {
            const int x = threadIdx.x + j * kCavThreads;
            if (x >= nx) continue;
            const double rho = g0[j] + ap[j] + am[j];
            if (fit) {
                sc[j] += rho * cw;
                ss[j] += rho * sw;
            }
            if (x == 0 || x == nx - 1) {
                g0[j] = phi * g0[j];
                np_[j] = phi * am[j];
                nm_[j] = phi * ap[j];
            } else if (x == 1) {
                const double J = ap[j] - am[j];
                g0[j] = rs * (1.0 - c0sq);
                np_[j] = 0.5 * (c0sq * rs + J);
                nm_[j] = 0.5 * (c0sq * rs - J);
            } else {
                g0[j] = 2.0 * (1.0 - c0sq) * rho - g0[j];
                np_[j] = c0sq * rho - am[j];
                nm_[j] = c0sq * rho - ap[j];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kCavPer; ++j) {
        const int x = threadIdx.x + j * kCavThreads;
        if (x < nx) {
            lockin[x] = sc[j];
            lockin[nx + x] = ss[j];
        }
    }
}

}  // namespace lbw
