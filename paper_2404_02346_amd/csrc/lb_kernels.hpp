// Device code of the wave lattice Boltzmann library (gfx950).
//
// Method: Castro-Avila et al., "A lattice Boltzmann approach for acoustic
// manipulation" (arXiv 2404.02346), Sec. "Lattice-Boltzmann for acoustics"
// and Sec. "Wave-particle interaction and interpolation".
//
// Population storage is structure-of-arrays: plane i (velocity i) holds the
// cells row by row, x fastest, rows `pitch` elements apart (pitch is a
// multiple of 64 elements, so every row starts on a 256-byte boundary for
// 4-byte storage).  Two state buffers alternate: the step that starts at t
// reads buffer t & 1 (f^new of step t-1) and writes buffer (t + 1) & 1.
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

struct InstDev {
    int32_t dim, nx, ny, nz;
    int32_t pitch, xbc;
    int64_t plane;           // elements per population plane
    void *buf[2];            // state buffers (plane 0)
    double c0sq;             // fluid c0^2 (outside the box)
    int32_t bb_lo[3];        // sound-speed box origin
    int32_t bb_n[3];         // sound-speed box extent (0 -> no box)
    const void *c2box;       // c^2 over the box in the compute type, x fastest
    double src_amp;          // rho_a times the storage scale
    double omega, wall_phi;
    int64_t max_steps;       // frozen for t >= max_steps
    // measurement
    int32_t mb_lo[3];        // moment box origin (cells whose rho, J the surface reads)
    int32_t mb_n[3];         // moment box extent (0 -> no measurement)
    void *mom[2];            // moment boxes (rho, Jx, Jy, Jz per cell, compute type) by step parity
    int32_t n_surf, n_chunks;  // surface elements, 64-element chunks
    const SurfPt *surf;
    double *part;            // 2 x n_chunks x 4 per-chunk flux sums by step parity
    double c0sq_force;       // c0^2 in the surface integral
    double force_scale;      // -1 / (rho0 * scale^2)
    int64_t avg_start;
    AccDev *acc;
    double *trace;           // trace_cap x 3
    int64_t trace_cap;
};

struct SegInfo {
    int32_t task0;      // first wave task of the run
    int32_t first;      // first (internal) instance of the run
    int32_t nx, ny, nz; // shape shared by the run
    int32_t xsegs;      // wave tasks per row
    int32_t tpi;        // wave tasks per instance
    int32_t pad;
};

// One launch = [reducer blocks][surface blocks][lattice blocks], a
// three-stage pipeline over consecutive steps:
//  * lattice blocks advance step t and store rho1, J1 of f(t) in the moment
//    box of parity t & 1;
//  * surface blocks interpolate F(t_meas = t - 1) from the moment box of
//    parity t_meas & 1 and write one partial sum per 64 elements;
//  * reducer blocks sum the partials of F(t_red = t - 2) in a fixed order,
//    scale, trace and accumulate.
// Every stage reads what an earlier launch wrote, so no stage waits on
// another inside a launch.
// The lattice step of a launch is t = *tp + dt: the counter lives in device
// memory so that a captured sequence of launches can be replayed at any t.
struct StepArgs {
    const InstDev *inst;
    const int64_t *tp;        // device step counter
    int32_t dt;               // offset of this launch from *tp
    int32_t meas_off;         // surface stage measures t - meas_off
    int32_t red_off;          // reducer stage reduces t - red_off
    int32_t nseg;
    int32_t ntask;
    int32_t n_red, n_sb;
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
template <int DIM, typename S, int CPL, int XM, int NT>
__device__ inline void lattice_task(const StepArgs &a, const int64_t t, int task, int lane)
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
    const gptr<C> mom = to_global<C>(I.mom[t & 1]);
    const C phi = (C)I.wall_phi;
    const double src_amp = I.src_amp, omega = I.omega;
    const gptr<const R> src = to_global<R>(static_cast<const void *>(I.buf[t & 1]));
    const gptr<R> dst = to_global<R>(I.buf[(t + 1) & 1]);

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
        } else if (driven && (x == 0 || x == nx - 1)) {
            // damped bounce-back of the pre-collision populations (eq. bounce-back)
            out[0] = phi * f[0][c];
#pragma unroll
            for (int i = 1; i < Q; i += 2) {
                out[i] = phi * f[i + 1][c];
                out[i + 1] = phi * f[i][c];
            }
        } else if (driven && x == 1) {
            // imposed density with the cell's own momentum (eq. imposingfields)
            const C rs = (C)(src_amp * sin(omega * (double)t));
            const C h = (C)0.5;
            out[0] = rs * ((C)1 - (C)DIM * c2);
#pragma unroll
            for (int i = 1; i < Q; i += 2) {
                const C Ja = f[i][c] - f[i + 1][c];
                out[i] = h * (c2 * rs + Ja);
                out[i + 1] = h * (c2 * rs - Ja);
            }
        } else {
            const C c2rho = c2 * rho;
            out[0] = (C)2 * ((C)1 - (C)DIM * c2) * rho - f[0][c];
#pragma unroll
            for (int i = 1; i < Q; i += 2) {
                out[i] = c2rho - f[i + 1][c];
                out[i + 1] = c2rho - f[i][c];
            }
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
    const gptr<const C> mom = to_global<C>(static_cast<const void *>(I.mom[t_meas & 1]));
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
        double *o = I.part + ((t_meas & 1) * I.n_chunks + chunk) * 4;
        o[0] = fx;
        o[1] = fy;
        o[2] = fz;
    }
}

// Reducer: F(t_red) of one instance from its chunk partials (written by the
// previous launch), scaled, traced and accumulated.
__device__ inline void reduce_block(const StepArgs &a, const int64_t t, int ii)
{
    if (threadIdx.x != 0) return;
    const InstDev &I = a.inst[ii];
    if (I.n_surf == 0) return;
    if (I.max_steps > 0 && t >= I.max_steps) return;
    const double *p = I.part + (t & 1) * I.n_chunks * 4;
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

template <int DIM, typename S, int CPL, int XM, int NT>
__global__ void __launch_bounds__(kStepThreads) step_kernel(StepArgs a)
{
    __shared__ double lds[4][64][4];
    const int64_t t = *a.tp + a.dt;
    const int b = blockIdx.x;
    if (b < a.n_red) {
        reduce_block(a, t - a.red_off, b);
        return;
    }
    if (b < a.n_red + a.n_sb) {
        const int sb = b - a.n_red;
        const InstDev &I = a.inst[a.sb_inst[sb]];
        const int64_t t_meas = t - a.meas_off;
        if (I.max_steps > 0 && t_meas >= I.max_steps) return;
        surface_block<DIM, typename StoreTraits<S>::C>(a, t_meas, sb, lds);
        return;
    }
    const int wave = wave_uniform(threadIdx.x >> 6);
    const int task = (b - a.n_red - a.n_sb) * (kStepThreads / 64) + wave;
    if (task >= a.ntask) return;
    lattice_task<DIM, S, CPL, XM, NT>(a, t, task, threadIdx.x & 63);
}

// Device step counter: set, or advance after a replayed sequence.
__global__ void set_step_kernel(int64_t *tp, int64_t v)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *tp = v;
}
__global__ void advance_step_kernel(int64_t *tp, int64_t k)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *tp = *tp + k;
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
template <int UNR, bool NT>
__global__ void __launch_bounds__(256) copy_kernel(const uint4 *__restrict__ src,
                                                    uint4 *__restrict__ dst, int64_t n16)
{
    const int64_t base = (int64_t)blockIdx.x * 256 * UNR + threadIdx.x;
    uint4 v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n16) v[u] = vload<uint4, NT>(src + i);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
        const int64_t i = base + (int64_t)u * 256;
        if (i < n16) vstore<uint4, NT>(dst + i, v[u]);
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
