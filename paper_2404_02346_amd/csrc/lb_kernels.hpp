// Device code of the wave lattice Boltzmann library (gfx950).
//
// Method: Castro-Avila et al., "A lattice Boltzmann approach for acoustic
// manipulation" (arXiv 2404.02346), Sec. "Lattice-Boltzmann for acoustics"
// and Sec. "Wave-particle interaction and interpolation".
//
// Population storage is structure-of-arrays: plane i (velocity i) holds the
// cells row by row, x fastest, rows `pitch` elements apart (pitch is a
// multiple of 64 elements so every row starts on a 256-byte boundary for
// 4-byte storage).  Two state buffers alternate: the step that starts at
// t reads buffer t & 1 (f^new of step t-1) and writes buffer (t + 1) & 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbw {

constexpr int kMaxSeg = 8;          // same-shape instance runs handled by one launch
constexpr int kStepThreads = 256;   // 4 wavefronts of 64 lanes

// ---------------------------------------------------------------------------
// Storage types and conversions
// ---------------------------------------------------------------------------
struct bf16 {
    uint16_t bits;
};

template <typename S> struct StoreTraits;
template <> struct StoreTraits<double> {
    using C = double;  // compute type
    __device__ static inline double load(const double *p) { return *p; }
    __device__ static inline void store(double *p, double v) { *p = v; }
};
template <> struct StoreTraits<float> {
    using C = float;
    __device__ static inline float load(const float *p) { return *p; }
    __device__ static inline void store(float *p, float v) { *p = v; }
};
template <> struct StoreTraits<_Float16> {
    using C = float;
    __device__ static inline float load(const _Float16 *p) { return (float)*p; }
    __device__ static inline void store(_Float16 *p, float v) { *p = (_Float16)v; }
};
template <> struct StoreTraits<bf16> {
    using C = float;
    __device__ static inline float load(const bf16 *p) {
        return __uint_as_float(((uint32_t)p->bits) << 16);
    }
    __device__ static inline void store(bf16 *p, float v) {
        // round to nearest, ties to even
        uint32_t u = __float_as_uint(v);
        u += 0x7FFFu + ((u >> 16) & 1u);
        p->bits = (uint16_t)(u >> 16);
    }
};

// ---------------------------------------------------------------------------
// Per-instance data (lives in the workspace)
// ---------------------------------------------------------------------------
struct SurfPt {
    int32_t ix[3], iy[3], iz[3];  // stencil node coordinates (y, z already wrapped)
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
    int32_t n_surf, pad0;
    const SurfPt *surf;
    double *contrib;         // n_surf x 4 per-element flux (x, y, z, unused)
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

struct StepArgs {
    const InstDev *inst;
    int64_t t;
    int32_t nseg;
    int32_t ntask;
    SegInfo seg[kMaxSeg];
};

__device__ inline int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Fused pull-advection + collision + x sheets.  One wavefront task covers
// 64*VX consecutive cells of one row; lane l handles x = x0 + l + 64 j.
//
// Collision with tau = 1/2 (eq. LBM-Collision) and the equilibrium of
// eq. feq_waves reduce, for these velocity sets (w_i / c_s^2 = 1/2,
// f0^eq = rho (1 - dim c^2)), to
//   f^new_{+a} = c^2 rho - f_{-a},  f^new_{-a} = c^2 rho - f_{+a},
//   f^new_0    = 2 (1 - dim c^2) rho - f_0,
// with c = c(x) the local sound speed.
// ---------------------------------------------------------------------------
template <int DIM, typename S, int VX>
__global__ void __launch_bounds__(kStepThreads) step_kernel(StepArgs a)
{
    using T = StoreTraits<S>;
    using C = typename T::C;
    constexpr int Q = 2 * DIM + 1;

    const int wave = wave_uniform(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int task = blockIdx.x * (kStepThreads / 64) + wave;
    if (task >= a.ntask) return;

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
    const InstDev &I = a.inst[sg.first + il];
    if (I.max_steps > 0 && a.t >= I.max_steps) return;

    const int nx = sg.nx, ny = sg.ny, nz = sg.nz;
    const int pitch = I.pitch;
    const int64_t plane = I.plane;
    const S *src = static_cast<const S *>(I.buf[a.t & 1]);
    S *dst = static_cast<S *>(I.buf[(a.t + 1) & 1]);
    const bool driven = (I.xbc == 0);
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    const int zm = (z == 0) ? nz - 1 : z - 1;
    const int zp = (z == nz - 1) ? 0 : z + 1;
    const int64_t row = ((int64_t)z * ny + y) * pitch;
    const int64_t row_ym = ((int64_t)z * ny + ym) * pitch;
    const int64_t row_yp = ((int64_t)z * ny + yp) * pitch;
    const int64_t row_zm = ((int64_t)zm * ny + y) * pitch;
    const int64_t row_zp = ((int64_t)zp * ny + y) * pitch;
    const C c0sq = (C)I.c0sq;
    const bool in_box_yz = (I.bb_n[0] > 0) && (y >= I.bb_lo[1]) && (y < I.bb_lo[1] + I.bb_n[1]) &&
                           (DIM == 2 || ((z >= I.bb_lo[2]) && (z < I.bb_lo[2] + I.bb_n[2])));
    const C *c2box = static_cast<const C *>(I.c2box);

#pragma unroll
    for (int j = 0; j < VX; ++j) {
        const int x = xs * 64 * VX + j * 64 + lane;
        if (x >= nx) continue;
        C f[Q];
        f[0] = T::load(src + row + x);
        if (x > 0)
            f[1] = T::load(src + plane + row + x - 1);
        else
            f[1] = driven ? C(0) : T::load(src + plane + row + nx - 1);
        if (x < nx - 1)
            f[2] = T::load(src + 2 * plane + row + x + 1);
        else
            f[2] = driven ? C(0) : T::load(src + 2 * plane + row);
        f[3] = T::load(src + 3 * plane + row_ym + x);
        f[4] = T::load(src + 4 * plane + row_yp + x);
        if (DIM == 3) {
            f[5] = T::load(src + 5 * plane + row_zm + x);
            f[6] = T::load(src + 6 * plane + row_zp + x);
        }
        C rho = f[0];
#pragma unroll
        for (int i = 1; i < Q; ++i) rho += f[i];

        C c2 = c0sq;
        if (in_box_yz) {
            const int bx = x - I.bb_lo[0];
            if (bx >= 0 && bx < I.bb_n[0]) {
                const int by = y - I.bb_lo[1];
                const int bz = (DIM == 3) ? z - I.bb_lo[2] : 0;
                c2 = c2box[((int64_t)bz * I.bb_n[1] + by) * I.bb_n[0] + bx];
            }
        }

        C out[Q];
        if (driven && (x == 0 || x == nx - 1)) {
            // damped bounce-back of the pre-collision populations (eq. bounce-back)
            const C phi = (C)I.wall_phi;
            out[0] = phi * f[0];
#pragma unroll
            for (int i = 1; i < Q; i += 2) {
                out[i] = phi * f[i + 1];
                out[i + 1] = phi * f[i];
            }
        } else if (driven && x == 1) {
            // imposed density with the cell's own momentum (eq. imposingfields)
            const C rs = (C)(I.src_amp * sin(I.omega * (double)a.t));
            const C h = (C)0.5;
            out[0] = rs * ((C)1 - (C)DIM * c2);
#pragma unroll
            for (int i = 1; i < Q; i += 2) {
                const C Ja = f[i] - f[i + 1];
                out[i] = h * (c2 * rs + Ja);
                out[i + 1] = h * (c2 * rs - Ja);
            }
        } else {
            const C c2rho = c2 * rho;
            out[0] = (C)2 * ((C)1 - (C)DIM * c2) * rho - f[0];
#pragma unroll
            for (int i = 1; i < Q; i += 2) {
                out[i] = c2rho - f[i + 1];
                out[i + 1] = c2rho - f[i];
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) T::store(dst + i * plane + row + x, out[i]);
    }
}

// ---------------------------------------------------------------------------
// Surface interpolation (eq. InterpolatedFields with the 3-point kernel as a
// tensor product) and per-element flux of eq. arf_integral_LBM.  Block:
// 64 elements x NZ wavefronts, wavefront dz handles stencil plane dz.
// Reads the state buffer f^new(t); at the stencil nodes (never on an x
// sheet) its moments equal those of the advected populations f(t).
// ---------------------------------------------------------------------------
template <int DIM, typename S>
__global__ void __launch_bounds__(192) surface_interp_kernel(const InstDev *insts, int64_t t,
                                                             int first_inst)
{
    using T = StoreTraits<S>;
    constexpr int Q = 2 * DIM + 1;
    constexpr int NZ = (DIM == 3) ? 3 : 1;
    __shared__ double part[NZ][64][4];

    const InstDev &I = insts[first_inst + blockIdx.y];
    if (I.max_steps > 0 && t >= I.max_steps) return;
    const int lane = threadIdx.x & 63;
    const int dz = wave_uniform(threadIdx.x >> 6);
    const int k = blockIdx.x * 64 + lane;
    const bool live = k < I.n_surf;
    const S *src = static_cast<const S *>(I.buf[(t + 1) & 1]);
    const int64_t plane = I.plane;
    const int pitch = I.pitch;

    double rI = 0.0, Jx = 0.0, Jy = 0.0, Jz = 0.0;
    if (live) {
        const SurfPt &P = I.surf[k];
        const int zc = P.iz[dz];
        const double wz = P.w[6 + dz];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int64_t rowb = ((int64_t)zc * I.ny + P.iy[dy]) * pitch;
            const double wyz = P.w[3 + dy] * wz;
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const S *p = src + rowb + P.ix[dx];
                double f[Q];
#pragma unroll
                for (int i = 0; i < Q; ++i) f[i] = (double)T::load(p + i * plane);
                double rho = f[0];
#pragma unroll
                for (int i = 1; i < Q; ++i) rho += f[i];
                const double w = P.w[dx] * wyz;
                rI += w * rho;
                Jx += w * (f[1] - f[2]);
                Jy += w * (f[3] - f[4]);
                if (DIM == 3) Jz += w * (f[5] - f[6]);
            }
        }
    }
    part[dz][lane][0] = rI;
    part[dz][lane][1] = Jx;
    part[dz][lane][2] = Jy;
    part[dz][lane][3] = Jz;
    __syncthreads();
    if (dz != 0 || !live) return;
    rI = part[0][lane][0];
    Jx = part[0][lane][1];
    Jy = part[0][lane][2];
    Jz = part[0][lane][3];
#pragma unroll
    for (int q = 1; q < NZ; ++q) {
        rI += part[q][lane][0];
        Jx += part[q][lane][1];
        Jy += part[q][lane][2];
        Jz += part[q][lane][3];
    }
    const SurfPt &P = I.surf[k];
    // (-|J|^2/2 + c0^2 rho^2/2) n dS + J (J . n dS)
    const double iso = -0.5 * (Jx * Jx + Jy * Jy + Jz * Jz) + 0.5 * I.c0sq_force * rI * rI;
    const double Jn = Jx * P.nA[0] + Jy * P.nA[1] + Jz * P.nA[2];
    double *o = I.contrib + 4 * (int64_t)k;
    o[0] = iso * P.nA[0] + Jx * Jn;
    o[1] = iso * P.nA[1] + Jy * Jn;
    o[2] = iso * P.nA[2] + Jz * Jn;
}

// Sum of the per-element fluxes in a fixed order (deterministic), scaling,
// trace and time accumulation.  One block of 256 threads per instance.
__global__ void __launch_bounds__(256) surface_reduce_kernel(const InstDev *insts, int64_t t,
                                                             int first_inst)
{
    __shared__ double red[3][256];
    const InstDev &I = insts[first_inst + blockIdx.x];
    if (I.max_steps > 0 && t >= I.max_steps) return;
    if (I.n_surf == 0) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = threadIdx.x; k < I.n_surf; k += 256) {
        const double *o = I.contrib + 4 * (int64_t)k;
        s0 += o[0];
        s1 += o[1];
        s2 += o[2];
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    red[2][threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
            red[2][threadIdx.x] += red[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double F[3] = {red[0][0] * I.force_scale, red[1][0] * I.force_scale,
                       red[2][0] * I.force_scale};
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

// Fill with zeros (used instead of hipMemsetAsync so that every node of a
// captured sequence is a kernel).
__global__ void zero_kernel(uint4 *p, int64_t n16)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
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
    for (int j = 0; j < kCavPer; ++j) {
        const int x = threadIdx.x + j * kCavThreads;
        if (x < nx) {
            gp[x] = 0.0;
            gm[x] = 0.0;
        }
    }
    __syncthreads();
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
