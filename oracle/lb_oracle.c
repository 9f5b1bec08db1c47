/*
 * FP64 CPU oracle for the wave lattice Boltzmann computation of the acoustic
 * radiation force on a density-matched compressible object.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference the GPU library is checked against.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Paper: Castro-Avila, Malgaretti, Harting, Munoz, "A lattice Boltzmann
 * approach for acoustic manipulation" (arXiv 2404.02346).
 *
 * What is computed, in the paper's order (Sec. "Lattice-Boltzmann for
 * acoustics", Sec. "Wave-particle interaction and interpolation",
 * Sec. "Results and discussion"):
 *   - macroscopic fields rho1 = sum f_i, J1 = sum v_i f_i   (eq. MacroscopicFields)
 *   - equilibrium f^eq with the LOCAL sound speed c(x)       (eq. feq_waves)
 *   - BGK collision with tau = 1/2                           (eq. LBM-Collision)
 *   - damped bounce-back walls at x = 0 and x = Lx-1         (eq. bounce-back)
 *   - imposed density rho_a sin(omega t) at x = 1            (eq. imposingfields)
 *   - or, in periodic mode, at one node: the oscillating     (eq. waves_with_pointSource,
 *     point source of the first validation                    imposed like the sheet)
 *   - advection f_i(x + v_i) = f_i^new(x)                    (eq. LBM-Advection)
 *   - per-cell sound speed of the object                     (eq. sound_speed_object,
 *                                                             sign read so that c = c_p inside)
 *   - kernel interpolation of rho1, J1 onto surface points   (eq. InterpolatedFields and
 *                                                             the 3-point kernel after it,
 *                                                             applied as a tensor product)
 *   - surface integral of the momentum flux                  (eq. arf_integral_LBM)
 *   - time average over a window of steps                    (Sec. Results, force measured
 *                                                             at every step and averaged)
 *
 * Conventions (readings documented in the design notes):
 *   node (x, y, z) sits at integer coordinates; cell index (z*ny + y)*nx + x;
 *   populations are stored array-of-structures f[cell*Q + i];
 *   velocity order 0, +x, -x, +y, -y, +z, -z (Q = 5 in 2D, 7 in 3D);
 *   y and z are periodic; in "driven" mode x carries the paper's sheets,
 *   in "periodic" mode x is periodic too (used only for the algebraic pins);
 *   the state handed in and out is f^new (post-collision, before advection),
 *   the paper's read-out instant.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_XBC_DRIVEN 0
#define ORC_XBC_PERIODIC 1

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EGEOMETRY (-4)

typedef struct orc_desc {
    int32_t dim, nx, ny, nz;
    int32_t xbc;              /* ORC_XBC_DRIVEN or ORC_XBC_PERIODIC */
    double c0, rho0;          /* fluid sound speed and mean density */
    const double *c_field;    /* optional per-cell sound speed, NULL = analytic object */
    double center[3];         /* object centre r0 */
    double radius, cp, d;     /* object radius R_p, inner sound speed c_p, square thickness d */
    double rho_a, omega, wall_phi;  /* source amplitude, drive frequency, damping Phi */
    int32_t n_surf;           /* surface elements */
    const double *surf_xyz;   /* n_surf*3 element centres R_k */
    const double *surf_normal;/* n_surf*3 unit normals */
    const double *surf_area;  /* n_surf element sizes dS_k */
    int64_t avg_start;        /* accumulate F(t) for t >= avg_start */
    int32_t src_kind;         /* 0: the sheet x = 1 (driven mode); 1: the node src_cell */
    int32_t src_cell[3];      /* point-source node (periodic mode only) */
} orc_desc;

/* Velocity set: rest vector plus the 2*dim unit vectors (Sec. LBW, Fig. velocity_sets). */
static const int VEL[7][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const int OPP[7] = {0, 2, 1, 4, 3, 6, 5};

/*
 * Weights and c_s^2 (Sec. LBW, eq. velocity_properties and the sentence after
 * eq. feq_waves: c_s^2 = 1/3 for D2Q5 and 1/4 for D3Q7).  The figure holding
 * the weights is lost; with the moving weights equal by symmetry, sum w = 1
 * and sum w v_a v_b = c_s^2 delta_ab fix w_i = c_s^2 / 2 and w_0 = 1 - dim c_s^2.
 */
void orc_lattice(int dim, double *w, double *cs2, int *vel)
{
    const int Q = 2 * dim + 1;
    double c2s = (dim == 2) ? 1.0 / 3.0 : 1.0 / 4.0;
    *cs2 = c2s;
    w[0] = (dim == 2) ? 1.0 / 3.0 : 1.0 / 4.0;
    for (int i = 1; i < Q; ++i) w[i] = (dim == 2) ? 1.0 / 6.0 : 1.0 / 8.0;
    if (vel)
        for (int i = 0; i < Q; ++i)
            for (int a = 0; a < 3; ++a) vel[3 * i + a] = VEL[i][a];
}

/* Equilibrium of eq. feq_waves, with c^2 the local squared sound speed. */
void orc_feq(int dim, double c2, double rho, const double *J, double *feq)
{
    const int Q = 2 * dim + 1;
    double w[7], cs2;
    orc_lattice(dim, w, &cs2, NULL);
    feq[0] = rho * (1.0 + (1.0 / cs2) * c2 * (w[0] - 1.0));
    for (int i = 1; i < Q; ++i) {
        double vJ = 0.0;
        for (int a = 0; a < dim; ++a) vJ += VEL[i][a] * J[a];
        feq[i] = (1.0 / cs2) * w[i] * (c2 * rho + vJ);
    }
}

/* Moments of eq. MacroscopicFields at one cell. */
static void moments(int dim, const double *f, double *rho, double *J)
{
    const int Q = 2 * dim + 1;
    *rho = 0.0;
    J[0] = J[1] = J[2] = 0.0;
    for (int i = 0; i < Q; ++i) {
        *rho += f[i];
        for (int a = 0; a < 3; ++a) J[a] += VEL[i][a] * f[i];
    }
}

/* BGK collision of eq. LBM-Collision with tau = 1/2 and dt = 1 at one cell. */
void orc_collide_cell(int dim, double c2, const double *f, double *fnew)
{
    const int Q = 2 * dim + 1;
    const double dt = 1.0, tau = 0.5;
    double rho, J[3], feq[7];
    moments(dim, f, &rho, J);
    orc_feq(dim, c2, rho, J, feq);
    for (int i = 0; i < Q; ++i) fnew[i] = (1.0 - dt / tau) * f[i] + (dt / tau) * feq[i];
}

/* Three-point kernel printed after eq. InterpolatedFields (Roma et al.). */
double orc_roma(double r)
{
    double a = fabs(r);
    if (a <= 0.5) return (1.0 + sqrt(-3.0 * a * a + 1.0)) / 3.0;
    if (a <= 1.5) return (5.0 - 3.0 * a - sqrt(-3.0 * (1.0 - a) * (1.0 - a) + 1.0)) / 6.0;
    return 0.0;
}

/*
 * Sound speed of the density-matched object, eq. sound_speed_object with the
 * sign of the tanh term read so that c = c_p inside and c = c0 outside, as
 * the surrounding text and eq. c_plane_int state.
 */
double orc_sound_speed(const orc_desc *D, double x, double y, double z)
{
    double dx = x - D->center[0], dy = y - D->center[1];
    double dz = (D->dim == 3) ? z - D->center[2] : 0.0;
    double r2 = dx * dx + dy * dy + dz * dz;
    double th = tanh((r2 - D->radius * D->radius) / D->d);
    return D->c0 - 0.5 * (D->c0 - D->cp) * (1.0 - th);
}

static inline int64_t cell_index(const orc_desc *D, int x, int y, int z)
{
    return ((int64_t)z * D->ny + y) * D->nx + x;
}

/* Periodic index for -n <= i < 2n (every caller stays within one period). */
static inline int wrap(int i, int n)
{
    if (i < 0) return i + n;
    if (i >= n) return i - n;
    return i;
}

/*
 * Advection, eq. LBM-Advection: fout_i(x + v_i) = fin_i(x).  y and z wrap;
 * x wraps in periodic mode.  In driven mode populations leaving through
 * x < 0 or x >= nx are dropped and nothing enters from outside, so the
 * incoming slots of the end planes receive zero.
 */
void orc_stream(const orc_desc *D, const double *fin, double *fout)
{
    const int Q = 2 * D->dim + 1;
    const int64_t ncell = (int64_t)D->nx * D->ny * D->nz;
    memset(fout, 0, sizeof(double) * (size_t)(ncell * Q));
#pragma omp parallel for schedule(static)
    for (int z = 0; z < D->nz; ++z)
        for (int y = 0; y < D->ny; ++y)
            for (int x = 0; x < D->nx; ++x) {
                const int64_t src = cell_index(D, x, y, z);
                for (int i = 0; i < Q; ++i) {
                    int tx = x + VEL[i][0];
                    int ty = wrap(y + VEL[i][1], D->ny);
                    int tz = wrap(z + VEL[i][2], D->nz);
                    if (D->xbc == ORC_XBC_PERIODIC) {
                        tx = wrap(tx, D->nx);
                    } else if (tx < 0 || tx >= D->nx) {
                        continue;
                    }
                    fout[cell_index(D, tx, ty, tz) * Q + i] = fin[src * Q + i];
                }
            }
}

/*
 * Kernel interpolation of eq. InterpolatedFields at one point P from the
 * per-cell fields rho[cell], J[cell*3].  Every node within 1.5 cells along
 * each axis is visited and weighted by the product of the 1D kernel along
 * the axes (y, z periodic).  Returns ORC_EGEOMETRY if a needed node lies
 * outside 0 <= x < nx.
 */
int orc_interp(const orc_desc *D, const double *rho, const double *J, const double *P,
               double *rhoI, double *JI)
{
    const int dim = D->dim;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        if (a < dim) {
            lo[a] = (int)ceil(P[a] - 1.5);
            hi[a] = (int)floor(P[a] + 1.5);
        } else {
            lo[a] = hi[a] = 0;
        }
    }
    if (lo[0] < 0 || hi[0] >= D->nx) return ORC_EGEOMETRY;
    *rhoI = 0.0;
    JI[0] = JI[1] = JI[2] = 0.0;
    for (int z = lo[2]; z <= hi[2]; ++z)
        for (int y = lo[1]; y <= hi[1]; ++y)
            for (int x = lo[0]; x <= hi[0]; ++x) {
                double wgt = orc_roma(x - P[0]) * orc_roma(y - P[1]);
                if (dim == 3) wgt *= orc_roma(z - P[2]);
                int64_t c = cell_index(D, x, wrap(y, D->ny), wrap(z, D->nz));
                *rhoI += rho[c] * wgt;
                for (int a = 0; a < 3; ++a) JI[a] += J[3 * c + a] * wgt;
            }
    return ORC_OK;
}

/*
 * Surface integral of eq. arf_integral_LBM (without the time average) from
 * the interpolated fields at each element: per element the integrand
 *   (-|J|^2/2 + c0^2 rho^2/2) n_i + J_i (J . n),
 * times dS_k, summed over k in increasing order, times -1/rho0.
 */
void orc_surface_integral(const orc_desc *D, const double *rhoI, const double *JI, double *F)
{
    F[0] = F[1] = F[2] = 0.0;
    for (int k = 0; k < D->n_surf; ++k) {
        const double *n = D->surf_normal + 3 * k;
        const double *Jk = JI + 3 * k;
        double J2 = Jk[0] * Jk[0] + Jk[1] * Jk[1] + Jk[2] * Jk[2];
        double Jn = Jk[0] * n[0] + Jk[1] * n[1] + Jk[2] * n[2];
        double iso = -0.5 * J2 + 0.5 * D->c0 * D->c0 * rhoI[k] * rhoI[k];
        for (int i = 0; i < 3; ++i) F[i] += (iso * n[i] + Jk[i] * Jn) * D->surf_area[k];
    }
    for (int i = 0; i < 3; ++i) F[i] *= -1.0 / D->rho0;
}

/* Per-cell sound speed squared, from the given field or the analytic object. */
static void build_c2(const orc_desc *D, double *c2)
{
    for (int z = 0; z < D->nz; ++z)
        for (int y = 0; y < D->ny; ++y)
            for (int x = 0; x < D->nx; ++x) {
                int64_t c = cell_index(D, x, y, z);
                double cs = D->c_field ? D->c_field[c] : orc_sound_speed(D, x, y, z);
                c2[c] = cs * cs;
            }
}

/*
 * The full run.  fnew_init (optional, NULL = all zero) is the post-collision
 * state of step -1; each step t = 0 .. n_steps-1 then, cell by cell,
 *   1. gathers f(t) by advection of the previous f^new (eq. LBM-Advection,
 *      written as a pull: f_i(x) = f^new_i(x - v_i), zero where x - v_i
 *      lies outside 0 <= x < nx in driven mode),
 *   2. takes rho1, J1 of f(t),
 *   3. collides with its own c(x)^2 (eq. LBM-Collision), except that in
 *      driven mode the wall planes x = 0 and x = nx-1 take the damped
 *      bounce-back of the pre-collision populations (eq. bounce-back) and
 *      the source plane x = 1 takes f^eq(rho_a sin(omega t), J1(1, y, z))
 *      (eq. imposingfields); in periodic mode with src_kind = 1 the single
 *      node src_cell takes f^eq(rho_a sin(omega t), J1) in the same way;
 * and then
 *   4. interpolates rho1, J1 of f(t) onto the surface and evaluates F(t)
 *      (eq. arf_integral_LBM); for t >= avg_start adds F(t) to the FP64
 *      accumulator.
 * Outputs (each optional): fnew_out = f^new of the last step, F_trace
 * (n_steps*3), F_avg (3) and n_acc, rho_line (rho1 along x at y = z = 0 for
 * steps line_t0 .. line_t0+line_n-1, line_n*nx values), rho_probe (rho1 at
 * the n_probe cell indices probe[] for the same steps, line_n*n_probe values).
 */
/* The steps t = t0 .. t0 + n_steps - 1 of the loop above on the state *prev (f^new of step
 * t0 - 1), swapping *prev and *next after each step, adding F(t) for t >= avg_start to acc and
 * nacc, and recording the optional outputs of orc_run (trace index t - t0). */
static int run_steps(const orc_desc *D, int64_t t0, int64_t n_steps, double **prev_io,
                     double **next_io, const double *c2, double *rho, double *J, double *rhoI,
                     double *JI, double acc[3], int64_t *nacc, double *F_trace, double *rho_line,
                     int64_t line_t0, int64_t line_n, const int64_t *probe, int64_t n_probe,
                     double *rho_probe)
{
    const int dim = D->dim, Q = 2 * dim + 1;
    const int driven = (D->xbc == ORC_XBC_DRIVEN);
    const int point = (D->src_kind == 1);
    double *prev = *prev_io, *next = *next_io;
    int status = ORC_OK;

    for (int64_t t = t0; t < t0 + n_steps && status == ORC_OK; ++t) {
        const double rho_src = D->rho_a * sin(D->omega * (double)t);
#pragma omp parallel for schedule(static)
        for (int z = 0; z < D->nz; ++z)
            for (int y = 0; y < D->ny; ++y)
                for (int x = 0; x < D->nx; ++x) {
                    const int64_t c = cell_index(D, x, y, z);
                    double f[7];
                    /* 1. pull advection */
                    for (int i = 0; i < Q; ++i) {
                        int sx = x - VEL[i][0];
                        int sy = wrap(y - VEL[i][1], D->ny);
                        int sz = wrap(z - VEL[i][2], D->nz);
                        if (!driven) {
                            sx = wrap(sx, D->nx);
                        } else if (sx < 0 || sx >= D->nx) {
                            f[i] = 0.0;
                            continue;
                        }
                        f[i] = prev[cell_index(D, sx, sy, sz) * Q + i];
                    }
                    /* 2. moments */
                    moments(dim, f, rho + c, J + 3 * c);
                    /* 3. collision, walls, source */
                    double *out = next + c * Q;
                    if (driven && (x == 0 || x == D->nx - 1)) {
                        for (int i = 0; i < Q; ++i) out[i] = D->wall_phi * f[OPP[i]];
                    } else if ((driven && x == 1) ||
                               (point && x == D->src_cell[0] && y == D->src_cell[1] &&
                                z == D->src_cell[2])) {
                        orc_feq(dim, c2[c], rho_src, J + 3 * c, out);
                    } else {
                        orc_collide_cell(dim, c2[c], f, out);
                    }
                }

        if (rho_line && t >= line_t0 && t < line_t0 + line_n)
            for (int x = 0; x < D->nx; ++x) rho_line[(t - line_t0) * D->nx + x] = rho[x];
        if (rho_probe && t >= line_t0 && t < line_t0 + line_n)
            for (int64_t j = 0; j < n_probe; ++j) rho_probe[(t - line_t0) * n_probe + j] = rho[probe[j]];

        /* 4. interpolation and surface integral */
        if (D->n_surf > 0) {
            for (int k = 0; k < D->n_surf && status == ORC_OK; ++k)
                status = orc_interp(D, rho, J, D->surf_xyz + 3 * k, rhoI + k, JI + 3 * k);
            if (status != ORC_OK) break;
            double F[3];
            orc_surface_integral(D, rhoI, JI, F);
            if (F_trace)
                for (int a = 0; a < 3; ++a) F_trace[3 * (t - t0) + a] = F[a];
            if (t >= D->avg_start) {
                for (int a = 0; a < 3; ++a) acc[a] += F[a];
                ++*nacc;
            }
        }
        double *tmp = prev;
        prev = next;
        next = tmp;
    }
    *prev_io = prev;
    *next_io = next;
    return status;
}

static int check_desc(const orc_desc *D)
{
    const int dim = D->dim;
    if (dim != 2 && dim != 3) return ORC_EINVAL;
    if (D->nx < 1 || D->ny < 1 || D->nz < 1 || (dim == 2 && D->nz != 1)) return ORC_EINVAL;
    if (D->xbc == ORC_XBC_DRIVEN && D->nx < 3) return ORC_EINVAL;
    const int driven = (D->xbc == ORC_XBC_DRIVEN);
    const int point = (D->src_kind == 1);
    if (D->src_kind != 0 && D->src_kind != 1) return ORC_EINVAL;
    if (point && (driven || D->src_cell[0] < 0 || D->src_cell[0] >= D->nx || D->src_cell[1] < 0 ||
                  D->src_cell[1] >= D->ny || D->src_cell[2] < 0 || D->src_cell[2] >= D->nz))
        return ORC_EINVAL;
    return ORC_OK;
}

int orc_run(const orc_desc *D, int64_t n_steps, const double *fnew_init, double *fnew_out,
            double *F_trace, double *F_avg, int64_t *n_acc, double *rho_line, int64_t line_t0,
            int64_t line_n, const int64_t *probe, int64_t n_probe, double *rho_probe)
{
    int status = check_desc(D);
    if (status != ORC_OK) return status;
    const int Q = 2 * D->dim + 1;
    const int64_t ncell = (int64_t)D->nx * D->ny * D->nz;
    for (int64_t j = 0; j < n_probe; ++j)
        if (probe[j] < 0 || probe[j] >= ncell) return ORC_EINVAL;

    double *prev = (double *)calloc((size_t)(ncell * Q), sizeof(double));
    double *next = (double *)malloc(sizeof(double) * (size_t)(ncell * Q));
    double *c2 = (double *)malloc(sizeof(double) * (size_t)ncell);
    double *rho = (double *)malloc(sizeof(double) * (size_t)ncell);
    double *J = (double *)malloc(sizeof(double) * (size_t)(ncell * 3));
    int n_s = D->n_surf > 0 ? D->n_surf : 1;
    double *rhoI = (double *)malloc(sizeof(double) * (size_t)n_s);
    double *JI = (double *)malloc(sizeof(double) * 3 * (size_t)n_s);
    if (!prev || !next || !c2 || !rho || !J || !rhoI || !JI) {
        free(prev); free(next); free(c2); free(rho); free(J); free(rhoI); free(JI);
        return ORC_ENOMEM;
    }
    if (fnew_init) memcpy(prev, fnew_init, sizeof(double) * (size_t)(ncell * Q));
    build_c2(D, c2);

    double acc[3] = {0.0, 0.0, 0.0};
    int64_t nacc = 0;
    status = run_steps(D, 0, n_steps, &prev, &next, c2, rho, J, rhoI, JI, acc, &nacc, F_trace,
                       rho_line, line_t0, line_n, probe, n_probe, rho_probe);

    if (status == ORC_OK) {
        if (fnew_out) memcpy(fnew_out, prev, sizeof(double) * (size_t)(ncell * Q));
        if (F_avg)
            for (int a = 0; a < 3; ++a) F_avg[a] = nacc > 0 ? acc[a] / (double)nacc : 0.0;
        if (n_acc) *n_acc = nacc;
    }
    free(prev); free(next); free(c2); free(rho); free(J); free(rhoI); free(JI);
    return status;
}

/* Steps t0 .. t0 + n_steps - 1 of orc_run from the state fnew_init (f^new of step t0 - 1,
 * required), continuing the FP64 force accumulator: acc (3 sums) and n_acc are read and
 * written back.  fnew_out (required) receives f^new of the last step.  Running steps 0 .. n-1
 * as consecutive segments this way gives the same sums, and so the same time average
 * acc / n_acc, as one orc_run of n steps. */
int orc_run_segment(const orc_desc *D, int64_t t0, int64_t n_steps, const double *fnew_init,
                    double *fnew_out, double *acc, int64_t *n_acc)
{
    int status = check_desc(D);
    if (status != ORC_OK) return status;
    if (!fnew_init || !fnew_out || !acc || !n_acc || t0 < 0 || n_steps < 0) return ORC_EINVAL;
    const int Q = 2 * D->dim + 1;
    const int64_t ncell = (int64_t)D->nx * D->ny * D->nz;
    double *prev = (double *)malloc(sizeof(double) * (size_t)(ncell * Q));
    double *next = (double *)malloc(sizeof(double) * (size_t)(ncell * Q));
    double *c2 = (double *)malloc(sizeof(double) * (size_t)ncell);
    double *rho = (double *)malloc(sizeof(double) * (size_t)ncell);
    double *J = (double *)malloc(sizeof(double) * (size_t)(ncell * 3));
    int n_s = D->n_surf > 0 ? D->n_surf : 1;
    double *rhoI = (double *)malloc(sizeof(double) * (size_t)n_s);
    double *JI = (double *)malloc(sizeof(double) * 3 * (size_t)n_s);
    if (!prev || !next || !c2 || !rho || !J || !rhoI || !JI) {
        free(prev); free(next); free(c2); free(rho); free(J); free(rhoI); free(JI);
        return ORC_ENOMEM;
    }
    memcpy(prev, fnew_init, sizeof(double) * (size_t)(ncell * Q));
    build_c2(D, c2);
    status = run_steps(D, t0, n_steps, &prev, &next, c2, rho, J, rhoI, JI, acc, n_acc, NULL,
                       NULL, 0, 0, NULL, 0, NULL);
    if (status == ORC_OK) memcpy(fnew_out, prev, sizeof(double) * (size_t)(ncell * Q));
    free(prev); free(next); free(c2); free(rho); free(J); free(rhoI); free(JI);
    return status;
}
