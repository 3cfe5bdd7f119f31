/*
 * lbm_oracle.c -- plain, slow, FP64 CPU oracle for one D2Q9 BGK lattice-Boltzmann
 * step with the velocity-interpolation-based bounce-back (VIBB) wall closure of
 * Zhang et al., "Velocity interpolation based Bounce-Back scheme for non-slip
 * boundary condition in Lattice Boltzmann Method" (arXiv:1903.01111).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library calls this file; only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no code, header, table or constant with the GPU path.
 *
 * The same source is compiled twice:
 *   - with real_t = double                 -> functions prefixed  orc_
 *   - with real_t = double _Complex (-DORC_COMPLEX) -> prefixed    orc_cs_
 * The complex build evaluates the identical arithmetic on complex numbers, so
 * a perturbation i*h of one input gives the exact derivative of the discrete
 * map as Im(out)/h (complex-step differentiation, Squire & Trapp 1998).
 * Every branch decides on real parts only.
 *
 * Layout (oracle-private, chosen for readability): populations are stored
 * node-major, fp[(y*nx + x)*9 + i], holding the post-collision value f+_i
 * of the paper, raw (not shifted by the weights).
 *
 * Readings of the paper that this file takes where the text is silent or
 * ambiguous are marked "reading:".
 *
 * Built with -fopenmp (a separate library used only to time the oracle and to
 * compare large workloads), the per-node loops of streaming, collision, the
 * open columns and the moments run over rows in parallel; every node's
 * arithmetic is the same, so the results are bitwise those of the serial build.
 * The link loop and the force sums stay serial.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <complex.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifdef ORC_COMPLEX
typedef double _Complex real_t;
#define ORC(name) orc_cs_##name
#define RE(x) creal(x)
#define SQRT(x) csqrt(x)
#else
typedef double real_t;
#define ORC(name) orc_##name
#define RE(x) (x)
#define SQRT(x) sqrt(x)
#endif

/* ---------------------------------------------------------------------------
 * Lattice (Section 2).  The paper lists the nine D2Q9 velocities by groups
 * only (rest, axis, diagonal); their order is fixed by the transform matrix M
 * of the MRT operator, whose rows for j_x and j_y are the x and y components
 * of e_i column by column.
 * ------------------------------------------------------------------------- */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1}; /* row j_x of M */
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1}; /* row j_y of M */

/* weights with C = dx = dt = 1 (Section 2, after the equilibrium) */
static double weight(int i)
{
    if (i == 0) return 4.0 / 9.0;
    if (i <= 4) return 1.0 / 9.0;
    return 1.0 / 36.0;
}

/* opposite direction i' of i: the index whose velocity is -e_i (found by search) */
static int opposite(int i)
{
    for (int j = 0; j < 9; ++j)
        if (EX[j] == -EX[i] && EY[j] == -EY[i]) return j;
    return -1;
}

/* equilibrium, Section 2 Eq. (feq) with C = 1:
 *   f^eq_i = w_i rho (1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u.u) */
real_t ORC(equilibrium)(int i, real_t rho, real_t ux, real_t uy)
{
    real_t eu = EX[i] * ux + EY[i] * uy;
    real_t uu = ux * ux + uy * uy;
    return weight(i) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
}

/* Macroscopic density and velocity of a post-collision node (Section 2, the
 * zeroth and first moments).  reading: with a body force g the post-collision
 * momentum carries half of the force density F = rho g (Guo forcing, see
 * collide()), so the physical velocity is u = (sum f+ e)/rho - g/2. */
static void moments_post(const real_t *f, double gx, double gy,
                         real_t *rho, real_t *ux, real_t *uy)
{
    real_t r = 0, jx = 0, jy = 0;
    for (int i = 0; i < 9; ++i) {
        r += f[i];
        jx += f[i] * EX[i];
        jy += f[i] * EY[i];
    }
    *rho = r;
    *ux = jx / r - 0.5 * gx;
    *uy = jy / r - 0.5 * gy;
}

void ORC(moments_node)(const real_t *f, double gx, double gy, real_t *out3)
{
    moments_post(f, gx, gy, &out3[0], &out3[1], &out3[2]);
}

/* ---------------------------------------------------------------------------
 * VIBB, Section 3.1.  The unknown population f_i(x_f, t+1) that would stream
 * out of the solid is obtained by bounce-back from the departure point d of
 * the molecule that leaves f with velocity e_{i'}:
 *   f_i(x_f,t+1) = f+_{i'}(x_d,t) + 6 w_{i'} rho0 e_i.u_w                (VIBB bounce-back)
 *   f+_{i'}(x_d,t) = f^eq_{i'}(rho_d, u_d) + f^neq_{i'}(x_d,t)           (eq./non-eq. split)
 *   rho_d = 2q rho_f + (1-2q) rho_ff                                      (density at d)
 *   f^neq_{i'}(x_d) = 2q f^neq_{i'}(x_f) rho_d/rho_f
 *                   + (1-2q) f^neq_{i'}(x_ff) rho_d/rho_ff                (non-eq. at d)
 *   u*_d  = 2q u_f + (1-2q) u_ff                   if q <= 1/2
 *         = (1-q)/q u_f + (2q-1)/q u_w             if q >  1/2
 *   u**_d = (1-q)/(1+q) u_ff + 2q/(1+q) u_w
 *   u_d   = u*_d/3 + 2 u**_d/3
 * reading: rho_d and f^neq use the same 2q, (1-2q) weights for every q, i.e.
 * they are extrapolated when q > 1/2; only the velocity brings in u_w.
 * reading: the q = 1/2 case takes the first branch of u*_d (both agree there).
 * reading: f^neq at a node is its post-collision population minus the
 * equilibrium of its own (rho, u), with u the physical velocity of
 * moments_post().
 * ------------------------------------------------------------------------- */
real_t ORC(vibb)(int ip, const real_t *fp_f, const real_t *fp_ff, real_t q,
                 real_t uwx, real_t uwy, double rho0, double gx, double gy)
{
    int i = opposite(ip);
    real_t rho_f, ufx, ufy, rho_ff, uffx, uffy;
    moments_post(fp_f, gx, gy, &rho_f, &ufx, &ufy);
    moments_post(fp_ff, gx, gy, &rho_ff, &uffx, &uffy);

    real_t rho_d = 2.0 * q * rho_f + (1.0 - 2.0 * q) * rho_ff;

    real_t fneq_f = fp_f[ip] - ORC(equilibrium)(ip, rho_f, ufx, ufy);
    real_t fneq_ff = fp_ff[ip] - ORC(equilibrium)(ip, rho_ff, uffx, uffy);
    real_t fneq_d = 2.0 * q * fneq_f * rho_d / rho_f
                  + (1.0 - 2.0 * q) * fneq_ff * rho_d / rho_ff;

    real_t us_x, us_y;
    if (RE(q) <= 0.5) {
        us_x = 2.0 * q * ufx + (1.0 - 2.0 * q) * uffx;
        us_y = 2.0 * q * ufy + (1.0 - 2.0 * q) * uffy;
    } else {
        us_x = (1.0 - q) / q * ufx + (2.0 * q - 1.0) / q * uwx;
        us_y = (1.0 - q) / q * ufy + (2.0 * q - 1.0) / q * uwy;
    }
    real_t uss_x = (1.0 - q) / (1.0 + q) * uffx + 2.0 * q / (1.0 + q) * uwx;
    real_t uss_y = (1.0 - q) / (1.0 + q) * uffy + 2.0 * q / (1.0 + q) * uwy;

    real_t ud_x = us_x / 3.0 + 2.0 * uss_x / 3.0;
    real_t ud_y = us_y / 3.0 + 2.0 * uss_y / 3.0;

    real_t fplus_d = ORC(equilibrium)(ip, rho_d, ud_x, ud_y) + fneq_d;
    real_t wall = 6.0 * weight(ip) * rho0 * (EX[i] * uwx + EY[i] * uwy);
    return fplus_d + wall;
}

/* Halfway bounce-back (Section 3): the wall is taken halfway between f and s,
 * f_i(x_f,t+1) = f+_{i'}(x_f,t), plus the same moving-wall momentum term. */
real_t ORC(hbb)(int ip, const real_t *fp_f, real_t uwx, real_t uwy, double rho0)
{
    int i = opposite(ip);
    return fp_f[ip] + 6.0 * weight(ip) * rho0 * (EX[i] * uwx + EY[i] * uwy);
}

/* Bouzidi's linear interpolated bounce-back (Section 3, the two equations for
 * q <= 1/2 and q > 1/2), with the same moving-wall term:
 *   q <= 1/2:  f_i(x_f,t+1) = 2q f+_{i'}(x_f) + (1-2q) f+_{i'}(x_ff) + wall
 *   q >  1/2:  f_i(x_f,t+1) = (f+_{i'}(x_f) + wall)/(2q) + (2q-1)/(2q) f+_i(x_f)
 * reading: the last term of the q > 1/2 equation, printed as f_i(x_f, t), is
 * the post-collision population f+_i(x_f, t) of the outgoing direction i (the
 * value that streams to x_ff at t+1).  For q > 1/2 the node ff is not used. */
real_t ORC(bouzidi)(int ip, const real_t *fp_f, const real_t *fp_ff, real_t q, real_t uwx, real_t uwy,
                    double rho0)
{
    int i = opposite(ip);
    real_t wall = 6.0 * weight(ip) * rho0 * (EX[i] * uwx + EY[i] * uwy);
    if (RE(q) <= 0.5) return 2.0 * q * fp_f[ip] + (1.0 - 2.0 * q) * fp_ff[ip] + wall;
    return (fp_f[ip] + wall) / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * fp_f[i];
}

/* Yu's unified interpolated bounce-back (Section 3): the population at the
 * wall point first, by linear interpolation of f+_{i'} between x_f and x_ff and
 * bounce-back with the moving-wall term,
 *   f_i(x_w, t+1) = q f+_{i'}(x_f) + (1-q) f+_{i'}(x_ff) + wall,
 * then the unknown at x_f by interpolation between x_w and x_ff,
 *   f_i(x_f, t+1) = [f_i(x_w, t+1) + q f_i(x_ff, t+1)] / (1+q).
 * reading: the second equation has an unbalanced parenthesis as printed; it is
 * read as the linear interpolation above (x_w at distance q from x_f on one
 * side, x_ff at distance 1 on the other).  f_i(x_ff, t+1) is what streams into
 * x_ff from x_f, i.e. f+_i(x_f, t). */
real_t ORC(yu)(int ip, const real_t *fp_f, const real_t *fp_ff, real_t q, real_t uwx, real_t uwy, double rho0)
{
    int i = opposite(ip);
    real_t wall = 6.0 * weight(ip) * rho0 * (EX[i] * uwx + EY[i] * uwy);
    real_t fw = q * fp_f[ip] + (1.0 - q) * fp_ff[ip] + wall;
    real_t fff = fp_f[i];
    return (fw + q * fff) / (1.0 + q);
}

/* ---------------------------------------------------------------------------
 * Geometry (Section 3, node classification and the wall fraction q).
 * Primitives, each given as (cx, cy, R): 0 disc solid inside |x-c| <= R;
 * 1 disc solid outside |x-c| >= R; 2 half-plane y <= cy solid; 3 half-plane
 * y >= cy solid.
 * Each primitive carries a wall velocity (ux, uy) plus a spin omega about its
 * centre, and an object id for the force.
 * reading: a node exactly on a circle is solid; periodic directions use the
 * minimum-image offset from the centre; q is the fraction of the link from
 * the fluid node to the first crossing of the boundary of a primitive that
 * holds the solid node; u_w is evaluated at x_w = x_f + q e_{i'}.
 * ------------------------------------------------------------------------- */
typedef struct {
    int nx, ny, x_open;
} orc_grid;

static double wrapd(double d, int n, int periodic)
{
    if (!periodic) return d;
    while (d >= 0.5 * n) d -= n;
    while (d < -0.5 * n) d += n;
    return d;
}

/* real-valued containment test, on the real part of the primitive */
static int inside(int type, const real_t *pc, const orc_grid *g, int x, int y)
{
    if (type == 0 || type == 1) {
        double dx = wrapd(x - RE(pc[0]), g->nx, !g->x_open);
        double dy = wrapd(y - RE(pc[1]), g->ny, 1);
        double rr = dx * dx + dy * dy, R = RE(pc[2]);
        return type == 0 ? (rr <= R * R) : (rr >= R * R);
    }
    if (type == 2) return y <= RE(pc[1]);
    return y >= RE(pc[1]);
}

/* link fraction s in (0,1] where x_f + s e enters the solid side of a primitive */
static real_t crossing(int type, const real_t *pc, const orc_grid *g, int x, int y,
                       int ex, int ey, real_t *rx, real_t *ry)
{
    if (type == 0 || type == 1) {
        /* offset from the centre, minimum image taken on the real part */
        double sx = wrapd(x - RE(pc[0]), g->nx, !g->x_open) - (x - RE(pc[0]));
        double sy = wrapd(y - RE(pc[1]), g->ny, 1) - (y - RE(pc[1]));
        real_t dx = (x - pc[0]) + sx, dy = (y - pc[1]) + sy;
        real_t a = ex * ex + ey * ey;
        real_t b = dx * ex + dy * ey;
        real_t k = dx * dx + dy * dy - pc[2] * pc[2];
        real_t disc = b * b - a * k;
        real_t s = (type == 0) ? (-b - SQRT(disc)) / a : (-b + SQRT(disc)) / a;
        *rx = dx + s * ex;
        *ry = dy + s * ey;
        return s;
    }
    real_t s = (pc[1] - y) / ey;
    *rx = 0;
    *ry = 0;
    return s;
}

/* Builds the solid mask and the list of fluid->solid links.  Returns the number
 * of links; arrays are written only if it does not exceed max_links. */
int64_t ORC(geometry)(int nx, int ny, int x_open, int nprim, const int32_t *ptype,
                      const real_t *pc, const real_t *pvel, const int32_t *pobj,
                      uint8_t *solid, int64_t max_links, int32_t *node, int8_t *dir,
                      real_t *q, real_t *uw, int32_t *obj)
{
    orc_grid g = {nx, ny, x_open};
    /* owner[n]: the one primitive holding node n, -1 none, -2 several.  Discs
     * are only tested over their bounding box (with periodic wrap). */
    int32_t *owner = (int32_t *)malloc(sizeof(int32_t) * (size_t)nx * ny);
    for (int n = 0; n < nx * ny; ++n) {
        solid[n] = 0;
        owner[n] = -1;
    }
    for (int p = 0; p < nprim; ++p) {
        int xa = 0, xb = nx - 1, ya = 0, yb = ny - 1;
        if (ptype[p] == 0) {
            xa = (int)floor(RE(pc[3 * p]) - RE(pc[3 * p + 2])) - 1;
            xb = (int)ceil(RE(pc[3 * p]) + RE(pc[3 * p + 2])) + 1;
            ya = (int)floor(RE(pc[3 * p + 1]) - RE(pc[3 * p + 2])) - 1;
            yb = (int)ceil(RE(pc[3 * p + 1]) + RE(pc[3 * p + 2])) + 1;
        }
        for (int yy = ya; yy <= yb; ++yy)
            for (int xx = xa; xx <= xb; ++xx) {
                int x = xx, y = ((yy % ny) + ny) % ny;
                if (x_open && (x < 0 || x >= nx)) continue;
                x = ((x % nx) + nx) % nx;
                if (!inside(ptype[p], pc + 3 * p, &g, x, y)) continue;
                int n = y * nx + x;
                if (owner[n] == p) continue;
                solid[n] = 1;
                owner[n] = owner[n] == -1 ? p : -2;
            }
    }
    int64_t n = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (solid[y * nx + x]) continue;
            if (x_open && (x == 0 || x == nx - 1)) continue; /* open columns are not streamed */
            for (int ip = 1; ip < 9; ++ip) {
                int xs = x + EX[ip], ys = y + EY[ip];
                if (x_open && (xs < 0 || xs >= nx)) continue;
                xs = (xs + nx) % nx;
                ys = (ys + ny) % ny;
                if (!solid[ys * nx + xs]) continue;
                real_t best = 0, brx = 0, bry = 0;
                int bp = -1;
                int own = owner[ys * nx + xs];
                for (int p = (own >= 0 ? own : 0); p < (own >= 0 ? own + 1 : nprim); ++p) {
                    if (!inside(ptype[p], pc + 3 * p, &g, xs, ys)) continue;
                    real_t rx, ry;
                    real_t s = crossing(ptype[p], pc + 3 * p, &g, x, y, EX[ip], EY[ip], &rx, &ry);
                    if (bp < 0 || RE(s) < RE(best)) {
                        best = s;
                        bp = p;
                        brx = rx;
                        bry = ry;
                    }
                }
                if (n < max_links) {
                    const real_t *v = pvel + 3 * bp;
                    node[n] = y * nx + x;
                    dir[n] = (int8_t)ip;
                    q[n] = best;
                    /* translation plus rotation omega x r about the centre */
                    uw[2 * n] = v[0] - v[2] * bry;
                    uw[2 * n + 1] = v[1] + v[2] * brx;
                    obj[n] = pobj[bp];
                }
                ++n;
            }
        }
    free(owner);
    return n;
}

/* ---------------------------------------------------------------------------
 * Time stepping.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t nx, ny;     /* node index y*nx + x */
    int32_t x_open;     /* 0: periodic in x; 1: inlet at x = 0 and outlet at x = nx-1 */
    int32_t n_obj;      /* number of force accumulators */
    double tau;         /* BGK relaxation time, tau = 3 nu + 1/2 (Section 2) */
    double gx, gy;      /* body acceleration (force density F = rho g) */
    double rho0;        /* reference density of the moving-wall term */
    int32_t collision;  /* 0: BGK; 1: MRT with the rates s[] (Section 2) */
    int32_t gi_mea;     /* 0: plain momentum exchange; 1: its Galilean-invariant form */
    double s[9];        /* MRT relaxation rates, one per moment of M (collision == 1) */
} orc_params;

/* threads of the OpenMP build (ignored by the serial build); returns the count
 * the parallel loops will use (1 in the serial build) */
#ifndef ORC_COMPLEX
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
#endif

/* f+ = f^eq(rho, u) at every fluid node; solid nodes hold zeros */
void ORC(init_equilibrium)(int nx, int ny, const uint8_t *solid, const real_t *rho,
                           const real_t *ux, const real_t *uy, real_t *fp)
{
    for (int n = 0; n < nx * ny; ++n)
        for (int i = 0; i < 9; ++i)
            fp[n * 9 + i] = solid[n] ? 0.0 : ORC(equilibrium)(i, rho[n], ux[n], uy[n]);
}

void ORC(moments)(const orc_params *p, const uint8_t *solid, const real_t *fp,
                  real_t *rho, real_t *ux, real_t *uy)
{
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int n = 0; n < p->nx * p->ny; ++n) {
        if (solid[n]) {
            rho[n] = ux[n] = uy[n] = 0;
            continue;
        }
        moments_post(fp + 9 * n, p->gx, p->gy, &rho[n], &ux[n], &uy[n]);
    }
}

/* ---------------------------------------------------------------------------
 * MRT collision (Section 2): Omega = M^-1 S (m^eq - m), m = M f, with the
 * transform matrix M as printed (moments rho, e, epsilon, j_x, q_x, j_y, q_y,
 * p_xx, p_xy) and the diagonal relaxation matrix S.
 * ------------------------------------------------------------------------- */
static const int MRT_M[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},       {-4, -1, -1, -1, -1, 2, 2, 2, 2}, {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},    {0, -2, 0, 2, 0, 1, -1, -1, 1},   {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},    {0, 1, -1, 1, -1, 0, 0, 0, 0},    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

#ifndef ORC_COMPLEX
void orc_mrt_matrix(int32_t *out81)
{
    for (int k = 0; k < 81; ++k) out81[k] = MRT_M[k / 9][k % 9];
}
#endif

/* M^-1 by Gauss-Jordan elimination with partial pivoting (computed once) */
static double MRT_MINV[9][9];
static int mrt_minv_ready = 0;

static void mrt_inverse(void)
{
    if (mrt_minv_ready) return;
    double a[9][18];
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 18; ++c) a[r][c] = c < 9 ? MRT_M[r][c] : (c - 9 == r ? 1.0 : 0.0);
    for (int c = 0; c < 9; ++c) {
        int piv = c;
        for (int r = c + 1; r < 9; ++r)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        for (int k = 0; k < 18; ++k) {
            double tmp = a[c][k];
            a[c][k] = a[piv][k];
            a[piv][k] = tmp;
        }
        double d = a[c][c];
        for (int k = 0; k < 18; ++k) a[c][k] /= d;
        for (int r = 0; r < 9; ++r) {
            if (r == c) continue;
            double m = a[r][c];
            for (int k = 0; k < 18; ++k) a[r][k] -= m * a[c][k];
        }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) MRT_MINV[r][c] = a[r][c + 9];
    mrt_minv_ready = 1;
}

#ifndef ORC_COMPLEX
void orc_mrt_inverse(double *out81)
{
    mrt_inverse();
    for (int k = 0; k < 81; ++k) out81[k] = MRT_MINV[k / 9][k % 9];
}
#endif

/* Equilibrium moments.  reading: the printed e^eq and epsilon^eq, rho(-2 + 3 j.j)
 * and rho(1 - 3 j.j), mix j = rho u with rho; they are taken as the moments of
 * the second-order equilibrium of Section 2, rho(-2 + 3 u.u) and rho(1 - 3 u.u);
 * likewise q^eq = -j, p_xx^eq = (j_x^2 - j_y^2)/rho, p_xy^eq = j_x j_y/rho. */
void ORC(mrt_meq)(real_t rho, real_t ux, real_t uy, real_t *m)
{
    real_t uu = ux * ux + uy * uy;
    m[0] = rho;
    m[1] = rho * (-2.0 + 3.0 * uu);
    m[2] = rho * (1.0 - 3.0 * uu);
    m[3] = rho * ux;
    m[4] = -rho * ux;
    m[5] = rho * uy;
    m[6] = -rho * uy;
    m[7] = rho * (ux * ux - uy * uy);
    m[8] = rho * ux * uy;
}

/* MRT collision with a body force.  reading: the paper names no forcing scheme;
 * Guo, Zheng & Shi's source term F_i = w_i [3(e_i - u) + 9 (e_i.u) e_i].F is
 * applied in moment space with the factor (I - S/2), the MRT form of Guo's
 * forcing, and u carries the half-force shift as in the BGK collision.  With
 * every s_k = 1/tau this is the BGK collision below. */
static void collide_mrt(real_t *f, const double *s, double gx, double gy)
{
    mrt_inverse();
    real_t rho = 0, jx = 0, jy = 0;
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += f[i] * EX[i];
        jy += f[i] * EY[i];
    }
    real_t Fx = rho * gx, Fy = rho * gy;
    real_t ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
    real_t meq[9], src[9], ms[9];
    ORC(mrt_meq)(rho, ux, uy, meq);
    for (int i = 0; i < 9; ++i) {
        real_t eu = EX[i] * ux + EY[i] * uy;
        src[i] = weight(i) * ((3.0 * (EX[i] - ux) + 9.0 * eu * EX[i]) * Fx +
                              (3.0 * (EY[i] - uy) + 9.0 * eu * EY[i]) * Fy);
    }
    for (int k = 0; k < 9; ++k) {
        real_t mk = 0, sk = 0;
        for (int i = 0; i < 9; ++i) {
            mk += MRT_M[k][i] * f[i];
            sk += MRT_M[k][i] * src[i];
        }
        ms[k] = mk - s[k] * (mk - meq[k]) + (1.0 - 0.5 * s[k]) * sk;
    }
    for (int i = 0; i < 9; ++i) {
        real_t v = 0;
        for (int k = 0; k < 9; ++k) v += MRT_MINV[i][k] * ms[k];
        f[i] = v;
    }
}

/* BGK collision with Guo, Zheng & Shi (2002) forcing.  Section 2 gives the BGK
 * operator Omega = (f^eq - f)/tau; reading: the paper drives its channel with a
 * body force without naming the scheme, so the force enters through Guo's
 * source term with the half-force velocity shift. */
static void collide(real_t *f, double tau, double gx, double gy)
{
    real_t rho = 0, jx = 0, jy = 0;
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += f[i] * EX[i];
        jy += f[i] * EY[i];
    }
    real_t Fx = rho * gx, Fy = rho * gy;
    real_t ux = (jx + 0.5 * Fx) / rho, uy = (jy + 0.5 * Fy) / rho;
    for (int i = 0; i < 9; ++i) {
        real_t feq = ORC(equilibrium)(i, rho, ux, uy);
        real_t eu = EX[i] * ux + EY[i] * uy;
        real_t src = (1.0 - 0.5 / tau) * weight(i) *
                     ((3.0 * (EX[i] - ux) + 9.0 * eu * EX[i]) * Fx +
                      (3.0 * (EY[i] - uy) + 9.0 * eu * EY[i]) * Fy);
        f[i] = f[i] - (f[i] - feq) / tau + src;
    }
}

static void collide_node(const orc_params *p, real_t *f)
{
    if (p->collision == 1) collide_mrt(f, p->s, p->gx, p->gy);
    else collide(f, p->tau, p->gx, p->gy);
}

/* one node's collision in place (pre-collision f in, post-collision out) */
void ORC(collide_node)(const orc_params *p, real_t *f) { collide_node(p, f); }

/* Scratch of one step: boundary values per node and direction, which of them a
 * link sets, the post-collision populations, the value of every link. */
typedef struct {
    real_t *fbc, *fnew, *val;
    uint8_t *have;
} orc_work;

static int work_alloc(orc_work *w, int nx, int ny, int64_t nl)
{
    size_t n9 = 9 * (size_t)nx * ny;
    w->fbc = (real_t *)malloc(sizeof(real_t) * n9);
    w->fnew = (real_t *)malloc(sizeof(real_t) * n9);
    w->val = (real_t *)malloc(sizeof(real_t) * (size_t)(nl > 0 ? nl : 1));
    w->have = (uint8_t *)malloc(n9);
    return w->fbc && w->fnew && w->val && w->have;
}

static void work_free(orc_work *w)
{
    free(w->fbc);
    free(w->fnew);
    free(w->val);
    free(w->have);
}

/* One time step t -> t+1 in place on fp.  force[2*obj] accumulates (+=) the
 * momentum-exchange force of the fluid on each object during this step;
 * link_out (may be NULL) receives the missing population of every link;
 * *n_fallback (may be NULL) is increased by the number of links that fall back to
 * halfway bounce-back.  Returns 0, or -2 if a fluid node pulls from a solid node
 * with no link. */
static int step_work(const orc_params *p, const uint8_t *solid, int64_t nl, const int32_t *lnode,
                     const int8_t *ldir, const real_t *lq, const real_t *luw, const int32_t *lobj,
                     const int8_t *lscheme, const real_t *uin, real_t *fp, real_t *force,
                     int64_t *n_fallback, real_t *link_out, orc_work *w)
{
    const int nx = p->nx, ny = p->ny, N = nx * ny;
    real_t *fbc = w->fbc, *fnew = w->fnew, *val = w->val;
    uint8_t *have = w->have;
    memset(have, 0, 9 * (size_t)N);

    /* 1-2. boundary value of every link from the state at time t (links are
     * independent: the OpenMP build evaluates them in parallel); the force sums
     * follow serially in link order */
    int64_t nfb = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(+ : nfb)
#endif
    for (int64_t l = 0; l < nl; ++l) {
        int nf = lnode[l], ip = ldir[l], i = opposite(ip);
        int xf = nf % nx, yf = nf / nx;
        int xff = xf - EX[ip], yff = yf - EY[ip];
        int ff_ok = 1;
        if (p->x_open && (xff < 0 || xff >= nx)) ff_ok = 0;
        xff = (xff + nx) % nx;
        yff = (yff + ny) % ny;
        int nff = yff * nx + xff;
        if (solid[nff]) ff_ok = 0;
        real_t uwx = luw ? luw[2 * l] : 0.0, uwy = luw ? luw[2 * l + 1] : 0.0;
        /* scheme: 0 VIBB (Section 3.1), 1 halfway bounce-back, 2 Bouzidi, 3 Yu */
        int sch = lscheme ? lscheme[l] : 0;
        /* reading: a scheme that needs the second fluid node falls back to halfway
         * bounce-back where x_ff is solid or off an open edge (Bouzidi needs it only
         * for q <= 1/2) */
        int needs_ff = sch == 0 || sch == 3 || (sch == 2 && RE(lq[l]) <= 0.5);
        if (needs_ff && !ff_ok) {
            ++nfb;
            sch = 1;
        }
        real_t v;
        if (sch == 0)
            v = ORC(vibb)(ip, fp + 9 * nf, fp + 9 * nff, lq[l], uwx, uwy, p->rho0, p->gx, p->gy);
        else if (sch == 2)
            v = ORC(bouzidi)(ip, fp + 9 * nf, fp + 9 * nff, lq[l], uwx, uwy, p->rho0);
        else if (sch == 3)
            v = ORC(yu)(ip, fp + 9 * nf, fp + 9 * nff, lq[l], uwx, uwy, p->rho0);
        else
            v = ORC(hbb)(ip, fp + 9 * nf, uwx, uwy, p->rho0);
        fbc[9 * nf + i] = v;
        have[9 * nf + i] = 1;
        val[l] = v;
    }
    if (n_fallback) *n_fallback += nfb;
    for (int64_t l = 0; l < nl; ++l) {
        int nf = lnode[l], ip = ldir[l];
        real_t v = val[l];
        real_t uwx = luw ? luw[2 * l] : 0.0, uwy = luw ? luw[2 * l + 1] : 0.0;
        if (link_out) link_out[l] = v;
        /* momentum exchange: the population f+_{i'} carried into the wall and the
         * returning f_i both push the solid along e_{i'}.  With gi_mea, the
         * Galilean-invariant form of Wen, Zhang, Tu, Wang & Fang (J. Comput. Phys.
         * 266, 2014): the momenta are taken relative to the wall,
         * (e_{i'} - u_w) f+_{i'} - (e_i - u_w) f_i, which adds
         * -u_w (f+_{i'} - f_i) to the plain form. */
        int o = lobj ? lobj[l] : 0;
        if (force) {
            real_t fin = fp[9 * nf + ip];
            real_t fx = EX[ip] * (fin + v), fy = EY[ip] * (fin + v);
            if (p->gi_mea) {
                fx -= uwx * (fin - v);
                fy -= uwy * (fin - v);
            }
            force[2 * o] += fx;
            force[2 * o + 1] += fy;
        }
    }

    /* 3-4. pull streaming then collision at every interior fluid node */
    int status = 0;
    if (p->collision == 1) mrt_inverse(); /* before the parallel loop */
#ifdef _OPENMP
#pragma omp parallel for schedule(static) reduction(min : status)
#endif
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            int n = y * nx + x;
            if (solid[n]) continue;
            if (p->x_open && (x == 0 || x == nx - 1)) continue;
            real_t f[9];
            for (int i = 0; i < 9; ++i) {
                int xs = (x - EX[i] + nx) % nx, ys = (y - EY[i] + ny) % ny;
                int ns = ys * nx + xs;
                if (!solid[ns]) {
                    f[i] = fp[9 * ns + i];
                } else if (have[9 * n + i]) {
                    f[i] = fbc[9 * n + i];
                } else {
                    f[i] = 0;
                    status = -2;
                }
            }
            collide_node(p, f);
            for (int i = 0; i < 9; ++i) fnew[9 * n + i] = f[i];
        }
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
    for (int n = 0; n < N; ++n) {
        int x = n % nx;
        if (solid[n] || (p->x_open && (x == 0 || x == nx - 1))) continue;
        for (int i = 0; i < 9; ++i) fp[9 * n + i] = fnew[9 * n + i];
    }

    /* 5. open columns (Section 4.3): non-equilibrium extrapolation velocity inlet
     * at x = 0 and a zero-gradient outlet at x = nx-1 that copies every
     * population from the nearest fluid column.  reading: both act on the
     * post-collision populations of the new time level; a column node is updated
     * only if it and its neighbour column node are fluid. */
    if (p->x_open) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static)
#endif
        for (int y = 0; y < ny; ++y) {
            int n0 = y * nx, n1 = y * nx + 1;
            if (!solid[n0] && !solid[n1]) {
                real_t rho1, u1x, u1y;
                moments_post(fp + 9 * n1, p->gx, p->gy, &rho1, &u1x, &u1y);
                for (int i = 0; i < 9; ++i)
                    fp[9 * n0 + i] = ORC(equilibrium)(i, rho1, uin[2 * y], uin[2 * y + 1]) +
                                     (fp[9 * n1 + i] - ORC(equilibrium)(i, rho1, u1x, u1y));
            }
            int ne = y * nx + nx - 1, nw = y * nx + nx - 2;
            if (!solid[ne] && !solid[nw])
                for (int i = 0; i < 9; ++i) fp[9 * ne + i] = fp[9 * nw + i];
        }
    }
    return status;
}

int ORC(step)(const orc_params *p, const uint8_t *solid, int64_t nl, const int32_t *lnode,
              const int8_t *ldir, const real_t *lq, const real_t *luw, const int32_t *lobj,
              const int8_t *lscheme, const real_t *uin, real_t *fp, real_t *force,
              int64_t *n_fallback, real_t *link_out)
{
    orc_work w = {NULL, NULL, NULL, NULL};
    if (!work_alloc(&w, p->nx, p->ny, nl)) {
        work_free(&w);
        return -3;
    }
    int st = step_work(p, solid, nl, lnode, ldir, lq, luw, lobj, lscheme, uin, fp, force, n_fallback, link_out,
                       &w);
    work_free(&w);
    return st;
}

/* nsteps steps; force_hist (nsteps*n_obj*2, may be NULL) receives the force of
 * every step, force_sum (n_obj*2, may be NULL) accumulates over all steps.
 * Returns 0, -2 as ORC(step), or -3 if the scratch could not be allocated. */
int ORC(run)(const orc_params *p, const uint8_t *solid, int64_t nl, const int32_t *lnode,
             const int8_t *ldir, const real_t *lq, const real_t *luw, const int32_t *lobj,
             const int8_t *lscheme, const real_t *uin, real_t *fp, int64_t nsteps,
             real_t *force_hist, real_t *force_sum, int64_t *n_fallback)
{
    int no = p->n_obj > 0 ? p->n_obj : 1;
    real_t *fs = (real_t *)malloc(sizeof(real_t) * 2 * no);
    orc_work w = {NULL, NULL, NULL, NULL};
    if (!fs || !work_alloc(&w, p->nx, p->ny, nl)) {
        free(fs);
        work_free(&w);
        return -3;
    }
    int st = 0;
    for (int64_t t = 0; t < nsteps && !st; ++t) {
        for (int k = 0; k < 2 * no; ++k) fs[k] = 0;
        st = step_work(p, solid, nl, lnode, ldir, lq, luw, lobj, lscheme, uin, fp, fs, t == 0 ? n_fallback : NULL,
                       NULL, &w);
        if (st) break;
        for (int k = 0; k < 2 * no; ++k) {
            if (force_hist) force_hist[t * 2 * no + k] = fs[k];
            if (force_sum) force_sum[k] += fs[k];
        }
    }
    free(fs);
    work_free(&w);
    return st;
}

/* total mass sum_{fluid nodes} sum_i f_i */
real_t ORC(mass)(int nx, int ny, const uint8_t *solid, const real_t *fp)
{
    real_t m = 0;
    for (int n = 0; n < nx * ny; ++n)
        if (!solid[n])
            for (int i = 0; i < 9; ++i) m += fp[9 * n + i];
    return m;
}

/* velocity set and weights, exported for the tests that pin them */
void ORC(lattice)(int32_t *ex, int32_t *ey, double *w, int32_t *opp)
{
    for (int i = 0; i < 9; ++i) {
        ex[i] = EX[i];
        ey[i] = EY[i];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}
