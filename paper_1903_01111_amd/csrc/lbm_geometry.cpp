// Host geometry: solid mask and fluid->solid links with wall fractions q from a
// union of discs, disc complements and half-planes (arXiv:1903.01111, Section 3:
// node classification and q = |x_f - x_w| / |x_f - x_s|).
//
// Nodes sit at integer coordinates; a node is solid when any primitive holds it
// (a node exactly on a circle is solid).  A link (x_f, i') is emitted for each
// fluid node x_f that is streamed and each direction whose neighbour
// x_s = x_f + e_{i'} is solid.  q is the smallest fraction s in (0, 1] at which
// x_f + s e_{i'} enters a primitive that holds x_s.  Circle roots are taken in
// the cancellation-free form.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "lbm.h"

extern "C" void lbm_set_thread_error(const char *msg);

namespace {

constexpr int EXG[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EYG[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

struct Prim {
    int kind;
    double cx, cy, r, ux, uy, om;
    int obj;
};

// offset d - c folded into [-n/2, n/2) along a periodic direction
double fold(double d, int n, bool periodic)
{
    if (!periodic) return d;
    return d - n * std::floor(d / n + 0.5);
}

bool holds(const Prim &p, double x, double y, int nx, int ny, bool px)
{
    switch (p.kind) {
    case LBM_PRIM_DISC:
    case LBM_PRIM_RING: {
        const double dx = fold(x - p.cx, nx, px), dy = fold(y - p.cy, ny, true);
        const double rr = dx * dx + dy * dy, R2 = p.r * p.r;
        return p.kind == LBM_PRIM_DISC ? rr <= R2 : rr >= R2;
    }
    case LBM_PRIM_BELOW: return y <= p.cy;
    default: return y >= p.cy;
    }
}

// fraction s at which x_f + s e enters the solid side of p; also the wall point
// relative to the centre (for the spin velocity)
double entry(const Prim &p, int x, int y, int ex, int ey, int nx, int ny, bool px, double *rx,
             double *ry)
{
    if (p.kind == LBM_PRIM_BELOW || p.kind == LBM_PRIM_ABOVE) {
        *rx = *ry = 0.0;
        return (p.cy - y) / ey;
    }
    const double dx = fold(x - p.cx, nx, px), dy = fold(y - p.cy, ny, true);
    const double a = ex * ex + ey * ey, b = dx * ex + dy * ey;
    const double k = dx * dx + dy * dy - p.r * p.r;  // > 0 outside the circle
    const double sq = std::sqrt(std::fmax(b * b - a * k, 0.0));
    double s;
    if (p.kind == LBM_PRIM_DISC) {
        // entering the disc from outside: smaller root (-b - sq)/a = k/(-b + sq)
        s = k / (-b + sq);
    } else {
        // leaving the disc from inside: larger root (-b + sq)/a
        s = b <= 0.0 ? (-b + sq) / a : -k / (b + sq);
    }
    *rx = dx + s * ex;
    *ry = dy + s * ey;
    return s;
}

}  // namespace

extern "C" lbm_status lbm_geometry(int32_t nx, int32_t ny, int32_t x_bc, int32_t n_prim,
                                   const int32_t *kind, const double *geo, const double *motion,
                                   const int32_t *prim_obj, uint8_t *mask_out, int64_t max_links,
                                   int32_t *node, int8_t *dir, double *q, double *uw, int32_t *obj,
                                   int64_t *n_links_out)
{
    return lbm_geometry_ex(nx, ny, x_bc, n_prim, kind, geo, motion, prim_obj, mask_out, max_links, node,
                           dir, q, uw, obj, nullptr, nullptr, n_links_out);
}

extern "C" lbm_status lbm_geometry_ex(int32_t nx, int32_t ny, int32_t x_bc, int32_t n_prim,
                                      const int32_t *kind, const double *geo, const double *motion,
                                      const int32_t *prim_obj, uint8_t *mask_out, int64_t max_links,
                                      int32_t *node, int8_t *dir, double *q, double *uw, int32_t *obj,
                                      int32_t *prim, double *dq, int64_t *n_links_out)
{
    if (nx < 1 || ny < 1 || (int64_t)nx * ny > ((int64_t)1 << 31) - 1 || n_prim < 0 ||
        (n_prim > 0 && (!kind || !geo)) || !mask_out || !n_links_out ||
        (x_bc != LBM_X_PERIODIC && x_bc != LBM_X_OPEN)) {
        lbm_set_thread_error("lbm_geometry: invalid size or null argument");
        return LBM_E_ARG;
    }
    std::vector<Prim> P(n_prim);
    for (int k = 0; k < n_prim; ++k) {
        if (kind[k] < LBM_PRIM_DISC || kind[k] > LBM_PRIM_ABOVE || !std::isfinite(geo[3 * k]) ||
            !std::isfinite(geo[3 * k + 1]) || !std::isfinite(geo[3 * k + 2]) ||
            ((kind[k] == LBM_PRIM_DISC || kind[k] == LBM_PRIM_RING) && !(geo[3 * k + 2] > 0.0))) {
            char m[128];
            std::snprintf(m, sizeof m, "lbm_geometry: invalid primitive %d", k);
            lbm_set_thread_error(m);
            return LBM_E_ARG;
        }
        P[k] = {kind[k], geo[3 * k], geo[3 * k + 1], geo[3 * k + 2],
                motion ? motion[3 * k] : 0.0, motion ? motion[3 * k + 1] : 0.0,
                motion ? motion[3 * k + 2] : 0.0, prim_obj ? prim_obj[k] : 0};
    }
    const bool px = x_bc == LBM_X_PERIODIC;
    // node classification; discs only visit their bounding box.  owner[n] is the
    // primitive holding node n, or -2 when several do (then all are scanned).
    const int64_t N = (int64_t)nx * ny;
    std::vector<int32_t> owner((size_t)N, -1);
    for (int64_t n = 0; n < N; ++n) mask_out[n] = 0;
    auto mark = [&](int k, int x, int y) {
        const int64_t n = (int64_t)y * nx + x;
        if (owner[n] == k) return;
        mask_out[n] = 1;
        owner[n] = owner[n] == -1 ? k : -2;
    };
    for (int k = 0; k < n_prim; ++k) {
        const Prim &p = P[k];
        if (p.kind == LBM_PRIM_DISC) {
            const int x0 = (int)std::floor(p.cx - p.r) - 1, x1 = (int)std::ceil(p.cx + p.r) + 1;
            const int y0 = (int)std::floor(p.cy - p.r) - 1, y1 = (int)std::ceil(p.cy + p.r) + 1;
            for (int yy = y0; yy <= y1; ++yy)
                for (int xx = x0; xx <= x1; ++xx) {
                    int x = xx;
                    const int y = ((yy % ny) + ny) % ny;
                    if (px) x = ((xx % nx) + nx) % nx;
                    else if (xx < 0 || xx >= nx) continue;
                    if (holds(p, x, y, nx, ny, px)) mark(k, x, y);
                }
        } else {
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x)
                    if (holds(p, x, y, nx, ny, px)) mark(k, x, y);
        }
    }
    // links; q from the primitive(s) that hold x_s
    int64_t count = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (mask_out[(int64_t)y * nx + x]) continue;
            if (!px && (x == 0 || x == nx - 1)) continue;
            for (int ip = 1; ip < 9; ++ip) {
                int xs = x + EXG[ip];
                const int ys = (y + EYG[ip] + ny) % ny;
                if (px) xs = (xs + nx) % nx;
                if (!mask_out[(int64_t)ys * nx + xs]) continue;
                if (count < max_links) {
                    const int32_t own = owner[(int64_t)ys * nx + xs];
                    const int k0 = own >= 0 ? own : 0, k1 = own >= 0 ? own + 1 : n_prim;
                    double best = 2.0, brx = 0.0, bry = 0.0;
                    int bp = -1;
                    for (int k = k0; k < k1; ++k) {
                        if (!holds(P[k], xs, ys, nx, ny, px)) continue;
                        double rx, ry;
                        const double s = entry(P[k], x, y, EXG[ip], EYG[ip], nx, ny, px, &rx, &ry);
                        if (bp < 0 || s < best) {
                            best = s;
                            bp = k;
                            brx = rx;
                            bry = ry;
                        }
                    }
                    const Prim &p = P[bp];
                    node[count] = y * nx + x;
                    dir[count] = (int8_t)ip;
                    q[count] = best;
                    uw[2 * count] = p.ux - p.om * bry;
                    uw[2 * count + 1] = p.uy + p.om * brx;
                    obj[count] = p.obj;
                    if (prim) prim[count] = bp;
                    if (dq) {
                        // derivatives of q with respect to (cx, cy, r) of the primitive, from
                        // |x_f + q e - c| = r (circles: with p = x_w - c, dq/dc = p/(p.e),
                        // dq/dr = +-r/(p.e)) or x_f.y + q e.y = cy (lines: dq/dcy = 1/e.y)
                        double *d = dq + 3 * count;
                        if (p.kind == LBM_PRIM_DISC || p.kind == LBM_PRIM_RING) {
                            const double pe = brx * EXG[ip] + bry * EYG[ip];
                            d[0] = brx / pe;
                            d[1] = bry / pe;
                            d[2] = p.r / pe;
                        } else {
                            d[0] = 0.0;
                            d[1] = 1.0 / EYG[ip];
                            d[2] = 0.0;
                        }
                    }
                }
                ++count;
            }
        }
    *n_links_out = count;
    return LBM_OK;
}
