// Host-side geometry of the directional diffusion splitting method (FP64):
// the bounding-box grid (eq. (20)), the domain, the unit fields b and p
// (Sec. 3), seeding on the inflow sets (eq. (12)), the curve families
// (eq. (13)-(14)), the per-node line-element data (eq. (17), (19)), the gather
// stencils (eq. (21)-(23)) and the crossing-record scatter of Sec. 6.
//
// Readings where the paper is silent: curves are integrated in arc length with
// classical RK4 and step h (the finer grid spacing); a step that leaves the
// closed domain is shortened by 44 bisections and its end projected onto Gamma;
// a last element shorter than 0.1 h is merged into the previous one.  Seeds
// sit at mid-increments h of the measure int |n.b| ds on every connected
// inflow arc (midpoint rule on sub-segments of length <= h/4).  At a grid node
// the scatter takes the plain average of its horizontal and vertical
// estimates; where only one of them is local (both brackets within
// kLocalEdges edges of the node) that one alone.
//
// The interpolation-free transfer (the conclusions' second improvement): the
// segments of the two families are intersected (candidates: the pairs whose
// bounding boxes share a grid cell), and each interior node of a target curve
// takes the linear interpolant, in arc length along its curve, between the
// nearest intersections at or before and at or after it (the curve's end on a
// side without one).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <memory>

#include "adr_internal.h"

namespace adr {
namespace {

constexpr double kCeilTol = 1e-9;
constexpr int kBisect = 44;
constexpr double kMerge = 0.1;
constexpr double kNodeMargin = 1e-9;
constexpr int kLocalEdges = 4;  // a scatter bracket further out is not local

[[noreturn]] void fail(adr_status c, const std::string &m) { throw Error{c, m}; }

// ---------------------------------------------------------------- domains
struct Sub {  // boundary sub-segment
    double x0, y0, x1, y1, xm, ym, nx, ny, len, t0, t1;
};

struct Domain {
    virtual ~Domain() = default;
    virtual bool inside(double x, double y) const = 0;
    virtual double dist(double x, double y) const = 0;
    virtual bool exits(double x0, double y0, double x1, double y1) const = 0;
    virtual void project(double &x, double &y) const = 0;
    virtual double first_hit(double x0, double y0, double x1, double y1) const = 0;
    virtual void subsegments(double h, std::vector<Sub> &out) const = 0;
    virtual void point(const Sub &s, double frac, double &x, double &y) const = 0;
    double perimeter = 0.0;
};

struct Polygon final : Domain {
    std::vector<double> vx, vy;
    bool is_box = false, convex = true;
    int m = 0;
    Polygon(const std::vector<double> &xy, bool box) : is_box(box) {
        m = static_cast<int>(xy.size() / 2);
        for (int q = 0; q < m; ++q) { vx.push_back(xy[2 * q]); vy.push_back(xy[2 * q + 1]); }
        for (int q = 0; q < m; ++q) {
            int r = (q + 1) % m, s = (q + 2) % m;
            double ex = vx[r] - vx[q], ey = vy[r] - vy[q];
            double fx = vx[s] - vx[r], fy = vy[s] - vy[r];
            if (ex * fy - ey * fx < 0) convex = false;
            perimeter += std::hypot(ex, ey);
        }
    }
    bool inside(double x, double y) const override {
        if (is_box) return x > vx[0] && x < vx[2] && y > vy[0] && y < vy[2];
        bool in = false;
        for (int q = 0; q < m; ++q) {
            int r = (q + 1) % m;
            bool cond = (vy[q] > y) != (vy[r] > y);
            if (cond) {
                double xint = vx[q] + (y - vy[q]) * (vx[r] - vx[q]) / (vy[r] - vy[q]);
                if (x < xint) in = !in;
            }
        }
        return in;
    }
    double dist(double x, double y) const override {
        double best = std::numeric_limits<double>::infinity();
        for (int q = 0; q < m; ++q) {
            int r = (q + 1) % m;
            double ex = vx[r] - vx[q], ey = vy[r] - vy[q];
            double t = ((x - vx[q]) * ex + (y - vy[q]) * ey) / (ex * ex + ey * ey);
            t = std::min(1.0, std::max(0.0, t));
            best = std::min(best, std::hypot(x - (vx[q] + t * ex), y - (vy[q] + t * ey)));
        }
        return best;
    }
    bool chord_crosses(double x0, double y0, double x1, double y1) const {
        double dx = x1 - x0, dy = y1 - y0;
        for (int q = 0; q < m; ++q) {
            int r = (q + 1) % m;
            double ex = vx[r] - vx[q], ey = vy[r] - vy[q];
            double den = dx * ey - dy * ex;
            if (den == 0) continue;
            double t = ((vx[q] - x0) * ey - (vy[q] - y0) * ex) / den;
            double u = ((vx[q] - x0) * dy - (vy[q] - y0) * dx) / den;
            if (t > 1e-9 && t <= 1.0 && u >= 0.0 && u <= 1.0) return true;
        }
        return false;
    }
    bool exits(double x0, double y0, double x1, double y1) const override {
        if (!inside(x1, y1)) return true;
        return !convex && chord_crosses(x0, y0, x1, y1);
    }
    void project(double &x, double &y) const override {
        double best = std::numeric_limits<double>::infinity(), px = x, py = y;
        for (int q = 0; q < m; ++q) {
            int r = (q + 1) % m;
            double ex = vx[r] - vx[q], ey = vy[r] - vy[q];
            double t = ((x - vx[q]) * ex + (y - vy[q]) * ey) / (ex * ex + ey * ey);
            t = std::min(1.0, std::max(0.0, t));
            double cx = vx[q] + t * ex, cy = vy[q] + t * ey;
            double dd = std::hypot(x - cx, y - cy);
            if (dd < best) { best = dd; px = cx; py = cy; }
        }
        x = px; y = py;
    }
    double first_hit(double x0, double y0, double x1, double y1) const override {
        double best = 1.0, dx = x1 - x0, dy = y1 - y0;
        for (int q = 0; q < m; ++q) {
            int r = (q + 1) % m;
            double ex = vx[r] - vx[q], ey = vy[r] - vy[q];
            double den = dx * ey - dy * ex;
            if (den == 0) continue;
            double t = ((vx[q] - x0) * ey - (vy[q] - y0) * ex) / den;
            double u = ((vx[q] - x0) * dy - (vy[q] - y0) * dx) / den;
            if (t > 0.0 && t <= 1.0 && u >= 0.0 && u <= 1.0 && t < best) best = t;
        }
        return best;
    }
    void subsegments(double h, std::vector<Sub> &out) const override {
        for (int q = 0; q < m; ++q) {
            int r = (q + 1) % m;
            double ell = std::hypot(vx[r] - vx[q], vy[r] - vy[q]);
            int K = std::max(1, static_cast<int>(std::ceil(ell / (0.25 * h) - kCeilTol)));
            double nxo = (vy[r] - vy[q]) / ell, nyo = -(vx[r] - vx[q]) / ell;
            for (int k = 0; k < K; ++k) {
                double s0 = static_cast<double>(k) / K, s1 = static_cast<double>(k + 1) / K;
                Sub s;
                s.x0 = vx[q] + s0 * (vx[r] - vx[q]); s.y0 = vy[q] + s0 * (vy[r] - vy[q]);
                s.x1 = vx[q] + s1 * (vx[r] - vx[q]); s.y1 = vy[q] + s1 * (vy[r] - vy[q]);
                s.xm = 0.5 * (s.x0 + s.x1); s.ym = 0.5 * (s.y0 + s.y1);
                s.nx = nxo; s.ny = nyo; s.len = ell / K; s.t0 = s.t1 = 0.0;
                out.push_back(s);
            }
        }
    }
    void point(const Sub &s, double frac, double &x, double &y) const override {
        x = s.x0 + frac * (s.x1 - s.x0);
        y = s.y0 + frac * (s.y1 - s.y0);
    }
};

struct Disc final : Domain {
    double cx, cy, r;
    Disc(double a, double b, double c) : cx(a), cy(b), r(c) { perimeter = 2.0 * M_PI * r; }
    bool inside(double x, double y) const override {
        return (x - cx) * (x - cx) + (y - cy) * (y - cy) < r * r;
    }
    double dist(double x, double y) const override { return std::fabs(r - std::hypot(x - cx, y - cy)); }
    bool exits(double, double, double x1, double y1) const override { return !inside(x1, y1); }
    void project(double &x, double &y) const override {
        double dx = x - cx, dy = y - cy, rho = std::hypot(dx, dy);
        x = cx + r * dx / rho;
        y = cy + r * dy / rho;
    }
    double first_hit(double x0, double y0, double x1, double y1) const override {
        double dx = x1 - x0, dy = y1 - y0, px = x0 - cx, py = y0 - cy;
        double A = dx * dx + dy * dy, B = px * dx + py * dy, C = px * px + py * py - r * r;
        double disc = std::max(B * B - A * C, 0.0);
        double t = (-B + std::sqrt(disc)) / A;
        return std::min(1.0, std::max(0.0, t));
    }
    void subsegments(double h, std::vector<Sub> &out) const override {
        int K = std::max(1, static_cast<int>(std::ceil(perimeter / (0.25 * h) - kCeilTol)));
        for (int k = 0; k < K; ++k) {
            Sub s;
            s.t0 = 2.0 * M_PI * k / K;
            s.t1 = 2.0 * M_PI * (k + 1) / K;
            double tm = 0.5 * (s.t0 + s.t1);
            s.x0 = cx + r * std::cos(s.t0); s.y0 = cy + r * std::sin(s.t0);
            s.x1 = cx + r * std::cos(s.t1); s.y1 = cy + r * std::sin(s.t1);
            s.xm = cx + r * std::cos(tm); s.ym = cy + r * std::sin(tm);
            s.nx = std::cos(tm); s.ny = std::sin(tm);
            s.len = r * 2.0 * M_PI / K;
            out.push_back(s);
        }
    }
    void point(const Sub &s, double frac, double &x, double &y) const override {
        double t = s.t0 + frac * (s.t1 - s.t0);
        x = cx + r * std::cos(t);
        y = cy + r * std::sin(t);
    }
};

// ---------------------------------------------------------------- flow field
struct Flow {
    const Grid *g;
    const double *B1, *B2;
    // unit direction b (family 0) or p = (b2, -b1) (family 1)
    void unit(double x, double y, int fam, double &ux, double &uy) const {
        double b1 = g->interp(B1, x, y), b2 = g->interp(B2, x, y);
        double n = std::hypot(b1, b2);
        if (!(n > 0.0)) fail(ADR_EBETA, "|beta| vanishes on a curve: direction b undefined");
        b1 /= n; b2 /= n;
        if (fam == 0) { ux = b1; uy = b2; } else { ux = b2; uy = -b1; }
    }
    void rk4(double x, double y, double s, int fam, double &ox, double &oy) const {
        double k1x, k1y, k2x, k2y, k3x, k3y, k4x, k4y;
        unit(x, y, fam, k1x, k1y);
        unit(x + 0.5 * s * k1x, y + 0.5 * s * k1y, fam, k2x, k2y);
        unit(x + 0.5 * s * k2x, y + 0.5 * s * k2y, fam, k3x, k3y);
        unit(x + s * k3x, y + s * k3y, fam, k4x, k4y);
        ox = x + s / 6.0 * (k1x + 2.0 * k2x + 2.0 * k3x + k4x);
        oy = y + s / 6.0 * (k1y + 2.0 * k2y + 2.0 * k3y + k4y);
    }
};

// Seeds on the inflow set of family fam (eq. (12)).
void make_seeds(const Flow &fl, const Domain &dom, int fam, double hperp, std::vector<double> &sx,
                std::vector<double> &sy) {
    std::vector<Sub> sub;
    dom.subsegments(fl.g->h, sub);
    const int K = static_cast<int>(sub.size());
    std::vector<double> w(K);
    bool any = false, all = true;
    for (int s = 0; s < K; ++s) {
        double ux, uy;
        fl.unit(sub[s].xm, sub[s].ym, fam, ux, uy);
        double q = std::max(0.0, -(sub[s].nx * ux + sub[s].ny * uy));
        w[s] = q * sub[s].len;
        if (w[s] > 0) any = true; else all = false;
    }
    if (!any) return;
    if (all) fail(ADR_EBETA, "the whole boundary is an inflow boundary");
    int start = 0;
    while (w[start] > 0) ++start;
    std::vector<int> run;
    auto flush = [&]() {
        if (run.empty()) return;
        std::vector<double> cum(run.size());
        double acc = 0.0;
        for (size_t t = 0; t < run.size(); ++t) { acc += w[run[t]]; cum[t] = acc; }
        const double lam = acc;
        const int n = static_cast<int>(std::floor(lam / hperp + 0.5));
        for (int k = 0; k < n; ++k) {
            double target = (k + 0.5) * lam / n;
            size_t r = std::lower_bound(cum.begin(), cum.end(), target) - cum.begin();
            if (r >= run.size()) r = run.size() - 1;
            double before = r > 0 ? cum[r - 1] : 0.0;
            double frac = (target - before) / w[run[r]];
            double px, py;
            dom.point(sub[run[r]], frac, px, py);
            sx.push_back(px);
            sy.push_back(py);
        }
        run.clear();
    };
    for (int t = 0; t < K; ++t) {
        int s = (start + t) % K;
        if (w[s] > 0) run.push_back(s); else flush();
    }
    flush();
}

// Integral curves from the seeds (eq. (13)-(14)).
void trace(const Flow &fl, const Domain &dom, const std::vector<double> &sx, const std::vector<double> &sy,
           int fam, double hl, Family &out) {
    const int64_t max_steps = static_cast<int64_t>(std::ceil(4.0 * dom.perimeter / hl)) + 2;
    out.off.assign(1, 0);
    std::vector<double> lx, ly;
    for (size_t s = 0; s < sx.size(); ++s) {
        lx.assign(1, sx[s]);
        ly.assign(1, sy[s]);
        double cx = sx[s], cy = sy[s];
        bool closed = false;
        for (int64_t step = 0; step < max_steps; ++step) {
            double nx, ny;
            fl.rk4(cx, cy, hl, fam, nx, ny);
            if (!dom.exits(cx, cy, nx, ny)) {
                lx.push_back(nx); ly.push_back(ny);
                cx = nx; cy = ny;
                continue;
            }
            double lo = 0.0, hi = hl;
            for (int it = 0; it < kBisect; ++it) {
                double mid = 0.5 * (lo + hi), mx, my;
                fl.rk4(cx, cy, mid, fam, mx, my);
                if (dom.exits(cx, cy, mx, my)) hi = mid; else lo = mid;
            }
            double ex, ey;
            fl.rk4(cx, cy, hi, fam, ex, ey);
            dom.project(ex, ey);
            if (std::hypot(ex - cx, ey - cy) < kMerge * hl && lx.size() >= 2) {
                lx.back() = ex; ly.back() = ey;
            } else {
                lx.push_back(ex); ly.push_back(ey);
            }
            closed = true;
            break;
        }
        if (!closed) fail(ADR_EBETA, "a curve did not leave the domain within four perimeters");
        if (lx.size() < 3) continue;  // no interior node
        out.x.insert(out.x.end(), lx.begin(), lx.end());
        out.y.insert(out.y.end(), ly.begin(), ly.end());
        out.off.push_back(static_cast<int64_t>(out.x.size()));
    }
}

// ---------------------------------------------------------------- scatter
struct Crossing {
    double coord;  // coordinate along the grid line
    int64_t k;     // first node of the segment
    double t;      // (1-t) v[k] + t v[k+1]
};

struct Bracket {
    int kind;      // 0 line record, 1 boundary point
    double coord;
    int64_t k;
    double t;
    int depth;     // edges from the node to the edge holding the bracket (1 = own edge)
};

// gdata: nodal Dirichlet data (NULL: zero); a boundary point's share of a node's
// value is summed into the stencil's gb.
void build_scatter(const Grid &g, const Domain &dom, const std::vector<uint8_t> &inner,
                   const std::vector<int32_t> &inner_list, const Family &F, const double *gdata,
                   std::vector<Rec4> &out) {
    const int nx = g.nx, ny = g.ny;
    // edges of vertical grid lines: line i, edge j (ny-1 per line); horizontal: line j, edge i
    const int64_t nvE = static_cast<int64_t>(nx) * (ny - 1), nhE = static_cast<int64_t>(ny) * (nx - 1);
    std::vector<int64_t> vmin(nvE, -1), vmax(nvE, -1), hmin(nhE, -1), hmax(nhE, -1);
    std::vector<Crossing> vrec, hrec;
    const int nl = static_cast<int>(F.off.size()) - 1;
    for (int axis = 0; axis < 2; ++axis) {
        std::vector<Crossing> &rec = axis == 0 ? vrec : hrec;
        std::vector<int64_t> &emin = axis == 0 ? vmin : hmin, &emax = axis == 0 ? vmax : hmax;
        const double org = axis == 0 ? g.a : g.c, hh = axis == 0 ? g.hx : g.hy;
        const double qorg = axis == 0 ? g.c : g.a, qh = axis == 0 ? g.hy : g.hx;
        const int nlines = axis == 0 ? nx : ny, nedges = axis == 0 ? ny - 1 : nx - 1;
        for (int l = 0; l < nl; ++l) {
            for (int64_t k = F.off[l]; k + 1 < F.off[l + 1]; ++k) {
                double p0 = axis == 0 ? F.x[k] : F.y[k], p1 = axis == 0 ? F.x[k + 1] : F.y[k + 1];
                double q0 = axis == 0 ? F.y[k] : F.x[k], q1 = axis == 0 ? F.y[k + 1] : F.x[k + 1];
                if (p0 == p1) continue;
                long lo = static_cast<long>(std::floor((std::min(p0, p1) - org) / hh)) - 1;
                long hi = static_cast<long>(std::ceil((std::max(p0, p1) - org) / hh)) + 1;
                lo = std::max(0L, std::min<long>(lo, nlines - 1));
                hi = std::max(0L, std::min<long>(hi, nlines - 1));
                for (long c = lo; c <= hi; ++c) {
                    double gl = org + hh * c;
                    if ((gl - p0) * (gl - p1) > 0.0) continue;
                    double t = (gl - p0) / (p1 - p0);
                    double coord = q0 + t * (q1 - q0);
                    long e = static_cast<long>(std::floor((coord - qorg) / qh));
                    e = std::max(0L, std::min<long>(e, nedges - 1));
                    int64_t eid = c * static_cast<int64_t>(nedges) + e;
                    int64_t id = static_cast<int64_t>(rec.size());
                    rec.push_back({coord, k, t});
                    if (emin[eid] < 0 || coord < rec[emin[eid]].coord) emin[eid] = id;
                    if (emax[eid] < 0 || coord >= rec[emax[eid]].coord) emax[eid] = id;
                }
            }
        }
    }
    out.resize(inner_list.size());
    auto is_in = [&](int i, int j) { return inner[static_cast<size_t>(j) * nx + i] != 0; };
    for (size_t n = 0; n < inner_list.size(); ++n) {
        const int gi = inner_list[n] % nx, gj = inner_list[n] / nx;
        Bracket br[2][2];  // [direction: 0 horizontal, 1 vertical][side: 0 low, 1 high]
        for (int dir = 0; dir < 2; ++dir) {
            // dir 0: along row gj (positions i, edges (e, e+1) on horizontal line gj)
            // dir 1: along column gi
            const int pos = dir == 0 ? gi : gj;
            const int nE = dir == 0 ? nx - 1 : ny - 1;
            const std::vector<int64_t> &emin = dir == 0 ? hmin : vmin, &emax = dir == 0 ? hmax : vmax;
            const std::vector<Crossing> &rec = dir == 0 ? hrec : vrec;
            const int64_t base = static_cast<int64_t>(dir == 0 ? gj : gi) * nE;
            auto node_in = [&](int p) { return dir == 0 ? is_in(p, gj) : is_in(gi, p); };
            auto coord_of = [&](int p) { return dir == 0 ? g.x(p) : g.y(p); };
            auto boundary = [&](int nearp, int farp) {
                double x0 = dir == 0 ? g.x(nearp) : g.x(gi), y0 = dir == 0 ? g.y(gj) : g.y(nearp);
                double x1 = dir == 0 ? g.x(farp) : g.x(gi), y1 = dir == 0 ? g.y(gj) : g.y(farp);
                double t = dom.first_hit(x0, y0, x1, y1);
                return dir == 0 ? x0 + t * (x1 - x0) : y0 + t * (y1 - y0);
            };
            // low side: edges e = pos-1, pos-2, ...
            bool found = false;
            for (int e = pos - 1; e >= 0 && !found; --e) {
                int64_t r = emax[base + e];
                if (r >= 0) {
                    br[dir][0] = {0, rec[r].coord, rec[r].k, rec[r].t, pos - e};
                    found = true;
                } else if (!node_in(e)) {
                    br[dir][0] = {1, boundary(e + 1, e), -1, 0.0, pos - e};
                    found = true;
                }
            }
            if (!found) fail(ADR_EINVAL, "interior grid node without a bracketing record");
            found = false;
            for (int e = pos; e < nE && !found; ++e) {
                int64_t r = emin[base + e];
                if (r >= 0) {
                    br[dir][1] = {0, rec[r].coord, rec[r].k, rec[r].t, e - pos + 1};
                    found = true;
                } else if (!node_in(e + 1)) {
                    br[dir][1] = {1, boundary(e, e + 1), -1, 0.0, e - pos + 1};
                    found = true;
                }
            }
            if (!found) fail(ADR_EINVAL, "interior grid node without a bracketing record");
            (void)coord_of;
        }
        // Sec. 6: the node value is the average of the two estimates. An
        // estimate whose bracket lies beyond the kLocalEdges nearest edges is
        // not local (curves along a grid line); where only one estimate is
        // local it is used alone.
        double cl[2], cr[2];
        bool local[2];
        for (int dir = 0; dir < 2; ++dir) {
            double p = dir == 0 ? g.x(gi) : g.y(gj);
            double dL = p - br[dir][0].coord, dR = br[dir][1].coord - p;
            double span = dL + dR;
            if (span > 0) { cl[dir] = dR / span; cr[dir] = dL / span; }
            else { cl[dir] = 0.5; cr[dir] = 0.5; }
            local[dir] = br[dir][0].depth <= kLocalEdges && br[dir][1].depth <= kLocalEdges;
        }
        const double Wh = local[0] == local[1] ? 0.5 : (local[0] ? 1.0 : 0.0);
        const double Ws[2] = {Wh, 1.0 - Wh};
        Rec4 &R = out[n];
        R.gb = 0.0;
        R.wh = Wh;
        R.lam[0] = cl[0];
        R.lam[1] = cl[1];
        for (int dir = 0; dir < 2; ++dir) {
            for (int side = 0; side < 2; ++side) {
                int slot = dir * 2 + side;
                const Bracket &b = br[dir][side];
                double coef = Ws[dir] * (side == 0 ? cl[dir] : cr[dir]);
                if (b.kind == 0) {
                    R.k[slot] = static_cast<int32_t>(b.k);
                    R.ca[slot] = coef * (1.0 - b.t);
                    R.cb[slot] = coef * b.t;
                    R.t[slot] = b.t;
                } else {  // boundary point: carries the Dirichlet data there
                    R.k[slot] = -1;
                    R.ca[slot] = 0.0;
                    R.cb[slot] = 0.0;
                    R.t[slot] = 0.0;
                    if (gdata && coef != 0.0) {
                        const double px = dir == 0 ? b.coord : g.x(gi), py = dir == 0 ? g.y(gj) : b.coord;
                        R.gb += coef * g.interp(gdata, px, py);
                    }
                }
            }
        }
    }
}

// beta = (psi_y, -psi_x) at the nodes: central differences inside, the
// second-order one-sided formula (-3 f0 + 4 f1 - f2) / (2 h) on the grid's edges.
void beta_from_psi(const double *psi, int nx, int ny, double hx, double hy, std::vector<double> &b1,
                   std::vector<double> &b2) {
    b1.assign(static_cast<size_t>(nx) * ny, 0.0);
    b2.assign(static_cast<size_t>(nx) * ny, 0.0);
    auto P = [&](int i, int j) { return psi[static_cast<size_t>(j) * nx + i]; };
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double dx, dy;
            if (i == 0) dx = (-3.0 * P(0, j) + 4.0 * P(1, j) - P(2, j)) / (2.0 * hx);
            else if (i == nx - 1) dx = (3.0 * P(nx - 1, j) - 4.0 * P(nx - 2, j) + P(nx - 3, j)) / (2.0 * hx);
            else dx = (P(i + 1, j) - P(i - 1, j)) / (2.0 * hx);
            if (j == 0) dy = (-3.0 * P(i, 0) + 4.0 * P(i, 1) - P(i, 2)) / (2.0 * hy);
            else if (j == ny - 1) dy = (3.0 * P(i, ny - 1) - 4.0 * P(i, ny - 2) + P(i, ny - 3)) / (2.0 * hy);
            else dy = (P(i, j + 1) - P(i, j - 1)) / (2.0 * hy);
            b1[static_cast<size_t>(j) * nx + i] = dy;
            b2[static_cast<size_t>(j) * nx + i] = -dx;
        }
}

bool finite_all(const double *p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

}  // namespace

void Grid::cell(double px, double py, int &i, int &j, double &lx, double &ly) const {
    double X = (px - a) / hx, Y = (py - c) / hy;
    double fi = std::floor(X), fj = std::floor(Y);
    fi = std::min(static_cast<double>(nx - 2), std::max(0.0, fi));
    fj = std::min(static_cast<double>(ny - 2), std::max(0.0, fj));
    i = static_cast<int>(fi);
    j = static_cast<int>(fj);
    lx = X - fi;
    ly = Y - fj;
}

double Grid::interp(const double *F, double px, double py) const {
    int i, j;
    double lx, ly;
    cell(px, py, i, j, lx, ly);
    const double *r0 = F + static_cast<size_t>(j) * nx, *r1 = r0 + nx;
    return (1 - ly) * (1 - lx) * r0[i] + (1 - ly) * lx * r0[i + 1] + ly * (1 - lx) * r1[i] + ly * lx * r1[i + 1];
}

void build_instance(const adr_problem &p, InstanceGeo &G) {
    if (p.nx < 3 || p.ny < 3) fail(ADR_EINVAL, "nx and ny must be >= 3");
    if (!(p.b > p.a) || !(p.d > p.c)) fail(ADR_EINVAL, "empty bounding box");
    if (!(p.mu > 0.0)) fail(ADR_EINVAL, "mu must be > 0");
    if (!(p.sigma >= 0.0)) fail(ADR_EINVAL, "sigma must be >= 0");
    if (!p.f) fail(ADR_EINVAL, "f is required");
    if ((!p.beta1 || !p.beta2) && !(!p.beta1 && !p.beta2 && p.psi))
        fail(ADR_EINVAL, "give beta1 and beta2, or psi with both beta arrays NULL");
    const size_t nn = static_cast<size_t>(p.nx) * p.ny;
    if (nn > (1u << 30)) fail(ADR_EINVAL, "grid too large");
    std::vector<double> b1v, b2v;
    const double *beta1 = p.beta1, *beta2 = p.beta2;
    if (!beta1) {
        if (!finite_all(p.psi, nn)) fail(ADR_ENONFINITE, "non-finite psi");
        beta_from_psi(p.psi, p.nx, p.ny, (p.b - p.a) / (p.nx - 1), (p.d - p.c) / (p.ny - 1), b1v, b2v);
        beta1 = b1v.data();
        beta2 = b2v.data();
    }
    if (!finite_all(beta1, nn) || !finite_all(beta2, nn) || !finite_all(p.f, nn))
        fail(ADR_ENONFINITE, "non-finite beta or f");
    if (p.g && !finite_all(p.g, nn)) fail(ADR_ENONFINITE, "non-finite g");
    Grid &g = G.g;
    g.a = p.a; g.b = p.b; g.c = p.c; g.d = p.d; g.nx = p.nx; g.ny = p.ny;
    g.hx = (p.b - p.a) / (p.nx - 1);
    g.hy = (p.d - p.c) / (p.ny - 1);
    g.h = std::min(g.hx, g.hy);
    G.mu = p.mu;
    G.sigma = p.sigma;

    std::unique_ptr<Domain> dom;
    if (p.domain == ADR_DOM_BOX) {
        dom.reset(new Polygon({p.a, p.c, p.b, p.c, p.b, p.d, p.a, p.d}, true));
    } else if (p.domain == ADR_DOM_DISC) {
        if (p.n_dom_params != 3 || !p.dom_params || !(p.dom_params[2] > 0))
            fail(ADR_EINVAL, "disc needs cx, cy, r > 0");
        dom.reset(new Disc(p.dom_params[0], p.dom_params[1], p.dom_params[2]));
    } else if (p.domain == ADR_DOM_POLYGON) {
        if (p.n_dom_params < 6 || (p.n_dom_params % 2) || !p.dom_params)
            fail(ADR_EINVAL, "polygon needs >= 3 vertices");
        dom.reset(new Polygon(std::vector<double>(p.dom_params, p.dom_params + p.n_dom_params), false));
    } else {
        fail(ADR_EINVAL, "unknown domain kind");
    }

    G.inner.assign(nn, 0);
    G.inner_list.clear();
    for (int j = 0; j < p.ny; ++j)
        for (int i = 0; i < p.nx; ++i) {
            double x = g.x(i), y = g.y(j);
            if (dom->inside(x, y) && dom->dist(x, y) > kNodeMargin * g.h) {
                G.inner[static_cast<size_t>(j) * p.nx + i] = 1;
                G.inner_list.push_back(j * p.nx + i);
            }
        }

    Flow fl{&g, beta1, beta2};
    for (int fam = 0; fam < 2; ++fam) {
        std::vector<double> sx, sy;
        make_seeds(fl, *dom, fam, g.h, sx, sy);
        trace(fl, *dom, sx, sy, fam, g.h, G.fam[fam]);
        const Family &F = G.fam[fam];
        if (F.off.size() < 2)
            fail(ADR_EBETA, fam == 0 ? "no beta-curve enters the domain (closed streamlines?)"
                                     : "no gamma-curve enters the domain");
        const size_t n = F.x.size();
        G.hk[fam].assign(n, 0.0);
        G.cellk[fam].assign(n, -1);
        G.lxk[fam].assign(n, 0.0);
        G.lyk[fam].assign(n, 0.0);
        const int nl = static_cast<int>(F.off.size()) - 1;
        for (int l = 0; l < nl; ++l) {
            for (int64_t k = F.off[l]; k < F.off[l + 1]; ++k) {
                if (k > F.off[l]) G.hk[fam][k] = std::hypot(F.x[k] - F.x[k - 1], F.y[k] - F.y[k - 1]);
                if (k > F.off[l] && k + 1 < F.off[l + 1]) {
                    int ci, cj;
                    double lx, ly;
                    g.cell(F.x[k], F.y[k], ci, cj, lx, ly);
                    G.cellk[fam][k] = cj * p.nx + ci;
                    G.lxk[fam][k] = lx;
                    G.lyk[fam][k] = ly;
                }
            }
        }
        if (fam == 0) {
            G.wk.assign(n, 0.0);
            for (size_t k = 0; k < n; ++k) {
                double b1 = g.interp(beta1, F.x[k], F.y[k]), b2 = g.interp(beta2, F.x[k], F.y[k]);
                G.wk[k] = std::hypot(b1, b2);
            }
        }
        build_scatter(g, *dom, G.inner, G.inner_list, F, p.g, G.rec[fam]);
        // Dirichlet data at the curve ends (they lie on Gamma)
        G.gend[fam].assign(2 * (F.off.size() - 1), 0.0);
        if (p.g)
            for (int l = 0; l < nl; ++l) {
                const int64_t k0 = F.off[l], k1 = F.off[l + 1] - 1;
                G.gend[fam][2 * l] = g.interp(p.g, F.x[k0], F.y[k0]);
                G.gend[fam][2 * l + 1] = g.interp(p.g, F.x[k1], F.y[k1]);
            }
    }
    G.has_g = p.g != nullptr;
    compute_load(p, G);
}

void compute_load(const adr_problem &p, InstanceGeo &G) {
    // eq. (17): <l_i, phi_k> with f taken as its P1 interpolant on the beta-curve
    const Grid &g = G.g;
    const Family &F = G.fam[0];
    const size_t n = F.x.size();
    G.mu = p.mu;
    G.sigma = p.sigma;
    G.Lk.assign(n, 0.0);
    std::vector<double> fk(n);
    for (size_t k = 0; k < n; ++k) fk[k] = g.interp(p.f, F.x[k], F.y[k]);
    const int nl = static_cast<int>(F.off.size()) - 1;
    for (int l = 0; l < nl; ++l)
        for (int64_t k = F.off[l] + 1; k + 1 < F.off[l + 1]; ++k) {
            double hl = G.hk[0][k], hr = G.hk[0][k + 1];
            G.Lk[k] = (hl + hr) / 3.0 * fk[k] + hl / 6.0 * fk[k - 1] + hr / 6.0 * fk[k + 1];
        }
}

void load_from_positions(const Grid &g, const Family &F, const double *f, std::vector<double> &L) {
    // same chords and load as compute_load, the chords recomputed from the nodes
    const size_t n = F.x.size();
    L.assign(n, 0.0);
    std::vector<double> fk(n);
    for (size_t k = 0; k < n; ++k) fk[k] = g.interp(f, F.x[k], F.y[k]);
    const int nl = static_cast<int>(F.off.size()) - 1;
    for (int l = 0; l < nl; ++l)
        for (int64_t k = F.off[l] + 1; k + 1 < F.off[l + 1]; ++k) {
            const double hl = std::hypot(F.x[k] - F.x[k - 1], F.y[k] - F.y[k - 1]);
            const double hr = std::hypot(F.x[k + 1] - F.x[k], F.y[k + 1] - F.y[k]);
            L[k] = (hl + hr) / 3.0 * fk[k] + hl / 6.0 * fk[k - 1] + hr / 6.0 * fk[k + 1];
        }
}

void rebuild_for_source(const InstanceGeo &base, const adr_problem &p, InstanceGeo &G) {
    if (!(p.mu > 0.0)) fail(ADR_EINVAL, "mu must be > 0");
    if (!(p.sigma >= 0.0)) fail(ADR_EINVAL, "sigma must be >= 0");
    if (!p.f) fail(ADR_EINVAL, "f is required");
    if (!finite_all(p.f, static_cast<size_t>(p.nx) * p.ny)) fail(ADR_ENONFINITE, "non-finite f");
    G = base;
    compute_load(p, G);
}


// ------------------------------------------------------- direct transfer
namespace {
#pragma clang fp contract(off)
struct Hit {
    int64_t kt;   // first node of the target segment
    double s;     // position on it
    int64_t ks;   // first node of the source segment
    double t;     // position on it
};

void cell_range(double p0, double p1, double org, double h, int n_cells, int &lo, int &hi) {
    lo = static_cast<int>(std::floor((std::min(p0, p1) - org) / h));
    hi = static_cast<int>(std::floor((std::max(p0, p1) - org) / h));
    lo = std::min(std::max(lo, 0), n_cells - 1);
    hi = std::min(std::max(hi, 0), n_cells - 1);
}

std::vector<int64_t> segment_starts(const Family &F) {
    std::vector<int64_t> k;
    const int nl = static_cast<int>(F.off.size()) - 1;
    for (int l = 0; l < nl; ++l)
        for (int64_t q = F.off[l]; q + 1 < F.off[l + 1]; ++q) k.push_back(q);
    return k;
}
}  // namespace

void build_direct(const Grid &g, const Family &tgt, const std::vector<double> &htgt, const Family &src,
                  std::vector<DirRec> &out) {
    const int ncx = g.nx - 1, ncy = g.ny - 1;
    const std::vector<int64_t> kt_all = segment_starts(tgt), ks_all = segment_starts(src);
    // source segments by cell (compressed rows)
    const size_t nsrc = ks_all.size();
    std::vector<int> si0(nsrc), si1(nsrc), sj0(nsrc), sj1(nsrc);
    std::vector<int64_t> cnt(static_cast<size_t>(ncx) * ncy + 1, 0);
    for (size_t e = 0; e < nsrc; ++e) {
        const int64_t k = ks_all[e];
        cell_range(src.x[k], src.x[k + 1], g.a, g.hx, ncx, si0[e], si1[e]);
        cell_range(src.y[k], src.y[k + 1], g.c, g.hy, ncy, sj0[e], sj1[e]);
        for (int j = sj0[e]; j <= sj1[e]; ++j)
            for (int i = si0[e]; i <= si1[e]; ++i) ++cnt[static_cast<size_t>(j) * ncx + i + 1];
    }
    for (size_t c = 1; c < cnt.size(); ++c) cnt[c] += cnt[c - 1];
    std::vector<int> members(static_cast<size_t>(cnt.back()));
    {
        std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
        for (size_t e = 0; e < nsrc; ++e)
            for (int j = sj0[e]; j <= sj1[e]; ++j)
                for (int i = si0[e]; i <= si1[e]; ++i) members[fill[static_cast<size_t>(j) * ncx + i]++] = static_cast<int>(e);
    }
    // intersections per target segment, in target order; within a segment by (s, source segment)
    std::vector<Hit> hits;
    std::vector<Hit> seg_hits;
    for (const int64_t k : kt_all) {
        const double px0 = tgt.x[k], py0 = tgt.y[k], px1 = tgt.x[k + 1], py1 = tgt.y[k + 1];
        int i0, i1, j0, j1;
        cell_range(px0, px1, g.a, g.hx, ncx, i0, i1);
        cell_range(py0, py1, g.c, g.hy, ncy, j0, j1);
        seg_hits.clear();
        for (int j = j0; j <= j1; ++j)
            for (int i = i0; i <= i1; ++i) {
                const size_t c = static_cast<size_t>(j) * ncx + i;
                for (int64_t m = cnt[c]; m < cnt[c + 1]; ++m) {
                    const int e = members[static_cast<size_t>(m)];
                    // each pair once: in the first cell both boxes share
                    if (i != std::max(i0, si0[e]) || j != std::max(j0, sj0[e])) continue;
                    const int64_t q = ks_all[static_cast<size_t>(e)];
                    const double rx = px1 - px0, ry = py1 - py0;
                    const double qx = src.x[q + 1] - src.x[q], qy = src.y[q + 1] - src.y[q];
                    const double wx = src.x[q] - px0, wy = src.y[q] - py0;
                    const double den = rx * qy - ry * qx;
                    if (den == 0.0) continue;
                    const double sp = (wx * qy - wy * qx) / den;
                    const double tp = (wx * ry - wy * rx) / den;
                    if (sp >= 0.0 && sp <= 1.0 && tp >= 0.0 && tp <= 1.0) seg_hits.push_back(Hit{k, sp, q, tp});
                }
            }
        std::sort(seg_hits.begin(), seg_hits.end(), [](const Hit &x, const Hit &y) {
            return x.s != y.s ? x.s < y.s : x.ks < y.ks;
        });
        hits.insert(hits.end(), seg_hits.begin(), seg_hits.end());
    }
    // arc coordinates of the target nodes and of the intersections
    const size_t nt = tgt.x.size();
    std::vector<double> sig(nt, 0.0);
    const int nl = static_cast<int>(tgt.off.size()) - 1;
    for (int l = 0; l < nl; ++l) {
        double acc = 0.0;
        for (int64_t q = tgt.off[l] + 1; q < tgt.off[l + 1]; ++q) {
            acc = acc + htgt[static_cast<size_t>(q)];
            sig[static_cast<size_t>(q)] = acc;
        }
    }
    out.assign(nt, DirRec{{-1, -1}, {0.0, 0.0, 0.0, 0.0}});
    size_t h0 = 0;
    std::vector<double> xs;
    for (int l = 0; l < nl; ++l) {
        const int64_t a = tgt.off[l], b = tgt.off[l + 1];
        size_t h1 = h0;
        while (h1 < hits.size() && hits[h1].kt < b - 1) ++h1;
        xs.resize(h1 - h0);
        for (size_t e = h0; e < h1; ++e) xs[e - h0] = sig[static_cast<size_t>(hits[e].kt)] + hits[e].s * htgt[static_cast<size_t>(hits[e].kt + 1)];
        const double send = sig[static_cast<size_t>(b - 1)];
        for (int64_t q = a + 1; q < b - 1; ++q) {
            const double sq = sig[static_cast<size_t>(q)];
            const int64_t iL = (std::upper_bound(xs.begin(), xs.end(), sq) - xs.begin()) - 1;  // last <= sq
            const int64_t iR = std::lower_bound(xs.begin(), xs.end(), sq) - xs.begin();          // first >= sq
            const double sL = iL >= 0 ? xs[static_cast<size_t>(iL)] : 0.0;
            const double sR = iR < static_cast<int64_t>(xs.size()) ? xs[static_cast<size_t>(iR)] : send;
            double wL = 1.0, wR = 0.0;
            if (sR > sL) {
                wL = (sR - sq) / (sR - sL);
                wR = (sq - sL) / (sR - sL);
            }
            DirRec &R = out[static_cast<size_t>(q)];
            if (iL >= 0) {
                const Hit &H = hits[h0 + static_cast<size_t>(iL)];
                R.k[0] = static_cast<int32_t>(H.ks);
                R.w[0] = wL * (1.0 - H.t);
                R.w[1] = wL * H.t;
            } else {
                R.k[0] = -1;
                R.w[0] = wL;
                R.w[1] = 0.0;
            }
            if (iR < static_cast<int64_t>(xs.size())) {
                const Hit &H = hits[h0 + static_cast<size_t>(iR)];
                R.k[1] = static_cast<int32_t>(H.ks);
                R.w[2] = wR * (1.0 - H.t);
                R.w[3] = wR * H.t;
            } else {
                R.k[1] = -1;
                R.w[2] = wR;
                R.w[3] = 0.0;
            }
        }
        h0 = h1;
    }
}

}  // namespace adr
