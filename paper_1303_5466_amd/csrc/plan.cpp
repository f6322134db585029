// Host planning: tree (Sec. 2.2), skeleton sets (Sec. 3.1), proxy rings.
#include "plan.hpp"
#include "hostpool.hpp"


#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

namespace rsd {

int layers_for_tol(double tol) {
    if (tol >= 1e-6) return 1;
    if (tol >= 1e-11) return 2;
    return 3;
}

static int n_splits(int64_t side, int leaf) {
    int d = 0;
    while ((side + (int64_t(1) << d) - 1) / (int64_t(1) << d) > leaf) ++d;
    return d;
}

namespace {

struct Pt { int u, v; };

// depth of a point below the boundary of an a x b box
inline int depth_in(int u, int v, int a, int b) {
    return std::min(std::min(u, a - 1 - u), std::min(v, b - 1 - v));
}

// Skeleton points ordered cyclically around the box (angle about the centre,
// then depth, then coordinates); residual points along the interface (the
// coordinate along the cut first) or row-major for a leaf's interior.
void order_points(std::vector<int>& sk, std::vector<int>& rs, const std::vector<Pt>& pts,
                  int a, int b, int split) {
    const double cu = 0.5 * (a - 1), cv = 0.5 * (b - 1);
    std::vector<double> ang(pts.size());
    for (size_t q = 0; q < pts.size(); ++q) ang[q] = std::atan2(pts[q].v - cv, pts[q].u - cu);
    std::sort(sk.begin(), sk.end(), [&](int x, int y) {
        if (ang[x] != ang[y]) return ang[x] < ang[y];
        int dx = depth_in(pts[x].u, pts[x].v, a, b), dy = depth_in(pts[y].u, pts[y].v, a, b);
        if (dx != dy) return dx < dy;
        if (pts[x].u != pts[y].u) return pts[x].u < pts[y].u;
        return pts[x].v < pts[y].v;
    });
    std::sort(rs.begin(), rs.end(), [&](int x, int y) {
        int ax_ = pts[x].u, bx = pts[x].v, ay_ = pts[y].u, by = pts[y].v;
        if (split == 0) { std::swap(ax_, bx); std::swap(ay_, by); }  // along v first
        if (ax_ != ay_) return ax_ < ay_;
        return bx < by;
    });
}

struct Builder {
    Plan& P;
    std::map<std::tuple<int, int, int, int, int, int>, int> layout_of;
    explicit Builder(Plan& p) : P(p) {}

    int leaf_layout(int a, int b, bool root) {
        auto key = std::make_tuple(a, b, -1, -1, -1, root ? 1 : 0);
        auto it = layout_of.find(key);
        if (it != layout_of.end()) return it->second;
        Layout L;
        L.ax = a; L.ay = b; L.split = -1; L.root = root;
        std::vector<Pt> pts;
        for (int u = 0; u < a; ++u)
            for (int v = 0; v < b; ++v) pts.push_back({u, v});
        std::vector<int> sk, rs;
        for (int q = 0; q < (int)pts.size(); ++q)
            (root || depth_in(pts[q].u, pts[q].v, a, b) < P.m ? sk : rs).push_back(q);
        order_points(sk, rs, pts, a, b, -1);
        finish(L, pts, sk, rs, {}, {});
        int id = (int)P.layouts.size();
        P.layouts.push_back(std::move(L));
        layout_of[key] = id;
        return id;
    }

    int parent_layout(int a, int b, int split, int l1, int l2, int a1, int b1, bool root) {
        auto key = std::make_tuple(a, b, split, l1, l2, root ? 1 : 0);
        auto it = layout_of.find(key);
        if (it != layout_of.end()) return it->second;
        Layout L;
        L.ax = a; L.ay = b; L.split = split; L.root = root;
        L.child[0] = l1; L.child[1] = l2;
        L.child_ax1 = split == 0 ? a1 : 0;
        L.child_ay1 = split == 1 ? b1 : 0;
        std::vector<Pt> pts;
        std::vector<int> srcc, srci;
        for (int c = 0; c < 2; ++c) {
            const Layout& C = P.layouts[c == 0 ? l1 : l2];
            int du = c == 0 ? 0 : L.child_ax1, dv = c == 0 ? 0 : L.child_ay1;
            for (int i = 0; i < C.k; ++i) {
                pts.push_back({C.u[i] + du, C.v[i] + dv});
                srcc.push_back(c);
                srci.push_back(i);
            }
        }
        std::vector<int> sk, rs;
        if (root) {
            // block elimination at the top: residual = first child, skeleton = second
            for (int q = 0; q < (int)pts.size(); ++q) (srcc[q] == 0 ? rs : sk).push_back(q);
        } else {
            for (int q = 0; q < (int)pts.size(); ++q) {
                const bool keep = depth_in(pts[q].u, pts[q].v, a, b) < P.m ||
                                  on_interface(pts[q], a, b, split, split == 0 ? a1 : b1);
                (keep ? sk : rs).push_back(q);
            }
            order_points(sk, rs, pts, a, b, split);
        }
        finish(L, pts, sk, rs, srcc, srci);
        int id = (int)P.layouts.size();
        P.layouts.push_back(std::move(L));
        layout_of[key] = id;
        return id;
    }

    // Interface skeleton points (Sec. 5.3: a few points per wavelength kept on
    // the cut between the children): on the two grid lines either side of
    // the cut at c (u = c - 1, c for a cut across u; v likewise), those whose
    // distance past the boundary layers along the cut is iface / 2 modulo
    // iface.  Off when iface = 0.
    bool on_interface(const Pt& p, int a, int b, int split, int c) const {
        if (P.iface <= 0 || split < 0) return false;
        const int across = split == 0 ? p.u : p.v;
        if (across != c - 1 && across != c) return false;
        const int along = split == 0 ? p.v : p.u, len = split == 0 ? b : a;
        const int past = std::min(along, len - 1 - along) - P.m;
        return past >= 0 && past % P.iface == P.iface / 2;
    }

    void finish(Layout& L, const std::vector<Pt>& pts, const std::vector<int>& sk,
                const std::vector<int>& rs, const std::vector<int>& srcc,
                const std::vector<int>& srci) {
        L.k = (int)sk.size();
        L.r = (int)rs.size();
        for (int pass = 0; pass < 2; ++pass)
            for (int q : (pass == 0 ? sk : rs)) {
                L.u.push_back(pts[q].u);
                L.v.push_back(pts[q].v);
                if (!srcc.empty()) {
                    L.src_c.push_back(srcc[q]);
                    L.src_i.push_back(srci[q]);
                }
            }
    }

    void add_idp(int lid) {
        Layout& L = P.layouts[lid];
        if (L.root || L.r == 0 || L.idp >= 0) return;
        IDProblem I;
        I.layout = lid;
        I.k = L.k;
        I.r = L.r;
        const size_t ring = (size_t)(L.ax + 2 * P.m) * (L.ay + 2 * P.m) - (size_t)L.ax * L.ay;
        I.zu.reserve(ring);
        I.zv.reserve(ring);
        for (int zu = -P.m; zu < L.ax + P.m; ++zu)
            for (int zv = -P.m; zv < L.ay + P.m; ++zv) {
                bool inside = zu >= 0 && zu < L.ax && zv >= 0 && zv < L.ay;
                if (inside) continue;
                I.zu.push_back(zu);
                I.zv.push_back(zv);
            }
        I.p = (int)I.zu.size();
        if (L.ax % 2 == 0 || L.ay % 2 == 0) find_symmetry(L, I);
        L.idp = (int)P.idps.size();
        P.idps.push_back(std::move(I));
    }

    static void find_symmetry(const Layout& L, IDProblem& I) {
        const int ax = L.ax, ay = L.ay;
        const int k = L.k, r = L.r;
        // every point of the three sets lies in the rectangle the proxy ring
        // spans (mirror images of points in it stay in it): dense marks and
        // representative numbers over that rectangle
        int u0 = 0, v0 = 0, u1 = ax - 1, v1 = ay - 1;
        for (int i = 0; i < I.p; ++i) {
            u0 = std::min(u0, I.zu[i]); u1 = std::max(u1, I.zu[i]);
            v0 = std::min(v0, I.zv[i]); v1 = std::max(v1, I.zv[i]);
        }
        // a reflection along an axis can apply only when the side is even
        // (no fixed points) and the ring is mirror-symmetric along it
        int grp = 0;
        if (ax % 2 == 0 && u0 + u1 == ax - 1) grp |= 1;
        if (ay % 2 == 0 && v0 + v1 == ay - 1) grp |= 2;
        if (!grp) return;
        const int nu = u1 - u0 + 1, nv = v1 - v0 + 1;
        auto at = [&](int u, int v) { return (int64_t)(u - u0) * nv + (v - v0); };
        std::vector<int32_t> mark((size_t)nu * nv, -1);
        // the reflections (of those in grp) mapping a set onto itself
        auto closed = [&](const int32_t* U, const int32_t* V, int n, int tag) {
            for (int i = 0; i < n; ++i) mark[at(U[i], V[i])] = tag;
            int ok = grp;
            for (int i = 0; i < n && ok; ++i) {
                if ((ok & 1) && mark[at(ax - 1 - U[i], V[i])] != tag) ok &= ~1;
                if ((ok & 2) && mark[at(U[i], ay - 1 - V[i])] != tag) ok &= ~2;
            }
            return ok;
        };
        grp &= closed(I.zu.data(), I.zv.data(), I.p, 0);
        if (grp) grp &= closed(L.u.data(), L.v.data(), k, 1);
        if (grp) grp &= closed(L.u.data() + k, L.v.data() + k, r, 2);
        if (!grp) return;
        const int ord = grp == 3 ? 4 : 2;
        const bool ru_ = grp & 1, rv_ = grp & 2;
        // representatives in list order, then orbit / reflection of every point
        auto orbits = [&](const int32_t* U, const int32_t* V, int n, std::vector<int32_t>& ru,
                          std::vector<int32_t>& rv, std::vector<int32_t>* orb, std::vector<int32_t>* g) {
            for (int i = 0; i < n; ++i)
                if ((!ru_ || U[i] < ax / 2) && (!rv_ || V[i] < ay / 2)) {
                    mark[at(U[i], V[i])] = (int)ru.size();
                    ru.push_back(U[i]);
                    rv.push_back(V[i]);
                }
            if (!orb) return;
            orb->reserve(n);
            g->reserve(n);
            for (int i = 0; i < n; ++i) {
                const int gx = ru_ && U[i] >= ax / 2 ? 1 : 0, gy = rv_ && V[i] >= ay / 2 ? 1 : 0;
                const int fu = gx ? ax - 1 - U[i] : U[i], fv = gy ? ay - 1 - V[i] : V[i];
                orb->push_back(mark[at(fu, fv)]);
                g->push_back(gx + 2 * gy);
            }
        };
        orbits(I.zu.data(), I.zv.data(), I.p, I.zr_u, I.zr_v, nullptr, nullptr);
        orbits(L.u.data(), L.v.data(), k, I.skr_u, I.skr_v, &I.sk_orb, &I.sk_g);
        orbits(L.u.data() + k, L.v.data() + k, r, I.rsr_u, I.rsr_v, &I.rs_orb, &I.rs_g);
        if ((int)I.zr_u.size() * ord != I.p || (int)I.skr_u.size() * ord != k ||
            (int)I.rsr_u.size() * ord != r) {
            I.zr_u.clear(); I.zr_v.clear(); I.skr_u.clear(); I.skr_v.clear(); I.rsr_u.clear(); I.rsr_v.clear();
            I.sk_orb.clear(); I.sk_g.clear(); I.rs_orb.clear(); I.rs_g.clear();
            return;
        }
        I.sym = true;
        I.grp = grp;
    }
};

}  // namespace

Plan make_plan(int64_t nx, int64_t ny, int leaf, int m, int iface) {
    if (nx < 1 || ny < 1 || leaf < 1 || m < 1 || iface < 0) throw std::runtime_error("invalid plan arguments");
    if (nx > (1 << 20) || ny > (1 << 20)) throw std::runtime_error("grid too large");
    Plan P;
    P.nx = nx; P.ny = ny; P.leaf = leaf; P.m = m; P.iface = iface;
    const int sx = n_splits(nx, leaf), sy = n_splits(ny, leaf);
    // global split schedule: longer remaining segment first, x on ties
    std::vector<int> sched;
    for (int dx = 0, dy = 0; dx < sx || dy < sy;) {
        int64_t lx = (nx + (int64_t(1) << dx) - 1) >> dx;
        int64_t ly = (ny + (int64_t(1) << dy) - 1) >> dy;
        if (dx < sx && (dy >= sy || lx >= ly)) { sched.push_back(0); ++dx; }
        else { sched.push_back(1); ++dy; }
    }
    const int depth = (int)sched.size();
    // top-down boxes by depth
    struct TB { int x0, y0, ax, ay, parent, c0, c1; };
    std::vector<std::vector<TB>> bydepth(depth + 1);
    bydepth[0].push_back({0, 0, (int)nx, (int)ny, -1, -1, -1});
    for (int d = 0; d < depth; ++d) {
        for (int i = 0; i < (int)bydepth[d].size(); ++i) {
            TB& b = bydepth[d][i];
            TB c0 = b, c1 = b;
            c0.parent = c1.parent = i;
            c0.c0 = c0.c1 = c1.c0 = c1.c1 = -1;
            if (sched[d] == 0) {
                int h = b.ax / 2;
                c0.ax = h; c1.x0 = b.x0 + h; c1.ax = b.ax - h;
            } else {
                int h = b.ay / 2;
                c0.ay = h; c1.y0 = b.y0 + h; c1.ay = b.ay - h;
            }
            b.c0 = (int)bydepth[d + 1].size();
            bydepth[d + 1].push_back(c0);
            b.c1 = (int)bydepth[d + 1].size();
            bydepth[d + 1].push_back(c1);
        }
    }
    Builder B(P);
    // bottom-up numbering: level t = depth - d
    std::vector<std::vector<int>> gid(depth + 1);
    P.levels.resize(depth + 1);
    for (int d = depth; d >= 0; --d) {
        int t = depth - d;
        gid[d].resize(bydepth[d].size());
        for (int i = 0; i < (int)bydepth[d].size(); ++i) {
            const TB& tb = bydepth[d][i];
            Box bx;
            bx.x0 = tb.x0; bx.y0 = tb.y0; bx.ax = tb.ax; bx.ay = tb.ay;
            bx.level = t;
            const bool is_root = (d == 0);
            if (d == depth) {
                bx.layout = B.leaf_layout(tb.ax, tb.ay, is_root);  // a root leaf keeps every point
            } else {
                int g0 = gid[d + 1][tb.c0], g1 = gid[d + 1][tb.c1];
                bx.child[0] = g0; bx.child[1] = g1;
                const Box& C0 = P.boxes[g0];
                bx.layout = B.parent_layout(tb.ax, tb.ay, sched[d], C0.layout, P.boxes[g1].layout,
                                            C0.ax, C0.ay, is_root);
            }
            const Layout& L = P.layouts[bx.layout];
            bx.k = L.k;
            bx.r = L.r;
            int id = (int)P.boxes.size();
            gid[d][i] = id;
            P.boxes.push_back(bx);
            P.levels[t].push_back(id);
            if (d < depth) {
                P.boxes[bx.child[0]].parent = id;
                P.boxes[bx.child[1]].parent = id;
                P.boxes[bx.child[0]].pos_in_parent = 0;
                P.boxes[bx.child[1]].pos_in_parent = 1;
            }
        }
    }
    P.root = (int)P.boxes.size() - 1;
    for (auto& bx : P.boxes)
        if (&bx != &P.boxes[P.root]) B.add_idp(bx.layout);
    // arenas
    int64_t offF = 0, offV = 0;
    for (auto& bx : P.boxes) {
        int64_t mm = bx.k + bx.r;
        bx.offF = offF;
        offF += mm * mm;
        bx.offV = offV;
        offV += mm;
    }
    P.F_elems = offF;
    P.V_elems = offV;
    return P;
}

std::vector<int64_t> box_points(const Plan& p, int box) {
    const Box& b = p.boxes.at(box);
    const Layout& L = p.layouts[b.layout];
    std::vector<int64_t> out(L.k + L.r);
    for (int q = 0; q < L.k + L.r; ++q)
        out[q] = int64_t(b.x0 + L.u[q]) * p.ny + (b.y0 + L.v[q]);
    return out;
}

bool detect_grid(const double* pts, int64_t n, int64_t& nx, int64_t& ny, double& h,
                 double& x0, double& y0, std::vector<int64_t>& perm, std::string& why) {
    if (n < 1) { why = "no points"; return false; }
    // one pass for the extent, one for the second grid line of each axis (the
    // smallest coordinate above the minimum), which gives the spacing; the
    // placement pass below then checks every point against that grid.  Each
    // pass runs over chunks of points on the host pool; chunks combine their
    // partial results under a lock.
    HostPool& pool = HostPool::get();
    // below about 10^5 points waking the pool costs more than the passes
    const int64_t GRAIN = n >= (int64_t(1) << 17) ? 16384 : n;
    std::mutex mu;
    double xmin = pts[0], xmax = pts[0], ymin = pts[1], ymax = pts[1];
    bool finite = true;
    pool.parallel_for(n, GRAIN, [&](int64_t lo, int64_t hi) {
        double a0 = pts[2 * lo], a1 = a0, b0 = pts[2 * lo + 1], b1 = b0;
        bool ok = true;
        for (int64_t i = lo; i < hi; ++i) {
            const double x = pts[2 * i], y = pts[2 * i + 1];
            ok = ok && std::isfinite(x) && std::isfinite(y);
            a0 = std::min(a0, x); a1 = std::max(a1, x);
            b0 = std::min(b0, y); b1 = std::max(b1, y);
        }
        std::lock_guard<std::mutex> lk(mu);
        finite = finite && ok;
        xmin = std::min(xmin, a0); xmax = std::max(xmax, a1);
        ymin = std::min(ymin, b0); ymax = std::max(ymax, b1);
    });
    if (!finite) { why = "non-finite coordinate"; return false; }
    const double span = std::max(xmax - xmin, ymax - ymin);
    const double eps = 1e-9 * std::max(1.0, span);
    double x1 = HUGE_VAL, y1 = HUGE_VAL;
    pool.parallel_for(n, GRAIN, [&](int64_t lo, int64_t hi) {
        double a = HUGE_VAL, b = HUGE_VAL;
        for (int64_t i = lo; i < hi; ++i) {
            const double x = pts[2 * i], y = pts[2 * i + 1];
            if (x - xmin > eps) a = std::min(a, x);
            if (y - ymin > eps) b = std::min(b, y);
        }
        std::lock_guard<std::mutex> lk(mu);
        x1 = std::min(x1, a);
        y1 = std::min(y1, b);
    });
    auto lines = [&](double lo, double hi, double second, int64_t& cnt) {
        if (second == HUGE_VAL) { cnt = 1; return true; }
        const double q = (hi - lo) / (second - lo);
        if (!(q < (double)n)) return false;          // more lines than points
        cnt = (int64_t)std::llround(q) + 1;
        return true;
    };
    if (!lines(xmin, xmax, x1, nx) || !lines(ymin, ymax, y1, ny) || nx * ny != n) {
        why = "point count is not nx * ny";
        return false;
    }
    if (nx == 1 && ny == 1) { why = "a single point is not a grid"; return false; }
    const double hx = nx > 1 ? (xmax - xmin) / double(nx - 1) : 0.0;
    const double hy = ny > 1 ? (ymax - ymin) / double(ny - 1) : 0.0;
    h = nx > 1 ? hx : hy;
    if (nx > 1 && ny > 1 && std::fabs(hx - hy) > 1e-9 * h) { why = "spacing differs in x and y"; return false; }
    if (!(h > 0)) { why = "zero spacing"; return false; }
    x0 = xmin;
    y0 = ymin;
    perm.assign(n, -1);
    const double ih = 1.0 / h;
    std::atomic<int> off{0}, dup{0};
    int64_t* pm = perm.data();
    pool.parallel_for(n, GRAIN, [&](int64_t lo, int64_t hi) {
        for (int64_t p = lo; p < hi; ++p) {
            // fi, fj >= 0 (x0, y0 are the minima): truncation rounds to nearest
            const double fi = (pts[2 * p] - x0) * ih, fj = (pts[2 * p + 1] - y0) * ih;
            const int64_t i = (int64_t)(fi + 0.5), j = (int64_t)(fj + 0.5);
            if (std::fabs(fi - i) > 1e-6 || std::fabs(fj - j) > 1e-6 || i < 0 || j < 0 || i >= nx || j >= ny) {
                off.store(1, std::memory_order_relaxed);
                return;
            }
            int64_t expect = -1;
            if (!__atomic_compare_exchange_n(pm + i * ny + j, &expect, p, false, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED)) {
                dup.store(1, std::memory_order_relaxed);
                return;
            }
        }
    });
    if (off.load()) { why = "point off the uniform grid"; return false; }
    if (dup.load()) { why = "duplicate grid point"; return false; }
    return true;
}

}  // namespace rsd
