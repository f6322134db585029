// Host-side planning of the recursive-skeletonisation factorisation:
// grid detection, the binary tree of boxes (Sec. 2.2), boundary-layer
// skeleton and residual sets (Sec. 3.1), proxy rings (Sec. 2.2, Sec. 3.3.2)
// and the canonical point orderings every device kernel relies on.
//
// Everything here is integer bookkeeping computed once per grid shape; no
// kernel values are formed on the host.
#pragma once

#include <cstdint>
#include <map>
#include <string>
#include <tuple>
#include <vector>

namespace rsd {

// Canonical ordering of the active points of one box type.  Every box of the
// same shape, split direction and child types shares one Layout, so one
// interpolation matrix T and one assembly map serve all of them.
struct Layout {
    int ax = 0, ay = 0;      // box size in grid points
    int split = -1;          // -1 leaf, 0 split in x, 1 split in y
    bool root = false;       // root: residual = first child, skeleton = second
    int k = 0, r = 0;        // |I^sk|, |I^rs|; active size k + r
    int child[2] = {-1, -1}; // child layouts
    int child_ax1 = 0, child_ay1 = 0;  // offset of the second child
    // relative coordinates of the active points in [sk; rs] order
    std::vector<int32_t> u, v;
    // non-leaf: source of each active position (child, index in child's sk)
    std::vector<int32_t> src_c, src_i;
    // index of the interpolation problem solving for T (-1: none)
    int idp = -1;
};

// One proxy least-squares problem  K(Z, X^sk) T = K(Z, X^rs)  (Sec. 3.1).
struct IDProblem {
    int layout = -1;
    int p = 0, k = 0, r = 0;
    std::vector<int32_t> zu, zv;   // proxy nodes relative to the box origin
    // Mirror symmetry: when reflections of the box (u -> ax-1-u along an
    // even side ax, v -> ay-1-v along an even side ay) map Z, I^sk and I^rs
    // onto themselves (no fixed points, the sides being even), every point
    // lies in an orbit of the group they generate (grp: bit 0 the u
    // reflection, bit 1 the v reflection; order 2 or 4), and the problem
    // splits into that many independent sector problems of 1/order the size.
    // Orbit representatives are the points in the lower half along every
    // reflected axis; g (bit 0: u, bit 1: v) names the reflection carrying
    // the representative to the point.
    bool sym = false;
    int grp = 0;
    int nsec() const { return sym ? (grp == 3 ? 4 : 2) : 1; }
    std::vector<int32_t> zr_u, zr_v;           // Z representatives (p / nsec)
    std::vector<int32_t> skr_u, skr_v;         // I^sk representatives (k / nsec)
    std::vector<int32_t> rsr_u, rsr_v;         // I^rs representatives (r / nsec)
    std::vector<int32_t> sk_orb, sk_g;         // per skeleton position: orbit, reflection
    std::vector<int32_t> rs_orb, rs_g;         // per residual position
};

struct Box {
    int x0 = 0, y0 = 0, ax = 0, ay = 0;
    int level = 0;            // height above the leaves
    int parent = -1;
    int child[2] = {-1, -1};
    int layout = -1;
    int k = 0, r = 0;
    int64_t offF = 0;         // offset (elements) of its (k+r)^2 F block
    int64_t offV = 0;         // offset (elements per rhs) of its vector block
    int pos_in_parent = 0;    // 0/1: which child of its parent
};

struct Plan {
    int64_t nx = 0, ny = 0;
    int leaf = 8, m = 2;
    int iface = 0;                        // spacing of the interface skeleton points (0: none)
    std::vector<Box> boxes;               // level by level from the leaves
    std::vector<std::vector<int>> levels; // box ids per level (0 = leaves)
    std::vector<Layout> layouts;
    std::vector<IDProblem> idps;
    int root = -1;
    int64_t F_elems = 0;      // total F arena size (elements)
    int64_t V_elems = 0;      // total vector arena size per rhs
    int64_t Vr_elems = 0;     // residual-part scratch per rhs
};

// Build the plan for an nx x ny grid; throws std::runtime_error on bad input.
Plan make_plan(int64_t nx, int64_t ny, int leaf, int m, int iface = 0);

// Active point ids (grid index i * ny + j) of a box in [sk; rs] order.
std::vector<int64_t> box_points(const Plan& p, int box);

// Detect a complete uniform grid.  perm[g] = caller index of grid point g.
// Returns false (and a reason) when the points are not such a grid.
bool detect_grid(const double* pts, int64_t n, int64_t& nx, int64_t& ny, double& h,
                 double& x0, double& y0, std::vector<int64_t>& perm, std::string& why);

int layers_for_tol(double tol);

}  // namespace rsd
