// Host-side geometry and interpolation tables of the spherical tree code.
//
// Triangle tree (Sec. 3, overview and grids on a sphere): the 20 faces of an
// icosahedron, each split into four children level by level.  The recipe is
// fixed so that decisions (point location, MAC) are reproducible bit for bit:
//  * icosahedron vertices (0,+-1,+-phi), (+-1,+-phi,0), (+-phi,0,+-1) in
//    lexicographic (x,y,z) order, normalised p / sqrt((px*px + py*py) + pz*pz);
//    faces = adjacent triples i<j<k, lexicographic, counter-clockwise outward;
//  * children of (v1,v2,v3): (v1,m12,m31), (m12,v2,m23), (m31,m23,v3),
//    (m12,m23,m31) with m_ab = (a+b)/|a+b|;
//  * circumcentre c = normalise((v2-v1) x (v3-v1)); radius r = max_k |c - v_k|
//    (Sec. 3, dual tree traversal).
// This file must be compiled with floating-point contraction off.
#pragma once

#include <cstdint>
#include <vector>

namespace stc {

// 22 doubles per node: vertices, circumcentre, radius, rows of M^{-1} with
// M = [v1 v2 v3] (spherical barycentric coordinates b = M^{-1} y, Sec. 3,
// interpolation in triangles).
struct NodeGeo {
    double v[3][3];
    double c[3];
    double r;
    double minv[3][3];
};

// The traversal's view of a node: circumcentre and radius (32 bytes).
struct NodeMac {
    double cx, cy, cz, r;
};

inline int64_t level_offset(int level) { return 20 * ((int64_t(1) << (2 * level)) - 1) / 3; }
inline int64_t total_nodes(int max_level) { return level_offset(max_level + 1); }

// Geometry of every node of the complete tree down to max_level, indexed by
// node id = level_offset(level) + key.
void build_tree_geometry(int max_level, std::vector<NodeGeo>& out);

// Interpolation tables of degree d (readings of Sec. 3, interpolation in
// triangles): Lobatto triangle points of Blyth & Pozrikidis, the
// multinomial-scaled SBB basis, and the inverse of the reference Vandermonde
// matrix V_ref[m][k] = B_k(b_m), computed in extended precision.
struct RefTables {
    int degree = 0;
    int np = 0;
    std::vector<double> points;    // np x 3 planar barycentrics b_m
    std::vector<int> expo;         // np x 3 exponents (i, j, k)
    std::vector<double> coef;      // np multinomials d!/(i!j!k!)
    std::vector<double> vinv;      // np x np, [k * np + m] = (V_ref^{-1})_{km}
    double max_abs_vinv = 0;
};

bool build_reference_tables(int degree, RefTables& out);

}  // namespace stc
