// Host-side geometry and interpolation tables (see geometry.hpp).
// Compiled with -ffp-contract=off: every value here feeds the bitwise
// reproducible decisions of point location and the MAC.
#include "geometry.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <tuple>

namespace stc {

namespace {

using V3 = std::array<double, 3>;

V3 normalize(const V3& p) {
    double n = std::sqrt((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]);
    return {p[0] / n, p[1] / n, p[2] / n};
}

V3 add(const V3& a, const V3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
V3 sub(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
V3 cross(const V3& a, const V3& b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
double dot(const V3& a, const V3& b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

void icosahedron(std::vector<V3>& verts, std::vector<std::array<int, 3>>& faces) {
    const double phi = (1.0 + std::sqrt(5.0)) / 2.0;
    std::vector<V3> raw;
    for (double s1 : {-1.0, 1.0})
        for (double s2 : {-1.0, 1.0}) {
            raw.push_back({0.0, s1, s2 * phi});
            raw.push_back({s1, s2 * phi, 0.0});
            raw.push_back({s2 * phi, 0.0, s1});
        }
    std::sort(raw.begin(), raw.end());
    verts.clear();
    for (auto& p : raw) verts.push_back(normalize(p));
    faces.clear();
    auto adjacent = [&](int i, int j) {
        V3 d = sub(raw[i], raw[j]);
        return std::fabs(dot(d, d) - 4.0) < 1e-9;
    };
    for (int i = 0; i < 12; ++i)
        for (int j = i + 1; j < 12; ++j)
            for (int k = j + 1; k < 12; ++k)
                if (adjacent(i, j) && adjacent(i, k) && adjacent(j, k)) {
                    double o = dot(cross(sub(raw[j], raw[i]), sub(raw[k], raw[i])), raw[i]);
                    if (o > 0) faces.push_back({i, j, k});
                    else faces.push_back({i, k, j});
                }
}

void fill_node(NodeGeo& g, const V3& v1, const V3& v2, const V3& v3) {
    const V3* v[3] = {&v1, &v2, &v3};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) g.v[a][b] = (*v[a])[b];
    V3 c = normalize(cross(sub(v2, v1), sub(v3, v1)));
    double r = 0.0;
    for (int k = 0; k < 3; ++k) {
        V3 d = sub(c, *v[k]);
        double rk = std::sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
        r = (k == 0) ? rk : std::max(r, rk);
    }
    for (int b = 0; b < 3; ++b) g.c[b] = c[b];
    g.r = r;
    // rows of M^{-1}, M = [v1 v2 v3]: (v2 x v3, v3 x v1, v1 x v2) / det
    V3 r1 = cross(v2, v3), r2 = cross(v3, v1), r3 = cross(v1, v2);
    double det = dot(v1, r1);
    for (int b = 0; b < 3; ++b) {
        g.minv[0][b] = r1[b] / det;
        g.minv[1][b] = r2[b] / det;
        g.minv[2][b] = r3[b] / det;
    }
}

}  // namespace

void build_tree_geometry(int max_level, std::vector<NodeGeo>& out) {
    std::vector<V3> verts;
    std::vector<std::array<int, 3>> faces;
    icosahedron(verts, faces);
    out.assign(size_t(total_nodes(max_level)), NodeGeo{});
    // vertices of the current level
    std::vector<std::array<V3, 3>> cur(20), nxt;
    for (int f = 0; f < 20; ++f) cur[f] = {verts[faces[f][0]], verts[faces[f][1]], verts[faces[f][2]]};
    for (int lvl = 0; lvl <= max_level; ++lvl) {
        int64_t off = level_offset(lvl);
        for (size_t k = 0; k < cur.size(); ++k) fill_node(out[off + k], cur[k][0], cur[k][1], cur[k][2]);
        if (lvl == max_level) break;
        nxt.resize(cur.size() * 4);
        for (size_t k = 0; k < cur.size(); ++k) {
            const V3& v1 = cur[k][0];
            const V3& v2 = cur[k][1];
            const V3& v3 = cur[k][2];
            V3 m12 = normalize(add(v1, v2));
            V3 m23 = normalize(add(v2, v3));
            V3 m31 = normalize(add(v3, v1));
            nxt[4 * k + 0] = {v1, m12, m31};
            nxt[4 * k + 1] = {m12, v2, m23};
            nxt[4 * k + 2] = {m31, m23, v3};
            nxt[4 * k + 3] = {m12, m23, m31};
        }
        cur.swap(nxt);
    }
}

namespace {

// Legendre P_n and its derivative at t (long double recurrences).
void legendre(int n, long double t, long double& p, long double& dp) {
    long double p0 = 1.0L, p1 = t;
    if (n == 0) { p = 1.0L; dp = 0.0L; return; }
    for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * t * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    dp = n * (t * p1 - p0) / (t * t - 1.0L);
}

// Gauss-Lobatto-Legendre nodes on [0,1]: endpoints and roots of P_d'.
std::vector<long double> gll01(int d) {
    std::vector<long double> t(d + 1);
    const long double pi = 3.141592653589793238462643383279502884L;
    t[0] = -1.0L;
    t[d] = 1.0L;
    for (int k = 1; k < d; ++k) {
        long double x = -std::cos(pi * k / d);  // Chebyshev-Gauss-Lobatto start
        for (int it = 0; it < 100; ++it) {
            // Newton on q(t) = (1 - t^2) P_d'(t): q' = -d(d+1) P_d
            long double p, dp;
            legendre(d, x, p, dp);
            long double q = (1.0L - x * x) * dp;
            long double qp = -(long double)d * (d + 1) * p;
            long double dx = q / qp;
            x -= dx;
            if (std::fabs(dx) < 1e-19L) break;
        }
        t[k] = x;
    }
    std::sort(t.begin(), t.end());
    std::vector<long double> v(d + 1);
    for (int k = 0; k <= d; ++k) v[k] = 0.5L * (1.0L + t[k]);
    return v;
}

long double fact(int n) {
    long double f = 1.0L;
    for (int k = 2; k <= n; ++k) f *= k;
    return f;
}

}  // namespace

bool build_reference_tables(int d, RefTables& out) {
    if (d < 1 || d > 16) return false;
    out.degree = d;
    int np = (d + 1) * (d + 2) / 2;
    out.np = np;
    std::vector<long double> v = gll01(d);
    std::vector<std::array<int, 3>> idx;
    for (int i = 0; i <= d; ++i)
        for (int j = 0; j <= d - i; ++j) idx.push_back({i, j, d - i - j});
    std::vector<long double> b(np * 3), coef(np);
    out.points.resize(np * 3);
    out.expo.resize(np * 3);
    out.coef.resize(np);
    for (int m = 0; m < np; ++m) {
        int i = idx[m][0], j = idx[m][1], k = idx[m][2];
        b[3 * m + 0] = (1 + 2 * v[i] - v[j] - v[k]) / 3.0L;
        b[3 * m + 1] = (1 + 2 * v[j] - v[i] - v[k]) / 3.0L;
        b[3 * m + 2] = (1 + 2 * v[k] - v[i] - v[j]) / 3.0L;
        coef[m] = fact(d) / (fact(i) * fact(j) * fact(k));
        for (int a = 0; a < 3; ++a) {
            out.points[3 * m + a] = double(b[3 * m + a]);
            out.expo[3 * m + a] = idx[m][a];
        }
        out.coef[m] = double(coef[m]);
    }
    // V_ref[m][k] = coef_k * b_m1^i_k * b_m2^j_k * b_m3^k_k, inverted by
    // Gauss-Jordan elimination with partial pivoting in long double.
    std::vector<long double> A(size_t(np) * np), I(size_t(np) * np, 0.0L);
    for (int m = 0; m < np; ++m) {
        for (int k = 0; k < np; ++k) {
            long double val = coef[k];
            for (int a = 0; a < 3; ++a) {
                for (int e = 0; e < idx[k][a]; ++e) val *= b[3 * m + a];
            }
            A[size_t(m) * np + k] = val;
        }
        I[size_t(m) * np + m] = 1.0L;
    }
    for (int col = 0; col < np; ++col) {
        int piv = col;
        for (int r = col + 1; r < np; ++r)
            if (std::fabs(A[size_t(r) * np + col]) > std::fabs(A[size_t(piv) * np + col])) piv = r;
        if (std::fabs(A[size_t(piv) * np + col]) < 1e-30L) return false;
        if (piv != col)
            for (int c = 0; c < np; ++c) {
                std::swap(A[size_t(piv) * np + c], A[size_t(col) * np + c]);
                std::swap(I[size_t(piv) * np + c], I[size_t(col) * np + c]);
            }
        long double inv = 1.0L / A[size_t(col) * np + col];
        for (int c = 0; c < np; ++c) {
            A[size_t(col) * np + c] *= inv;
            I[size_t(col) * np + c] *= inv;
        }
        for (int r = 0; r < np; ++r) {
            if (r == col) continue;
            long double f = A[size_t(r) * np + col];
            if (f == 0.0L) continue;
            for (int c = 0; c < np; ++c) {
                A[size_t(r) * np + c] -= f * A[size_t(col) * np + c];
                I[size_t(r) * np + c] -= f * I[size_t(col) * np + c];
            }
        }
    }
    // I now holds V_ref^{-1}: row k (basis), column m (point)
    out.vinv.resize(size_t(np) * np);
    out.max_abs_vinv = 0;
    for (size_t t = 0; t < out.vinv.size(); ++t) {
        out.vinv[t] = double(I[t]);
        out.max_abs_vinv = std::max(out.max_abs_vinv, std::fabs(out.vinv[t]));
    }
    return true;
}

}  // namespace stc
