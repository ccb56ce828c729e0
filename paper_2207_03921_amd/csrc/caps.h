// The paper's ball approximations restricted to one inner element
// (Sec. 2.2, Def. 2.3 nocaps and Def. 2.4 approximate caps).
//
// nocaps: the convex hull of all crossings of the circle |y - x| = delta
// with the element edges of the mesh.  Two consecutive crossings (by angle)
// bound an arc that runs inside a single element, so the hull's chord
// between them lies in that element and no vertex lies in the cap it cuts
// off; hence
//   T_l n B_ncp(x) = conv(vertices of T_l in the closed disc
//                         u crossings of T_l's edges with the circle).
// approxcaps adds the midpoint of every arc of the circle inside T_l (the
// cap centre).  The region is convex and is listed counter-clockwise: along
// each edge v_i -> v_i+1 the vertex v_i when inside, then the crossings in
// order of the edge parameter t, roots of
//   A t^2 + 2 B t + C = 0,  A = e.e, B = (v_i - x).e, C = |v_i - x|^2 - delta^2,
// D = B^2 - A C: leaving the disc t = (-B + sqrt D)/A, entering
// t = (-B - sqrt D)/A (clamped to [0, 1]); an edge with both ends outside
// has two crossings iff D > 0 and 0 < -B < A.  With approximate caps the
// cap centre follows every leaving crossing: of the two points
// x +- delta m/|m|, m = u1 + u2 (u1, u2 the leaving and the next entering
// crossing minus x; u1 turned by +90 degrees when m = 0), the one deeper
// inside T_l (larger smallest edge function; ties to +), which also settles
// the zero-length arc of a circle through a vertex.  All vertices inside:
// the element itself (stored order).  No crossing otherwise: empty.
//
// The inclusion decision of the pair search (shoelace area > 0) must equal
// the plain definition's in every case, so the arithmetic follows that
// definition operation by operation, without contraction.
#pragma once

#include "nlfem_internal.h"

namespace nlfem {

constexpr int kMaxCaps = 12;   // 6 crossings + 3 vertices or 3 cap centres

// the approaches of Def. 2.3 / 2.4: 0 none, 1 nocaps, 2 approximate caps
inline int caps_mode(int approach)
{
    return approach == NLFEM_A_NOCAPS ? 1 : approach == NLFEM_A_APPROXCAPS ? 2 : 0;
}

// Writes the polygon to (px, py)[0..n) and returns n.
__device__ inline int caps_polygon(double x, double y, const double vx[3], const double vy[3], double delta,
                                   bool approx, double *px, double *py)
{
#pragma clang fp contract(off)
    const double d2 = delta * delta;
    const double sa = (vx[1] - vx[0]) * (vy[2] - vy[0]) - (vx[2] - vx[0]) * (vy[1] - vy[0]);
    const int o1 = sa >= 0.0 ? 1 : 2, o2 = sa >= 0.0 ? 2 : 1;
    const double Px[3] = {vx[0], vx[o1], vx[o2]}, Py[3] = {vy[0], vy[o1], vy[o2]};
    bool in[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double dx = Px[i] - x, dy = Py[i] - y;
        in[i] = dx * dx + dy * dy <= d2;
    }
    if (in[0] && in[1] && in[2]) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            px[i] = vx[i];
            py[i] = vy[i];
        }
        return 3;
    }
    double qx[9], qy[9];
    int kind[9];   // 0 vertex, 1 entering, 2 leaving
    int n = 0, ncross = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int i1 = i == 2 ? 0 : i + 1;
        if (in[i]) {
            qx[n] = Px[i];
            qy[n] = Py[i];
            kind[n++] = 0;
        }
        const double ex = Px[i1] - Px[i], ey = Py[i1] - Py[i];
        const double ax = Px[i] - x, ay = Py[i] - y;
        const double A = ex * ex + ey * ey;
        const double B = ax * ex + ay * ey;
        const double C = ax * ax + ay * ay - d2;
        const double D = B * B - A * C;
        const double sq = sqrt(D > 0.0 ? D : 0.0);
        double t0 = 0.0, t1 = 0.0;
        int k0 = 0, m = 0;
        if (in[i] && !in[i1]) {
            t0 = (-B + sq) / A;
            k0 = 2;
            m = 1;
        } else if (!in[i] && in[i1]) {
            t0 = (-B - sq) / A;
            k0 = 1;
            m = 1;
        } else if (!in[i] && !in[i1] && D > 0.0 && -B > 0.0 && -B < A) {
            t0 = (-B - sq) / A;
            t1 = (-B + sq) / A;
            k0 = 1;
            m = 2;
        }
        for (int c = 0; c < m; ++c) {
            const double t = c == 0 ? t0 : t1;
            const double tc = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
            qx[n] = Px[i] + tc * ex;
            qy[n] = Py[i] + tc * ey;
            kind[n++] = c == 0 ? k0 : 2;
            ++ncross;
        }
    }
    if (ncross == 0) return 0;
    int cnt = 0;
    for (int j = 0; j < n; ++j) {
        px[cnt] = qx[j];
        py[cnt] = qy[j];
        ++cnt;
        if (!approx || kind[j] != 2) continue;
        int jn = j + 1 == n ? 0 : j + 1;
        while (kind[jn] != 1) jn = jn + 1 == n ? 0 : jn + 1;
        const double u1x = qx[j] - x, u1y = qy[j] - y;
        const double u2x = qx[jn] - x, u2y = qy[jn] - y;
        double mx = u1x + u2x, my = u1y + u2y;
        if (mx == 0.0 && my == 0.0) {
            mx = -u1y;
            my = u1x;
        }
        const double mn = sqrt(mx * mx + my * my);
        const double ux = delta * (mx / mn), uy = delta * (my / mn);
        const double cx[2] = {x + ux, x - ux}, cy[2] = {y + uy, y - uy};
        double depth[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            depth[c] = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int i1 = i == 2 ? 0 : i + 1;
                const double f = (Px[i1] - Px[i]) * (cy[c] - Py[i]) - (Py[i1] - Py[i]) * (cx[c] - Px[i]);
                if (i == 0 || f < depth[c]) depth[c] = f;
            }
        }
        const int pick = depth[0] >= depth[1] ? 0 : 1;
        px[cnt] = cx[pick];
        py[cnt] = cy[pick];
        ++cnt;
    }
    return cnt;
}

// twice the signed area by the shoelace sum, halved (the decision is its
// absolute value > 0)
__device__ inline double caps_area(const double *px, const double *py, int n)
{
#pragma clang fp contract(off)
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        const int i1 = i + 1 == n ? 0 : i + 1;
        s += px[i] * py[i1] - px[i1] * py[i];
    }
    return 0.5 * s;
}

}  // namespace nlfem
