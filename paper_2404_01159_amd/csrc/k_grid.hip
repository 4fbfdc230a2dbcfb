// k_grid.hip -- association (Alg. 1, Eq. 2) through an index of the
// reference vectors, three objectives.
//
// The association of a row is the vector of largest cosine (lowest index on
// ties).  Here each row looks only at a short candidate list that provably
// holds that vector and every vector tied with it, and computes the binary64
// cosines of those candidates exactly as the full re-rank does, so the
// result is the same as a scan of all K vectors.
//
// Index.  A direction x >= 0 is mapped to the simplex point q of x / r
// (componentwise; r > 0 is the range vector of the last adaptation, scaled
// to max 1, so that the adapted lattice is again a uniform lattice in q) and
// q (its first two coordinates) to a cell of a G x G grid over [0, 1]^2.  A
// cell C is the square clipped to the simplex, a polygon of at most five
// vertices; the directions of the rows that land in C form the cone over
// that polygon (up to rounding).  Distances between directions are chord
// lengths |u - v| of unit vectors (a metric, monotone in the angle), so no
// inverse trigonometric function is needed.  For each cell, built whenever
// V changes:
//   u_c    the unit direction of the polygon's vertex mean; rho the largest
//          distance from u_c to a vertex (the largest to any point of the
//          cell: the distance to a fixed direction is quasi-convex on the
//          plane of q, so its maximum over the polygon is at a vertex)
//   b      an upper bound of the distance from any point of C to its nearest
//          vector: min over the vectors k of the cells around C of the largest
//          distance from a vertex to v_k (again attained at a vertex)
//   box    the smallest square of cells around C whose boundary (clipped to
//          the simplex) is farther than b + rho from u_c: that ball around
//          u_c is convex in q, so it lies inside the box
//   P      the vectors in the box whose distance to the cell is at most b
//          (the least over its edges, each the distance to a great-circle
//          arc; the cell's own vectors always): any vector that is the
//          nearest for some row direction in C is within b of it
//   list   P without the vectors that a champion (the vector of largest
//          cosine at a vertex or at u_c) beats at every vertex by more than
//          1e-12: the cosine difference is linear on the cone, so such a
//          vector loses to the champion for every row direction in C, with
//          a margin far above binary64 rounding
// Lists longer than kSlot, cells whose box would pass kStage cells from
// C, and cells with no vector within kNear cells are marked for a full scan
// (correct for any vector set, counted as full rescans).  The same pass
// gives Eq. 5's gamma of each vector whose nearest other vector provably lies
// in its cell's staged neighbourhood (the nearest staged one is closer than
// the neighbourhood's boundary); if any vector is left, it asks for the full
// gamma pass.  Each cell's list
// has a slot of kSlot records of its own; the cells' ranges of vector
// positions are allocated by one atomic add per wavefront, so the order of
// the vectors in memory varies from build to build (no result depends on it).
//
// Two objectives.  The index is a line: a direction x >= 0 maps to its share
// u = (x1 / r1) / (x0 / r0 + x1 / r1) of the scaled simplex (u = j / H for
// the adapted lattice again) and u to one of G = K equal cells.  In the
// quadrant the angle of a direction is monotone in u, so a row needs no
// candidate list: it scans its own cell and the cells on either side, then
// keeps stepping outward on a side while the cosine to the direction of that
// side's next cell boundary (moved outward by far more than u's rounding)
// is not below the best cosine found by more than 1e-12.  Every vector
// beyond that boundary has a smaller cosine than the boundary direction, so
// the vector of largest cosine and all vectors tied with it have been seen.
// A walk past kLineWalk cells on a side, or any vector outside the quadrant
// (which the bucket leaves out and flags), makes the row scan all vectors
// (counted).  Eq. 5's gamma of each vector comes from the same walk, with
// the vector as the row, itself and the vectors parallel to it skipped; a
// walk past the limit leaves it to the full pass.
#include <algorithm>

#include "rvea_dev.h"
#include "rvea_index.h"
#include "rvea_internal.h"

namespace rvea {

constexpr int kSlot = 24;      // list records per cell (longer lists: a full scan)
constexpr int kChamps = 6;     // champions per cell: five vertices and the centre
constexpr int kGridRowLanes = 4;  // lanes per row of the association
constexpr double kDomMargin = 1e-12;

struct D3 {
    double x, y, z;
};
__device__ __forceinline__ D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__device__ __forceinline__ double dot3(const D3 &a, const D3 &b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
__device__ __forceinline__ D3 sub3(const D3 &a, const D3 &b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ D3 unit3(const D3 &a)
{
    const double inv = 1.0 / sqrt(dot3(a, a));
    return d3(a.x * inv, a.y * inv, a.z * inv);
}

// Binary32 versions for the geometric tests of the build.  Those tests only
// have to keep every possible candidate, so they run in single precision
// with hardware square root and reciprocal (1 ulp) and a slack kSlack on
// every comparison, far above their rounding (chords of unit vectors in
// [0, 2], each off by well under 1e-6); the tests that decide exclusion
// for good (domination) stay in binary64.
constexpr float kSlack = 4e-6f;
struct F3 {
    float x, y, z;
};
__device__ __forceinline__ F3 f3(float x, float y, float z) { return F3{x, y, z}; }
__device__ __forceinline__ F3 f3of(const D3 &a) { return F3{(float)a.x, (float)a.y, (float)a.z}; }
__device__ __forceinline__ float fdot(const F3 &a, const F3 &b)
{
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
__device__ __forceinline__ F3 fsub(const F3 &a, const F3 &b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ F3 fcross(const F3 &a, const F3 &b)
{
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ F3 funit(const F3 &a)
{
    const float inv = __builtin_amdgcn_rcpf(fsqrt(fdot(a, a)));
    return f3(a.x * inv, a.y * inv, a.z * inv);
}
// squared chord, and the chord (minima and maxima of chords are taken on
// the squares, with one square root at the end: the square root is
// monotone, so the result moves by at most its last-bit rounding)
__device__ __forceinline__ float fchord2(const F3 &a, const F3 &b)
{
    const F3 d = fsub(a, b);
    return fdot(d, d);
}
__device__ __forceinline__ float fchord(const F3 &a, const F3 &b) { return fsqrt(fchord2(a, b)); }
__device__ float farc_chord(const F3 &u, const F3 &a, const F3 &b, const F3 &n, bool valid)
{
    const float ends2 = fminf(fchord2(u, a), fchord2(u, b));
    if (!valid) return fsqrt(ends2);
    const float un = fdot(u, n);
    const F3 w = f3(u.x - un * n.x, u.y - un * n.y, u.z - un * n.z);
    const float wn = fsqrt(fdot(w, w));
    if (wn > 0.0f && fdot(fcross(a, w), n) >= 0.0f && fdot(fcross(w, b), n) >= 0.0f)
        return fsqrt(fminf(ends2, 2.0f * un * un * __builtin_amdgcn_rcpf(1.0f + wn)));
    return fsqrt(ends2);
}
__device__ float farc_chord_of(const F3 &u, const F3 &A, const F3 &B)
{
    const F3 a = funit(A), b = funit(B);
    const F3 n = fcross(a, b);
    const float nn = fsqrt(fdot(n, n));
    const bool valid = nn > 1e-30f;
    const float inv = valid ? __builtin_amdgcn_rcpf(nn) : 0.0f;
    return farc_chord(u, a, b, f3(n.x * inv, n.y * inv, n.z * inv), valid);
}
__device__ __forceinline__ F3 flift(float q1, float q2, const double *r)
{
    return f3((float)r[0] * q1, (float)r[1] * q2, (float)r[2] * (1.0f - q1 - q2));
}

// the direction of simplex point (q1, q2) scaled back by r
__device__ __forceinline__ D3 lift(double q1, double q2, const double *r)
{
    return d3(r[0] * q1, r[1] * q2, r[2] * (1.0 - q1 - q2));
}


// One cell's geometry, held in LDS by the cell's workgroup: the square
// [a, a+h] x [b, b+h] clipped to q1 + q2 <= 1 as five vertices in order
// (with corner sums s0 <= s1 = s3 <= s2: the whole square when s2 <= 1, a
// pentagon when only the far corner is cut, a triangle (or a point) when
// s1 > 1; fewer distinct vertices repeat the last, which adds only
// zero-length edges), their unit directions in binary64 (champions and
// domination) and binary32 (the geometric tests), the unit normals of the
// edges' planes, u_c and rho.
constexpr int kNv = 5;
struct CellGeo {
    double X[kNv][3];
    float Xf[kNv][3], Nf[kNv][3];
    int nok[kNv];
    double uc[3];
    float ucf[3];
    float rho;
};

__device__ __forceinline__ F3 ld3(const float (&a)[3]) { return f3(a[0], a[1], a[2]); }
__device__ __forceinline__ D3 ld3(const double (&a)[3]) { return d3(a[0], a[1], a[2]); }

// the cell's vertex v (v < kNv) in q, for a cell (ci, cj) with ci + cj <= G
// (its corner (a, b) on or below the diagonal; at ci + cj = G all five are
// that corner, up to rounding)
__device__ __forceinline__ void cell_vertex(int G, int c, int v, double &px, double &py)
{
    const double h = 1.0 / G;
    const double a = (c / G) * h, b = (c % G) * h;
    const double s1 = a + h + b, s2 = a + b + 2.0 * h;
    if (s2 <= 1.0) {  // the whole square
        const double x[kNv] = {a, a + h, a + h, a, a}, y[kNv] = {b, b, b + h, b + h, b + h};
        px = x[v];
        py = y[v];
    } else if (s1 <= 1.0) {  // the corner (a+h, b+h) cut off
        const double x[kNv] = {a, a + h, a + h, 1.0 - b - h, a};
        const double y[kNv] = {b, b, 1.0 - a - h, b + h, b + h};
        px = x[v];
        py = y[v];
    } else {  // only the corner (a, b) inside
        const double x[kNv] = {a, 1.0 - b, a, a, a}, y[kNv] = {b, b, 1.0 - a, 1.0 - a, 1.0 - a};
        px = x[v];
        py = y[v];
    }
}

// the geometry of a live cell, by the workgroup: lanes 0..4 the vertices,
// lane 5 u_c; then lanes 0..4 the edge normals and rho (g.rho as the bits
// of a non-negative float, combined by an LDS max)
__device__ void cell_geo(const RunView &R, int c, CellGeo &g, int lane)
{
    if (lane <= kNv) {
        double px = 0.0, py = 0.0;
        if (lane < kNv) {
            cell_vertex(R.gG, c, lane, px, py);
        } else {
            for (int v = 0; v < kNv; ++v) {
                double x, y;
                cell_vertex(R.gG, c, v, x, y);
                px += x;
                py += y;
            }
            px /= kNv;
            py /= kNv;
        }
        const D3 X = unit3(lift(px, py, R.gr));
        const F3 Xf = f3of(X);
        double *dst = lane < kNv ? g.X[lane] : g.uc;
        float *dsf = lane < kNv ? g.Xf[lane] : g.ucf;
        dst[0] = X.x;
        dst[1] = X.y;
        dst[2] = X.z;
        dsf[0] = Xf.x;
        dsf[1] = Xf.y;
        dsf[2] = Xf.z;
    }
    if (lane == 0) g.rho = 0.0f;
    __syncthreads();
    if (lane < kNv) {
        const F3 p = ld3(g.Xf[lane]), q = ld3(g.Xf[(lane + 1) % kNv]);
        const F3 n = fcross(p, q);
        const float nn = fsqrt(fdot(n, n));
        g.nok[lane] = nn > 1e-30f;
        const float inv = g.nok[lane] ? __builtin_amdgcn_rcpf(nn) : 0.0f;
        g.Nf[lane][0] = n.x * inv;
        g.Nf[lane][1] = n.y * inv;
        g.Nf[lane][2] = n.z * inv;
        atomicMax(reinterpret_cast<unsigned int *>(&g.rho),
                  __float_as_uint(fchord(ld3(g.ucf), p)));
    }
    __syncthreads();
}

// least distance from unit v to the cell (v outside it: the least over the
// polygon's edges, each an arc of a great circle)
__device__ float cell_dist(const CellGeo &g, const F3 &v)
{
    float d = INFINITY;
    for (int e = 0; e < kNv; ++e)
        d = fminf(d, farc_chord(v, ld3(g.Xf[e]), ld3(g.Xf[(e + 1) % kNv]), ld3(g.Nf[e]),
                                g.nok[e] != 0));
    return d;
}

__device__ __forceinline__ D3 gvh_at(const RunView &R, int64_t p)
{
    const double4 v = reinterpret_cast<const double4 *>(R.gvh)[p];
    return d3(v.x, v.y, v.z);
}

// a vector of the box belongs to P (cell c's own vectors always do); b
// already holds its slack
__device__ __forceinline__ bool in_p(const CellGeo &g, const D3 &v, bool own, float b)
{
    if (own) return true;
    const F3 vf = f3of(v);
    // a lower bound of the distance first
    if (fchord(ld3(g.ucf), vf) - g.rho - 2.0f * kSlack > b) return false;
    return cell_dist(g, vf) - kSlack <= b;
}

// the champions of a cell (LDS): unit directions and vector ids (-1: none)
struct Champs {
    double v[kChamps][3];
    int32_t j[kChamps];
};

// some champion beats v at every vertex by more than the margin
__device__ __forceinline__ bool dominated(const CellGeo &g, const Champs &ch, const D3 &v, int32_t j)
{
    for (int d = 0; d < kChamps; ++d) {
        if (ch.j[d] < 0 || ch.j[d] == j) continue;
        const D3 w = sub3(ld3(ch.v[d]), v);
        bool all = true;
        for (int e = 0; e < kNv; ++e) all = all && dot3(ld3(g.X[e]), w) > kDomMargin;
        if (all) return true;
    }
    return false;
}

// first position of a range of n items allocated by the whole wavefront
// with one atomic add on *total (every lane active; lanes without items pass 0)
__device__ __forceinline__ int64_t wave_alloc(int n, unsigned long long *total)
{
    const int incl = wave_incl_scan(n);
    const int sum = __builtin_amdgcn_readlane(incl, 63);
    unsigned long long base = 0;
    if ((threadIdx.x & 63) == 0 && sum > 0) base = atomicAdd(total, (unsigned long long)sum);
    base = __shfl(base, 0, 64);
    return (int64_t)base + incl - n;
}

// ------------------------------------------------------------- line
constexpr int kLineWalk = 64;        // cells a row steps outward on a side at most
constexpr double kLineEps = 1e-12;   // outward shift of a boundary's u
constexpr double kLineTau = 1e-12;   // cosine margin of the stopping test


// binary64 cosine of f (norm nrm) and the direction of share u
__device__ __forceinline__ double line_bound(double f0, double f1, double nrm, double u,
                                             const double *r)
{
    const double b0 = (1.0 - u) * r[0], b1 = u * r[1];
    return (f0 * b0 + f1 * b1) / (nrm * sqrt(b0 * b0 + b1 * b1));
}

// ------------------------------------------------------------- build
// vectors per cell (counts start at zero: the last build cleared them); a
// rebuild after an adaptation skips this pass, the adaptation having
// counted each vector as it wrote it (k_vectors.hip)
__device__ __forceinline__ void grid_bucket_body(const RunView &R, int64_t bx, int gate)
{
    if (!gate && *R.vchanged == 0) return;
    const int64_t j = bx * 256 + threadIdx.x;
    if (j == 0) {
        R.gtot[1] = 0;  // the full gamma pass not needed (yet)
        R.gtot[2] = 0;  // no vector outside the line (yet)
    }
    if (j >= R.K) return;
    int c;
    if (R.m == 3) {
        c = cell_of(R.V[j * 3], R.V[j * 3 + 1], R.V[j * 3 + 2], R.gr, R.gG);
        if (c < 0) c = 0;  // cannot happen for a nonzero vector >= 0
    } else {
        double u;
        c = line_cell_of(R.V[j * 2], R.V[j * 2 + 1], R.gr, R.gG, u);
    }
    R.gcell[j] = c;
    if (c >= 0) atomicAdd(&R.gcnt[c], 1);
}

// each cell's range of positions (one atomic add per wavefront); the
// counts become the fill cursors (grid: counting up from zero, cleared again
// by the cells pass; line: counting down to zero)
__device__ __forceinline__ void grid_ranges_body(const RunView &R, int64_t bx, int gate)
{
    if (!gate && *R.vchanged == 0) return;
    const int64_t c = bx * 256 + threadIdx.x;
    const int64_t cells = index_cells(R.m, R.gG);
    const int n = c < cells ? R.gcnt[c] : 0;
    const int64_t st = wave_alloc(n, &R.gtot[0]);
    if (c < cells) {
        R.gstart[c] = (int32_t)st;
        R.gnum[c] = n;
        if (R.m == 3) R.gcnt[c] = 0;
    }
}

// vectors into their cells' ranges, with their unit directions (grid) or
// (v, |v|) (line, whose build ends here: the range allocator cleared)
__device__ __forceinline__ void grid_fill_body(const RunView &R, int64_t bx, int gate)
{
    if (!gate && *R.vchanged == 0) return;
    const int64_t j = bx * 256 + threadIdx.x;
    if (R.m != 3 && j == 0) R.gtot[0] = 0;
    if (j >= R.K) return;
    const int c = R.gcell[j];
    if (c < 0) {  // outside the line: every row scans all vectors
        R.gtot[2] = 1;
        return;
    }
    const int64_t p = R.m == 3 ? R.gstart[c] + atomicAdd(&R.gcnt[c], 1)
                               : R.gstart[c] + atomicSub(&R.gcnt[c], 1) - 1;
    R.gvec[p] = (int32_t)j;
    if (R.m != 3) {
        reinterpret_cast<double4 *>(R.gvh)[p] =
            make_double4(R.V[j * 2], R.V[j * 2 + 1], R.vn[j], 0.0);
        return;
    }
    const double inv = 1.0 / R.vn[j];
    reinterpret_cast<double4 *>(R.gvh)[p] =
        make_double4(R.V[j * 3] * inv, R.V[j * 3 + 1] * inv, R.V[j * 3 + 2] * inv, 0.0);
}

// Wavefront-wide minimum / best (largest value, lowest id on ties) over
// the 64 lanes (every lane active): the pairings of partner32 within each
// half, then the two halves' results read out and combined (the result is
// uniform).
__device__ __forceinline__ double wave_fmin(double v)
{
    v = fmin(v, partner32<0>(v));
    v = fmin(v, partner32<1>(v));
    v = fmin(v, partner32<2>(v));
    v = fmin(v, partner32<3>(v));
    v = fmin(v, partner32<4>(v));
    RVEA_ASSERT_FULL_WAVE();
    const double a = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                      __builtin_amdgcn_readlane(__double2loint(v), 0));
    const double b = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 32),
                                      __builtin_amdgcn_readlane(__double2loint(v), 32));
    return fmin(a, b);
}
__device__ __forceinline__ int wave_imin(int v)
{
    v = min(v, partner32<0>(v));
    v = min(v, partner32<1>(v));
    v = min(v, partner32<2>(v));
    v = min(v, partner32<3>(v));
    v = min(v, partner32<4>(v));
    RVEA_ASSERT_FULL_WAVE();
    return min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 32));
}
template <int L>
__device__ __forceinline__ void best_step(double &v, int32_t &j, int32_t &p)
{
    const double ov = partner32<L>(v);
    const int32_t oj = partner32<L>((int)j), op = partner32<L>((int)p);
    if (ov > v || (ov == v && oj < j)) {
        v = ov;
        j = oj;
        p = op;
    }
}
__device__ __forceinline__ void wave_best(double &v, int32_t &j, int32_t &p)
{
    best_step<0>(v, j, p);
    best_step<1>(v, j, p);
    best_step<2>(v, j, p);
    best_step<3>(v, j, p);
    best_step<4>(v, j, p);
    RVEA_ASSERT_FULL_WAVE();
    const double v0 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 0),
                                       __builtin_amdgcn_readlane(__double2loint(v), 0));
    const double v1 = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 32),
                                       __builtin_amdgcn_readlane(__double2loint(v), 32));
    const int32_t j0 = __builtin_amdgcn_readlane(j, 0), j1 = __builtin_amdgcn_readlane(j, 32);
    const int32_t p0 = __builtin_amdgcn_readlane(p, 0), p1 = __builtin_amdgcn_readlane(p, 32);
    const bool second = v1 > v0 || (v1 == v0 && j1 < j0);
    v = second ? v1 : v0;
    j = second ? j1 : j0;
    p = second ? p1 : p0;
}

constexpr int kNear = 3;  // the covering search looks at the (2 kNear + 1)^2 cells around

// The vectors of the (2 kStage + 1)^2 cells around a cell, staged in LDS by
// its workgroup: unit direction, id, raw vector and norm (the list record),
// and the cell offset.  kStageCap entries at most.
constexpr int kStage = 4;
constexpr int kStageW = 2 * kStage + 1;
constexpr int kStageCap = 192;
struct Stage {
    double vh[kStageCap][3];
    double rec[kStageCap][4];
    int32_t j[kStageCap];
    int8_t di[kStageCap], dj[kStageCap];
    int n;
};

// least distance from unit u to the boundary of the box of cells of radius
// k around (ci, cj), clipped to the simplex (sides on the grid's edge, where
// the simplex ends, do not count): the sides are exact grid lines in
// binary64 (their ends on the simplex's edge), lifted in binary32, so the
// callers compare it with their slack
__device__ float box_side_min(const RunView &R, int ci, int cj, int k, const F3 &u)
{
    const int G = R.gG;
    const int i0 = max(0, ci - k), i1 = min(G - 1, ci + k);
    const int j0 = max(0, cj - k), j1 = min(G - 1, cj + k);
    const double h = 1.0 / G;
    float lo = INFINITY;
    if (i0 > 0) {
        const double x = i0 * h, ya = j0 * h, yb = fmin((j1 + 1) * h, 1.0 - x);
        if (yb >= ya)
            lo = fminf(lo, farc_chord_of(u, flift((float)x, (float)ya, R.gr),
                                         flift((float)x, (float)yb, R.gr)));
    }
    if (i1 < G - 1) {
        const double x = (i1 + 1) * h, ya = j0 * h, yb = fmin((j1 + 1) * h, 1.0 - x);
        if (yb >= ya)
            lo = fminf(lo, farc_chord_of(u, flift((float)x, (float)ya, R.gr),
                                         flift((float)x, (float)yb, R.gr)));
    }
    if (j0 > 0) {
        const double y = j0 * h, xa = i0 * h, xb = fmin((i1 + 1) * h, 1.0 - y);
        if (xb >= xa)
            lo = fminf(lo, farc_chord_of(u, flift((float)xa, (float)y, R.gr),
                                         flift((float)xb, (float)y, R.gr)));
    }
    if (j1 < G - 1) {
        const double y = (j1 + 1) * h, xa = i0 * h, xb = fmin((i1 + 1) * h, 1.0 - y);
        if (xb >= xa)
            lo = fminf(lo, farc_chord_of(u, flift((float)xa, (float)y, R.gr),
                                         flift((float)xb, (float)y, R.gr)));
    }
    return lo;
}

// The cells a row or a vector can land in: ci + cj <= G (cell_of clamps q
// to the simplex, so floor(q1 G) + floor(q2 G) <= G); the others lie outside
// it, hold no vector and are never read.  Row ci of them holds G cells for
// ci <= 1 and G - ci + 1 after; t-th such cell in row order.
__device__ __forceinline__ int64_t tri_start(int G, int ci)
{
    return ci == 0 ? 0 : (int64_t)G + (int64_t)(ci - 1) * (G + 1) - (int64_t)(ci - 1) * ci / 2;
}
static int64_t grid_live_cells(int G) { return (int64_t)G + (int64_t)G * (G + 1) / 2 - 1; }

// One wavefront per cell (the simplex's cells only, in row order): the
// neighbourhood staged in LDS; b from the cells within kNear; the box
// radius (lane k tests radius k, at most kStage); the champions and the
// list from the staged box vectors, written into the cell's slot at each
// lane's prefix.
// A neighbourhood over kStageCap vectors or a box over kStage marks the cell
// for a full scan.  Also clears the cell's fill cursor and the range
// allocator for the next build.
__device__ __forceinline__ void grid_cells_body(const RunView &R, int64_t bx, int gate)
{
    if (!gate && *R.vchanged == 0) return;
    const int G = R.gG;
    const int lane = threadIdx.x;
    if (bx >= (int64_t)G + (int64_t)G * (G + 1) / 2 - 1) return;  // uniform
    int ci = 0;  // the row of cell bx: the last row starting at or before it
    for (int hi = G - 1; ci < hi;) {
        const int mid = (ci + hi + 1) >> 1;
        if (tri_start(G, mid) <= bx) ci = mid; else hi = mid - 1;
    }
    const int cj = (int)(bx - tri_start(G, ci));
    const int c = ci * G + cj;
    __shared__ CellGeo g;
    __shared__ Champs ch;
    __shared__ Stage st;
    if (lane == 0) {
        if (c == 0) R.gtot[0] = 0;
        R.gcnt[c] = 0;
    }
    // stage: each lane's cells of the neighbourhood, their vector counts
    // scanned over the wave, then the vectors
    int cnt[2] = {0, 0}, from[2] = {0, 0};
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int t = lane + 64 * u;
        if (t < kStageW * kStageW) {
            const int i = ci - kStage + t / kStageW, jj = cj - kStage + t % kStageW;
            if (i >= 0 && i < G && jj >= 0 && jj < G) {
                from[u] = R.gstart[i * G + jj];
                cnt[u] = R.gnum[i * G + jj];
            }
        }
    }
    const int mine0 = cnt[0] + cnt[1];
    const int incl0 = wave_incl_scan(mine0);
    const int nst = __builtin_amdgcn_readlane(incl0, 63);
    cell_geo(R, c, g, lane);
    bool full = nst > kStageCap;
    if (!full) {
        int q = incl0 - mine0;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = lane + 64 * u;
            for (int k = 0; k < cnt[u]; ++k, ++q) {
                const int p = from[u] + k;
                const int32_t j = R.gvec[p];
                const D3 v = gvh_at(R, p);
                st.vh[q][0] = v.x;
                st.vh[q][1] = v.y;
                st.vh[q][2] = v.z;
                st.j[q] = j;
                st.di[q] = (int8_t)(t / kStageW - kStage);
                st.dj[q] = (int8_t)(t % kStageW - kStage);
                st.rec[q][0] = R.V[(int64_t)j * 3];
                st.rec[q][1] = R.V[(int64_t)j * 3 + 1];
                st.rec[q][2] = R.V[(int64_t)j * 3 + 2];
                st.rec[q][3] = R.vn[j];
            }
        }
    }
    __syncthreads();
    // the least distance from u_c to the boundary of the box of cells of
    // radius k, on lane k <= kStage: for the box test below and, at radius
    // kStage, for the own vectors' gamma
    float bsm = INFINITY;
    if (!full && lane <= kStage) bsm = box_side_min(R, ci, cj, lane, ld3(g.ucf));
    // Eq. 5's gamma of the cell's own vectors: the largest binary64 cosine
    // to another vector that is not parallel to it (cosine below 1, as the
    // full pass computes it), kept when the staged neighbourhood provably
    // holds that vector (the nearest staged one is closer than the
    // neighbourhood's boundary: every own vector lies within rho of u_c, so
    // its distance to that boundary is at least u_c's less rho); otherwise
    // the full gamma pass is asked for
    {
        const int own = kStage * kStageW + kStage;  // the centre cell's lane
        const int oq0 = __builtin_amdgcn_readlane(incl0 - mine0, own);
        const int on = full ? 0 : __builtin_amdgcn_readlane(cnt[0], own);
        bool need = full && __builtin_amdgcn_readlane(cnt[0], own) > 0;
        const float lo =
            __int_as_float(__builtin_amdgcn_readlane(__float_as_int(bsm), kStage)) - g.rho -
            kSlack;
        for (int o = oq0; o < oq0 + on; ++o) {  // uniform
            const int32_t id = st.j[o];
            const double vi[3] = {st.rec[o][0], st.rec[o][1], st.rec[o][2]};
            const double vni = st.rec[o][3];
            const F3 ui = f3(st.vh[o][0], st.vh[o][1], st.vh[o][2]);
            double gb = -INFINITY;
            float dmin = INFINITY;
            for (int q = lane; q < nst; q += 64) {
                if (st.j[q] == id) continue;
                double sd = vi[0] * st.rec[q][0];
                sd = fma(vi[1], st.rec[q][1], sd);
                sd = fma(vi[2], st.rec[q][2], sd);
                const double cv = sd / (vni * st.rec[q][3]);
                if (cv >= 1.0) continue;
                gb = fmax(gb, cv);
                dmin = fminf(dmin, fchord2(ui, f3(st.vh[q][0], st.vh[q][1], st.vh[q][2])));
            }
            gb = -wave_fmin(-gb);
            dmin = fsqrt((float)wave_fmin((double)dmin));  // the squared minimum's root
            if (dmin < INFINITY && lo > dmin + 2.0f * kSlack) {
                if (lane == 0) R.gamma[id] = acos(gb < -1.0 ? -1.0 : gb);
            } else {
                need = true;
            }
        }
        if (need && lane == 0) R.gtot[1] = 1;
    }
    // b: the best covering vector among the cells within kNear
    float best = INFINITY;
    if (!full) {
        for (int q = lane; q < nst; q += 64) {
            if (abs(st.di[q]) > kNear || abs(st.dj[q]) > kNear) continue;
            const F3 v = f3(st.vh[q][0], st.vh[q][1], st.vh[q][2]);
            float cov = 0.0f;
            for (int e = 0; e < kNv; ++e) cov = fmaxf(cov, fchord2(ld3(g.Xf[e]), v));
            best = fminf(best, cov);  // squared
        }
    }
    best = fsqrt((float)wave_fmin((double)best));
    full = full || !(best < INFINITY);
    const float b = best + kSlack;
    int kc = 0x7fffffff;
    if (!full) {  // lane k: does the box of radius k hold the ball of radius b + rho?
        const int k = lane;
        const bool ok = k <= kStage && bsm > b + g.rho + 2.0f * kSlack;
        kc = wave_imin(ok ? k : 0x7fffffff);
        full = kc == 0x7fffffff;
    }
    if (!full) {
        // members of P among this lane's staged entries (q = lane + 64 u),
        // and the champions: largest cosine at each vertex and at u_c
        uint32_t mem = 0;
        double bv[kChamps];
        int32_t bj[kChamps], bq[kChamps];
#pragma unroll
        for (int d = 0; d < kChamps; ++d) {
            bv[d] = -INFINITY;
            bj[d] = 0x7fffffff;
            bq[d] = -1;
        }
        for (int u = 0; lane + 64 * u < nst; ++u) {
            const int q = lane + 64 * u;
            if (abs(st.di[q]) > kc || abs(st.dj[q]) > kc) continue;
            const D3 v = ld3(st.vh[q]);
            if (!in_p(g, v, st.di[q] == 0 && st.dj[q] == 0, b)) continue;
            mem |= 1u << u;
            const int32_t j = st.j[q];
#pragma unroll
            for (int d = 0; d < kChamps; ++d) {
                const double cv = dot3(d < kNv ? ld3(g.X[d]) : ld3(g.uc), v);
                if (cv > bv[d] || (cv == bv[d] && j < bj[d])) {
                    bv[d] = cv;
                    bj[d] = j;
                    bq[d] = q;
                }
            }
        }
#pragma unroll
        for (int d = 0; d < kChamps; ++d) wave_best(bv[d], bj[d], bq[d]);
        if (lane < kChamps) {
            int32_t q = -1;
#pragma unroll
            for (int d = 0; d < kChamps; ++d) q = lane == d ? bq[d] : q;
            ch.j[lane] = q < 0 ? -1 : st.j[q];
            ch.v[lane][0] = q < 0 ? 0.0 : st.vh[q][0];
            ch.v[lane][1] = q < 0 ? 0.0 : st.vh[q][1];
            ch.v[lane][2] = q < 0 ? 0.0 : st.vh[q][2];
        }
        __syncthreads();
        // the list: members no champion beats on the whole cell
        uint32_t keep = 0;
        int mine = 0;
        for (int u = 0; lane + 64 * u < nst; ++u) {
            const int q = lane + 64 * u;
            if (((mem >> u) & 1u) && !dominated(g, ch, ld3(st.vh[q]), st.j[q])) {
                keep |= 1u << u;
                ++mine;
            }
        }
        const int incl = wave_incl_scan(mine);
        const int n = __builtin_amdgcn_readlane(incl, 63);
        full = n > kSlot;
        // the cell's records in its own slot, each lane at its prefix
        const int64_t base = (int64_t)c * kSlot;
        if (!full) {
            int64_t o = base + incl - mine;
            for (int u = 0; lane + 64 * u < nst; ++u) {
                if (!((keep >> u) & 1u)) continue;
                const int q = lane + 64 * u;
                reinterpret_cast<double4 *>(R.lrec)[o] =
                    make_double4(st.rec[q][0], st.rec[q][1], st.rec[q][2], st.rec[q][3]);
                R.lidx[o] = st.j[q];
                ++o;
            }
            if (lane == 0) {
                R.lstart[c] = (int32_t)base;
                R.lcnt[c] = n;
            }
        }
    }
    if (full && lane == 0) {
        R.lstart[c] = -1;
        R.lcnt[c] = -1;
    }
}

// ----------------------------------------------------------- association
// kGridRowLanes lanes per merged row: f' = F - z* in binary64 and |f'| as
// the re-rank forms them, the row's cell, the binary64 cosines of the
// cell's list (or of every vector for a cell marked for a full scan), the
// best with the lowest index on ties, then as the re-rank: angle, APD of
// Eq. 4 and the per-vector minimum of (APD, row).
__device__ __forceinline__ void assoc_grid_body(const RunView &R, int64_t bx)
{
    const int sub = threadIdx.x % kGridRowLanes;
    const int64_t i = (bx * 256 + threadIdx.x) / kGridRowLanes;
    const bool in = i < R.M;
    const int64_t pop = *R.t_done;
    const uint32_t *zb = zbuf(R, pop + 1);
    const float *Fm = fm_of(R, pop);
    float rf[3] = {0.f, 0.f, 0.f};
    if (in)
        for (int k = 0; k < 3; ++k) rf[k] = Fm[i * 3 + k];
    const bool act = in && R.mvalid[i];
    double f[3];
    for (int k = 0; k < 3; ++k) {
        const float zk = ord_dec(zb[k]);
        f[k] = act ? (double)rf[k] - (double)zk : 0.0;
    }
    double n2 = f[0] * f[0];
    n2 = fma(f[1], f[1], n2);
    n2 = fma(f[2], f[2], n2);
    const double nrm = sqrt(n2);
    const bool live = act && nrm > 0.0;
    int32_t st = -1, n = 0;
    if (live) {
        const int c = cell_of(f[0], f[1], f[2], R.gr, R.gG);
        if (c >= 0) {
            st = R.lstart[c];
            n = R.lcnt[c];
        }
    }
    const bool full = live && (st < 0 || n <= 0);
    // the best cosine, its vector and that vector's gamma (loaded with the
    // candidate, so the APD needs no further round trip)
    double best = -INFINITY, bg = 0.0;
    int64_t bj = R.K;
    if (live && !full) {
        const double4 *rec = reinterpret_cast<const double4 *>(R.lrec) + st;
        for (int e = sub; e < n; e += kGridRowLanes) {
            const double4 v = rec[e];
            const int64_t j = R.lidx[st + e];
            const double gj = R.gamma[j];
            double s = f[0] * v.x;
            s = fma(f[1], v.y, s);
            s = fma(f[2], v.z, s);
            const double cv = s / (nrm * v.w);
            if (cv > best || (cv == best && j < bj)) {
                best = cv;
                bj = j;
                bg = gj;
            }
        }
    } else if (full) {
        for (int64_t j = sub; j < R.K; j += kGridRowLanes) {
            double s = f[0] * R.V[j * 3];
            s = fma(f[1], R.V[j * 3 + 1], s);
            s = fma(f[2], R.V[j * 3 + 2], s);
            const double cv = s / (nrm * R.vn[j]);
            if (cv > best || (cv == best && j < bj)) {
                best = cv;
                bj = j;
                bg = R.gamma[j];
            }
        }
    }
    // the row's four lanes are a quad: combine them by the quad swaps of
    // partner32 (every lane active)
    static_assert(kGridRowLanes == 4, "rows are quads");
    {
        double ob = partner32<0>(best), og = partner32<0>(bg);
        int64_t oj = partner32<0>(bj);
        if (ob > best || (ob == best && oj < bj)) {
            best = ob;
            bj = oj;
            bg = og;
        }
        ob = partner32<1>(best);
        og = partner32<1>(bg);
        oj = partner32<1>(bj);
        if (ob > best || (ob == best && oj < bj)) {
            best = ob;
            bj = oj;
            bg = og;
        }
    }
    if (!in || sub != 0) return;
    if (!act) {
        R.assoc[i] = -1;
        R.apd[i] = INFINITY;
        return;
    }
    if (!live) {  // the row is the ideal point: vector 0, APD 0
        R.assoc[i] = 0;
        R.apd[i] = 0.0;
        atomicMin(&R.key[0], (unsigned long long)i);
        return;
    }
    if (full) atomicAdd(&R.counters[1], 1ull);
    const double gj = bj < R.K ? bg : R.gamma[0];
    if (bj >= R.K) bj = 0;
    const double cc = best > 1.0 ? 1.0 : (best < -1.0 ? -1.0 : best);
    const double th = acos(cc);
    const double a = (1.0 + *R.pen * th / gj) * nrm;
    R.assoc[i] = (int32_t)bj;
    R.apd[i] = a;
    const unsigned long long ab = (unsigned long long)__double_as_longlong(a);
    atomicMin(&R.key[bj], ((ab >> R.kb) << R.kb) | (unsigned long long)i);
}

// One lane per merged row (two objectives): f' and |f'| as the re-rank forms
// them, the row's cell on the line, the walk outward (or a scan of every
// vector if the walk is too long or the line incomplete), then as the
// re-rank: angle, APD of Eq. 4 and the per-vector minimum of (APD, row).
__device__ __forceinline__ void assoc_line_body(const RunView &R, int64_t bx)
{
    const int64_t i = bx * 256 + threadIdx.x;
    if (i >= R.M) return;
    if (!R.mvalid[i]) {
        R.assoc[i] = -1;
        R.apd[i] = INFINITY;
        return;
    }
    const int64_t pop = *R.t_done;
    const uint32_t *zb = zbuf(R, pop + 1);
    const float *Fm = fm_of(R, pop);
    const double f0 = (double)Fm[i * 2] - (double)ord_dec(zb[0]);
    const double f1 = (double)Fm[i * 2 + 1] - (double)ord_dec(zb[1]);
    double n2 = f0 * f0;
    n2 = fma(f1, f1, n2);
    const double nrm = sqrt(n2);
    if (!(nrm > 0.0)) {  // the row is the ideal point: vector 0, APD 0
        R.assoc[i] = 0;
        R.apd[i] = 0.0;
        atomicMin(&R.key[0], (unsigned long long)i);
        return;
    }
    const int G = R.gG;
    const double *r = R.gr;
    double best = -INFINITY;
    int64_t bj = R.K;
    double u;
    const int c = line_cell_of(f0, f1, r, G, u);
    bool full = c < 0 || R.gtot[2] != 0;
    if (!full) {
        const double4 *rec = reinterpret_cast<const double4 *>(R.gvh);
        // scan one cell's vectors into (best, bj)
        auto scan = [&](int cc) {
            const int st = R.gstart[cc], n = R.gnum[cc];
            for (int e = 0; e < n; ++e) {
                const double4 v = rec[st + e];
                const int64_t j = R.gvec[st + e];
                double s = f0 * v.x;
                s = fma(f1, v.y, s);
                const double cv = s / (nrm * v.z);
                if (cv > best || (cv == best && j < bj)) {
                    best = cv;
                    bj = j;
                }
            }
        };
        scan(c);
        // the cells on either side always; beyond them while the boundary
        // direction (moved outward by kLineEps in u) could still tie
        int lo = c, hi = c, steps = 0;
        while (lo > 0 && !full) {
            if (lo < c && line_bound(f0, f1, nrm, (double)lo / G + kLineEps, r) + kLineTau < best)
                break;
            scan(--lo);
            full = ++steps > kLineWalk;
        }
        steps = 0;
        while (hi < G - 1 && !full) {
            if (hi > c &&
                line_bound(f0, f1, nrm, (double)(hi + 1) / G - kLineEps, r) + kLineTau < best)
                break;
            scan(++hi);
            full = ++steps > kLineWalk;
        }
    }
    if (full) {
        best = -INFINITY;
        bj = R.K;
        for (int64_t j = 0; j < R.K; ++j) {
            double s = f0 * R.V[j * 2];
            s = fma(f1, R.V[j * 2 + 1], s);
            const double cv = s / (nrm * R.vn[j]);
            if (cv > best || (cv == best && j < bj)) {
                best = cv;
                bj = j;
            }
        }
        atomicAdd(&R.counters[1], 1ull);
    }
    if (bj >= R.K) bj = 0;
    const double gj = R.gamma[bj];
    const double cc = best > 1.0 ? 1.0 : (best < -1.0 ? -1.0 : best);
    const double th = acos(cc);
    const double a = (1.0 + *R.pen * th / gj) * nrm;
    R.assoc[i] = (int32_t)bj;
    R.apd[i] = a;
    const unsigned long long ab = (unsigned long long)__double_as_longlong(a);
    atomicMin(&R.key[bj], ((ab >> R.kb) << R.kb) | (unsigned long long)i);
}

// Eq. 5's gamma of each vector on the line (one lane per vector): the walk
// of the association with the vector as the row, skipping itself and the
// vectors exactly parallel to it (binary64 cosine 1 or more), as the full
// gamma pass does; the largest cosine's angle (pi/2 without another
// vector).  A vector outside the line or a walk past kLineWalk cells on a
// side asks for the full gamma pass instead.
__device__ __forceinline__ void line_gamma_body(const RunView &R, int64_t bx, int gate)
{
    if (!gate && *R.vchanged == 0) return;
    const int64_t i = bx * 256 + threadIdx.x;
    if (i >= R.K) return;
    const double f0 = R.V[i * 2], f1 = R.V[i * 2 + 1], nrm = R.vn[i];
    const int G = R.gG;
    const double *r = R.gr;
    double u;
    const int c = line_cell_of(f0, f1, r, G, u);
    if (c < 0 || R.gtot[2] != 0) {
        R.gtot[1] = 1;
        return;
    }
    const double4 *rec = reinterpret_cast<const double4 *>(R.gvh);
    double best = -INFINITY;
    auto scan = [&](int cc) {
        const int st = R.gstart[cc], n = R.gnum[cc];
        for (int e = 0; e < n; ++e) {
            if (R.gvec[st + e] == (int32_t)i) continue;
            const double4 v = rec[st + e];
            double s = f0 * v.x;
            s = fma(f1, v.y, s);
            const double cv = s / (nrm * v.z);
            if (cv >= 1.0) continue;
            best = fmax(best, cv);
        }
    };
    scan(c);
    int lo = c, hi = c, steps = 0;
    bool full = false;
    while (lo > 0 && !full) {
        if (lo < c && line_bound(f0, f1, nrm, (double)lo / G + kLineEps, r) + kLineTau < best)
            break;
        scan(--lo);
        full = ++steps > kLineWalk;
    }
    steps = 0;
    while (hi < G - 1 && !full) {
        if (hi > c && line_bound(f0, f1, nrm, (double)(hi + 1) / G - kLineEps, r) + kLineTau < best)
            break;
        scan(++hi);
        full = ++steps > kLineWalk;
    }
    if (full) {
        R.gtot[1] = 1;
        return;
    }
    R.gamma[i] = best > -INFINITY ? acos(best < -1.0 ? -1.0 : best) : 1.5707963267948966;
}

// ------------------------------------------------------------- kernels
__global__ __launch_bounds__(256) void k_grid_bucket(RunView R, int gate)
{
    grid_bucket_body(R, blockIdx.x, gate);
}
__global__ __launch_bounds__(256) void k_grid_ranges(RunView R, int gate)
{
    grid_ranges_body(R, blockIdx.x, gate);
}
__global__ __launch_bounds__(256) void k_grid_fill(RunView R, int gate)
{
    grid_fill_body(R, blockIdx.x, gate);
}
__global__ __launch_bounds__(64) void k_grid_cells(RunView R, int gate)
{
    grid_cells_body(R, blockIdx.x, gate);
}
__global__ __launch_bounds__(256) void k_assoc_grid(RunView R) { assoc_grid_body(R, blockIdx.x); }
__global__ __launch_bounds__(256) void k_assoc_line(RunView R) { assoc_line_body(R, blockIdx.x); }
__global__ __launch_bounds__(256) void k_line_gamma(RunView R, int gate)
{
    line_gamma_body(R, blockIdx.x, gate);
}

// batched: blockIdx.x decoded into (run, local block) through the span
// table; the build phases run for the runs whose vectors changed
__global__ __launch_bounds__(256) void kb_grid_ranges(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    grid_ranges_body(runs[sp[s].run], blockIdx.x - sp[s].start, 0);
}
__global__ __launch_bounds__(256) void kb_grid_fill(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    grid_fill_body(runs[sp[s].run], blockIdx.x - sp[s].start, 0);
}
// one cell per workgroup: more per workgroup would keep more registers live
// in this heavy body, and it is the open generations' cost that matters here
__global__ __launch_bounds__(64) void kb_grid_cells(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    grid_cells_body(runs[sp[s].run], blockIdx.x - sp[s].start, 0);
}
__global__ __launch_bounds__(256) void kb_assoc_grid(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    assoc_grid_body(runs[sp[s].run], blockIdx.x - sp[s].start);
}
__global__ __launch_bounds__(256) void kb_assoc_line(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    assoc_line_body(runs[sp[s].run], blockIdx.x - sp[s].start);
}
__global__ __launch_bounds__(256) void kb_line_gamma(const RunView *runs, const Span *sp, int n)
{
    const int s = find_span(sp, n, blockIdx.x);
    line_gamma_body(runs[sp[s].run], blockIdx.x - sp[s].start, 0);
}

// ------------------------------------------------------------- launchers
hipError_t launch_grid_build(const RunView &R, hipStream_t s, int force)
{
    if (R.gG <= 0) return hipSuccess;
    const unsigned vb = (unsigned)((R.K + 255) / 256);
    const int64_t cells = index_cells(R.m, R.gG);
    k_grid_bucket<<<vb, 256, 0, s>>>(R, force);
    k_grid_ranges<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(R, force);
    k_grid_fill<<<vb, 256, 0, s>>>(R, force);
    if (R.m == 3)
        k_grid_cells<<<(unsigned)grid_live_cells(R.gG), 64, 0, s>>>(R, force);
    else
        k_line_gamma<<<vb, 256, 0, s>>>(R, force);
    return hipGetLastError();
}

hipError_t launch_grid_rebuild(const RunView &R, hipStream_t s)
{
    if (R.gG <= 0) return hipSuccess;
    const unsigned vb = (unsigned)((R.K + 255) / 256);
    const int64_t cells = index_cells(R.m, R.gG);
    k_grid_ranges<<<(unsigned)((cells + 255) / 256), 256, 0, s>>>(R, 0);
    k_grid_fill<<<vb, 256, 0, s>>>(R, 0);
    if (R.m == 3)
        k_grid_cells<<<(unsigned)grid_live_cells(R.gG), 64, 0, s>>>(R, 0);
    else
        k_line_gamma<<<vb, 256, 0, s>>>(R, 0);
    return hipGetLastError();
}

hipError_t launch_assoc_grid(const RunView &R, hipStream_t s)
{
    if (R.m == 3) {
        const int64_t threads = R.M * kGridRowLanes;
        k_assoc_grid<<<(unsigned)((threads + 255) / 256), 256, 0, s>>>(R);
    } else {
        k_assoc_line<<<(unsigned)((R.M + 255) / 256), 256, 0, s>>>(R);
    }
    return hipGetLastError();
}

hipError_t launch_batch_grid(int phase, int cls, const RunView *runs, const Span *sp, int n,
                             int64_t blocks, hipStream_t s)
{
    const dim3 g((unsigned)blocks);
    switch (phase) {
    case BP_ASSOC:
        if (cls == (kIndexedClass | 3))
            kb_assoc_grid<<<g, 256, 0, s>>>(runs, sp, n);
        else
            kb_assoc_line<<<g, 256, 0, s>>>(runs, sp, n);
        break;
    case BP_GRID_RANGES: kb_grid_ranges<<<g, 256, 0, s>>>(runs, sp, n); break;
    case BP_GRID_FILL: kb_grid_fill<<<g, 256, 0, s>>>(runs, sp, n); break;
    case BP_GRID_CELLS:  // class: the objective count (3: cells, 2: the line's gamma)
        if (cls == 3)
            kb_grid_cells<<<g, 64, 0, s>>>(runs, sp, n);
        else
            kb_line_gamma<<<g, 256, 0, s>>>(runs, sp, n);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t grid_phase_blocks(int phase, const RunView &R)
{
    if (R.gG <= 0) return 0;
    const int64_t cells = index_cells(R.m, R.gG);
    switch (phase) {
    case BP_ASSOC: return ((R.m == 3 ? R.M * kGridRowLanes : R.M) + 255) / 256;
    case BP_GRID_FILL: return (R.K + 255) / 256;
    case BP_GRID_RANGES: return (cells + 255) / 256;
    case BP_GRID_CELLS: return R.m == 3 ? grid_live_cells(R.gG) : (R.K + 255) / 256;
    }
    return 0;
}

int grid_slot() { return kSlot; }

int grid_side(int m, int64_t K)
{
    if (m == 2) return K < 2 ? 2 : (int)K;  // a line of K cells
    if (m != 3) return 0;
    int G = (int)ceil(1.0 * sqrt((double)K));
    return G < 2 ? 2 : G;
}

}  // namespace rvea
