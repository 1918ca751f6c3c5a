/*
 * lidar_oracle.c -- TEST INFRASTRUCTURE, not part of the product path.
 *
 * A plain, slow, single-threaded FP64 reference of what the hot path computes
 * for one spinning-Lidar sweep (Mukherjee et al., "Fast Geometric Surface based
 * Segmentation of Point Cloud from Lidar Data", PReMI 2019):
 *
 *   1. bin the sweep into its (ring, azimuth) lattice            -- Section 2, opening
 *   2. keep every s-th azimuth firing (sub-sampling)             -- Section 2, opening
 *   3. mesh by joining lattice neighbours; the map M              -- Section 2, Mesh Construction
 *   4. per-vertex normal from weighted consecutive cross products -- Section 2, Normal Estimation
 *   5. Algorithm 1: depth-first label propagation                 -- Section 2, Algorithm 1
 *   6. labels for the points the sub-sampling skipped, and removal of
 *      segments with too few points (optional)                    -- Section 2, Segmentation
 *   7. edge scores of the segments against ground-truth surfaces  -- Section 3 (evaluation)
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * this library.  It shares no source, header or table with the GPU library.
 *
 * Grid convention (also the order Algorithm 1 visits M): cell (i, k) -- ring i
 * (0 = topmost laser), sampled column k -- is stored at k*H + i, i.e. in firing
 * order, shot by shot, because the paper builds M while the sensor spins.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - a point belongs to the ring whose elevation is nearest to atan2(z, rho)
 *     (tie: lower ring index) -- or to the ring the sensor reported for it, when
 *     given (a reported ring beyond the lattice: the point is not used) -- and to
 *     the azimuth firing round((phi - phi0)/dphi) mod W, round half away from zero;
 *   - "within range" is r_min^2 <= x^2+y^2+z^2 <= r_max^2 in FP64;
 *   - two returns in one cell: the smaller float(r^2) wins, then the lower index;
 *   - "consecutive vectors" are cycle-adjacent pairs (A,B),(B,C),...,(F,A) with
 *     both neighbours present, i.e. the incident triangles;
 *   - the weighted sum is normalised to unit length; a vertex with no incident
 *     triangle (or a zero sum) has no normal, and no edge touching it is similar;
 *   - the label counter is incremented after each seed's flood;
 *   - the similarity test reads the normal map N as stored (FP32) and takes
 *     each component difference exactly in FP64, strict '<'; the optional
 *     cosine test is n_p . n_q > cos_min with the dot product summed in FP64 as
 *     (x x' + y y') + z z';
 *   - a point's label is that of the nearest vertex (sampled, kept point) in its
 *     ring along the sweep, by firing distance (around the cylinder when it is
 *     closed), the earlier firing on a tie; 0 if its ring has no vertex or the
 *     point was not used;
 *   - a segment has "too few points" when fewer than min_segment vertices carry
 *     its label; its vertices (and the points that took its label) get label 0;
 *   - the evaluation's "edge points" are the vertices with a mesh join to a
 *     vertex of another label (or, for the ground truth, of another surface);
 *     "dilated" means grown by R lattice steps in ring and in column (Chebyshev
 *     distance, columns around the cylinder when it is closed).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared -o liblidar_oracle.so lidar_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* Neighbour t of (i, k): A,B,C,D,E,F in the paper's anticlockwise order
 * (Section 2, Normal Estimation): A=(i+1,k) B=(i+1,k+1) C=(i,k+1)
 * D=(i-1,k) E=(i-1,k-1) F=(i,k-1). */
static const int NB_DI[6] = {+1, +1, 0, -1, -1, 0};
static const int NB_DK[6] = {0, +1, +1, 0, -1, -1};

/* Cell of neighbour t of (i,k), or -1 when off the lattice.  Rings do not wrap;
 * columns wrap when the cylinder is closed (Mesh Construction, last joins). */
static int64_t neighbour_cell(int32_t H, int32_t Wp, int32_t wrap, int32_t i, int32_t k, int t)
{
    int32_t ii = i + NB_DI[t];
    int32_t kk = k + NB_DK[t];
    if (ii < 0 || ii >= H) return -1;
    if (kk < 0 || kk >= Wp) {
        if (!wrap) return -1;
        kk = (kk + Wp) % Wp;
    }
    return (int64_t)kk * H + ii;
}

/* ------------------------------------------------------------------------ */
/* Steps 1-2: binning and sub-sampling.
 * The lattice position of one point: its ring (nearest elevation, the upper ring
 * on a tie -- or the ring the sensor reported, given >= 0) and firing (nearest
 * azimuth sample, round half away from zero, modulo W), both decided in FP64.
 * Returns 0 when the point is not used (non-finite, outside the range window,
 * or a reported ring beyond the lattice), 1 otherwise; r2 receives x^2+y^2+z^2. */
static int bin_decide(const float* q, int32_t given, int32_t H, int32_t W, const double* elev, double az0,
                      double rmin2, double rmax2, int32_t* ring_out, int64_t* firing_out, double* r2_out)
{
    double x = q[0], y = q[1], z = q[2];
    if (!isfinite(x) || !isfinite(y) || !isfinite(z)) return 0;
    double rho2 = x * x + y * y;
    double r2 = rho2 + z * z;
    if (r2 < rmin2 || r2 > rmax2) return 0;                /* "within range of the Lidar" */

    int32_t ring = 0;
    if (given >= 0) {
        if (given >= H) return 0;
        ring = given;
    } else {
        /* ring: nearest elevation, first (upper) ring on a tie */
        double el = atan2(z, sqrt(rho2));
        double best = fabs(el - elev[0]);
        for (int32_t i = 1; i < H; ++i) {
            double d = fabs(el - elev[i]);
            if (d < best) { best = d; ring = i; }
        }
    }

    /* firing: nearest azimuth sample of the spin */
    double dphi = 2.0 * M_PI / (double)W;
    double jf = (atan2(y, x) - az0) / dphi;
    int64_t j = (int64_t)round(jf);
    j %= W;
    if (j < 0) j += W;
    *ring_out = ring;
    *firing_out = j;
    *r2_out = r2;
    return 1;
}

/* cell_point[c] = index of the point kept in cell c, or -1.  Returns #occupied.
 * ring_ids: each point's reported ring, or NULL to decide rings by elevation. */
int64_t oracle_bin(const float* xyz, const uint8_t* ring_ids, int64_t n, int32_t H, int32_t W, int32_t s,
                   const double* elev, double az0, double r_min, double r_max,
                   int64_t* cell_point)
{
    const int32_t Wp = W / s;
    const int64_t ncell = (int64_t)H * Wp;
    float* best_r2 = (float*)malloc(sizeof(float) * (size_t)(ncell > 0 ? ncell : 1));
    const double rmin2 = r_min * r_min;
    const double rmax2 = r_max * r_max;
    int64_t occupied = 0;

    for (int64_t c = 0; c < ncell; ++c) cell_point[c] = -1;

    for (int64_t p = 0; p < n; ++p) {
        int32_t ring;
        int64_t j;
        double r2;
        if (!bin_decide(xyz + 3 * p, ring_ids ? ring_ids[p] : -1, H, W, elev, az0, rmin2, rmax2, &ring, &j, &r2))
            continue;
        if (j % s != 0) continue;                           /* sub-sampling */
        int64_t c = (j / s) * H + ring;

        float r2f = (float)r2;
        if (cell_point[c] < 0) {
            cell_point[c] = p; best_r2[c] = r2f; ++occupied;
        } else if (r2f < best_r2[c]) {                      /* ties keep the lower index */
            cell_point[c] = p; best_r2[c] = r2f;
        }
    }
    free(best_r2);
    return occupied;
}

/* Every point's ring and firing (full resolution, before sub-sampling), or
 * ring = firing = -1 for a point that is not used. */
void oracle_point_cells(const float* xyz, const uint8_t* ring_ids, int64_t n, int32_t H, int32_t W,
                        const double* elev, double az0, double r_min, double r_max, int32_t* ring, int32_t* firing)
{
    for (int64_t p = 0; p < n; ++p) {
        int32_t i;
        int64_t j;
        double r2;
        if (bin_decide(xyz + 3 * p, ring_ids ? ring_ids[p] : -1, H, W, elev, az0, r_min * r_min, r_max * r_max, &i,
                       &j, &r2)) {
            ring[p] = i;
            firing[p] = (int32_t)j;
        } else {
            ring[p] = firing[p] = -1;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Step 3 helper: vertex index of every cell (firing order), -1 if empty. */
int64_t oracle_vertex_index(int32_t H, int32_t Wp, const uint8_t* valid, int32_t* vidx)
{
    int64_t v = 0;
    for (int64_t c = 0; c < (int64_t)H * Wp; ++c) vidx[c] = valid[c] ? (int32_t)v++ : -1;
    return v;
}

/* Step 3: the map M -- for every cell, a 6-bit mask of existing neighbours,
 * bit t = neighbour t (A..F) is a vertex and the cell itself is a vertex. */
void oracle_mesh_mask(int32_t H, int32_t Wp, int32_t wrap, const uint8_t* valid, uint8_t* mask)
{
    for (int32_t k = 0; k < Wp; ++k)
        for (int32_t i = 0; i < H; ++i) {
            int64_t c = (int64_t)k * H + i;
            uint8_t m = 0;
            if (valid[c])
                for (int t = 0; t < 6; ++t) {
                    int64_t q = neighbour_cell(H, Wp, wrap, i, k, t);
                    if (q >= 0 && valid[q]) m |= (uint8_t)(1u << t);
                }
            mask[c] = m;
        }
}

/* Step 3 (surface triangles): for each anchor (i,k) in firing order with i+1 < H,
 *   T_a = (p, A, B) and T_b = (p, B, C), each kept iff its three corners exist.
 * These are the six cycle-adjacent pairs seen from their anchor, so every
 * triangle is listed once.  Returns the triangle count; tri may be NULL. */
int64_t oracle_triangles(int32_t H, int32_t Wp, int32_t wrap, const uint8_t* valid,
                         int32_t* tri)
{
    int32_t* vidx = (int32_t*)malloc(sizeof(int32_t) * (size_t)((int64_t)H * Wp + 1));
    oracle_vertex_index(H, Wp, valid, vidx);
    int64_t T = 0;
    for (int32_t k = 0; k < Wp; ++k)
        for (int32_t i = 0; i < H; ++i) {
            int64_t p = (int64_t)k * H + i;
            if (!valid[p]) continue;
            int64_t a = neighbour_cell(H, Wp, wrap, i, k, 0);
            int64_t b = neighbour_cell(H, Wp, wrap, i, k, 1);
            int64_t cc = neighbour_cell(H, Wp, wrap, i, k, 2);
            if (a >= 0 && b >= 0 && valid[a] && valid[b]) {
                if (tri) { tri[3 * T] = vidx[p]; tri[3 * T + 1] = vidx[a]; tri[3 * T + 2] = vidx[b]; }
                ++T;
            }
            if (b >= 0 && cc >= 0 && valid[b] && valid[cc]) {
                if (tri) { tri[3 * T] = vidx[p]; tri[3 * T + 1] = vidx[b]; tri[3 * T + 2] = vidx[cc]; }
                ++T;
            }
        }
    free(vidx);
    return T;
}

/* ------------------------------------------------------------------------ */
/* Step 4: normals (Section 2, Normal Estimation).
 * V_t = q_t - p for each existing neighbour; for every cycle-adjacent pair
 * (t, t+1 mod 6) with both present, add (V_t x V_{t+1}) / (|V_t| + |V_{t+1}|);
 * the normal is that sum scaled to unit length.  FP64 throughout.
 * cell_xyz: [cells][3] float; normals: [cells][3] double; has_normal: [cells]. */
int64_t oracle_normals(int32_t H, int32_t Wp, int32_t wrap, const float* cell_xyz,
                       const uint8_t* valid, double* normals, uint8_t* has_normal)
{
    int64_t count = 0;
    for (int32_t k = 0; k < Wp; ++k)
        for (int32_t i = 0; i < H; ++i) {
            int64_t c = (int64_t)k * H + i;
            normals[3 * c] = normals[3 * c + 1] = normals[3 * c + 2] = 0.0;
            has_normal[c] = 0;
            if (!valid[c]) continue;

            double px = cell_xyz[3 * c], py = cell_xyz[3 * c + 1], pz = cell_xyz[3 * c + 2];
            double V[6][3], len[6];
            int present[6];
            for (int t = 0; t < 6; ++t) {
                int64_t q = neighbour_cell(H, Wp, wrap, i, k, t);
                present[t] = (q >= 0 && valid[q]);
                if (present[t]) {
                    V[t][0] = cell_xyz[3 * q] - px;
                    V[t][1] = cell_xyz[3 * q + 1] - py;
                    V[t][2] = cell_xyz[3 * q + 2] - pz;
                    len[t] = sqrt(V[t][0] * V[t][0] + V[t][1] * V[t][1] + V[t][2] * V[t][2]);
                }
            }
            double ax = 0.0, ay = 0.0, az = 0.0;
            int pairs = 0;
            for (int t = 0; t < 6; ++t) {
                int u = (t + 1) % 6;
                if (!present[t] || !present[u]) continue;
                double cx = V[t][1] * V[u][2] - V[t][2] * V[u][1];
                double cy = V[t][2] * V[u][0] - V[t][0] * V[u][2];
                double cz = V[t][0] * V[u][1] - V[t][1] * V[u][0];
                double w = 1.0 / (len[t] + len[u]);
                ax += w * cx;
                ay += w * cy;
                az += w * cz;
                ++pairs;
            }
            if (pairs == 0) continue;
            double norm = sqrt(ax * ax + ay * ay + az * az);
            if (!(norm > 0.0)) continue;
            normals[3 * c] = ax / norm;
            normals[3 * c + 1] = ay / norm;
            normals[3 * c + 2] = az / norm;
            has_normal[c] = 1;
            ++count;
        }
    return count;
}

/* ------------------------------------------------------------------------ */
/* Step 5: Algorithm 1 (Section 2, Segmentation by Surface Homogeneity).
 * labels[c] = 0 for empty cells, else 1..K.  Seeds are visited in firing order;
 * a popped vertex p floods each unlabelled mesh neighbour q when both have
 * normals and the test holds: pred 0 -- every normal component differs by less
 * than thr (strict); pred 1 -- n_p . n_q > cos_min.
 * normals32: the stored normal map N, [cells][3] float.  Returns K. */
static int similar_normals(const float* a, const float* b, int32_t pred, const double* thr, double cos_min)
{
    if (pred == 1) {
        double dot = ((double)a[0] * (double)b[0] + (double)a[1] * (double)b[1]) + (double)a[2] * (double)b[2];
        return dot > cos_min;
    }
    double dx = fabs((double)a[0] - (double)b[0]);
    double dy = fabs((double)a[1] - (double)b[1]);
    double dz = fabs((double)a[2] - (double)b[2]);
    return dx < thr[0] && dy < thr[1] && dz < thr[2];
}

int64_t oracle_labels_pred(int32_t H, int32_t Wp, int32_t wrap, const uint8_t* valid,
                           const uint8_t* has_normal, const float* normals32, int32_t pred,
                           const double* thr, double cos_min, int32_t* labels)
{
    const int64_t ncell = (int64_t)H * Wp;
    int64_t* stack = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ncell + 1));
    int64_t sp = 0;
    int32_t label = 1;
    for (int64_t c = 0; c < ncell; ++c) labels[c] = 0;

    for (int32_t k0 = 0; k0 < Wp; ++k0)
        for (int32_t i0 = 0; i0 < H; ++i0) {
            int64_t seed = (int64_t)k0 * H + i0;
            if (!valid[seed] || labels[seed] != 0) continue;
            labels[seed] = label;
            stack[sp++] = seed;
            while (sp > 0) {
                int64_t p = stack[--sp];
                int32_t pi = (int32_t)(p % H), pk = (int32_t)(p / H);
                for (int t = 0; t < 6; ++t) {
                    int64_t q = neighbour_cell(H, Wp, wrap, pi, pk, t);
                    if (q < 0 || !valid[q] || labels[q] != 0) continue;
                    if (!has_normal[p] || !has_normal[q]) continue;
                    if (similar_normals(normals32 + 3 * p, normals32 + 3 * q, pred, thr, cos_min)) {
                        labels[q] = label;
                        stack[sp++] = q;
                    }
                }
            }
            ++label;
        }
    free(stack);
    return (int64_t)label - 1;
}

int64_t oracle_labels(int32_t H, int32_t Wp, int32_t wrap, const uint8_t* valid,
                      const uint8_t* has_normal, const float* normals32, const double* thr,
                      int32_t* labels)
{
    return oracle_labels_pred(H, Wp, wrap, valid, has_normal, normals32, 0, thr, 0.0, labels);
}

/* ------------------------------------------------------------------------ */
/* Step 6a (Section 2, Segmentation, last paragraph): optional removal of
 * segments with too few points.  labels: [V] vertex labels 1..K; a label carried
 * by fewer than min_size vertices becomes 0.  min_size <= 1 keeps everything. */
void oracle_prune(int32_t* labels, int64_t V, int64_t K, int32_t min_size)
{
    if (min_size <= 1) return;
    int64_t* size = (int64_t*)calloc((size_t)K + 1, sizeof(int64_t));
    for (int64_t v = 0; v < V; ++v) size[labels[v]] += 1;
    for (int64_t v = 0; v < V; ++v)
        if (labels[v] > 0 && size[labels[v]] < min_size) labels[v] = 0;
    free(size);
}

/* Step 6b (Section 2, Segmentation): the points the sub-sampling skipped get
 * the label of the nearest labelled point along the horizontal sweep.  For each
 * point with ring i and firing j (ring < 0: not used -> label 0), every vertex
 * of ring i is a candidate: sampled column k at firing k s, at distance
 * |j - k s| (around the cylinder, min(d, W - d), when it is closed); the
 * nearest wins, the one at firing j - d (the earlier along the sweep) on a tie.
 * cell_label: [H * W/s] label of each cell's vertex, -1 for an empty cell. */
void oracle_backfill(int64_t n, const int32_t* ring, const int32_t* firing, int32_t H, int32_t W,
                     int32_t s, int32_t wrap, const int32_t* cell_label, int32_t* point_labels)
{
    const int32_t Wp = W / s;
    for (int64_t p = 0; p < n; ++p) {
        point_labels[p] = 0;
        if (ring[p] < 0) continue;
        const int32_t i = ring[p], j = firing[p];
        int64_t best_d = -1;
        int32_t best_label = 0;
        int best_left = 0;
        for (int32_t k = 0; k < Wp; ++k) {
            const int32_t lab = cell_label[(int64_t)k * H + i];
            if (lab < 0) continue;
            const int64_t jk = (int64_t)k * s;
            int64_t d_left, d_right;          /* the vertex before / after the point along the sweep */
            if (wrap) {
                d_left = ((int64_t)j - jk + W) % W;
                d_right = (jk - (int64_t)j + W) % W;
            } else {
                d_left = jk <= j ? j - jk : -1;
                d_right = jk >= j ? jk - j : -1;
            }
            /* its distance: the shorter way round; reached from the left on a tie */
            int64_t d;
            int left;
            if (d_left >= 0 && (d_right < 0 || d_left <= d_right)) { d = d_left; left = 1; }
            else { d = d_right; left = 0; }
            if (best_d < 0 || d < best_d || (d == best_d && left && !best_left)) {
                best_d = d; best_label = lab; best_left = left;
            }
        }
        point_labels[p] = best_label;
    }
}

/* ------------------------------------------------------------------------ */
/* The whole path on one sweep.  Outputs are compact, in vertex (firing) order:
 *   vertices [V][3] float (the kept input point, bit-exact)
 *   normals  [V][3] float (FP64 result rounded once; zero = no normal)
 *   labels   [V] int32 (1..K, 0 after segment removal), triangles [T][3] int32,
 *   vertex_point [V] int32, counts {V, T, K}
 *   point_labels [n] int32 (optional): every input point's label (step 6b)
 * pred / cos_min select the similarity test (Algorithm 1's component test, or
 * the cosine test); min_segment > 1 removes smaller segments (step 6a).
 * Capacity: V <= H*(W/s), T <= 2*H*(W/s).  normals64 (optional, [V][3]) receives
 * the unrounded FP64 normals.  Returns 0, or -1 on a bad argument. */
int oracle_mesh_segment_ex(const float* xyz, const uint8_t* ring_ids, int64_t n, int32_t H, int32_t W, int32_t s,
                           int32_t wrap, const double* elev, double az0, double r_min,
                           double r_max, int32_t pred, const double* thr, double cos_min,
                           int32_t min_segment, float* vertices, float* normals, int32_t* labels,
                           int32_t* triangles, int32_t* vertex_point, int64_t* counts,
                           double* normals64, int32_t* point_labels)
{
    if (H < 1 || W < 1 || s < 1 || W % s != 0) return -1;
    const int32_t Wp = W / s;
    if (wrap && Wp < 3) return -1;
    const int64_t ncell = (int64_t)H * Wp;
    int64_t* cell_point = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
    uint8_t* valid = (uint8_t*)malloc((size_t)ncell);
    uint8_t* hasn = (uint8_t*)malloc((size_t)ncell);
    float* cxyz = (float*)malloc(sizeof(float) * 3 * (size_t)ncell);
    double* n64 = (double*)malloc(sizeof(double) * 3 * (size_t)ncell);
    float* n32 = (float*)malloc(sizeof(float) * 3 * (size_t)ncell);
    int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)ncell);

    oracle_bin(xyz, ring_ids, n, H, W, s, elev, az0, r_min, r_max, cell_point);
    for (int64_t c = 0; c < ncell; ++c) {
        valid[c] = cell_point[c] >= 0;
        for (int d = 0; d < 3; ++d)
            cxyz[3 * c + d] = valid[c] ? xyz[3 * cell_point[c] + d] : 0.0f;
    }
    oracle_normals(H, Wp, wrap, cxyz, valid, n64, hasn);
    for (int64_t q = 0; q < 3 * ncell; ++q) n32[q] = (float)n64[q];
    int64_t K = oracle_labels_pred(H, Wp, wrap, valid, hasn, n32, pred, thr, cos_min, lab);
    int64_t T = oracle_triangles(H, Wp, wrap, valid, triangles);

    int64_t V = 0;
    for (int64_t c = 0; c < ncell; ++c) {
        if (!valid[c]) continue;
        for (int d = 0; d < 3; ++d) {
            vertices[3 * V + d] = cxyz[3 * c + d];
            normals[3 * V + d] = n32[3 * c + d];
            if (normals64) normals64[3 * V + d] = n64[3 * c + d];
        }
        labels[V] = lab[c];
        if (vertex_point) vertex_point[V] = (int32_t)cell_point[c];
        ++V;
    }
    oracle_prune(labels, V, K, min_segment);
    if (point_labels) {
        /* the cell labels after removal, then every point from its ring and firing */
        int64_t v = 0;
        for (int64_t c = 0; c < ncell; ++c) lab[c] = valid[c] ? labels[v++] : -1;
        int32_t* pr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        int32_t* pf = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
        oracle_point_cells(xyz, ring_ids, n, H, W, elev, az0, r_min, r_max, pr, pf);
        oracle_backfill(n, pr, pf, H, W, s, wrap, lab, point_labels);
        free(pr); free(pf);
    }
    counts[0] = V;
    counts[1] = T;
    counts[2] = K;
    free(cell_point); free(valid); free(hasn); free(cxyz); free(n64); free(n32); free(lab);
    return 0;
}

int oracle_mesh_segment(const float* xyz, int64_t n, int32_t H, int32_t W, int32_t s,
                        int32_t wrap, const double* elev, double az0, double r_min,
                        double r_max, const double* thr, float* vertices, float* normals,
                        int32_t* labels, int32_t* triangles, int32_t* vertex_point,
                        int64_t* counts, double* normals64)
{
    return oracle_mesh_segment_ex(xyz, NULL, n, H, W, s, wrap, elev, az0, r_min, r_max, 0, thr, 0.0, 0,
                                  vertices, normals, labels, triangles, vertex_point, counts, normals64,
                                  NULL);
}

/* ------------------------------------------------------------------------ */
/* Step 7: edge scores (Section 3: the segments are compared with the ground
 * truth through their edge points, each side dilated, and scored by
 * precision, recall and F1).
 * label[c] is the label of cell c's vertex (-1: empty cell), truth[c] its
 * ground-truth surface id.  A vertex is a segment edge when one of its mesh
 * joins (the six neighbours A..F) reaches a vertex of another label, a truth
 * edge when one reaches a vertex of another truth id.  A segment edge is
 * found when some truth edge lies within R rings and R columns of it; a truth
 * edge is recalled when some segment edge does.
 * out = {segment edges, truth edges, found, recalled}. */
static int col_within(int32_t Wp, int32_t wrap, int32_t k, int32_t k2, int32_t R)
{
    int32_t d = k > k2 ? k - k2 : k2 - k;
    if (wrap && Wp - d < d) d = Wp - d;
    return d <= R;
}

void oracle_edge_scores(int32_t H, int32_t Wp, int32_t wrap, const int32_t* label, const int32_t* truth,
                        int32_t R, int64_t* out)
{
    const int64_t cells = (int64_t)H * Wp;
    uint8_t* seg_edge = calloc((size_t)(cells > 0 ? cells : 1), 1);
    uint8_t* tru_edge = calloc((size_t)(cells > 0 ? cells : 1), 1);
    out[0] = out[1] = out[2] = out[3] = 0;
    for (int32_t k = 0; k < Wp; ++k)
        for (int32_t i = 0; i < H; ++i) {
            const int64_t c = (int64_t)k * H + i;
            if (label[c] < 0) continue;
            for (int t = 0; t < 6; ++t) {
                const int64_t q = neighbour_cell(H, Wp, wrap, i, k, t);
                if (q < 0 || label[q] < 0) continue;
                if (label[q] != label[c]) seg_edge[c] = 1;
                if (truth[q] != truth[c]) tru_edge[c] = 1;
            }
            out[0] += seg_edge[c];
            out[1] += tru_edge[c];
        }
    /* every pair of edge cells within the window, by brute force */
    for (int32_t k = 0; k < Wp; ++k)
        for (int32_t i = 0; i < H; ++i) {
            const int64_t c = (int64_t)k * H + i;
            if (!seg_edge[c] && !tru_edge[c]) continue;
            int found = 0, recalled = 0;
            for (int32_t k2 = 0; k2 < Wp; ++k2) {
                if (!col_within(Wp, wrap, k, k2, R)) continue;
                for (int32_t i2 = i - R; i2 <= i + R; ++i2) {
                    if (i2 < 0 || i2 >= H) continue;
                    const int64_t q = (int64_t)k2 * H + i2;
                    if (tru_edge[q]) found = 1;
                    if (seg_edge[q]) recalled = 1;
                }
            }
            if (seg_edge[c] && found) ++out[2];
            if (tru_edge[c] && recalled) ++out[3];
        }
    free(seg_edge);
    free(tru_edge);
}
