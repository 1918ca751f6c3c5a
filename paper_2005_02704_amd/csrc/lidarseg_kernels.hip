// HIP kernels for gfx950 (MI355X): bin -> sub-sample -> mesh -> normals -> labels.
//
// One batch of frames runs as a chain of nine grid-stride kernels (eleven when
// point labels, segment removal or edge scores are asked for); each kernel
// walks its work items (point blocks, lattice tiles, border slots, blocks of
// vertex slots or frames) across every frame of the batch, reading the
// per-frame descriptors from device memory, so the same launches (and the same
// captured graph) serve any batch that fits the workspace.  No kernel waits for
// another workgroup, and no work item is handed out through a shared counter.
//
// Stage map (Mukherjee et al., PReMI 2019, Section 2):
//   k_bin      points -> (ring, firing) cell, sub-sampling, nearest return     [opening paragraph]
//   k_count    vertices, triangles and occupancy bits of each tile             [Mesh Construction]
//   k_geom     per tile in LDS: vertex and triangle numbering, mesh triangles,
//              normals                                                         [Mesh Construction,
//                                                                               Normal Estimation]
//   k_cc       per tile in LDS: similarity of joins, local segments           [Algorithm 1]
//   k_merge    unions of the similar joins that cross tile borders             [Algorithm 1]
//   k_compress pointer jumping on the segments joined across borders
//   k_flatten  segment roots flagged and counted; key cells reset
//   k_scan     per frame: roots before each labelling item (their rank base)
//   k_resolve  every vertex's root; label = 1 + rank of that root; segment sizes
//   k_post     (when asked for) segment removal and every input point's label  [Segmentation, last paragraph]
//   k_score    (when asked for) edge scores of the labels against truth ids   [Section 3, evaluation]
//
// Algorithm 1 floods through neighbours whose normal components differ by less
// than the thresholds; that test is symmetric, so the flood's label classes are
// the connected components of the similar-join graph, and numbering them by the
// first vertex in the visiting order gives the same labels.  Union-find here
// always links the larger root under the smaller, so a root is the smallest
// vertex of its segment and the labels follow from ranking the roots.
#include <functional>

#include "lidarseg_internal.h"

namespace lidarseg {
namespace {

constexpr int WALK_LIMIT = 1 << 20;          // steps of any pointer walk (parents strictly
                                             // decrease, so a walk is far shorter; the cap
                                             // only guarantees that every loop ends)
constexpr float COL_GUARD = 0.02f;           // firings: FP32 firing estimate decides outside this band
constexpr int COL_GUARD_MAX_W = 16384;       // wider sweeps always decide the firing in FP64
constexpr double LEN2_FLOOR = 1e-300;        // added to squared edge lengths: an absent edge
                                             // (zero vector) gets a tiny positive length

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Number of set bits of `mask` in the lanes below this one.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ int wave_sum(int x) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) x += __shfl_xor(x, d, 64);
    return x;
}

// A frame descriptor's pointer as a global-memory pointer.  Pointers read from
// device memory are generic to the compiler, which then emits flat accesses;
// those also count against the LDS wait counter, so every wait for an LDS read
// would wait for them as well.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Dense outputs that no later stage reads (vertices, vertex points, labels,
// point labels) are written with non-temporal stores, so they do not displace
// what the next stages read back (the normals, the forest) from the caches.
// The normals stay ordinary stores (k_cc reads them), and so do the
// triangles: a lane writes one only where the triangle exists, and streamed
// partial lines would cost whole-line writes.

__device__ __forceinline__ const FrameDesc* frames_of(const BatchHeader* h) {
    return reinterpret_cast<const FrameDesc*>(h + 1);
}

// A cell is occupied when its key names one of the frame's points (the bound
// also keeps a stale key from ever indexing outside the frame's points).
__device__ __forceinline__ bool occupied(uint64_t key, int64_t n_points) {
    return key != KEY_EMPTY && (int64_t)(uint32_t)key < n_points;
}

// The point index of cell c's key: the key's low 32 bits (0xFFFFFFFF when the
// cell is empty).  Reading the index alone keeps half the registers.
__device__ __forceinline__ uint32_t key_index(const uint64_t* keys, int64_t c) {
    return reinterpret_cast<const uint32_t*>(keys)[2 * c];
}

__device__ __forceinline__ bool occupied_index(uint32_t idx, int64_t n_points) {
    return (int64_t)idx < n_points;
}

// Largest frame f with F[f].*off <= x (offsets ascend with f).
template <int32_t FrameDesc::*OFF>
__device__ __forceinline__ int frame_of(const FrameDesc* F, int nf, int x) {
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (F[mid].*OFF <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// x / H for the small non-negative LDS indices used here (x < 2^13, H <= 128).
__device__ __forceinline__ int div_small(int x, float inv_h) {
    return (int)(((float)x + 0.5f) * inv_h);
}

// Nearest ring elevation, ties to the upper (lower-index) ring.  e is strictly
// descending.  The nearest of a sorted table is one of the two that bracket el.
__device__ __forceinline__ int nearest_ring(const double* e, int H, double el) {
    if (el >= e[0]) return 0;
    if (el <= e[H - 1]) return H - 1;
    // first j with e[j] <= el; 1 <= j <= H-1
    int lo = 1, hi = H - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (e[mid] <= el) hi = mid; else lo = mid + 1;
    }
    const double d_up = fabs(el - e[lo - 1]);
    const double d_dn = fabs(el - e[lo]);
    return (d_dn < d_up) ? lo : lo - 1;
}

// The FP64 decisions, out of line.  They run only for points whose FP32
// estimate falls inside a guard band, in a pass after the fast one.
__device__ __attribute__((noinline)) int ring_fp64(const double* e, int H, double z, double rho2) {
    return nearest_ring(e, H, atan2(z, sqrt(rho2)));
}

__device__ __attribute__((noinline)) int firing_fp64(double x, double y, double az0, double dphi) {
    return (int)round((atan2(y, x) - az0) / dphi);
}

// The cell of a used point (firing j in [0, W), ring i), its key, and the record
// j * H + i for point labels: shared by the fast and the exact pass.
__device__ __forceinline__ void bin_store(unsigned long long* keys, int32_t* pcell, int64_t p, int ring, int j, int W,
                                          int H, int s, double r2) {
    if (j < 0) j += W;
    if (j < 0) j += W;
    if (j >= W) j -= W;
    if (j >= W) j -= W;
    if (pcell) pcell[p] = j * H + ring;
    int k = j;
    if (s > 1) {
        k = j / s;
        if (k * s != j) return;
    }
    const unsigned long long key =
        ((unsigned long long)__float_as_uint((float)r2) << 32) | (unsigned long long)(uint32_t)p;
    atomicMin(keys + (int64_t)k * H + ring, key);
}

// atan(q) ~= q * P(q^2) on [0, 1]: a degree-8 polynomial in q^2 fitted for this
// library (weighted least squares on Chebyshev nodes); largest error 6e-9 rad
// in exact arithmetic, 1e-7 rad evaluated in FP32.
__constant__ float ATAN_P[9] = {0.99999988634662018f, -0.3333259686572097f, 0.19985904654765521f, -0.14161216713985597f, 0.10498906521530744f, -0.072347856186199572f, 0.039780477295818122f, -0.014400943859970152f, 0.0024566295904995218f};

// atan2 in FP32 from the polynomial above: reduce to q = min/max in [0, 1], then
// reflect by octant.  Error below 5e-7 rad; NaN when x = y = 0.
__device__ __forceinline__ float atan2_poly(float y, float x) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float q = fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay));
    const float s = q * q;
    float p = ATAN_P[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) p = fmaf(p, s, ATAN_P[k]);
    float a = q * p;
    if (ay > ax) a = 1.57079632679489662f - a;
    if (x < 0.0f) a = 3.14159265358979324f - a;
    return copysignf(a, y);
}

constexpr int RING_LUT = 1024;   // buckets of the ring lookup table (tan of elevation)

// ---------------------------------------------------------------------------
// Binning and sub-sampling.  One work item = POINT_BLOCK points of one frame;
// each workgroup takes a contiguous range of items, so its per-frame tables
// change rarely.  The cell keeps min((bits(float(r^2)) << 32) | point), i.e.
// the nearest return, then the lower index: independent of thread order.
//
// The ring and firing are FP64 decisions (nearest ring elevation; firing =
// round((atan2(y, x) - az0) / dphi)).  Each is first decided in FP32: the ring
// from t = z / sqrt(x^2 + y^2) against the tangents of the midpoints between
// ring elevations (tan is increasing, so the comparison is the same), through a
// lookup table over t; the firing from a polynomial atan2.  The estimates are
// within a few 1e-7 (relative for t, radians for the azimuth), so when they lie
// farther than a guard band from every decision boundary the FP64 decision is
// the same and is not computed.  Inside a band the FP64 expression decides.
template <int NT>
__global__ __launch_bounds__(NT, 6) void k_bin(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int PPT = POINT_BLOCK / NT;  // points per thread per item
    static_assert(PPT <= 4, "the given rings of a thread's points fit one word");
    __shared__ double s_elev[MAX_RINGS];
    __shared__ float s_T[MAX_RINGS];       // s_T[i]: tan of the midpoint of rings i and i+1 (descending)
    __shared__ uint8_t s_lut[RING_LUT];    // ring at the lower edge of each t bucket
    __shared__ float s_lo, s_inv;          // t at the first bucket's lower edge, buckets per unit t
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int nb = hdr->total_pblk;
    const int per = (nb + (int)gridDim.x - 1) / (int)gridDim.x;
    const int b0 = blockIdx.x * per, b1 = min(nb, b0 + per);
    int cur = -1;
    for (int b = b0; b < b1; ++b) {
        const int f = frame_of<&FrameDesc::pblk_off>(F, nf, b);
        const FrameDesc* fd = F + f;
        const int H = fd->H;
        if (f != cur) {
            __syncthreads();
            for (int i = threadIdx.x; i < H; i += NT) s_elev[i] = ws.elev[fd->elev_off + i];
            __syncthreads();
            for (int i = threadIdx.x; i + 1 < H; i += NT) s_T[i] = (float)tan(0.5 * (s_elev[i] + s_elev[i + 1]));
            __syncthreads();
            // buckets span the boundaries with a margin; outside them the table's
            // end values (ring H-1 below, 0 above) are exact
            const float thi = H > 1 ? s_T[0] : 0.0f, tlo = H > 1 ? s_T[H - 2] : 0.0f;
            const float pad = 0.01f * (thi - tlo) + 1e-3f;
            const float lo = tlo - pad, inv = (float)RING_LUT / (thi - tlo + 2.0f * pad);
            for (int k = threadIdx.x; k < RING_LUT; k += NT) {
                const float e = lo + (float)k / inv;
                // rings whose upper boundary lies above e: first i with s_T[i] <= e
                int a = 0, c = H - 1;
                while (a < c) {
                    const int m = (a + c) >> 1;
                    if (s_T[m] <= e) c = m; else a = m + 1;
                }
                s_lut[k] = (uint8_t)a;
            }
            if (threadIdx.x == 0) { s_lo = lo; s_inv = inv; }
            __syncthreads();
            cur = f;
        }
        const int W = fd->W, s = fd->s;
        const double az0 = fd->az0, dphi = fd->dphi, rmin2 = fd->rmin2, rmax2 = fd->rmax2;
        const float az0f = (float)az0;
        const float inv_dphif = (float)(1.0 / dphi);
        const bool col_fast = W <= COL_GUARD_MAX_W;
        const float lo = s_lo, inv = s_inv;
        const auto xyz = gmem(fd->xyz);
        unsigned long long* keys = reinterpret_cast<unsigned long long*>(ws.keys + fd->cell_off);
        const int64_t p0 = (int64_t)(b - fd->pblk_off) * POINT_BLOCK + threadIdx.x;
        const int64_t np = fd->n_points;
        // all loads of the item first, so their latencies overlap: unconditional
        // (a lane past the frame's last point reads that point and drops it
        // below), since a load under a lane mask is waited for at once
        float px[PPT], py[PPT], pz[PPT];
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
            const int64_t p = p0 + r * NT;
            const auto q = xyz + 3 * (p < np ? p : np - 1);   // np >= 1: the item holds a point
            px[r] = q[0];
            py[r] = q[1];
            pz[r] = q[2];
        }
        int32_t* const pcell = fd->point_labels ? ws.pcell + fd->pt_off : nullptr;
        const auto rings = gmem(fd->rings);   // the sensor's own ring of each point, if given
        // the given rings of the item's points, one byte each, loaded with the
        // points (a load inside the pass below would also wait for the atomics
        // issued before it)
        uint32_t given4 = 0;
        if (rings) {
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
                const int64_t p = p0 + r * NT;
                given4 |= (uint32_t)rings[p < np ? p : np - 1] << (8 * r);
            }
        }
        // fast pass: FP32 estimates; a point inside a guard band is only flagged
        uint32_t hard = 0;
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
            const int64_t p = p0 + r * NT;
            const float xf = px[r], yf = py[r], zf = pz[r];
            bool used = p < np && isfinite(xf) && isfinite(yf) && isfinite(zf);
            const double x = xf, y = yf, z = zf;
            const double rho2 = x * x + y * y;   // products of floats are exact in FP64
            const double r2 = rho2 + z * z;
            used = used && r2 >= rmin2 && r2 <= rmax2;
            const int given = rings ? (int)((given4 >> (8 * r)) & 0xffu) : -1;
            used = used && given < H;
            if (!used) {
                if (pcell && p < np) pcell[p] = -1;
                continue;
            }
            // ring: the reported one, or t against the midpoint tangents, through
            // the bucket table
            const float t = zf * __builtin_amdgcn_rsqf(fmaf(xf, xf, yf * yf));
            int ring = given;
            bool exact = given < 0 && !isfinite(t);
            if (given < 0 && !exact) {
                const float bf = fminf(fmaxf((t - lo) * inv, 0.0f), (float)(RING_LUT - 1));
                ring = s_lut[(int)bf];
                for (int k = 0; k < MAX_RINGS && ring > 0 && t > s_T[ring - 1]; ++k) --ring;
                exact = (ring > 0 && fabsf(t - s_T[ring - 1]) <= 2e-6f * fabsf(s_T[ring - 1]) + 1e-7f) ||
                        (ring + 1 < H && fabsf(t - s_T[ring]) <= 2e-6f * fabsf(s_T[ring]) + 1e-7f);
            }
            // firing: |az0| <= 2 pi, so the rounded firing lies in [-2W, 2W)
            const float jff = (atan2_poly(yf, xf) - az0f) * inv_dphif;
            exact = exact || !(col_fast && fabsf(jff - floorf(jff) - 0.5f) > COL_GUARD);
            if (exact) {
                hard |= 1u << r;
                continue;
            }
            bin_store(keys, pcell, p, ring, (int)floorf(jff + 0.5f), W, H, s, r2);
        }
        // exact pass (rare): both decisions of the flagged points in FP64
        if (hard) {
#pragma unroll 1
            for (int r = 0; r < PPT; ++r) {
                if (!((hard >> r) & 1u)) continue;
                const int64_t p = p0 + r * NT;
                const double x = xyz[3 * p], y = xyz[3 * p + 1], z = xyz[3 * p + 2];
                const double rho2 = x * x + y * y;
                const double r2 = rho2 + z * z;
                const int ring = rings ? (int)rings[p] : ring_fp64(s_elev, H, z, rho2);
                bin_store(keys, pcell, p, ring, firing_fp64(x, y, az0, dphi), W, H, s, r2);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Vertices and triangles owned by each tile (from the key grid alone), so that
// the tile stages can number their vertices and triangles without waiting on
// other tiles, and the occupancy bits of the tile's cells.
// A vertex is an occupied cell; own anchor (i, k) with i+1 < H has triangle
// T_a = (p, A, B) and T_b = (p, B, C) when all three corners are occupied.
template <int NT, int MAXC>
__global__ __launch_bounds__(NT) void k_count(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int NO = MAXC + MAX_RINGS;      // own cells + right column
    constexpr int RO = (NO + NT - 1) / NT;
    constexpr int NW = NT / 64;
    __shared__ uint8_t socc[NO];
    __shared__ int s_red[2][NW];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of<&FrameDesc::tile_off>(F, nf, t);
        const int H = fd->H, Wp = fd->Wp;
        const float inv_h = 1.0f / (float)H;
        const int k0 = (t - fd->tile_off) * fd->TW;
        const int TWe = min(fd->TW, Wp - k0);
        const int nown = H * TWe;
        const bool inside = k0 + TWe < Wp;
        const bool right = inside || fd->wrap;
        const int64_t rbase = (int64_t)(inside ? k0 + TWe : 0) * H;
        const uint64_t* keys = ws.keys + fd->cell_off;
        const int64_t np = fd->n_points;
        if (fd->scores && t == fd->tile_off && threadIdx.x < 4) fd->scores[threadIdx.x] = 0;
        __syncthreads();  // the previous tile's readers are done
        uint32_t key[RO];
#pragma unroll
        for (int r = 0; r < RO; ++r) {
            const int l = threadIdx.x + r * NT;
            key[r] = ~0u;
            if (l < nown) key[r] = key_index(keys, (int64_t)k0 * H + l);
            else if (l < nown + H && right) key[r] = key_index(keys, rbase + (l - nown));
        }
#pragma unroll
        for (int r = 0; r < RO; ++r) {
            const int l = threadIdx.x + r * NT;
            if (l < nown + H) socc[l] = occupied_index(key[r], np) ? 1 : 0;
        }
        __syncthreads();
        int nv = 0, nt = 0;
#pragma unroll
        for (int r = 0; r < RO; ++r) {
            const int l = threadIdx.x + r * NT;
            if (l < nown && socc[l]) {
                ++nv;
                const int i = l - div_small(l, inv_h) * H;
                if (i + 1 < H) {
                    const int a = socc[l + 1], b = socc[l + H + 1], c = socc[l + H];
                    nt += (a & b) + (b & c);
                }
            }
        }
        // occupancy words of the own cells (64-cell chunk r * NW + wv is one ballot)
#pragma unroll
        for (int r = 0; r < RO; ++r) {
            const int l = threadIdx.x + r * NT;
            const int chunk = r * NW + wv;
            const uint64_t m = __ballot(l < nown && socc[l]);
            if (lane == 0 && chunk < MAXC / 64) ws.occ[(int64_t)t * OCC_WORDS + chunk] = m;
        }
        nv = wave_sum(nv);
        nt = wave_sum(nt);
        if (lane == 0) {
            s_red[0][wv] = nv;
            s_red[1][wv] = nt;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int sv = 0, st = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                sv += s_red[0][w];
                st += s_red[1][w];
            }
            ws.tile_v[t] = sv;
            ws.tile_t[t] = st;
        }
    }
}

// ---------------------------------------------------------------------------
// LDS union-find: links the larger root under the smaller (atomicMin), so every
// root is the smallest cell of its tree.  Path halving only rewrites non-roots.
__device__ __forceinline__ int lds_find(int* P, int x) {
    for (int it = 0; it < WALK_LIMIT; ++it) {
        const int p = P[x];
        if (p == x) return x;
        const int gp = P[p];
        if (gp != p) P[x] = gp;
        x = gp;
    }
    return x;
}

__device__ __forceinline__ void lds_union(int* P, int a, int b) {
    for (int it = 0; it < WALK_LIMIT; ++it) {
        a = lds_find(P, a);
        b = lds_find(P, b);
        if (a == b) return;
        if (a > b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(&P[b], a);
        if (old == b) return;
        b = old;
    }
}

// Algorithm 1's test: both vertices have normals and every component differs by
// strictly less than its threshold (differences of two floats are exact in
// FP64); or, as the alternative test, the dot product of the two normals
// exceeds cos_min.  A vertex without a normal carries NaN components here,
// which fail every comparison.
struct SimTest {
    int pred;               // 0: components (Algorithm 1), 1: cosine
    double tx, ty, tz, cmin;
};

__device__ __forceinline__ bool similar(float4 a, float4 b, const SimTest& q) {
    if (q.pred) {
        // products of floats are exact in FP64; the sum is (x x' + y y') + z z'
        const double d = ((double)a.x * (double)b.x + (double)a.y * (double)b.y) + (double)a.z * (double)b.z;
        return d > q.cmin;
    }
    // all three comparisons, combined without branches
    const bool x = fabs((double)a.x - (double)b.x) < q.tx;
    const bool y = fabs((double)a.y - (double)b.y) < q.ty;
    const bool z = fabs((double)a.z - (double)b.z) < q.tz;
    return x & y & z;
}

// FP64 reciprocal, reciprocal square root and square root: the hardware estimate
// (about 2^-23 relative error) plus one Newton step (about 2^-46).  Weights and
// the final scaling need no correctly rounded division: the normal is rounded
// to FP32.
__device__ __forceinline__ double rcp_dp(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

__device__ __forceinline__ double rsq_dp(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return fma(y, fma(-0.5 * x * y, y, 0.5), y);
}

__device__ __forceinline__ double sqrt_dp(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double s = x * y;
    return fma(fma(-s, s, x), 0.5 * y, s);
}

// Weighted normal of LDS cell lx (ring i): sum over cycle-adjacent present pairs
// (A,B),(B,C),(C,D),(D,E),(E,F),(F,A) of (V_t x V_u) / (|V_t| + |V_u|), scaled to
// unit length (Section 2, Normal Estimation).  Edge vectors are exact in FP64.
// Branch-free: an absent neighbour (off the ring range, or an empty cell, whose
// coordinates are NaN) is replaced by the vertex itself, so its edge vector is
// zero, its cross products vanish and its length is a tiny positive number.
// Neighbours are visited once in cycle order, keeping only the previous edge
// live; the first edge is formed again to close the cycle (same arithmetic, same
// bits), which keeps the register footprint small.
__device__ __forceinline__ void vertex_edge(const float4* sc, int lx, int t, int H, bool up, bool dn, float4 P,
                                            double& vx, double& vy, double& vz, double& lv, bool& pv) {
    const int off = t == 0 ? 1 : t == 1 ? H + 1 : t == 2 ? H : t == 3 ? -1 : t == 4 ? -H - 1 : -H;
    const bool inr = (t <= 1) ? dn : (t == 3 || t == 4) ? up : true;
    const float4 Q = sc[inr ? lx + off : lx];
    pv = inr && (Q.x == Q.x);
    vx = (double)(pv ? Q.x : P.x) - (double)P.x;
    vy = (double)(pv ? Q.y : P.y) - (double)P.y;
    vz = (double)(pv ? Q.z : P.z) - (double)P.z;
    lv = sqrt_dp(fma(vx, vx, fma(vy, vy, fma(vz, vz, LEN2_FLOOR))));
}

__device__ __forceinline__ void vertex_normal(const float4* sc, int lx, int i, int H, float& onx, float& ony,
                                              float& onz) {
    const bool up = i >= 1, dn = i + 1 < H;
    const float4 P = sc[lx];
    double ux, uy, uz, lu;
    bool pu;
    vertex_edge(sc, lx, 0, H, up, dn, P, ux, uy, uz, lu, pu);
    double ax = 0.0, ay = 0.0, az = 0.0;
    bool any = false;
#pragma unroll
    for (int t = 1; t <= 6; ++t) {
        double vx, vy, vz, lv;
        bool pv;
        vertex_edge(sc, lx, t % 6, H, up, dn, P, vx, vy, vz, lv, pv);
        const double w = rcp_dp(lu + lv);
        ax = fma(w, fma(uy, vz, -uz * vy), ax);
        ay = fma(w, fma(uz, vx, -ux * vz), ay);
        az = fma(w, fma(ux, vy, -uy * vx), az);
        any |= pu && pv;
        ux = vx; uy = vy; uz = vz; lu = lv; pu = pv;
    }
    const double n2 = ax * ax + ay * ay + az * az;
    if (any && n2 > 0.0) {
        const double inv = rsq_dp(n2);
        onx = (float)(ax * inv);
        ony = (float)(ay * inv);
        onz = (float)(az * inv);
    } else {
        onx = ony = onz = 0.0f;
    }
}

__device__ __forceinline__ int vid_of(float4 c) { return __float_as_int(c.w); }

// ---------------------------------------------------------------------------
// Vertex ids of the l-sequence of a tile (own cells, then the right column)
// from per-lane occupancy: wave prefixes from ballots, the (round, wave) totals
// scanned by every wave itself after one barrier.  vid[r] holds the rank within
// the round on entry (-1 = empty) and the frame's vertex id on exit.
template <int NT, int RN>
__device__ __forceinline__ void number_cells(int (&vid)[RN], const int* s_cnt, int vbase, int vbase_next,
                                             int own_v, int nown, int lane, int wv) {
    constexpr int NW = NT / 64;
    const int c = lane < RN * NW ? (s_cnt[lane] & 0xffff) : 0;
    int inc = c;
#pragma unroll
    for (int d = 1; d < RN * NW; d <<= 1) {
        const int y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    const int exc = inc - c;
#pragma unroll
    for (int r = 0; r < RN; ++r) {
        const int pre = __shfl(exc, r * NW + wv, 64);
        const int l = (int)threadIdx.x + NT * r;
        if (vid[r] < 0) continue;
        const int rank = pre + vid[r];
        vid[r] = (l < nown) ? vbase + rank : vbase_next + (rank - own_v);
    }
}

// Mesh stage, per tile in LDS.  Columns lc = -1 .. TWe of the tile (global
// column k0 + lc, wrapped on a closed cylinder) hold the kept points'
// coordinates (NaN = empty cell) and vertex ids; LDS cell lx = (lc + 1) * H + i.
// Own cells are lc in [0, TWe); the right column lc = TWe belongs to the next
// tile (its vertex ids are needed by the triangles that reach into it).  Index
// l = lx - H runs over own cells and then the right column; thread x handles
// l = x + r * NT in round r, so every 64-cell chunk is one wave's round.
// Writes vertices, vertex_point, triangles and normals.
// 6 waves per SIMD at up to 4 cells per thread (one more wave than the
// registers of the unconstrained build allow; it hides more load latency)
template <int NT, int MAXC>
__global__ __launch_bounds__(NT, (MAXC / NT <= 4 ? 6 : 1)) void k_geom(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int XC = MAXC + 2 * MAX_RINGS;  // coordinate cells incl. halo
    constexpr int NC = MAXC + MAX_RINGS;      // own cells + right column
    constexpr int RX = (XC + NT - 1) / NT;
    constexpr int NW = NT / 64;
    constexpr int RN = (NC + NT - 1) / NT;
    static_assert(RN * NW <= 64, "one lane per (round, wave) in the prefix scan");
    __shared__ float4 sc[XC];         // (x, y, z, vertex id) by lx
    __shared__ int saux[MAXC];        // kept point index, then triangle start
    __shared__ int s_cnt[RN * NW];    // per round and wave: vertices | triangles << 16
    __shared__ int s_misc[4];         // vertex base, triangle base, own vertices, own triangles

    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of<&FrameDesc::tile_off>(F, nf, t);
        const int H = fd->H, Wp = fd->Wp, wrap = fd->wrap;
        const float inv_h = 1.0f / (float)H;
        const int lt = t - fd->tile_off;
        const int k0 = lt * fd->TW;
        const int TWe = min(fd->TW, Wp - k0);
        const int nx = H * (TWe + 2);
        const int nown = H * TWe;
        const int nscan = nown + H;
        const uint64_t* keys = ws.keys + fd->cell_off;
        const auto xyz = gmem(fd->xyz);
        const auto nin = gmem(fd->normals_in);
        const int64_t np = fd->n_points;
        const int step_i = NT % H, step_c = NT / H;   // (column, ring) advance per round
        const int i0 = (int)threadIdx.x - div_small(threadIdx.x, inv_h) * H;
        __syncthreads();  // LDS of the previous tile is free

        // The loads of phases 1-3 go out at raised wave priority, so that a
        // workgroup starting a tile gets its memory requests in flight ahead of
        // the normal arithmetic of the other workgroups on the compute unit.
        __builtin_amdgcn_s_setprio(3);
        // 1. keys of the tile and its halo columns (lx = tid + r * NT)
        uint64_t key[RX];
        {
            int col = div_small(threadIdx.x, inv_h);
            int i = i0;
#pragma unroll
            for (int r = 0; r < RX; ++r) {
                const int lx = threadIdx.x + r * NT;
                key[r] = KEY_EMPTY;
                if (lx < nx) {
                    int k = k0 + col - 1;
                    bool in = true;
                    if (k < 0 || k >= Wp) {
                        if (wrap) k = (k < 0) ? k + Wp : k - Wp;
                        else in = false;
                    }
                    if (in) key[r] = keys[(int64_t)k * H + i];
                }
                i += step_i;
                col += step_c;
                if (i >= H) { i -= H; ++col; }
            }
        }
        // 2. vertex and triangle bases: the counts of the frame's earlier tiles
        if (wv == 0) {
            int sv = 0, st = 0;
#pragma unroll 4
            for (int j = fd->tile_off + lane; j < t; j += 64) {
                sv += ws.tile_v[j];
                st += ws.tile_t[j];
            }
            sv = wave_sum(sv);
            st = wave_sum(st);
            if (lane == 0) {
                s_misc[0] = sv;
                s_misc[1] = st;
                s_misc[2] = ws.tile_v[t];
                s_misc[3] = ws.tile_t[t];
            }
        }
        // 3. the kept points
        {
            float cx[RX], cy[RX], cz[RX];
#pragma unroll
            for (int r = 0; r < RX; ++r) {
                cx[r] = cy[r] = cz[r] = __builtin_nanf("");
                if (occupied(key[r], np)) {
                    const auto q = xyz + 3 * (int64_t)(uint32_t)key[r];
                    cx[r] = q[0];
                    cy[r] = q[1];
                    cz[r] = q[2];
                }
            }
#pragma unroll
            for (int r = 0; r < RX; ++r) {
                const int lx = threadIdx.x + r * NT;
                if (lx < nx) {
                    sc[lx] = make_float4(cx[r], cy[r], cz[r], __int_as_float(-1));
                    if (lx >= H && lx < H + nown) saux[lx - H] = (int)(uint32_t)key[r];
                }
            }
        }
        __syncthreads();

        __builtin_amdgcn_s_setprio(0);
        // 4. numbering in firing order (own cells, then the right column)
        int vid[RN], ltr[RN];
        {
            int i = i0;
#pragma unroll
            for (int r = 0; r < RN; ++r) {
                const int l = threadIdx.x + NT * r;
                bool v = false;
                int ntri = 0;
                if (l < nscan) {
                    const int lx = l + H;
                    v = sc[lx].x == sc[lx].x;
                    if (v && l < nown && i + 1 < H) {
                        const bool a = sc[lx + 1].x == sc[lx + 1].x;
                        const bool b = sc[lx + H + 1].x == sc[lx + H + 1].x;
                        const bool c = sc[lx + H].x == sc[lx + H].x;
                        ntri = (int)(a && b) + (int)(b && c);
                    }
                }
                const uint64_t bv = __ballot(v);
                const uint64_t b1 = __ballot(ntri & 1);
                const uint64_t b2 = __ballot(ntri >> 1);
                vid[r] = v ? lanes_below(bv) : -1;
                ltr[r] = lanes_below(b1) + 2 * lanes_below(b2);
                if (lane == 0) s_cnt[r * NW + wv] = __popcll(bv) | ((__popcll(b1) + 2 * __popcll(b2)) << 16);
                i += step_i;
                if (i >= H) i -= H;
            }
        }
        __syncthreads();
        const int vbase = s_misc[0], tbase = s_misc[1], own_v = s_misc[2];
        const bool last_tile = lt + 1 == fd->n_tiles;
        if (threadIdx.x == 0) {
            ws.tile_vbase[t] = vbase;  // for the segment stage
            if (last_tile) {
                fd->counts[0] = vbase + own_v;
                fd->counts[1] = tbase + s_misc[3];
            }
        }
        {
            // triangle starts: the same scan over the upper halves
            const int c = lane < RN * NW ? (s_cnt[lane] >> 16) : 0;
            int inc = c;
#pragma unroll
            for (int d = 1; d < RN * NW; d <<= 1) {
                const int y = __shfl_up(inc, d, 64);
                if (lane >= d) inc += y;
            }
            const int exc = inc - c;
#pragma unroll
            for (int r = 0; r < RN; ++r) ltr[r] += tbase + __shfl(exc, r * NW + wv, 64);
        }
        number_cells<NT, RN>(vid, s_cnt, vbase, last_tile ? 0 : vbase + own_v, own_v, nown, lane, wv);

        // 5. vertices, their points and triangle starts (and, for point labels,
        //    every own cell's vertex id)
        if (fd->point_labels || fd->scores) {
            int32_t* const cvid = ws.cvid + fd->cell_off + (int64_t)k0 * H;
#pragma unroll
            for (int r = 0; r < RN; ++r) {
                const int l = threadIdx.x + NT * r;
                if (l < nown) cvid[l] = vid[r];
            }
        }
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + NT * r;
            if (vid[r] < 0) continue;
            const int lx = l + H;
            sc[lx].w = __int_as_float(vid[r]);
            if (l < nown) {
                const float4 p = sc[lx];
                const auto vo = gmem(fd->vertices) + 3 * (int64_t)vid[r];
                __builtin_nontemporal_store(p.x, &vo[0]);
                __builtin_nontemporal_store(p.y, &vo[1]);
                __builtin_nontemporal_store(p.z, &vo[2]);
                if (fd->vpoint) __builtin_nontemporal_store(saux[l], &gmem(fd->vpoint)[vid[r]]);
                if (fd->scores) ws.vtruth[fd->cell_off + vid[r]] = gmem(fd->truth)[saux[l]];
                saux[l] = ltr[r];
            }
        }
        __syncthreads();

        // 6. triangles T_a = (p, A, B), T_b = (p, B, C) of each own anchor, and
        //    the normals of the own vertices (or the given ones, copied).  Vertex
        //    ids and triangle starts are read back from LDS, so no per-round
        //    state stays in registers across the normal stencil.
        {
            int ir = i0;
#pragma unroll 1
            for (int l = threadIdx.x; l < nown; l += NT) {
                const int lx = l + H;
                const int i = ir;
                ir += step_i;
                if (ir >= H) ir -= H;
                const int v = vid_of(sc[lx]);
                if (v < 0) continue;
                if (i + 1 < H) {
                    const int a = vid_of(sc[lx + 1]), b = vid_of(sc[lx + H + 1]), c = vid_of(sc[lx + H]);
                    int ti = saux[l];
                    if (a >= 0 && b >= 0) {
                        const auto to = gmem(fd->tris) + 3 * (int64_t)ti;
                        to[0] = v; to[1] = a; to[2] = b;
                        ++ti;
                    }
                    if (b >= 0 && c >= 0) {
                        const auto to = gmem(fd->tris) + 3 * (int64_t)ti;
                        to[0] = v; to[1] = b; to[2] = c;
                    }
                }
                float nx_, ny_, nz_;
                if (nin) {
                    nx_ = nin[3 * (int64_t)v];
                    ny_ = nin[3 * (int64_t)v + 1];
                    nz_ = nin[3 * (int64_t)v + 2];
                } else {
                    vertex_normal(sc, lx, i, H, nx_, ny_, nz_);
                }
                const auto no = gmem(fd->normals) + 3 * (int64_t)v;
                no[0] = nx_;
                no[1] = ny_;
                no[2] = nz_;
            }
        }
    }
}

// Local segments, per tile in LDS: the similar joins of the own cells (from
// the normals k_geom wrote), vertical runs, unions across the tile's columns,
// the joins that leave the tile into its border slots, and every own vertex's
// local root in the forest.  sn[l] = (normal, vertex id) for l over own cells
// and the right column, NaN components for a vertex without a normal or an
// empty cell.
// 6 waves per SIMD at up to 4 cells per thread (at 4, a few registers spill;
// 5 waves without the spill ran slower)
template <int NT, int MAXC>
__global__ __launch_bounds__(NT, (MAXC / NT <= 4 ? 6 : 1)) void k_cc(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int NC = MAXC + MAX_RINGS;      // own cells + right column
    constexpr int NW = NT / 64;
    constexpr int RN = (NC + NT - 1) / NT;
    static_assert(RN * NW <= 64, "one lane per (round, wave) in the prefix scan");
    constexpr int NB = (3 * NC > 2 * MAXC) ? 3 * NC : 2 * MAXC;
    __shared__ int s_buf[NB];         // normals (3 floats per cell), later the join list
    __shared__ int svid[NC];          // vertex id of own cells and the right column, -1 empty
    __shared__ int sparent[MAXC];     // union-find parent of own cells
    __shared__ uint8_t sedge[MAXC];   // similar joins of own cells: bit 0 A (down), 1 C (right), 2 B (diagonal)
    __shared__ int s_cnt[RN * NW];
    __shared__ int s_misc[2];         // vertex base, own vertices
    __shared__ int s_nj;
    float* const sn3 = reinterpret_cast<float*>(s_buf);
    int* const s_join = s_buf;        // unions inside the tile: cell | cell << 16
    auto nrm_of = [&](int l) { return make_float4(sn3[3 * l], sn3[3 * l + 1], sn3[3 * l + 2], 0.0f); };

    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of<&FrameDesc::tile_off>(F, nf, t);
        const int H = fd->H, Wp = fd->Wp;
        const float inv_h = 1.0f / (float)H;
        const int lt = t - fd->tile_off;
        const int k0 = lt * fd->TW;
        const int TWe = min(fd->TW, Wp - k0);
        const int nown = H * TWe;
        const int nscan = nown + H;
        SimTest sim;
        sim.pred = fd->pred;
        sim.tx = fd->thr[0];
        sim.ty = fd->thr[1];
        sim.tz = fd->thr[2];
        sim.cmin = fd->cos_min;
        const int cell_off = (int)fd->cell_off;
        const bool last_tile = lt + 1 == fd->n_tiles;
        // the tile holding the right column: the next one, or the frame's first on a closed cylinder
        const int tn = !last_tile ? t + 1 : (fd->wrap ? fd->tile_off : -1);
        const int step_i = NT % H;
        const int i0 = (int)threadIdx.x - div_small(threadIdx.x, inv_h) * H;
        __syncthreads();  // LDS of the previous tile is free
        if (threadIdx.x == 0) s_nj = 0;

        // 1. occupancy of own cells and the right column, vertex bases
        if (threadIdx.x == 0) {
            s_misc[0] = ws.tile_vbase[t];  // k_geom summed the counts of the tiles before
            s_misc[1] = ws.tile_v[t];
        }
        // (every word is loaded, a cell past the scan reading the tile's first,
        // so that the loads of all rounds are in flight together)
        uint64_t ow[RN];
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + NT * r;
            const int j = l - nown;
            const int64_t w = l < nown ? (int64_t)t * OCC_WORDS + (l >> 6)
                            : (l < nscan && tn >= 0) ? (int64_t)tn * OCC_WORDS + (j >> 6)
                                                     : (int64_t)t * OCC_WORDS;
            ow[r] = ws.occ[w];
        }
        int vid[RN];
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + NT * r;
            const int j = l - nown;
            const bool v = l < nown ? ((ow[r] >> (l & 63)) & 1ull) != 0
                         : (l < nscan && tn >= 0) ? ((ow[r] >> (j & 63)) & 1ull) != 0 : false;
            const uint64_t bv = __ballot(v);
            vid[r] = v ? lanes_below(bv) : -1;
            if (lane == 0) s_cnt[r * NW + wv] = __popcll(bv);
        }
        __syncthreads();
        const int vbase = s_misc[0], own_v = s_misc[1];
        number_cells<NT, RN>(vid, s_cnt, vbase, last_tile ? 0 : vbase + own_v, own_v, nown, lane, wv);

        // 2. normals by vertex id (all rounds' loads in flight together: a cell
        //    without a vertex reads vertex 0's, which exists when any vertex of
        //    the frame does, and drops it)
        const auto nrm = gmem(fd->normals);
        float gx[RN], gy[RN], gz[RN];
        if (fd->counts[0] > 0) {
#pragma unroll
            for (int r = 0; r < RN; ++r) {
                const auto q = nrm + 3 * (int64_t)max(vid[r], 0);
                gx[r] = q[0];
                gy[r] = q[1];
                gz[r] = q[2];
            }
        } else {
#pragma unroll
            for (int r = 0; r < RN; ++r) gx[r] = gy[r] = gz[r] = 0.0f;
        }
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + NT * r;
            if (l >= nscan) continue;
            const float q = __builtin_nanf("");
            float ax = q, ay = q, az = q;
            if (vid[r] >= 0) {
                const float x = gx[r], y = gy[r], z = gz[r];
                if (!(x == 0.0f && y == 0.0f && z == 0.0f)) { ax = x; ay = y; az = z; }
            }
            sn3[3 * l] = ax;
            sn3[3 * l + 1] = ay;
            sn3[3 * l + 2] = az;
            svid[l] = vid[r];
        }
        __syncthreads();

        // 3. similar joins of own cells (A down, C right, B diagonal; C and B into
        //    the right column leave the tile); NaN components never compare
        {
            int i = i0;
#pragma unroll
            for (int r = 0; r < RN; ++r) {
                const int l = threadIdx.x + NT * r;
                const int ir = i;
                i += step_i;
                if (i >= H) i -= H;
                if (l >= nown) continue;
                // every test is evaluated (off the ring range against the cell
                // itself) and masked, so the wave does not branch
                const bool dn = ir + 1 < H;
                const float4 a = nrm_of(l);
                const float4 qa = nrm_of(dn ? l + 1 : l);
                const float4 qc = nrm_of(l + H);
                const float4 qb = nrm_of(dn ? l + H + 1 : l);
                const int e = (int)(dn & similar(a, qa, sim)) | ((int)similar(a, qc, sim) << 1) |
                              ((int)(dn & similar(a, qb, sim)) << 2);
                sedge[l] = (uint8_t)e;
            }
        }
        __syncthreads();

        // 4. vertical runs: every own cell's parent is the top cell of its run of
        //    A joins, found with a ballot of run starts over each 64-cell chunk;
        //    a run that enters the chunk from above takes the previous chunk's head
        {
            int i = i0;
#pragma unroll
            for (int r = 0; r < RN; ++r) {
                const int l = threadIdx.x + NT * r;
                const int above = sedge[min(max(l - 1, 0), MAXC - 1)];
                const bool start = !((l < nown) & (i >= 1) & ((above & 1) != 0));
                i += step_i;
                if (i >= H) i -= H;
                const uint64_t S = __ballot(start);
                const uint64_t mine = S & ((lane == 63) ? ~0ull : ((2ull << lane) - 1ull));
                const int head = mine ? (l - lane) + 63 - __builtin_clzll(mine) : -1;
                if (l < nown) sparent[l] = head;
            }
        }
        __syncthreads();
        if (64 % H != 0) {
            // a run of at most 128 cells spans at most three chunks: two passes
            for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
                for (int r = 0; r < RN; ++r) {
                    const int l = threadIdx.x + NT * r;
                    if (l < nown && sparent[l] < 0) {
                        const int h = sparent[(l & ~63) - 1];
                        if (h >= 0) sparent[l] = h;
                    }
                }
                __syncthreads();
            }
        }

        // 6. joins leaving through the right edge, with the same implication
        //    rules (A joins of the right column from its normals), into the
        //    tile's border slots: 2i for the C join of ring i, 2i+1 for its B join
        {
            int2* const slots = ws.border + fd->border_off + (int64_t)lt * 2 * H;
            for (int i = threadIdx.x; i < H; i += NT) {
                const int l = (TWe - 1) * H + i;
                const int e = sedge[l];
                const int a = cell_off + svid[l];
                int2 jc = make_int2(-1, -1), jb = make_int2(-1, -1);
                if ((e & 2) && !(i >= 1 && (sedge[l - 1] & 3) == 3 && similar(nrm_of(l - 1 + H), nrm_of(l + H), sim)))
                    jc = make_int2(a, cell_off + svid[l + H]);
                if ((e & 4) && !(((e & 1) && (sedge[l + 1] & 2)) ||
                                 ((e & 2) && similar(nrm_of(l + H), nrm_of(l + H + 1), sim))))
                    jb = make_int2(a, cell_off + svid[l + H + 1]);
                slots[2 * i] = jc;
                slots[2 * i + 1] = jb;
            }
        }

        __syncthreads();  // the normals are read; their space becomes the join list

        // 5. unions across columns inside the tile.  A right (C) join is implied
        //    when the cell above has one and both cells continue their runs
        //    downwards; a diagonal (B) join is implied by A then C, or C then A.
        //    The joins left are first gathered into one list (both ends as
        //    16-bit cell indices), then spread over all threads.
        {
            int i = i0;
#pragma unroll
            for (int r = 0; r < RN; ++r) {
                const int l = threadIdx.x + NT * r;
                const int ir = i;
                i += step_i;
                if (i >= H) i -= H;
                // (branch-free: every read is in range, the results are masked)
                const bool inside = l + H < nown;   // the right neighbour column is own
                const int lc = inside ? l : 0;
                const int e = sedge[lc];
                const int eu = sedge[lc >= 1 ? lc - 1 : 0], eur = sedge[lc >= 1 ? lc - 1 + H : 0];
                const int ed = sedge[lc + 1], er = sedge[lc + H];
                const bool jc = inside & ((e & 2) != 0) & !((ir >= 1) & ((eu & 3) == 3) & ((eur & 1) != 0));
                const bool jb = inside & ((e & 4) != 0) &
                                !((((e & 1) != 0) & ((ed & 2) != 0)) | (((e & 2) != 0) & ((er & 1) != 0)));
                const uint64_t mc = __ballot(jc), mb = __ballot(jb);
                const int n = __popcll(mc) + __popcll(mb);
                if (n) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(&s_nj, n);
                    base = __shfl(base, 0, 64);
                    if (jc) s_join[base + lanes_below(mc)] = l | ((l + H) << 16);
                    if (jb) s_join[base + __popcll(mc) + lanes_below(mb)] = l | ((l + H + 1) << 16);
                }
            }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < s_nj; j += NT) {
            const int uv = s_join[j];
            lds_union(sparent, uv & 0xffff, uv >> 16);
        }
        __syncthreads();

        // 7. local roots: the smallest cell of each local tree.  Two passes of
        //    pointer jumping first (each roughly halves every path; a parent is
        //    only ever replaced by an ancestor, so concurrent readers still reach
        //    the root), then each cell's walk.
        for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
            for (int r = 0; r < RN; ++r) {
                const int l = threadIdx.x + NT * r;
                if (l >= nown) continue;
                const int p = sparent[l];
                const int gp = sparent[p];
                if (gp != p) sparent[l] = gp;
            }
            __syncthreads();
        }
        int* const forest = ws.forest;
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + NT * r;
            if (l >= nown || vid[r] < 0) continue;
            int x = sparent[l];
            for (int it = 0; it < nown && sparent[x] != x; ++it) x = sparent[x];
            forest[cell_off + vid[r]] = cell_off + svid[x];
        }
    }
}

// ---------------------------------------------------------------------------
// Global union-find on the batch's forest (batch-wide positions).
__device__ __forceinline__ int g_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void g_store(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int g_find(int* P, int x) {
    for (int it = 0; it < WALK_LIMIT; ++it) {
        const int p = g_load(P + x);
        if (p == x) return x;
        const int gp = g_load(P + p);
        if (gp != p) g_store(P + x, gp);
        x = gp;
    }
    return x;
}

__device__ __forceinline__ void g_union(int* P, int a, int b) {
    for (int it = 0; it < WALK_LIMIT; ++it) {
        a = g_find(P, a);
        b = g_find(P, b);
        if (a == b) return;
        if (a > b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(P + b, a);
        if (old == b) return;
        b = old;
    }
}

// Pointer jumping on one node: its parent becomes its grandparent until it
// points at a root.  Run by many threads on the nodes of one chain at once, the
// distance each node covers doubles per step.
__device__ __forceinline__ void g_jump(int* P, int x) {
    for (int it = 0; it < WALK_LIMIT; ++it) {
        const int p = g_load(P + x);
        const int gp = g_load(P + p);
        if (gp == p) return;
        g_store(P + x, gp);
    }
}

// Union of two local roots from a border join.  The larger of the two is
// usually still a root (the right tile's segment, not yet joined to anything):
// then one compare-and-swap links it under the smaller, with no walk up the
// left tile's tree.  Several joins across one border often pair the same two
// segments: when the swap finds the larger already linked to the smaller, the
// union is done as well.  Otherwise the general union runs.
__device__ __forceinline__ void g_union_fast(int* P, int a, int b) {
    const int x = max(a, b), y = min(a, b);
    if (x == y) return;
    const int old = atomicCAS(P + x, x, y);
    if (old == x || old == y) return;
    g_union(P, a, b);
}

// The tile's 2H border slots (written by k_cc), gathered into consecutive
// lanes of one wave: returns their number; lane j < n then holds join j.
template <int NW>
__device__ __forceinline__ int gather_joins(const FrameDesc* fd, int t, const int2* border, int2* list,
                                            int lane) {
    constexpr int RS = 2 * MAX_RINGS / 64;   // slots per lane
    const int ns = 2 * fd->H;
    const int2* slots = border + fd->border_off + (int64_t)(t - fd->tile_off) * ns;
    int2 ab[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const int j = lane + 64 * r;
        ab[r] = slots[min(j, ns - 1)];   // unconditional, so the loads overlap
        if (j >= ns) ab[r] = make_int2(-1, -1);
    }
    int n = 0;
#pragma unroll
    for (int r = 0; r < RS; ++r) {
        const uint64_t m = __ballot(ab[r].x >= 0);
        if (ab[r].x >= 0) list[n + lanes_below(m)] = ab[r];
        n += __popcll(m);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    return n;
}

// One wave per tile: the joins of its border slots, all unioned at once.
template <int NT>
__global__ __launch_bounds__(NT) void k_merge(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int NW = NT / 64;
    __shared__ int2 s_j[NW][2 * MAX_RINGS];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int lane = lane_id();
    // the wave's tile index is uniform: held in scalar registers, so the frame
    // search and the frame's fields are scalar loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int* const P = ws.forest;
    for (int t = blockIdx.x * NW + wv; t < hdr->total_tiles; t += gridDim.x * NW) {
        const FrameDesc* fd = F + frame_of<&FrameDesc::tile_off>(F, nf, t);
        const int n = gather_joins<NW>(fd, t, ws.border, s_j[wv], lane);
        for (int j = lane; j < n; j += 64) {
            const int2 e = s_j[wv][j];
            g_union_fast(P, g_load(P + e.x), g_load(P + e.y));
        }
        __builtin_amdgcn_wave_barrier();  // the wave's LDS list is reused by its next tile
    }
}

// Concurrent unions of neighbouring tiles' segments link each tile's root to
// its left neighbour's: a chain as long as the frame.  Every local root that
// took part in a join jumps (parent := grandparent) until it points at a root;
// all of a chain's nodes jump at once, so each covers twice the distance per
// step and the chains collapse in about log2(length) steps.
template <int NT>
__global__ __launch_bounds__(NT) void k_compress(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int NW = NT / 64;
    __shared__ int2 s_j[NW][2 * MAX_RINGS];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int lane = lane_id();
    // the wave's tile index is uniform: held in scalar registers, so the frame
    // search and the frame's fields are scalar loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int* const P = ws.forest;
    for (int t = blockIdx.x * NW + wv; t < hdr->total_tiles; t += gridDim.x * NW) {
        const FrameDesc* fd = F + frame_of<&FrameDesc::tile_off>(F, nf, t);
        const int n = gather_joins<NW>(fd, t, ws.border, s_j[wv], lane);
        for (int j = lane; j < n; j += 64) {
            const int2 e = s_j[wv][j];
            int x = g_load(P + e.x), y = g_load(P + e.y);
            // both local roots jump together, one step each per pass
            for (int it = 0; it < WALK_LIMIT; ++it) {
                const int px = g_load(P + x), py = g_load(P + y);
                const int gx = g_load(P + px), gy = g_load(P + py);
                const bool mx = gx != px, my = gy != py;
                if (mx) g_store(P + x, gx);
                if (my) g_store(P + y, gy);
                if (!mx && !my) break;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
}

// Roots.  Item b of a frame covers vertex slots [1024 b, 1024 b + 1024).  A
// vertex is a segment root when its forest entry points at itself.  The roots
// of each 64-slot word are flagged in rootbits, each word gets the item's roots
// before it, and the item its root count.  The item's key cells are reset for
// the next call.  (No walk is needed here: k_resolve finds each vertex's root.)
template <int NT>
__global__ __launch_bounds__(NT) void k_flatten(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int RV = VITEM / NT;
    constexpr int NW = NT / 64;
    static_assert(RV * NW == VITEM_WORDS, "one word per wave and round");
    __shared__ int s_w[VITEM_WORDS];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    const int* const P = ws.forest;
    for (int b = blockIdx.x; b < hdr->total_vitems; b += gridDim.x) {
        const FrameDesc* fd = F + frame_of<&FrameDesc::vitem_off>(F, nf, b);
        const int lb = b - fd->vitem_off;
        const int V = (int)max<int64_t>(fd->counts[0], 0);
        const int base = (int)fd->cell_off;
        const int v0 = lb * VITEM;
        const int64_t wbase = (int64_t)b * VITEM_WORDS;   // == vitem_off * 16 + lb * 16
        __syncthreads();  // s_w of the previous item has been read
        int par[RV];
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int v = v0 + r * NT + threadIdx.x;
            par[r] = v < V ? P[base + v] : -1;
        }
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int v = v0 + r * NT + threadIdx.x;
            const uint64_t bits = __ballot(v < V && par[r] == base + v);
            if (lane == 0) {
                ws.rootbits[wbase + r * NW + wv] = bits;
                s_w[r * NW + wv] = __popcll(bits);
            }
        }
        __syncthreads();
        if (wv == 0) {
            const int c = lane < VITEM_WORDS ? s_w[lane] : 0;
            int inc = c;
#pragma unroll
            for (int d = 1; d < VITEM_WORDS; d <<= 1) {
                const int y = __shfl_up(inc, d, 64);
                if (lane >= d) inc += y;
            }
            if (lane < VITEM_WORDS) ws.wprefix[wbase + lane] = (uint32_t)(inc - c);
            if (lane == VITEM_WORDS - 1) ws.vitem_roots[b] = inc;
        }
        const int c1 = min(v0 + VITEM, fd->H * fd->Wp);
        uint64_t* keys = ws.keys + fd->cell_off;
        for (int c = v0 + threadIdx.x; c < c1; c += NT) keys[c] = KEY_EMPTY;
        if (fd->min_seg > 1) {
            int32_t* size = ws.segsize + fd->cell_off;
            for (int c = v0 + threadIdx.x; c < c1; c += NT) size[c] = 0;
        }
    }
}

// Mesh-only calls (no labelling stages): the key cells of every labelling
// item go back to empty for the next call, as k_flatten does in a full chain,
// and each frame's label count K is written as 0.
template <int NT>
__global__ __launch_bounds__(NT) void k_reset(const BatchHeader* __restrict__ hdr, Workspace ws) {
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    for (int b = blockIdx.x; b < hdr->total_vitems; b += gridDim.x) {
        const FrameDesc* fd = F + frame_of<&FrameDesc::vitem_off>(F, nf, b);
        const int v0 = (b - fd->vitem_off) * VITEM;
        if (v0 == 0 && threadIdx.x == 0) fd->counts[2] = 0;
        const int c1 = min(v0 + VITEM, fd->H * fd->Wp);
        uint64_t* keys = ws.keys + fd->cell_off;
        for (int c = v0 + threadIdx.x; c < c1; c += NT) keys[c] = KEY_EMPTY;
    }
}

// Rank bases, one frame per workgroup: each labelling item's root count is
// replaced by the roots of the frame before the item (an exclusive scan in
// firing order), and the frame's label count K is written.
template <int NT>
__global__ __launch_bounds__(NT) void k_scan(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int NW = NT / 64;
    __shared__ int s_tot[NW];
    const FrameDesc* F = frames_of(hdr);
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    for (int f = blockIdx.x; f < hdr->n_frames; f += gridDim.x) {
        const FrameDesc* fd = F + f;
        int32_t* const cnt = ws.vitem_roots + fd->vitem_off;
        const int n = fd->n_vitem;
        int run = 0;
        for (int c0 = 0; c0 < n; c0 += NT) {
            const int j = c0 + (int)threadIdx.x;
            const int mine = j < n ? cnt[j] : 0;
            int inc = mine;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int y = __shfl_up(inc, d, 64);
                if (lane >= d) inc += y;
            }
            __syncthreads();  // s_tot of the previous chunk has been read
            if (lane == 63) s_tot[wv] = inc;
            __syncthreads();
            int before = 0, total = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                if (w < wv) before += s_tot[w];
                total += s_tot[w];
            }
            if (j < n) cnt[j] = run + before + inc - mine;
            run += total;
        }
        if (threadIdx.x == 0) fd->counts[2] = run;
    }
}

// label = 1 + (roots of the frame before the vertex's root): the roots of the
// frame before the root's item, of the item before its word, and of the word
// before it.  The root is found by walking the forest: after k_compress every
// vertex is at most two links from its root (its local root, then the root its
// local root was joined to), and the walks of an item advance together, one
// step per pass, so their loads overlap.
template <int NT>
__global__ __launch_bounds__(NT) void k_resolve(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int RV = VITEM / NT;
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int* const P = ws.forest;
    for (int b = blockIdx.x; b < hdr->total_vitems; b += gridDim.x) {
        const FrameDesc* fd = F + frame_of<&FrameDesc::vitem_off>(F, nf, b);
        const int lb = b - fd->vitem_off;
        const int V = (int)max<int64_t>(fd->counts[0], 0);
        const int base = (int)fd->cell_off;
        const int v0 = lb * VITEM;
        const int64_t wframe = (int64_t)fd->vitem_off * VITEM_WORDS;
        const int32_t* const ibase = ws.vitem_roots + fd->vitem_off;
        // Loads of every round are issued before any is used, unconditionally
        // (a slot past the last vertex reads the frame's first forest entry, or
        // first root word, and drops it), so that their latencies overlap.
        int cur[RV];
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int v = v0 + r * NT + threadIdx.x;
            cur[r] = P[base + (v < V ? v : 0)];
        }
        uint32_t walking = 0;
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int v = v0 + r * NT + threadIdx.x;
            if (v >= V) cur[r] = -1;
            else if (cur[r] != base + v) walking |= 1u << r;
        }
        for (int it = 0; walking && it < WALK_LIMIT; ++it) {
            int nxt[RV];
#pragma unroll
            for (int r = 0; r < RV; ++r) nxt[r] = ((walking >> r) & 1u) ? P[cur[r]] : cur[r];
#pragma unroll
            for (int r = 0; r < RV; ++r) {
                if (((walking >> r) & 1u) && nxt[r] == cur[r]) walking &= ~(1u << r);
                cur[r] = nxt[r];
            }
        }
        uint64_t rbits[RV];
        int rbase[RV];
        uint32_t rpre[RV];
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int root = cur[r] >= 0 ? cur[r] - base : 0;
            const int64_t w = wframe + (root >> 6);
            rbits[r] = ws.rootbits[w];
            rbase[r] = ibase[root / VITEM];
            rpre[r] = ws.wprefix[w];
        }
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int v = v0 + r * NT + threadIdx.x;
            int lab = -1;
            if (v < V) {
                const int root = cur[r] - base;
                const uint64_t below = rbits[r] & ((1ull << (root & 63)) - 1ull);
                lab = 1 + rbase[r] + (int)rpre[r] + __popcll(below);
                __builtin_nontemporal_store(lab, &gmem(fd->labels)[v]);
            }
            if (fd->min_seg > 1) {
                // segment sizes: one atomic per distinct label of the wave
                int32_t* size = ws.segsize + fd->cell_off - 1;
                uint64_t todo = __ballot(lab > 0);
                while (todo) {
                    const int leader = __builtin_ctzll(todo);
                    const int L = __shfl(lab, leader, 64);
                    const uint64_t same = __ballot(lab == L);
                    if ((int)(threadIdx.x & 63) == leader) atomicAdd(size + L, (int)__popcll(same));
                    todo &= ~same;
                }
            }
        }
    }
}

// The label of input point p from its full-resolution cell (ring i, firing j):
// that of the nearest vertex of ring i along the sweep.  Sampled columns are
// visited outwards from j, the nearer side first (the earlier firing on a tie),
// until one holds a vertex; around the cylinder when it is closed, at most W'
// columns in all.  A label carried by fewer than min_seg vertices reads as 0.
__device__ __forceinline__ int backfill_label(const FrameDesc* fd, const Workspace& ws, int rec) {
    if (rec < 0) return 0;
    const int H = fd->H, s = fd->s, Wp = fd->Wp, wrap = fd->wrap;
    const int i = rec % H, j = rec / H;
    const int32_t* cvid = ws.cvid + fd->cell_off + i;
    int kl = j / s, kr = kl + 1;
    int dl = j - kl * s, dr = kr * s - j;
    int vid = -1;
    for (int n = 0; n < Wp; ++n) {
        const bool lok = wrap || kl >= 0, rok = wrap || kr < Wp;
        if (!lok && !rok) break;
        const bool left = lok && (!rok || dl <= dr);
        int k = left ? kl : kr;
        if (k < 0) k += Wp;
        if (k >= Wp) k -= Wp;
        const int v = cvid[(int64_t)k * H];
        if (v >= 0) { vid = v; break; }
        if (left) { --kl; dl += s; } else { ++kr; dr += s; }
    }
    if (vid < 0) return 0;
    const int lab = fd->labels[vid];
    if (fd->min_seg > 1 && lab > 0 && ws.segsize[fd->cell_off + lab - 1] < fd->min_seg) return 0;
    return lab;
}

// Segment removal (Section 2, Segmentation, last paragraph: labels carried by
// fewer than min_seg vertices become 0) over labelling items, and every input
// point's label (the points the sub-sampling skipped take the label of the
// nearest vertex of their ring along the sweep) over point blocks.
template <int NT>
__global__ __launch_bounds__(NT) void k_post(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int RV = VITEM / NT;
    constexpr int PPT = POINT_BLOCK / NT;
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int nv = hdr->total_vitems;
    for (int b = blockIdx.x; b < nv + hdr->total_pblk; b += gridDim.x) {
        if (b < nv) {
            const FrameDesc* fd = F + frame_of<&FrameDesc::vitem_off>(F, nf, b);
            if (fd->min_seg <= 1) continue;
            const int V = (int)max<int64_t>(fd->counts[0], 0);
            const int v0 = (b - fd->vitem_off) * VITEM;
            const int32_t* size = ws.segsize + fd->cell_off - 1;
#pragma unroll
            for (int r = 0; r < RV; ++r) {
                const int v = v0 + r * NT + threadIdx.x;
                if (v < V) {
                    const int lab = gmem(fd->labels)[v];
                    if (lab > 0 && size[lab] < fd->min_seg) gmem(fd->labels)[v] = 0;
                }
            }
        } else {
            const int pb = b - nv;
            const FrameDesc* fd = F + frame_of<&FrameDesc::pblk_off>(F, nf, pb);
            if (!fd->point_labels) continue;
            const int64_t p0 = (int64_t)(pb - fd->pblk_off) * POINT_BLOCK + threadIdx.x;
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
                const int64_t p = p0 + r * NT;
                if (p < fd->n_points)
                    __builtin_nontemporal_store(backfill_label(fd, ws, ws.pcell[fd->pt_off + p]),
                                                &gmem(fd->point_labels)[p]);
            }
        }
    }
}

// Edge scores of the final labels against the truth ids (the evaluation of
// Section 3: segment edges and ground-truth edges, each dilated by R lattice
// steps).  Per tile, columns lc = -R-1 .. TWe+R are staged in LDS (label and
// truth id of each cell's vertex, label -1 for an empty cell); edge flags are
// formed for lc = -R .. TWe+R-1 from the six mesh neighbours; every own edge
// cell then looks for an edge of the other kind in its (2R+1) x (2R+1) window.
// A closed sweep maps the staged columns around the cylinder, so a column may
// be staged twice when the tile's window spans the whole sweep; "any edge in
// the window" is unaffected.
template <int NT>
__global__ __launch_bounds__(NT) void k_score(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int NS = MAX_TILE_CELLS + (2 * MAX_SCORE_RADIUS + 2) * MAX_RINGS;
    __shared__ int s_lab[NS];
    __shared__ int s_tru[NS];
    __shared__ uint8_t s_flag[NS];
    __shared__ unsigned long long s_sum[4];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int lane = lane_id();
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of<&FrameDesc::tile_off>(F, nf, t);
        if (!fd->scores) continue;
        const int H = fd->H, Wp = fd->Wp, R = fd->score_r;
        const float inv_h = 1.0f / (float)H;
        const int k0 = (t - fd->tile_off) * fd->TW;
        const int TWe = min(fd->TW, Wp - k0);
        const int n = (TWe + 2 * R + 2) * H;
        const int32_t* cvid = ws.cvid + fd->cell_off;
        const int32_t* vtruth = ws.vtruth + fd->cell_off;
        __syncthreads();  // LDS of the previous tile is free
        if (threadIdx.x < 4) s_sum[threadIdx.x] = 0;
        for (int x = threadIdx.x; x < n; x += NT) {
            const int c = div_small(x, inv_h), i = x - c * H;
            int k = k0 + c - R - 1;
            int lab = -1, tru = -1;
            bool in = true;
            if (k < 0 || k >= Wp) {
                if (fd->wrap) k = ((k % Wp) + Wp) % Wp;
                else in = false;
            }
            if (in) {
                const int v = cvid[(int64_t)k * H + i];
                if (v >= 0) {
                    lab = fd->labels[v];
                    tru = vtruth[v];
                }
            }
            s_lab[x] = lab;
            s_tru[x] = tru;
        }
        __syncthreads();
        for (int x = H + (int)threadIdx.x; x < n - H; x += NT) {
            const int i = x - div_small(x, inv_h) * H;
            const int lab = s_lab[x], tru = s_tru[x];
            int fl = 0;
            if (lab >= 0) {
                // neighbours A..F: (i+1,c) (i+1,c+1) (i,c+1) (i-1,c) (i-1,c-1) (i,c-1)
                const int up = i > 0, dn = i + 1 < H;
                const int nb[6] = {x + 1, x + H + 1, x + H, x - 1, x - H - 1, x - H};
                const bool ok[6] = {(bool)dn, (bool)dn, true, (bool)up, (bool)up, true};
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    if (!ok[q]) continue;
                    const int l2 = s_lab[nb[q]];
                    if (l2 < 0) continue;
                    fl |= (l2 != lab ? 1 : 0) | (s_tru[nb[q]] != tru ? 2 : 0);
                }
            }
            s_flag[x] = (uint8_t)fl;
        }
        __syncthreads();
        int cnt[4] = {0, 0, 0, 0};
        for (int x = (R + 1) * H + (int)threadIdx.x; x < (R + 1 + TWe) * H; x += NT) {
            const int fl = s_flag[x];
            if (!fl) continue;
            const int i = x - div_small(x, inv_h) * H;
            const int ia = max(-R, -i), ib = min(R, H - 1 - i);
            int any = 0;
            for (int dc = -R; dc <= R; ++dc)
                for (int di = ia; di <= ib; ++di) any |= s_flag[x + dc * H + di];
            cnt[0] += fl & 1;
            cnt[1] += (fl >> 1) & 1;
            cnt[2] += (fl & 1) && (any & 2);
            cnt[3] += (fl & 2) && (any & 1);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int w = wave_sum(cnt[q]);
            if (lane == 0 && w) atomicAdd(&s_sum[q], (unsigned long long)w);
        }
        __syncthreads();
        if (threadIdx.x < 4 && s_sum[threadIdx.x])
            atomicAdd(reinterpret_cast<unsigned long long*>(fd->scores) + threadIdx.x, s_sum[threadIdx.x]);
    }
}

// The three tile kernels for one tile shape (TT threads, MAXC cells per tile).
template <int TT, int MAXC>
void launch_tile_stages(const BatchHeader* d_hdr, const Workspace& ws, int g_count, int g_geom, int g_cc,
                        bool mesh_only, hipStream_t stream, const std::function<void()>& mark) {
    k_count<TT, MAXC><<<g_count, TT, 0, stream>>>(d_hdr, ws);
    mark();
    k_geom<TT, MAXC><<<g_geom, TT, 0, stream>>>(d_hdr, ws);
    mark();
    if (!mesh_only) k_cc<TT, MAXC><<<g_cc, TT, 0, stream>>>(d_hdr, ws);
    mark();
}

}  // namespace

namespace {
__global__ __launch_bounds__(256) void k_fill_keys(uint64_t* __restrict__ keys, int64_t n) {
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) keys[c] = KEY_EMPTY;
}
}  // namespace

hipError_t fill_keys_empty(uint64_t* keys, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    k_fill_keys<<<(int)(blocks < 4096 ? blocks : 4096), 256, 0, stream>>>(keys, n);
    return hipGetLastError();
}

bool tile_shape_supported(int tile_cells, int tile_threads) {
    return (tile_threads == 256 && (tile_cells == 512 || tile_cells == 1024 || tile_cells == 2048)) ||
           (tile_threads == 512 && (tile_cells == 1024 || tile_cells == 2048));
}

hipError_t launch_chain(const BatchHeader* d_hdr, const Workspace& ws, const LaunchCfg& cfg,
                        hipStream_t stream, hipEvent_t* ev) {
    constexpr int NT = 256;
    // workgroups of a stage: its own setting, else its share of the grid, never
    // more than it has work items
    const auto pick = [&](int stage, int dflt, int items) {
        return max(1, min(cfg.stage_grid[stage] > 0 ? cfg.stage_grid[stage] : dflt, items));
    };
    const int border_items = (cfg.max_tiles + NT / 64 - 1) / (NT / 64);
    const int g_pblk = pick(0, cfg.grid, cfg.max_pblk);
    const int g_count = pick(1, 2 * cfg.grid, cfg.max_tiles);
    const int g_tiles = pick(2, cfg.grid, cfg.max_tiles);
    const int g_cc = pick(3, 2 * cfg.grid, cfg.max_tiles);
    const int g_merge = pick(4, 2 * cfg.grid, border_items);
    const int g_compress = pick(5, 2 * cfg.grid, border_items);
    const int g_vitem = pick(6, 2 * cfg.grid, cfg.max_vitems);
    const int g_frames = pick(7, cfg.grid, cfg.max_frames);
    const int g_label = pick(8, 2 * cfg.grid, cfg.max_vitems);
    const int g_score = pick(10, 2 * cfg.grid, cfg.max_tiles);
    int n = 0;
    hipError_t e = hipSuccess;
    const std::function<void()> mark = [&]() {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[n], stream);
        ++n;
    };
    mark();
    k_bin<NT><<<g_pblk, NT, 0, stream>>>(d_hdr, ws);
    mark();
    const int shape = cfg.tile_cells * 4 + cfg.tile_threads / 256;
    switch (shape) {
        case 512 * 4 + 1: launch_tile_stages<256, 512>(d_hdr, ws, g_count, g_tiles, g_cc, cfg.mesh_only, stream, mark); break;
        case 2048 * 4 + 1: launch_tile_stages<256, 2048>(d_hdr, ws, g_count, g_tiles, g_cc, cfg.mesh_only, stream, mark); break;
        case 1024 * 4 + 2: launch_tile_stages<512, 1024>(d_hdr, ws, g_count, g_tiles, g_cc, cfg.mesh_only, stream, mark); break;
        case 2048 * 4 + 2: launch_tile_stages<512, 2048>(d_hdr, ws, g_count, g_tiles, g_cc, cfg.mesh_only, stream, mark); break;
        default: launch_tile_stages<256, 1024>(d_hdr, ws, g_count, g_tiles, g_cc, cfg.mesh_only, stream, mark); break;
    }
    if (cfg.mesh_only) {
        // no labelling: the stage marks stay in place (zero time), and the key
        // reset is timed as the flatten stage, where a full chain does it
        mark();
        mark();
        k_reset<NT><<<g_vitem, NT, 0, stream>>>(d_hdr, ws);
        mark();
        mark();
        mark();
        mark();
        mark();
        const hipError_t le = hipGetLastError();
        return le != hipSuccess ? le : e;
    }
    k_merge<NT><<<g_merge, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_compress<NT><<<g_compress, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_flatten<NT><<<g_vitem, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_scan<NT><<<g_frames, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_resolve<NT><<<g_label, NT, 0, stream>>>(d_hdr, ws);
    mark();
    if (cfg.post) {
        const int64_t items = (int64_t)cfg.max_vitems + cfg.max_pblk;
        const int64_t want = cfg.stage_grid[9] > 0 ? cfg.stage_grid[9] : 2 * (int64_t)cfg.grid;
        const int g_post = (int)(items < want ? (items > 0 ? items : 1) : want);
        k_post<NT><<<g_post, NT, 0, stream>>>(d_hdr, ws);
    }
    mark();
    if (cfg.score) k_score<NT><<<g_score, NT, 0, stream>>>(d_hdr, ws);
    mark();
    const hipError_t le = hipGetLastError();
    return le != hipSuccess ? le : e;
}

}  // namespace lidarseg
