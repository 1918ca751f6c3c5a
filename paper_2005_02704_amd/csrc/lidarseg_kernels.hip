// HIP kernels for gfx950 (MI355X): bin -> sub-sample -> mesh -> normals -> labels.
//
// One batch of frames runs as a chain of four grid-stride kernels; each kernel
// walks its work items (point blocks or lattice tiles) across every frame of the
// batch, reading the per-frame descriptors from device memory, so the same
// launches (and the same captured graph) serve any batch that fits the workspace.
//
// Stage map (Mukherjee et al., PReMI 2019, Section 2):
//   k_bin           points -> (ring, firing) cell, sub-sampling, nearest return   [opening paragraph]
//   k_tile          per tile in LDS: gather, vertex + triangle numbering (single
//                   pass: decoupled look-back over tiles), mesh triangles, normals,
//                   similarity of joins, local union-find       [Mesh Construction, Normal Estimation, Algorithm 1]
//   k_merge         unions across tile borders and the azimuth seam               [Algorithm 1]
//   k_label         segment roots ranked in firing order (single pass, look-back
//                   over tiles); every vertex takes its root's label; key cells reset
//
// Algorithm 1 floods through neighbours whose normal components differ by less
// than the thresholds; that test is symmetric, so the flood's label classes are
// the connected components of the similar-join graph, and numbering them by the
// first vertex in the visiting order gives the same labels.  Union-find here
// always links the larger root under the smaller, so a root is the smallest
// vertex of its segment and the labels follow from ranking the roots.
//
// The two look-back kernels (k_tile, k_label) take tiles from an atomic ticket counter, so a tile
// only ever waits for tiles taken earlier by workgroups that are already running;
// the waits are bounded (SPIN_LIMIT) and a frame whose wait runs out reports
// counts of -1 instead of hanging.
#include "lidarseg_internal.h"

namespace lidarseg {
namespace {

constexpr int SPIN_LIMIT = 1 << 22;          // polls before a look-back gives up
constexpr int WALK_LIMIT = 1 << 20;          // steps of any pointer walk (parents strictly
                                             // decrease, so a walk is far shorter; the cap
                                             // only guarantees that every loop ends)
constexpr uint32_t POISON = (1u << 30) - 1;  // published prefix of a frame that failed
constexpr double EL_GUARD = 1e-5;            // rad: FP32 elevation estimate decides outside this band
constexpr float COL_GUARD = 0.02f;           // firings: FP32 firing estimate decides outside this band
constexpr int COL_GUARD_MAX_W = 16384;       // wider sweeps always decide the firing in FP64

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

__device__ __forceinline__ const FrameDesc* frames_of(const BatchHeader* h) {
    return reinterpret_cast<const FrameDesc*>(h + 1);
}

// A cell is occupied when its key names one of the frame's points (the bound
// also keeps a stale key from ever indexing outside the frame's points).
__device__ __forceinline__ bool occupied(uint64_t key, int64_t n_points) {
    return key != KEY_EMPTY && (int64_t)(uint32_t)key < n_points;
}

// Largest frame f with F[f].tile_off <= t.
__device__ __forceinline__ int frame_of_tile(const FrameDesc* F, int nf, int t) {
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (F[mid].tile_off <= t) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int frame_of_pblk(const FrameDesc* F, int nf, int b) {
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (F[mid].pblk_off <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Tile status words for the look-back: [epoch:32 | flag:2 | value:30].
// flag 1 = the tile's own count, 2 = inclusive prefix of its frame up to it.
__device__ __forceinline__ uint64_t st_pack(uint32_t epoch, uint32_t flag, uint32_t value) {
    return ((uint64_t)epoch << 32) | ((uint64_t)flag << 30) | (uint64_t)value;
}

__device__ __forceinline__ void st_store(uint64_t* p, uint64_t w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t st_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix over tiles [first, t) of the values published in st[],
// computed by one wave that inspects 64 predecessors at a time.  Returns -1 if
// a predecessor stayed silent for SPIN_LIMIT polls.
__device__ int lookback(const uint64_t* st, int t, int first, uint32_t epoch) {
    const int lane = lane_id();
    int acc = 0;
    int j = t - 1;
    int spins = 0;
    while (j >= first) {
        const int idx = j - lane;
        uint32_t flag = 2u, val = 0u;            // lanes past the frame's first tile: prefix 0
        if (idx >= first) {
            const uint64_t w = st_load(st + idx);
            if ((uint32_t)(w >> 32) == epoch) {
                flag = (uint32_t)(w >> 30) & 3u;
                val = (uint32_t)w & POISON;
            } else {
                flag = 0u;
            }
        }
        const uint64_t inc = __ballot(flag == 2u);
        const uint64_t avail = __ballot(flag != 0u);
        const int k = inc ? __builtin_ctzll(inc) : 64;          // nearest inclusive lane
        const uint64_t need = (k >= 63) ? ~0ull : ((2ull << k) - 1ull);
        if ((avail & need) != need) {
            if (++spins > SPIN_LIMIT) return -1;
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        acc += wave_sum(lane <= k ? (int)val : 0);
        if (k < 64) break;
        j -= 64;
    }
    return acc;
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

// The FP64 decisions, kept out of line: they run only for points whose FP32
// estimate falls inside a guard band.
__device__ __attribute__((noinline)) int ring_fp64(const double* e, int H, double z, double rho2) {
    return nearest_ring(e, H, atan2(z, sqrt(rho2)));
}

__device__ __attribute__((noinline)) int firing_fp64(double x, double y, double az0, double dphi) {
    return (int)round((atan2(y, x) - az0) / dphi);
}

// ---------------------------------------------------------------------------
// Binning and sub-sampling.  One work item = POINT_BLOCK points of one frame.
// The cell keeps min((bits(float(r^2)) << 32) | point), i.e. the nearest return,
// then the lower index: independent of thread order.
//
// The ring and firing are FP64 decisions.  Each is first estimated in FP32; the
// estimate is within ~1e-6 rad (atan2f error plus input rounding), so when it
// lies farther than the guard band from every decision boundary (midpoint of
// two ring elevations, half-integer firing) the FP64 decision is the same and
// is not computed.  Inside a band the FP64 expression decides.
template <int NT>
__global__ __launch_bounds__(NT) void k_bin(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int PPT = POINT_BLOCK / NT;  // points per thread per item
    __shared__ double s_elev[MAX_RINGS];
    __shared__ double s_mid[MAX_RINGS];    // s_mid[i]: midpoint of rings i and i+1
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ws.tickets[0] = 0;
        ws.tickets[1] = 0;
    }
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const int nb = hdr->total_pblk;
    int cur = -1;
    for (int b = blockIdx.x; b < nb; b += gridDim.x) {
        const int f = frame_of_pblk(F, nf, b);
        const FrameDesc* fd = F + f;
        const int H = fd->H;
        if (f != cur) {
            __syncthreads();
            for (int i = threadIdx.x; i < H; i += NT) s_elev[i] = ws.elev[fd->elev_off + i];
            __syncthreads();
            for (int i = threadIdx.x; i + 1 < H; i += NT) s_mid[i] = 0.5 * (s_elev[i] + s_elev[i + 1]);
            __syncthreads();
            cur = f;
        }
        const int W = fd->W, s = fd->s;
        const double az0 = fd->az0, dphi = fd->dphi, rmin2 = fd->rmin2, rmax2 = fd->rmax2;
        const float az0f = (float)az0;
        const float inv_dphif = (float)(1.0 / dphi);
        const bool col_fast = W <= COL_GUARD_MAX_W;
        const float* __restrict__ xyz = fd->xyz;
        unsigned long long* keys = reinterpret_cast<unsigned long long*>(ws.keys + fd->cell_off);
        const int64_t p0 = (int64_t)(b - fd->pblk_off) * POINT_BLOCK + threadIdx.x;
        const int64_t np = fd->n_points;
        // all loads of the item first, so their latencies overlap
        float px[PPT], py[PPT], pz[PPT];
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
            const int64_t p = p0 + r * NT;
            px[r] = py[r] = pz[r] = __builtin_nanf("");
            if (p < np) {
                px[r] = xyz[3 * p];
                py[r] = xyz[3 * p + 1];
                pz[r] = xyz[3 * p + 2];
            }
        }
#pragma unroll
        for (int r = 0; r < PPT; ++r) {
            const int64_t p = p0 + r * NT;
            const float xf = px[r], yf = py[r], zf = pz[r];
            if (!(isfinite(xf) && isfinite(yf) && isfinite(zf))) continue;
            const double x = xf, y = yf, z = zf;
            const double rho2 = x * x + y * y;   // products of floats are exact in FP64
            const double r2 = rho2 + z * z;
            if (r2 < rmin2 || r2 > rmax2) continue;

            const double elf = (double)atan2f(zf, sqrtf(xf * xf + yf * yf));
            int ring = nearest_ring(s_elev, H, elf);
            if ((ring > 0 && fabs(elf - s_mid[ring - 1]) < EL_GUARD) ||
                (ring + 1 < H && fabs(elf - s_mid[ring]) < EL_GUARD))
                ring = ring_fp64(s_elev, H, z, rho2);

            // |az0| <= 2 pi, so the rounded firing lies in [-2W, 2W)
            int j;
            const float jff = (atan2f(yf, xf) - az0f) * inv_dphif;
            if (col_fast && fabsf(jff - floorf(jff) - 0.5f) > COL_GUARD)
                j = (int)floorf(jff + 0.5f);
            else
                j = firing_fp64(x, y, az0, dphi);
            if (j < 0) j += W;
            if (j < 0) j += W;
            if (j >= W) j -= W;
            if (j >= W) j -= W;
            int k = j;
            if (s > 1) {
                k = j / s;
                if (k * s != j) continue;
            }
            const int64_t c = (int64_t)k * H + ring;
            const unsigned long long key =
                ((unsigned long long)__float_as_uint((float)r2) << 32) | (unsigned long long)(uint32_t)p;
            atomicMin(keys + c, key);
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

__device__ __forceinline__ bool similar(float ax, float ay, float az, float bx, float by, float bz,
                                        double tx, double ty, double tz) {
    const bool ha = !(ax == 0.0f && ay == 0.0f && az == 0.0f);
    const bool hb = !(bx == 0.0f && by == 0.0f && bz == 0.0f);
    // differences of two floats are exact in FP64
    return ha && hb && fabs((double)ax - (double)bx) < tx && fabs((double)ay - (double)by) < ty &&
           fabs((double)az - (double)bz) < tz;
}

// FP64 reciprocal and reciprocal square root: the hardware estimate (about 2^-26
// relative error) plus one Newton step (about 2^-50).  Weights and the final
// scaling need no correctly rounded division: the normal is rounded to FP32.
__device__ __forceinline__ double rcp_dp(double x) {
    const double y = __builtin_amdgcn_rcp(x);
    return fma(y, fma(-x, y, 1.0), y);
}

__device__ __forceinline__ double rsq_dp(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return fma(y, fma(-0.5 * x * y, y, 0.5), y);
}

// x / H for the small non-negative LDS indices used here (x < 2^13, H <= 128).
__device__ __forceinline__ int div_small(int x, float inv_h) {
    return (int)(((float)x + 0.5f) * inv_h);
}

// Weighted normal of LDS cell lx (ring i): sum over cycle-adjacent present pairs
// (A,B),(B,C),(C,D),(D,E),(E,F),(F,A) of (V_t x V_u) / (|V_t| + |V_u|), scaled to
// unit length (Section 2, Normal Estimation).  Edge vectors are exact in FP64;
// empty cells hold NaN coordinates.  Branch-free: an absent neighbour reads the
// cell itself and contributes zero.  Neighbours are visited once, in cycle order,
// keeping only the previous and the first edge vector live.
__device__ __forceinline__ void edge_vec(const float* sx, const float* sy, const float* sz, int q, bool ok,
                                         double px, double py, double pz, double& vx, double& vy,
                                         double& vz, double& len, bool& pres) {
    const float qx = sx[q], qy = sy[q], qz = sz[q];
    pres = ok && (qx == qx);
    vx = pres ? (double)qx - px : 0.0;
    vy = pres ? (double)qy - py : 0.0;
    vz = pres ? (double)qz - pz : 0.0;
    const double l2 = vx * vx + vy * vy + vz * vz;
    len = pres ? l2 * rsq_dp(l2) : 1.0;
}

__device__ __forceinline__ void vertex_normal(const float* sx, const float* sy, const float* sz,
                                              int lx, int i, int H, float& onx, float& ony, float& onz) {
    const bool up = i >= 1, dn = i + 1 < H;
    const int q[6] = {dn ? lx + 1 : lx, dn ? lx + H + 1 : lx, lx + H,
                      up ? lx - 1 : lx, up ? lx - H - 1 : lx, lx - H};
    const bool ok[6] = {dn, dn, true, up, up, true};
    const double px = sx[lx], py = sy[lx], pz = sz[lx];
    double v0x, v0y, v0z, l0;
    bool p0;
    edge_vec(sx, sy, sz, q[0], ok[0], px, py, pz, v0x, v0y, v0z, l0, p0);
    double ux = v0x, uy = v0y, uz = v0z, lu = l0;
    bool pu = p0;
    double ax = 0.0, ay = 0.0, az = 0.0;
    bool any = false;
#pragma unroll
    for (int t = 1; t <= 6; ++t) {
        double vx, vy, vz, lv;
        bool pv;
        if (t < 6) {
            edge_vec(sx, sy, sz, q[t], ok[t], px, py, pz, vx, vy, vz, lv, pv);
        } else {
            vx = v0x; vy = v0y; vz = v0z; lv = l0; pv = p0;
        }
        const bool both = pu && pv;
        const double w = both ? rcp_dp(lu + lv) : 0.0;
        ax = fma(w, uy * vz - uz * vy, ax);
        ay = fma(w, uz * vx - ux * vz, ay);
        az = fma(w, ux * vy - uy * vx, az);
        any |= both;
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

// ---------------------------------------------------------------------------
// The per-tile fused stage.  LDS columns lc = -1 .. TWe+1 of the tile (global
// column k0 + lc, wrapped on a closed cylinder) hold the kept points'
// coordinates (NaN = empty cell); LDS cell lx = (lc + 1) * H + i.  Own cells are
// lc in [0, TWe); the right column lc = TWe belongs to the next tile but its
// normals are needed for the joins that leave the tile.  Index l = lx - H runs
// over own cells and then the right column.
template <int NT, int MAXC>
__global__ __launch_bounds__(NT) void k_tile(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int XC = MAXC + 3 * MAX_RINGS;  // coordinate cells incl. halo
    constexpr int NC = MAXC + MAX_RINGS;      // own cells + right column
    constexpr int RX = (XC + NT - 1) / NT;
    constexpr int RN = (NC + NT - 1) / NT;
    constexpr int NW = NT / 64;
    // sx/sy/sz: coordinates, then (after the normal stage) normals indexed by l
    __shared__ float sx[XC], sy[XC], sz[XC];
    __shared__ int svid[NC];     // vertex index of l (frame-local), -1 = empty
    __shared__ int saux[MAXC];   // kept point index, then triangle start, then union-find parent
    __shared__ uint8_t sedge[MAXC];   // similar joins of own cells: bit 0 A (down), 1 C (right), 2 B (diagonal)
    __shared__ int s_cnt[3][RN][NW];  // per round and wave: vertices, own vertices, triangles
    __shared__ int s_misc[3];         // ticket, vertex base, triangle base

    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const uint32_t epoch = hdr->epoch;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    while (true) {
        __syncthreads();  // LDS of the previous tile is free
        if (threadIdx.x == 0) s_misc[0] = atomicAdd(ws.tickets, 1);
        __syncthreads();
        const int t = s_misc[0];
        if (t >= hdr->total_tiles) break;
        const FrameDesc* fd = F + frame_of_tile(F, nf, t);
        const int H = fd->H, Wp = fd->Wp, wrap = fd->wrap;
        const float inv_h = 1.0f / (float)H;
        const int lt = t - fd->tile_off;
        const int k0 = lt * fd->TW;
        const int TWe = min(fd->TW, Wp - k0);
        const int nx = H * (TWe + 3);
        const int nown = H * TWe;
        const int nscan = nown + H;
        const uint64_t* keys = ws.keys + fd->cell_off;
        const float* __restrict__ xyz = fd->xyz;
        const float* __restrict__ nin = fd->normals_in;
        const int64_t np = fd->n_points;
        const double tx = fd->thr[0], ty = fd->thr[1], tz = fd->thr[2];
        int* const forest = ws.forest + fd->cell_off;

        // 1. keys of the tile and its halo columns, then the kept points (loads
        //    issued back to back so their latencies overlap)
        uint64_t key[RX];
#pragma unroll
        for (int r = 0; r < RX; ++r) {
            const int lx = threadIdx.x + r * NT;
            key[r] = KEY_EMPTY;
            if (lx < nx) {
                const int col = div_small(lx, inv_h);
                const int i = lx - col * H;
                int k = k0 + col - 1;
                bool in = true;
                if (k < 0 || k >= Wp) {
                    if (wrap) k = (k < 0) ? k + Wp : k - Wp;
                    else in = false;
                }
                if (in) key[r] = keys[(int64_t)k * H + i];
            }
        }
        float cx[RX], cy[RX], cz[RX];
#pragma unroll
        for (int r = 0; r < RX; ++r) {
            cx[r] = cy[r] = cz[r] = __builtin_nanf("");
            if (occupied(key[r], np)) {
                const float* q = xyz + 3 * (int64_t)(uint32_t)key[r];
                cx[r] = q[0];
                cy[r] = q[1];
                cz[r] = q[2];
            }
        }
#pragma unroll
        for (int r = 0; r < RX; ++r) {
            const int lx = threadIdx.x + r * NT;
            if (lx < nx) {
                sx[lx] = cx[r];
                sy[lx] = cy[r];
                sz[lx] = cz[r];
                if (lx >= H && lx < H + nown) saux[lx - H] = (int)(uint32_t)key[r];
            }
        }
        __syncthreads();

        // 2. local numbering in firing order: own cells, then the right column.
        //    Wave prefixes from ballots; per-wave totals go through LDS.
        bool vv[RN];
        int lv[RN], ltr[RN];
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + r * NT;
            bool v = false;
            int ntri = 0;
            if (l < nscan) {
                const int lx = l + H;
                v = sx[lx] == sx[lx];
                const int i = l - div_small(l, inv_h) * H;
                if (v && l < nown && i + 1 < H) {
                    const bool a = sx[lx + 1] == sx[lx + 1];
                    const bool b = sx[lx + H + 1] == sx[lx + H + 1];
                    const bool c = sx[lx + H] == sx[lx + H];
                    ntri = (int)(a && b) + (int)(b && c);
                }
            }
            const uint64_t bv = __ballot(v);
            const uint64_t bo = __ballot(v && l < nown);
            const uint64_t b1 = __ballot(ntri & 1);
            const uint64_t b2 = __ballot(ntri >> 1);
            vv[r] = v;
            lv[r] = lanes_below(bv);
            ltr[r] = lanes_below(b1) + 2 * lanes_below(b2);
            if (lane == 0) {
                s_cnt[0][r][wv] = __popcll(bv);
                s_cnt[1][r][wv] = __popcll(bo);
                s_cnt[2][r][wv] = __popcll(b1) + 2 * __popcll(b2);
            }
        }
        __syncthreads();
        int own_v = 0, own_t = 0, run_v = 0, run_t = 0;
#pragma unroll
        for (int r = 0; r < RN; ++r) {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int cv = s_cnt[0][r][w], ct = s_cnt[2][r][w];
                own_v += s_cnt[1][r][w];
                own_t += ct;
                if (w == wv) { lv[r] += run_v; ltr[r] += run_t; }
                run_v += cv;
                run_t += ct;
            }
        }

        // 3. frame-wide bases: publish this tile's counts and look back at its
        //    predecessors; vertices on wave 0, triangles on wave 1
        if (wv < 2) {
            uint64_t* st = (wv == 0) ? ws.stat_v : ws.stat_t;
            const int own = (wv == 0) ? own_v : own_t;
            if (lane == 0) st_store(st + t, st_pack(epoch, lt == 0 ? 2u : 1u, (uint32_t)own));
            const int pre = (lt > 0) ? lookback(st, t, fd->tile_off, epoch) : 0;
            if (lane == 0) {
                const bool bad = pre < 0 || pre >= (int)POISON;
                if (lt > 0) st_store(st + t, st_pack(epoch, 2u, bad ? POISON : (uint32_t)(pre + own)));
                s_misc[1 + wv] = bad ? -1 : pre;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const bool bad = s_misc[1] < 0 || s_misc[2] < 0;
            ws.tile_v[t] = own_v;
            ws.tile_vbase[t] = bad ? -1 : s_misc[1];
            if (bad) {
                s_misc[1] = -1;
                fd->counts[0] = -1;
                fd->counts[1] = -1;
                fd->counts[2] = -1;
            } else if (lt + 1 == fd->n_tiles) {
                fd->counts[0] = s_misc[1] + own_v;
                fd->counts[1] = s_misc[2] + own_t;
            }
        }
        __syncthreads();
        const int vbase = s_misc[1], tbase = s_misc[2];
        if (vbase < 0) continue;  // the frame reports counts of -1
        const int vbase_next = (lt + 1 == fd->n_tiles) ? 0 : vbase + own_v;  // seam: column 0

        // 4. vertex ids; vertices, their points and triangle starts
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + r * NT;
            if (l < nscan) {
                int vid = -1;
                if (vv[r]) vid = (l < nown) ? vbase + lv[r] : vbase_next + (lv[r] - own_v);
                svid[l] = vid;
                if (l < nown && vv[r]) {
                    const int lx = l + H;
                    float* vo = fd->vertices + 3 * (int64_t)vid;
                    vo[0] = sx[lx];
                    vo[1] = sy[lx];
                    vo[2] = sz[lx];
                    if (fd->vpoint) fd->vpoint[vid] = saux[l];
                    saux[l] = tbase + ltr[r];
                }
            }
        }
        __syncthreads();

        // 5. triangles T_a = (p, A, B), T_b = (p, B, C) of each own anchor
        for (int l = threadIdx.x; l < nown; l += NT) {
            const int p = svid[l];
            const int i = l - div_small(l, inv_h) * H;
            if (p < 0 || i + 1 >= H) continue;
            const int a = svid[l + 1], b = svid[l + H + 1], c = svid[l + H];
            int ti = saux[l];
            if (a >= 0 && b >= 0) {
                int32_t* to = fd->tris + 3 * (int64_t)ti;
                to[0] = p; to[1] = a; to[2] = b;
                ++ti;
            }
            if (b >= 0 && c >= 0) {
                int32_t* to = fd->tris + 3 * (int64_t)ti;
                to[0] = p; to[1] = b; to[2] = c;
            }
        }

        // 6. normals of own cells and the right column (or the given ones), kept
        //    in registers until every thread is done reading coordinates
        float nrm[RN][3];
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + r * NT;
            nrm[r][0] = nrm[r][1] = nrm[r][2] = 0.0f;
            if (l < nscan && vv[r]) {
                const int vid = svid[l];
                if (nin) {
                    nrm[r][0] = nin[3 * (int64_t)vid];
                    nrm[r][1] = nin[3 * (int64_t)vid + 1];
                    nrm[r][2] = nin[3 * (int64_t)vid + 2];
                } else {
                    const int i = l - div_small(l, inv_h) * H;
                    vertex_normal(sx, sy, sz, l + H, i, H, nrm[r][0], nrm[r][1], nrm[r][2]);
                }
                if (l < nown) {
                    float* no = fd->normals + 3 * (int64_t)vid;
                    no[0] = nrm[r][0];
                    no[1] = nrm[r][1];
                    no[2] = nrm[r][2];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + r * NT;
            if (l < nscan) {
                sx[l] = nrm[r][0];
                sy[l] = nrm[r][1];
                sz[l] = nrm[r][2];
            }
        }
        __syncthreads();

        // 7. segments inside the tile.  Similar joins of own cells first (A down,
        //    C right, B diagonal; C and B into the right column leave the tile).
        for (int l = threadIdx.x; l < nown; l += NT) {
            const int i = l - div_small(l, inv_h) * H;
            const float ax = sx[l], ay = sy[l], az = sz[l];
            int e = 0;
            if (i + 1 < H && similar(ax, ay, az, sx[l + 1], sy[l + 1], sz[l + 1], tx, ty, tz)) e |= 1;
            if (similar(ax, ay, az, sx[l + H], sy[l + H], sz[l + H], tx, ty, tz)) e |= 2;
            if (i + 1 < H && similar(ax, ay, az, sx[l + H + 1], sy[l + H + 1], sz[l + H + 1], tx, ty, tz)) e |= 4;
            sedge[l] = (uint8_t)e;
        }
        __syncthreads();
        //    Vertical runs: each cell points at the cell above when joined to it,
        //    then pointer jumping makes every cell point at its run's top cell.
        int* const sparent = saux;
        for (int l = threadIdx.x; l < nown; l += NT) {
            const int i = l - div_small(l, inv_h) * H;
            sparent[l] = (i >= 1 && (sedge[l - 1] & 1)) ? l - 1 : l;
        }
        __syncthreads();
        for (int span = 1; span < H; span <<= 1) {
            for (int l = threadIdx.x; l < nown; l += NT) sparent[l] = sparent[sparent[l]];
            __syncthreads();
        }
        //    Unions across columns.  A right (C) join is implied when the cell above
        //    has one and both cells continue their runs downwards; a diagonal (B)
        //    join is implied by A then C, or C then A.
        for (int l = threadIdx.x; l < nown; l += NT) {
            const int i = l - div_small(l, inv_h) * H;
            const int lc = div_small(l, inv_h);
            if (lc + 1 >= TWe) continue;
            const int e = sedge[l];
            if (e & 2) {
                const bool implied = i >= 1 && (sedge[l - 1] & 3) == 3 && (sedge[l - 1 + H] & 1);
                if (!implied) lds_union(sparent, l, l + H);
            }
            if (e & 4) {
                const bool implied = ((e & 1) && (sedge[l + 1] & 2)) || ((e & 2) && (sedge[l + H] & 1));
                if (!implied) lds_union(sparent, l, l + H + 1);
            }
        }
        // joins leaving through the right edge: (last column, C) and (last column, B)
        int2* border = ws.border + fd->border_off + (int64_t)lt * 2 * H;
        for (int i = threadIdx.x; i < H; i += NT) {
            const int l = (TWe - 1) * H + i;
            const int e = sedge[l];
            border[2 * i] = (e & 2) ? make_int2(svid[l], svid[l + H]) : make_int2(-1, -1);
            border[2 * i + 1] = (e & 4) ? make_int2(svid[l], svid[l + H + 1]) : make_int2(-1, -1);
        }
        __syncthreads();
        // local roots: the smallest cell of each local tree (no writes while reading)
        for (int l = threadIdx.x; l < nown; l += NT) {
            const int vid = svid[l];
            if (vid < 0) continue;
            int r = l;
            for (int it = 0; it < nown && sparent[r] != r; ++it) r = sparent[r];
            forest[vid] = svid[r];
        }
    }
}

// ---------------------------------------------------------------------------
// Global union-find on a frame's label array (vertex-indexed parents).
__device__ __forceinline__ int g_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int g_find(int* P, int x) {
    for (int it = 0; it < WALK_LIMIT; ++it) {
        const int p = g_load(P + x);
        if (p == x) return x;
        const int gp = g_load(P + p);
        if (gp != p) __hip_atomic_store(P + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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

// Largest frame f with F[f].border_off <= e.
__device__ __forceinline__ int frame_of_border(const FrameDesc* F, int nf, int64_t e) {
    int lo = 0, hi = nf - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (F[mid].border_off <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// One thread per border slot of the batch (the similar joins leaving each tile
// through its right edge).  Both ends are replaced by their current parents (any
// ancestor works for a union), and a join whose (frame, parent pair) repeats one
// of the four slots before it -- usually the rows above, joining the same two
// segments -- is skipped, which keeps most threads off the same two roots.
template <int NT>
__global__ __launch_bounds__(NT) void k_merge(const BatchHeader* __restrict__ hdr, Workspace ws) {
    __shared__ int3 s_pair[NT];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const FrameDesc* last = F + nf - 1;
    const int64_t total = last->border_off + (int64_t)last->n_tiles * 2 * last->H;
    for (int64_t base = (int64_t)blockIdx.x * NT; base < total; base += (int64_t)gridDim.x * NT) {
        const int64_t e = base + threadIdx.x;
        int3 rr = make_int3(-1, -1, -1);
        int* L = nullptr;
        if (e < total) {
            const int f = frame_of_border(F, nf, e);
            const FrameDesc* fd = F + f;
            const int2 ab = ws.border[e];
            if (ab.x >= 0 && fd->counts[0] >= 0) {  // counts < 0: the frame failed in k_tile
                L = ws.forest + fd->cell_off;
                rr = make_int3(g_load(L + ab.x), g_load(L + ab.y), f);
            }
        }
        __syncthreads();
        s_pair[threadIdx.x] = rr;
        __syncthreads();
        if (rr.x >= 0) {
            bool dup = false;
#pragma unroll
            for (int d = 1; d <= 4; ++d) {
                if ((int)threadIdx.x >= d) {
                    const int3 q = s_pair[threadIdx.x - d];
                    dup |= (q.x == rr.x && q.y == rr.y && q.z == rr.z);
                }
            }
            if (!dup) g_union(L, rr.x, rr.y);
        }
    }
}

// Labels.  Per tile, in ticket order: the tile's segment roots (forest entry
// equal to itself) are ranked in firing order across the frame (look-back over
// tiles) and their forest entries become -(1 + rank).  Every other vertex walks
// its forest path until it meets a negative entry, which carries its segment's
// label.  A root is the smallest vertex of its segment, so every path stays in
// this tile or earlier ones; a root of an earlier tile that is not ranked yet is
// waited for (its tile holds an earlier ticket and never waits on later tiles).
// The tile's key cells are reset for the next call.
template <int NT>
__global__ __launch_bounds__(NT) void k_label(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int RV = 2048 / NT;   // vertex rounds: a tile owns at most 2048 vertices
    constexpr int NW = NT / 64;
    __shared__ int s_cnt[RV][NW];
    __shared__ int s_misc[2];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    const uint32_t epoch = hdr->epoch;
    const int lane = lane_id(), wv = threadIdx.x >> 6;
    while (true) {
        __syncthreads();
        if (threadIdx.x == 0) s_misc[0] = atomicAdd(ws.tickets + 1, 1);
        __syncthreads();
        const int t = s_misc[0];
        if (t >= hdr->total_tiles) break;
        const FrameDesc* fd = F + frame_of_tile(F, nf, t);
        const int lt = t - fd->tile_off;
        const bool frame_ok = fd->counts[0] >= 0;
        int* const P = ws.forest + fd->cell_off;
        int* const L = fd->labels;
        const int vb = ws.tile_vbase[t], nv = ws.tile_v[t];

        // 1. roots of the tile, ranked
        uint32_t mine = 0, roots = 0;
        int pre[RV], cur[RV];
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int k = threadIdx.x + r * NT;
            const int v = vb + k;
            cur[r] = v;
            bool isroot = false;
            if (frame_ok && k < nv) {
                mine |= 1u << r;
                cur[r] = P[v];
                isroot = cur[r] == v;
            }
            const uint64_t b = __ballot(isroot);
            pre[r] = lanes_below(b);
            if (lane == 0) s_cnt[r][wv] = __popcll(b);
            roots |= (uint32_t)isroot << r;
        }
        __syncthreads();
        int own_r = 0, run = 0;
#pragma unroll
        for (int r = 0; r < RV; ++r) {
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int c = s_cnt[r][w];
                own_r += c;
                if (w == wv) pre[r] += run;
                run += c;
            }
        }
        if (wv == 0) {
            if (lane == 0) st_store(ws.stat_r + t, st_pack(epoch, lt == 0 ? 2u : 1u, (uint32_t)own_r));
            const int pr = (lt > 0) ? lookback(ws.stat_r, t, fd->tile_off, epoch) : 0;
            const bool bad = pr < 0 || pr >= (int)POISON;
            if (lane == 0) {
                if (lt > 0) st_store(ws.stat_r + t, st_pack(epoch, 2u, bad ? POISON : (uint32_t)(pr + own_r)));
                if (bad) fd->counts[2] = -1;
                else if (lt + 1 == fd->n_tiles && frame_ok) fd->counts[2] = pr + own_r;
                s_misc[1] = bad ? -1 : pr;
            }
        }
        __syncthreads();
        const int rbase = s_misc[1];
        const bool ok = rbase >= 0 && frame_ok;
        if (ok) {
#pragma unroll
            for (int r = 0; r < RV; ++r) {
                if ((roots >> r) & 1u) {
                    const int v = vb + threadIdx.x + r * NT;
                    const int label = 1 + rbase + pre[r];
                    __hip_atomic_store(P + v, -label, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    L[v] = label;
                }
            }
        }
        __syncthreads();

        // 2. every other vertex: walk to a ranked root, all walks advancing together
        uint32_t walking = ok ? (mine & ~roots) : 0u;
        int spins = 0;
        while (walking) {
#pragma unroll
            for (int r = 0; r < RV; ++r) {
                if ((walking >> r) & 1u) {
                    const int y = g_load(P + cur[r]);
                    if (y < 0) {
                        L[vb + threadIdx.x + r * NT] = -y;
                        walking &= ~(1u << r);
                    } else if (y != cur[r]) {
                        cur[r] = y;
                    }
                }
            }
            if (walking && ++spins > SPIN_LIMIT) {
                fd->counts[2] = -1;
                break;
            }
        }

        const int H = fd->H;
        const int k0 = lt * fd->TW;
        const int TWe = min(fd->TW, fd->Wp - k0);
        uint64_t* keys = ws.keys + fd->cell_off + (int64_t)k0 * H;
        for (int l = threadIdx.x; l < H * TWe; l += NT) keys[l] = KEY_EMPTY;
    }
}

}  // namespace

hipError_t launch_chain(const BatchHeader* d_hdr, const Workspace& ws, const LaunchCfg& cfg,
                        hipStream_t stream, hipEvent_t* ev) {
    constexpr int NT = 256;
    const int g_tiles = max(1, min(cfg.grid, cfg.max_tiles));
    const int g_pblk = max(1, min(cfg.grid, cfg.max_pblk));
    int n = 0;
    hipError_t e = hipSuccess;
    auto mark = [&]() {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[n], stream);
        ++n;
    };
    mark();
    k_bin<NT><<<g_pblk, NT, 0, stream>>>(d_hdr, ws);
    mark();
    switch (cfg.tile_cells) {
        case 512: k_tile<NT, 512><<<g_tiles, NT, 0, stream>>>(d_hdr, ws); break;
        case 2048: k_tile<NT, 2048><<<g_tiles, NT, 0, stream>>>(d_hdr, ws); break;
        default: k_tile<NT, 1024><<<g_tiles, NT, 0, stream>>>(d_hdr, ws); break;
    }
    mark();
    k_merge<NT><<<g_tiles, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_label<NT><<<g_tiles, NT, 0, stream>>>(d_hdr, ws);
    mark();
    const hipError_t le = hipGetLastError();
    return le != hipSuccess ? le : e;
}

}  // namespace lidarseg
