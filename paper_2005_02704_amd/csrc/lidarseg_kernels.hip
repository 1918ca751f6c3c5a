// HIP kernels for gfx950 (MI355X): bin -> sub-sample -> mesh -> normals -> labels.
//
// One batch of frames runs as a chain of grid-stride kernels; each kernel walks
// its work items (point blocks or lattice tiles) across every frame of the batch,
// reading the per-frame descriptors from device memory, so the same launches (and
// the same captured graph) serve any batch that fits the workspace.
//
// Stage map (Mukherjee et al., PReMI 2019, Section 2):
//   k_bin         points -> (ring, firing) cell, sub-sampling, nearest return   [opening paragraph]
//   k_count       per tile: vertices and triangles                              [Mesh Construction]
//   k_scan_tiles  per frame: tile offsets for vertices / triangles / labels
//   k_tile        per tile in LDS: gather, vertex + triangle numbering, normals,
//                 similarity of joins, local union-find                        [Normal Estimation, Algorithm 1]
//   k_merge       unions across tile borders and the azimuth seam               [Algorithm 1]
//   k_flatten     every vertex -> its segment root; segment roots per tile
//   k_rank        roots take their label = 1 + rank of the root in firing order
//   k_final       every vertex takes its root's label
//
// Algorithm 1 floods through neighbours whose normal components differ by less
// than the thresholds; that test is symmetric, so the flood's label classes are
// the connected components of the similar-join graph, and numbering them by the
// first vertex in the visiting order gives the same labels.  Union-find here
// always links the larger root under the smaller, so a root is the smallest
// vertex of its segment and the labels follow from a scan over roots.
#include "lidarseg_internal.h"

namespace lidarseg {
namespace {

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Block-wide exclusive scan.  s_tmp: NT/64 ints.  Every thread must call it.
template <int NT>
__device__ __forceinline__ int block_excl_scan(int x, int& total, int* s_tmp) {
    const int w = threadIdx.x >> 6;
    const int inc = wave_incl_scan(x);
    if (lane_id() == 63) s_tmp[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        const int v = s_tmp[i];
        off += (i < w) ? v : 0;
        tot += v;
    }
    __syncthreads();
    total = tot;
    return off + inc - x;
}

template <int NT>
__device__ __forceinline__ int block_sum(int x, int* s_tmp) {
    int tot;
    block_excl_scan<NT>(x, tot, s_tmp);
    return tot;
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

// ---------------------------------------------------------------------------
// Binning and sub-sampling.  One work item = POINT_BLOCK points of one frame.
// The cell keeps min((bits(float(r^2)) << 32) | point), i.e. the nearest return,
// then the lower index: independent of thread order.
template <int NT>
__global__ __launch_bounds__(NT) void k_bin(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int PPT = POINT_BLOCK / NT;  // points per thread per item
    __shared__ double s_elev[MAX_RINGS];
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
            cur = f;
        }
        const int W = fd->W, s = fd->s;
        const double az0 = fd->az0, dphi = fd->dphi, rmin2 = fd->rmin2, rmax2 = fd->rmax2;
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
            if (!(isfinite(px[r]) && isfinite(py[r]) && isfinite(pz[r]))) continue;
            const double x = px[r], y = py[r], z = pz[r];
            const double rho2 = x * x + y * y;   // products of floats are exact in FP64
            const double r2 = rho2 + z * z;
            if (r2 < rmin2 || r2 > rmax2) continue;
            const int ring = nearest_ring(s_elev, H, atan2(z, sqrt(rho2)));
            long long j = (long long)round((atan2(y, x) - az0) / dphi);
            j %= W;
            if (j < 0) j += W;
            if (j % s) continue;
            const int64_t c = (j / s) * (int64_t)H + ring;
            const unsigned long long key =
                ((unsigned long long)__float_as_uint((float)r2) << 32) | (unsigned long long)(uint32_t)p;
            atomicMin(keys + c, key);
        }
    }
}

// ---------------------------------------------------------------------------
// Per tile: vertices owned and triangles anchored (T_a = p,A,B and T_b = p,B,C).
template <int NT>
__global__ __launch_bounds__(NT) void k_count(const BatchHeader* __restrict__ hdr, Workspace ws) {
    __shared__ int s_tmp[NT / 64];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of_tile(F, nf, t);
        const int H = fd->H, Wp = fd->Wp, wrap = fd->wrap;
        const int k0 = (t - fd->tile_off) * fd->TW;
        const int TWe = min(fd->TW, Wp - k0);
        const uint64_t* keys = ws.keys + fd->cell_off;
        const int64_t np = fd->n_points;
        int nv = 0, nt = 0;
        for (int l = threadIdx.x; l < H * TWe; l += NT) {
            const int kc = k0 + l / H;
            const int i = l - (l / H) * H;
            const int64_t c = (int64_t)kc * H + i;
            const bool v = occupied(keys[c], np);
            nv += v;
            if (v && i + 1 < H) {
                int kn = kc + 1;
                bool ok = true;
                if (kn == Wp) { if (wrap) kn = 0; else ok = false; }
                if (ok) {
                    const bool a = occupied(keys[c + 1], np);
                    const bool bb = occupied(keys[(int64_t)kn * H + i + 1], np);
                    const bool cc = occupied(keys[(int64_t)kn * H + i], np);
                    nt += (a && bb) + (bb && cc);
                }
            }
        }
        nv = block_sum<NT>(nv, s_tmp);
        nt = block_sum<NT>(nt, s_tmp);
        if (threadIdx.x == 0) { ws.tile_v[t] = nv; ws.tile_t[t] = nt; }
    }
}

// ---------------------------------------------------------------------------
// Per frame: exclusive scans over its tiles.  mode 0: vertex and triangle bases
// (and counts V, T); mode 1: root bases (and count K).
template <int NT>
__global__ __launch_bounds__(NT) void k_scan_tiles(const BatchHeader* __restrict__ hdr, Workspace ws,
                                                   int mode) {
    __shared__ int s_tmp[NT / 64];
    const FrameDesc* F = frames_of(hdr);
    for (int f = blockIdx.x; f < hdr->n_frames; f += gridDim.x) {
        const FrameDesc* fd = F + f;
        const int n = fd->n_tiles, off = fd->tile_off;
        int run0 = 0, run1 = 0;
        for (int base = 0; base < n; base += NT) {
            const int idx = base + threadIdx.x;
            const bool in = idx < n;
            int x, y = 0;
            if (mode == 0) {
                x = in ? ws.tile_v[off + idx] : 0;
                y = in ? ws.tile_t[off + idx] : 0;
            } else {
                x = in ? ws.tile_r[off + idx] : 0;
            }
            int tot0, tot1;
            const int e0 = block_excl_scan<NT>(x, tot0, s_tmp);
            const int e1 = block_excl_scan<NT>(y, tot1, s_tmp);
            if (in) {
                if (mode == 0) {
                    ws.tile_vbase[off + idx] = run0 + e0;
                    ws.tile_tbase[off + idx] = run1 + e1;
                } else {
                    ws.tile_rbase[off + idx] = run0 + e0;
                }
            }
            run0 += tot0;
            run1 += tot1;
        }
        if (threadIdx.x == 0) {
            if (mode == 0) { fd->counts[0] = run0; fd->counts[1] = run1; }
            else fd->counts[2] = run0;
        }
    }
}

// ---------------------------------------------------------------------------
// LDS union-find: links the larger root under the smaller (atomicMin), so every
// root is the smallest cell of its tree.  Path halving only rewrites non-roots.
__device__ __forceinline__ int lds_find(int* P, int x) {
    while (true) {
        const int p = P[x];
        if (p == x) return x;
        const int gp = P[p];
        if (gp != p) P[x] = gp;
        x = gp;
    }
}

__device__ __forceinline__ void lds_union(int* P, int a, int b) {
    while (true) {
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
// empty cells hold NaN coordinates.
__device__ __forceinline__ void vertex_normal(const float* sx, const float* sy, const float* sz,
                                              int lx, int i, int H, float& onx, float& ony, float& onz) {
    const bool up = i >= 1, dn = i + 1 < H;
    const int q[6] = {lx + 1, lx + H + 1, lx + H, lx - 1, lx - H - 1, lx - H};
    const bool ok[6] = {dn, dn, true, up, up, true};
    const double px = sx[lx], py = sy[lx], pz = sz[lx];
    double v0x = 0.0, v0y = 0.0, v0z = 0.0, l0 = 0.0;
    bool p0 = false;
    if (ok[0]) {
        const float qx = sx[q[0]];
        if (qx == qx) {
            p0 = true;
            v0x = (double)qx - px;
            v0y = (double)sy[q[0]] - py;
            v0z = (double)sz[q[0]] - pz;
            const double l2 = v0x * v0x + v0y * v0y + v0z * v0z;
            l0 = l2 * rsq_dp(l2);
        }
    }
    double vpx = v0x, vpy = v0y, vpz = v0z, lp = l0;
    bool pp = p0;
    double ax = 0.0, ay = 0.0, az = 0.0;
    bool any = false;
#pragma unroll
    for (int t = 1; t <= 6; ++t) {
        double vx = 0.0, vy = 0.0, vz = 0.0, lc = 0.0;
        bool pc = false;
        if (t == 6) {
            vx = v0x; vy = v0y; vz = v0z; lc = l0; pc = p0;
        } else if (ok[t]) {
            const float qx = sx[q[t]];
            if (qx == qx) {
                pc = true;
                vx = (double)qx - px;
                vy = (double)sy[q[t]] - py;
                vz = (double)sz[q[t]] - pz;
                const double l2 = vx * vx + vy * vy + vz * vz;
                lc = l2 * rsq_dp(l2);
            }
        }
        if (pp && pc) {
            const double w = rcp_dp(lp + lc);
            ax = fma(w, vpy * vz - vpz * vy, ax);
            ay = fma(w, vpz * vx - vpx * vz, ay);
            az = fma(w, vpx * vy - vpy * vx, az);
            any = true;
        }
        vpx = vx; vpy = vy; vpz = vz; lp = lc; pp = pc;
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
    // sx/sy/sz: coordinates, then (after the normal stage) normals indexed by l
    __shared__ float sx[XC], sy[XC], sz[XC];
    __shared__ int svid[NC];     // vertex index of l (frame-local), -1 = empty
    __shared__ int saux[MAXC];   // kept point index, then triangle start, then union-find parent
    __shared__ int s_tmp[NT / 64];

    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
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

        __syncthreads();  // LDS of the previous tile is free
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

        // 2. numbering: vertices in firing order (own cells, then the right column,
        //    which continues at the next tile's base) and triangles per anchor.
        const int vbase = ws.tile_vbase[t];
        const int own_v = ws.tile_v[t];
        int next_t = t + 1;
        if (lt + 1 == fd->n_tiles) next_t = fd->tile_off;  // seam: column 0 (used only if wrap)
        const int vbase_next = ws.tile_vbase[next_t];
        const int tbase = ws.tile_tbase[t];
        int carry_v = 0, carry_t = 0;
        for (int base = 0; base < nscan; base += NT) {
            const int l = base + threadIdx.x;
            int val = 0;
            if (l < nscan) {
                const int lx = l + H;
                if (sx[lx] == sx[lx]) {
                    int ntri = 0;
                    const int i = l - div_small(l, inv_h) * H;
                    if (l < nown && i + 1 < H) {
                        const bool a = sx[lx + 1] == sx[lx + 1];
                        const bool b = sx[lx + H + 1] == sx[lx + H + 1];
                        const bool c = sx[lx + H] == sx[lx + H];
                        ntri = (int)(a && b) + (int)(b && c);
                    }
                    val = 1 | (ntri << 16);
                }
            }
            int tot;
            const int ex = block_excl_scan<NT>(val, tot, s_tmp);
            if (l < nscan) {
                const int exv = (ex & 0xFFFF) + carry_v;
                const int ext = (ex >> 16) + carry_t;
                int vid = -1;
                if (val) vid = (l < nown) ? vbase + exv : vbase_next + (exv - own_v);
                svid[l] = vid;
                if (l < nown && val) {
                    const int lx = l + H;
                    float* vo = fd->vertices + 3 * (int64_t)vid;
                    vo[0] = sx[lx];
                    vo[1] = sy[lx];
                    vo[2] = sz[lx];
                    if (fd->vpoint) fd->vpoint[vid] = saux[l];
                    saux[l] = tbase + ext;
                }
            }
            carry_v += tot & 0xFFFF;
            carry_t += tot >> 16;
        }
        __syncthreads();

        // 3. triangles T_a = (p, A, B), T_b = (p, B, C) of each own anchor
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

        // 4. normals of own cells and the right column (or the given ones), kept
        //    in registers until every thread is done reading coordinates
        float nrm[RN][3];
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int l = threadIdx.x + r * NT;
            nrm[r][0] = nrm[r][1] = nrm[r][2] = 0.0f;
            if (l < nscan) {
                const int vid = svid[l];
                if (vid >= 0) {
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
        for (int l = threadIdx.x; l < nown; l += NT) saux[l] = l;
        __syncthreads();

        // 5. segments inside the tile: union over similar joins C, A, B
        int* const sparent = saux;
        for (int l = threadIdx.x; l < nown; l += NT) {
            const int lc = div_small(l, inv_h);
            const int i = l - lc * H;
            const float ax = sx[l], ay = sy[l], az = sz[l];
            if (ax == 0.0f && ay == 0.0f && az == 0.0f) continue;
            if (i + 1 < H && similar(ax, ay, az, sx[l + 1], sy[l + 1], sz[l + 1], tx, ty, tz))
                lds_union(sparent, l, l + 1);
            if (lc + 1 < TWe) {
                if (similar(ax, ay, az, sx[l + H], sy[l + H], sz[l + H], tx, ty, tz))
                    lds_union(sparent, l, l + H);
                if (i + 1 < H && similar(ax, ay, az, sx[l + H + 1], sy[l + H + 1], sz[l + H + 1], tx, ty, tz))
                    lds_union(sparent, l, l + H + 1);
            }
        }
        // joins leaving through the right edge: (last column, C) and (last column, B)
        int2* border = ws.border + fd->border_off + (int64_t)lt * 2 * H;
        for (int i = threadIdx.x; i < H; i += NT) {
            const int l = (TWe - 1) * H + i;
            int2 ec = make_int2(-1, -1), eb = make_int2(-1, -1);
            if (similar(sx[l], sy[l], sz[l], sx[l + H], sy[l + H], sz[l + H], tx, ty, tz))
                ec = make_int2(svid[l], svid[l + H]);
            if (i + 1 < H && similar(sx[l], sy[l], sz[l], sx[l + H + 1], sy[l + H + 1], sz[l + H + 1], tx, ty, tz))
                eb = make_int2(svid[l], svid[l + H + 1]);
            border[2 * i] = ec;
            border[2 * i + 1] = eb;
        }
        __syncthreads();
        // local roots: the smallest cell of each local tree (no writes while reading)
        for (int l = threadIdx.x; l < nown; l += NT) {
            const int vid = svid[l];
            if (vid < 0) continue;
            int r = l;
            while (sparent[r] != r) r = sparent[r];
            fd->labels[vid] = svid[r];
        }
    }
}

// ---------------------------------------------------------------------------
// Global union-find on a frame's label array (vertex-indexed parents).
__device__ __forceinline__ int g_load(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int g_find(int* P, int x) {
    while (true) {
        const int p = g_load(P + x);
        if (p == x) return x;
        const int gp = g_load(P + p);
        if (gp != p) __hip_atomic_store(P + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

__device__ __forceinline__ void g_union(int* P, int a, int b) {
    while (true) {
        a = g_find(P, a);
        b = g_find(P, b);
        if (a == b) return;
        if (a > b) { const int t = a; a = b; b = t; }
        const int old = atomicMin(P + b, a);
        if (old == b) return;
        b = old;
    }
}

// Per tile: the similar joins leaving through its right edge.  Both ends are
// replaced by their current parents (any ancestor works for a union), and a
// join whose parent pair repeats one of the previous slots (the rows above,
// usually the same two segments) is skipped, which keeps most threads of a
// border off the same two roots.
template <int NT>
__global__ __launch_bounds__(NT) void k_merge(const BatchHeader* __restrict__ hdr, Workspace ws) {
    static_assert(NT >= 2 * MAX_RINGS, "one border slot per thread");
    __shared__ int2 s_pair[2 * MAX_RINGS];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of_tile(F, nf, t);
        const int H = fd->H;
        int* L = fd->labels;
        const int2* border = ws.border + fd->border_off + (int64_t)(t - fd->tile_off) * 2 * H;
        const int e = threadIdx.x;
        int2 rr = make_int2(-1, -1);
        if (e < 2 * H) {
            const int2 ab = border[e];
            if (ab.x >= 0) rr = make_int2(g_load(L + ab.x), g_load(L + ab.y));
        }
        __syncthreads();
        if (e < 2 * H) s_pair[e] = rr;
        __syncthreads();
        if (rr.x >= 0) {
            bool dup = false;
#pragma unroll
            for (int d = 1; d <= 4; ++d) {
                if (e - d >= 0) {
                    const int2 q = s_pair[e - d];
                    dup |= (q.x == rr.x && q.y == rr.y);
                }
            }
            if (!dup) g_union(L, rr.x, rr.y);
        }
    }
}

// Every vertex points at its root; roots counted per tile; the tile's key cells
// are reset for the next call.
template <int NT>
__global__ __launch_bounds__(NT) void k_flatten(const BatchHeader* __restrict__ hdr, Workspace ws) {
    __shared__ int s_tmp[NT / 64];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of_tile(F, nf, t);
        int* L = fd->labels;
        const int vb = ws.tile_vbase[t], nv = ws.tile_v[t];
        int roots = 0;
        for (int v = vb + threadIdx.x; v < vb + nv; v += NT) {
            int r = v;
            while (true) {
                const int p = L[r];
                if (p == r) break;
                r = p;
            }
            L[v] = r;
            roots += (r == v);
        }
        roots = block_sum<NT>(roots, s_tmp);
        if (threadIdx.x == 0) ws.tile_r[t] = roots;
        const int H = fd->H;
        const int k0 = (t - fd->tile_off) * fd->TW;
        const int TWe = min(fd->TW, fd->Wp - k0);
        uint64_t* keys = ws.keys + fd->cell_off + (int64_t)k0 * H;
        for (int l = threadIdx.x; l < H * TWe; l += NT) keys[l] = KEY_EMPTY;
    }
}

// Roots take -(label): label = 1 + rank of the root among roots in firing order.
template <int NT>
__global__ __launch_bounds__(NT) void k_rank(const BatchHeader* __restrict__ hdr, Workspace ws) {
    __shared__ int s_tmp[NT / 64];
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of_tile(F, nf, t);
        int* L = fd->labels;
        const int vb = ws.tile_vbase[t], nv = ws.tile_v[t];
        int carry = ws.tile_rbase[t];
        for (int base = 0; base < nv; base += NT) {
            const int v = vb + base + threadIdx.x;
            const bool in = base + threadIdx.x < nv;
            const int root = in && (L[v] == v);
            int tot;
            const int ex = block_excl_scan<NT>(root, tot, s_tmp);
            if (root) L[v] = -(1 + carry + ex);
            carry += tot;
        }
    }
}

template <int NT>
__global__ __launch_bounds__(NT) void k_final(const BatchHeader* __restrict__ hdr, Workspace ws) {
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of_tile(F, nf, t);
        int* L = fd->labels;
        const int vb = ws.tile_vbase[t], nv = ws.tile_v[t];
        for (int v = vb + threadIdx.x; v < vb + nv; v += NT) {
            const int x = L[v];
            L[v] = (x < 0) ? -x : abs(L[x]);
        }
    }
}

}  // namespace

hipError_t launch_chain(const BatchHeader* d_hdr, const Workspace& ws, const LaunchCfg& cfg,
                        hipStream_t stream, hipEvent_t* ev) {
    constexpr int NT = 256;
    const int g_tiles = max(1, min(cfg.grid, cfg.max_tiles));
    const int g_pblk = max(1, min(cfg.grid, cfg.max_pblk));
    const int g_frames = max(1, min(cfg.max_frames, 1024));
    int n = 0;
    hipError_t e = hipSuccess;
    auto mark = [&]() {
        if (ev && e == hipSuccess) e = hipEventRecord(ev[n], stream);
        ++n;
    };
    mark();
    k_bin<NT><<<g_pblk, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_count<NT><<<g_tiles, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_scan_tiles<NT><<<g_frames, NT, 0, stream>>>(d_hdr, ws, 0);
    mark();
    switch (cfg.tile_cells) {
        case 512: k_tile<NT, 512><<<g_tiles, NT, 0, stream>>>(d_hdr, ws); break;
        case 2048: k_tile<NT, 2048><<<g_tiles, NT, 0, stream>>>(d_hdr, ws); break;
        default: k_tile<NT, 1024><<<g_tiles, NT, 0, stream>>>(d_hdr, ws); break;
    }
    mark();
    k_merge<NT><<<g_tiles, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_flatten<NT><<<g_tiles, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_scan_tiles<NT><<<g_frames, NT, 0, stream>>>(d_hdr, ws, 1);
    mark();
    k_rank<NT><<<g_tiles, NT, 0, stream>>>(d_hdr, ws);
    mark();
    k_final<NT><<<g_tiles, NT, 0, stream>>>(d_hdr, ws);
    mark();
    const hipError_t le = hipGetLastError();
    return le != hipSuccess ? le : e;
}

}  // namespace lidarseg
