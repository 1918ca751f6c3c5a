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
        const int64_t p0 = (int64_t)(b - fd->pblk_off) * POINT_BLOCK;
        const int64_t p1 = min(p0 + POINT_BLOCK, fd->n_points);
        for (int64_t p = p0 + threadIdx.x; p < p1; p += NT) {
            const float xf = xyz[3 * p], yf = xyz[3 * p + 1], zf = xyz[3 * p + 2];
            if (!(isfinite(xf) && isfinite(yf) && isfinite(zf))) continue;
            const double x = xf, y = yf, z = zf;
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

// Weighted normal of LDS cell lx (ring i): sum over cycle-adjacent present pairs
// (A,B),(B,C),(C,D),(D,E),(E,F),(F,A) of (V_t x V_u) / (|V_t| + |V_u|), scaled to
// unit length (Section 2, Normal Estimation).  Edge vectors are exact in FP64.
__device__ __forceinline__ void vertex_normal(const float* sx, const float* sy, const float* sz,
                                              const uint8_t* sflag, int lx, int i, int H,
                                              float& onx, float& ony, float& onz) {
    const bool up = i >= 1, dn = i + 1 < H;
    const int off[6] = {1, H + 1, H, -1, -H - 1, -H};
    bool pres[6];
    pres[0] = dn && sflag[lx + 1];
    pres[1] = dn && sflag[lx + H + 1];
    pres[2] = sflag[lx + H] != 0;
    pres[3] = up && sflag[lx - 1];
    pres[4] = up && sflag[lx - H - 1];
    pres[5] = sflag[lx - H] != 0;
    const double px = sx[lx], py = sy[lx], pz = sz[lx];
    double vx[6], vy[6], vz[6], len[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        if (pres[t]) {
            const int q = lx + off[t];
            vx[t] = (double)sx[q] - px;
            vy[t] = (double)sy[q] - py;
            vz[t] = (double)sz[q] - pz;
            len[t] = sqrt(vx[t] * vx[t] + vy[t] * vy[t] + vz[t] * vz[t]);
        } else {
            vx[t] = vy[t] = vz[t] = len[t] = 0.0;
        }
    }
    double ax = 0.0, ay = 0.0, az = 0.0;
    bool any = false;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const int u = (t + 1) % 6;
        if (pres[t] && pres[u]) {
            const double w = 1.0 / (len[t] + len[u]);
            ax += w * (vy[t] * vz[u] - vz[t] * vy[u]);
            ay += w * (vz[t] * vx[u] - vx[t] * vz[u]);
            az += w * (vx[t] * vy[u] - vy[t] * vx[u]);
            any = true;
        }
    }
    const double n2 = ax * ax + ay * ay + az * az;
    if (any && n2 > 0.0) {
        const double nrm = sqrt(n2);
        onx = (float)(ax / nrm);
        ony = (float)(ay / nrm);
        onz = (float)(az / nrm);
    } else {
        onx = ony = onz = 0.0f;
    }
}

// ---------------------------------------------------------------------------
// The per-tile fused stage.  LDS columns lc = -1 .. TWe+1 of the tile (global
// column k0 + lc, wrapped on a closed cylinder) hold validity and coordinates;
// LDS cell lx = (lc + 1) * H + i.  Own cells are lc in [0, TWe); the right
// column lc = TWe belongs to the next tile but its normals are needed for the
// joins that leave the tile.
template <int NT, int MAXC>
__global__ __launch_bounds__(NT) void k_tile(const BatchHeader* __restrict__ hdr, Workspace ws) {
    constexpr int XC = MAXC + 3 * MAX_RINGS;  // coordinate cells incl. halo
    constexpr int NC = MAXC + MAX_RINGS;      // own cells + right column
    __shared__ float sx[XC], sy[XC], sz[XC];
    __shared__ float snx[NC], sny[NC], snz[NC];
    __shared__ int svid[NC];
    __shared__ uint8_t sflag[XC];
    __shared__ int s_tmp[NT / 64];
    int* const sparent = reinterpret_cast<int*>(sx);   // after the normal stage
    int* const ssrc = reinterpret_cast<int*>(snx);     // before the normal stage
    int* const stri = reinterpret_cast<int*>(snx);     // same slots, after ssrc is read

    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of_tile(F, nf, t);
        const int H = fd->H, Wp = fd->Wp, wrap = fd->wrap;
        const int lt = t - fd->tile_off;
        const int k0 = lt * fd->TW;
        const int TWe = min(fd->TW, Wp - k0);
        const int nx = H * (TWe + 3);
        const int nown = H * TWe;
        const int nscan = nown + H;
        const uint64_t* keys = ws.keys + fd->cell_off;
        const float* __restrict__ xyz = fd->xyz;
        const float* __restrict__ nin = fd->normals_in;
        const double tx = fd->thr[0], ty = fd->thr[1], tz = fd->thr[2];

        __syncthreads();  // LDS of the previous tile is free
        // 1. validity and coordinates of the tile and its halo columns
        for (int lx = threadIdx.x; lx < nx; lx += NT) {
            const int col = lx / H;
            const int i = lx - col * H;
            int k = k0 + col - 1;
            bool in = true;
            if (k < 0 || k >= Wp) {
                if (wrap) k = (k < 0) ? k + Wp : k - Wp;
                else in = false;
            }
            const uint64_t key = in ? keys[(int64_t)k * H + i] : KEY_EMPTY;
            const bool v = occupied(key, fd->n_points);
            sflag[lx] = v;
            if (v) {
                const uint32_t src = (uint32_t)key;
                sx[lx] = xyz[3 * (int64_t)src];
                sy[lx] = xyz[3 * (int64_t)src + 1];
                sz[lx] = xyz[3 * (int64_t)src + 2];
                if (lx >= H && lx < H + nown) ssrc[lx - H] = (int)src;
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
            if (l < nscan && sflag[l + H]) {
                int ntri = 0;
                const int i = l - (l / H) * H;
                if (l < nown && i + 1 < H) {
                    const int lx = l + H;
                    const bool a = sflag[lx + 1], b = sflag[lx + H + 1], c = sflag[lx + H];
                    ntri = (int)(a && b) + (int)(b && c);
                }
                val = 1 | (ntri << 16);
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
                    if (fd->vpoint) fd->vpoint[vid] = ssrc[l];
                    stri[l] = tbase + ext;
                }
            }
            carry_v += tot & 0xFFFF;
            carry_t += tot >> 16;
        }
        __syncthreads();

        // 3. triangles T_a = (p, A, B), T_b = (p, B, C) of each own anchor
        for (int l = threadIdx.x; l < nown; l += NT) {
            const int p = svid[l];
            const int i = l - (l / H) * H;
            if (p < 0 || i + 1 >= H) continue;
            const int a = svid[l + 1], b = svid[l + H + 1], c = svid[l + H];
            int ti = stri[l];
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
        __syncthreads();

        // 4. normals of own cells and the right column (or the given ones)
        for (int l = threadIdx.x; l < nscan; l += NT) {
            const int lx = l + H;
            const int i = l - (l / H) * H;
            float nx_ = 0.0f, ny_ = 0.0f, nz_ = 0.0f;
            const int vid = svid[l];
            if (vid >= 0) {
                if (nin) {
                    nx_ = nin[3 * (int64_t)vid];
                    ny_ = nin[3 * (int64_t)vid + 1];
                    nz_ = nin[3 * (int64_t)vid + 2];
                } else {
                    vertex_normal(sx, sy, sz, sflag, lx, i, H, nx_, ny_, nz_);
                }
                if (l < nown) {
                    float* no = fd->normals + 3 * (int64_t)vid;
                    no[0] = nx_; no[1] = ny_; no[2] = nz_;
                }
            }
            snx[l] = nx_; sny[l] = ny_; snz[l] = nz_;
        }
        __syncthreads();

        // 5. segments inside the tile: union over similar joins C, A, B
        for (int l = threadIdx.x; l < nown; l += NT) sparent[l] = l;
        __syncthreads();
        for (int l = threadIdx.x; l < nown; l += NT) {
            const int i = l - (l / H) * H;
            const int lc = l / H;
            const float ax = snx[l], ay = sny[l], az = snz[l];
            if (ax == 0.0f && ay == 0.0f && az == 0.0f) continue;
            if (i + 1 < H && similar(ax, ay, az, snx[l + 1], sny[l + 1], snz[l + 1], tx, ty, tz))
                lds_union(sparent, l, l + 1);
            if (lc + 1 < TWe) {
                if (similar(ax, ay, az, snx[l + H], sny[l + H], snz[l + H], tx, ty, tz))
                    lds_union(sparent, l, l + H);
                if (i + 1 < H &&
                    similar(ax, ay, az, snx[l + H + 1], sny[l + H + 1], snz[l + H + 1], tx, ty, tz))
                    lds_union(sparent, l, l + H + 1);
            }
        }
        // joins leaving through the right edge: (last column, C) and (last column, B)
        int2* border = ws.border + fd->border_off + (int64_t)lt * 2 * H;
        for (int i = threadIdx.x; i < H; i += NT) {
            const int l = (TWe - 1) * H + i;
            int2 ec = make_int2(-1, -1), eb = make_int2(-1, -1);
            if (similar(snx[l], sny[l], snz[l], snx[l + H], sny[l + H], snz[l + H], tx, ty, tz))
                ec = make_int2(svid[l], svid[l + H]);
            if (i + 1 < H &&
                similar(snx[l], sny[l], snz[l], snx[l + H + 1], sny[l + H + 1], snz[l + H + 1], tx, ty, tz))
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

template <int NT>
__global__ __launch_bounds__(NT) void k_merge(const BatchHeader* __restrict__ hdr, Workspace ws) {
    const FrameDesc* F = frames_of(hdr);
    const int nf = hdr->n_frames;
    for (int t = blockIdx.x; t < hdr->total_tiles; t += gridDim.x) {
        const FrameDesc* fd = F + frame_of_tile(F, nf, t);
        const int H = fd->H;
        const int2* border = ws.border + fd->border_off + (int64_t)(t - fd->tile_off) * 2 * H;
        for (int e = threadIdx.x; e < 2 * H; e += NT) {
            const int2 ab = border[e];
            if (ab.x >= 0) g_union(fd->labels, ab.x, ab.y);
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
