// Cell-list neighbor build (neighborhoods of MLIP-3 paper Sec. II.A).
//
// Per configuration the cell is cut into n_k bins along each cell vector
// (n_k = floor(h_k / R_cut), h_k = height of the cell along axis k, coarsened
// so that a configuration never has more bins than atoms).  A bin is then at
// least R_cut high, and every neighbor of an atom lies within s_k =
// ceil(R_cut n_k / h_k) bins along axis k.  Periodic axes wrap bins and
// record the image shift; a bin visited twice through different wraps is a
// different image, so small cells (h_k < R_cut) come out right.
//
// Steps: geometry per configuration -> bin every atom (counting sort, then
// each bin sorted by atom index so the result is deterministic) -> per atom
// the distance tests against the 27 (or more) nearby bins, whose ballots give
// the per-species counts and every pair's place in the list, grouped by
// neighbor species (bins whose surroundings exceed one LDS window: a counting
// sweep, then a filling sweep) -> reverse-pair index for the atomic-free
// force gather.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "internal.hpp"

namespace mtp {
namespace {

struct CfgGeo {
    double H[9], Hi[9];
    int n[3], s[3], pbc[3], pad;
    long long bin_off, nbins;
};

__device__ inline double height(const double *H, int k) {
    const double *u = H + 3 * ((k + 1) % 3), *v = H + 3 * ((k + 2) % 3), *w = H + 3 * k;
    double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
    double vol = fabs(w[0] * cx + w[1] * cy + w[2] * cz);
    return vol / sqrt(cx * cx + cy * cy + cz * cz);
}

// Clears the bin counters and fill cursors (all threads) and the status
// words; thread 0 then walks all configurations (bin offsets are a running
// sum) and writes their geometry.
__global__ void nbr_prepare(int n_cfg, const int64_t *cfg_off, const double *cell, const uint8_t *pbc, double rc,
                            CfgGeo *geo, int *flags, int32_t *bin_count, int32_t *cursor, int64_t bins) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bins; i += (int64_t)gridDim.x * blockDim.x) {
        bin_count[i] = 0;
        cursor[i] = 0;
    }
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    for (int k = 0; k < 8; ++k) flags[k] = 0;
    long long off = 0;
    for (int c = 0; c < n_cfg; ++c) {
        CfgGeo g;
        for (int k = 0; k < 9; ++k) g.H[k] = cell[9 * c + k];
        const double *H = g.H;
        double a = H[0], b = H[1], cc = H[2], d = H[3], e = H[4], f = H[5], gg = H[6], h = H[7], kk = H[8];
        double det = a * (e * kk - f * h) - b * (d * kk - f * gg) + cc * (d * h - e * gg);
        if (!(fabs(det) > 1e-12)) {   // degenerate cell: flag it, keep every index in range
            atomicOr(&flags[3], 1);
            det = INFINITY;
        }
        g.Hi[0] = (e * kk - f * h) / det; g.Hi[1] = (cc * h - b * kk) / det; g.Hi[2] = (b * f - cc * e) / det;
        g.Hi[3] = (f * gg - d * kk) / det; g.Hi[4] = (a * kk - cc * gg) / det; g.Hi[5] = (cc * d - a * f) / det;
        g.Hi[6] = (d * h - e * gg) / det; g.Hi[7] = (b * gg - a * h) / det; g.Hi[8] = (a * e - b * d) / det;
        const long long natoms = cfg_off[c + 1] - cfg_off[c];
        double hk[3];
        for (int k = 0; k < 3; ++k) {
            hk[k] = height(H, k);
            g.pbc[k] = pbc ? (int)pbc[3 * c + k] : 1;
            int nk = (int)floor(hk[k] / rc);
            g.n[k] = nk < 1 ? 1 : (nk > 1024 ? 1024 : nk);
        }
        const long long cap = natoms > 1 ? natoms : 1;
        while ((long long)g.n[0] * g.n[1] * g.n[2] > cap) {
            int big = 0;
            for (int k = 1; k < 3; ++k)
                if (g.n[k] > g.n[big]) big = k;
            g.n[big] -= 1;
        }
        for (int k = 0; k < 3; ++k) {
            int s = (int)ceil(rc * g.n[k] / hk[k]);
            g.s[k] = s < 1 ? 1 : s;
        }
        g.pad = 0;
        g.bin_off = off;
        g.nbins = (long long)g.n[0] * g.n[1] * g.n[2];
        off += g.nbins;
        geo[c] = g;
    }
    flags[4] = (int)off;   // bins in use (<= the host-side capacity n_atoms + n_cfg)
}

// A position that is not finite (NaN, Inf) sets bit 16 of flags[3] and is
// binned at the origin of its cell (it then fails every distance test): the
// status check reports MTP_E_INVAL instead of an empty neighborhood.
__global__ void bin_kernel(int64_t n, int n_cfg, const int64_t *cfg_off, const double *pos, const CfgGeo *geo,
                           int32_t *atom_cfg, int32_t *atom_bin, int32_t *atom_wrap, int32_t *bin_count,
                           int32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // configuration of atom i: last c with cfg_off[c] <= i
    int lo = 0, hi = n_cfg - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (cfg_off[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const CfgGeo &g = geo[lo];
    double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    if (!(isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]))) {
        atomicOr(&flags[3], 16);
        x[0] = x[1] = x[2] = 0.0;
    }
    int b[3], w[3];
    for (int k = 0; k < 3; ++k) {
        double s = x[0] * g.Hi[k] + x[1] * g.Hi[3 + k] + x[2] * g.Hi[6 + k];
        if (g.pbc[k]) {
            double fw = floor(s);
            w[k] = (int)fw;
            s -= fw;
        } else {
            w[k] = 0;
        }
        int bk = (int)floor(s * g.n[k]);
        b[k] = bk < 0 ? 0 : (bk >= g.n[k] ? g.n[k] - 1 : bk);
    }
    const int bin = (int)(g.bin_off + ((long long)b[2] * g.n[1] + b[1]) * g.n[0] + b[0]);
    atom_cfg[i] = lo;
    atom_bin[i] = bin;
    atom_wrap[3 * i] = w[0];
    atom_wrap[3 * i + 1] = w[1];
    atom_wrap[3 * i + 2] = w[2];
    atomicAdd(&bin_count[bin], 1);
}

// Exclusive scan of the bin counts (only the bins in use, a few per 10
// atoms) by one block: chunks of 4096, four per thread, wave scans by
// shuffles and one LDS step across the 16 wavefronts.
constexpr int SCAN_T = 1024;

struct BinStart {
    const int32_t *loc;
    __device__ int32_t operator[](int64_t b) const { return loc[b]; }
};

__global__ __launch_bounds__(SCAN_T) void scan_bins(const int32_t *in, int32_t *out, const int32_t *n_dev) {
    __shared__ int32_t wsum[SCAN_T / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t n = *n_dev;
    int32_t carry = 0;
    for (int64_t base = 0; base < n; base += 4 * SCAN_T) {
        const int64_t i0 = base + 4 * (int64_t)threadIdx.x;
        int32_t v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = i0 + e < n ? in[i0 + e] : 0;
        const int32_t tot = v[0] + v[1] + v[2] + v[3];
        int32_t inc = tot;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t t = __shfl_up(inc, d, 64);
            if (lane >= d) inc += t;
        }
        if (lane == 63) wsum[wave] = inc;
        __syncthreads();
        if (wave == 0) {
            int32_t w = lane < SCAN_T / 64 ? wsum[lane] : 0, wi = w;
#pragma unroll
            for (int d = 1; d < SCAN_T / 64; d <<= 1) {
                const int32_t t = __shfl_up(wi, d, 64);
                if (lane >= d) wi += t;
            }
            if (lane < SCAN_T / 64) wsum[lane] = wi - w;   // exclusive over the wavefronts
        }
        __syncthreads();
        int32_t run = carry + wsum[wave] + inc - tot;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (i0 + e < n) out[i0 + e] = run;
            run += v[e];
        }
        // the running total after this chunk: the last thread's value
        __syncthreads();
        if (threadIdx.x == SCAN_T - 1) wsum[0] = run;
        __syncthreads();
        carry = wsum[0];
        __syncthreads();
    }
}

__global__ void fill_bins(int64_t n, const int32_t *atom_bin, BinStart start, int32_t *cursor, int32_t *bin_atoms) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = atom_bin[i];
    bin_atoms[start[b] + atomicAdd(&cursor[b], 1)] = (int32_t)i;
}

__device__ inline int pack_q(int x, int y, int z) { return (x + 512) | ((y + 512) << 10) | ((z + 512) << 20); }

struct Stage {
    const double *pos;
    const int32_t *type, *atom_cfg, *atom_wrap;
    const CfgGeo *geo;
    int n_types;
    double *sx;     // [3 n] x_j - w_j.H
    int32_t *sw;    // [n] pack_q(-w_j)
    int32_t *st;    // [n] species (0 where out of range: that is reported)
};

// slot u of the bin order holds atom j: wrapped position, packed -wrap, species
__device__ inline void stage_atom(const Stage &S, int64_t u, int j, bool &wide, bool &bad) {
    const CfgGeo &g = S.geo[S.atom_cfg[j]];
    const int w0 = S.atom_wrap[3 * (int64_t)j], w1 = S.atom_wrap[3 * (int64_t)j + 1],
              w2 = S.atom_wrap[3 * (int64_t)j + 2];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        S.sx[3 * u + k] = S.pos[3 * (int64_t)j + k] - (w0 * g.H[k] + w1 * g.H[3 + k] + w2 * g.H[6 + k]);
    if (w0 < -255 || w0 > 255 || w1 < -255 || w1 > 255 || w2 < -255 || w2 > 255) wide = true;
    S.sw[u] = pack_q(-w0, -w1, -w2);
    const int t = S.type[j];
    if (t < 0 || t >= S.n_types) bad = true;   // reported as an error; 0 keeps later indexing in range
    S.st[u] = (t < 0 || t >= S.n_types) ? 0 : t;
}

// One wavefront per bin: the bin's atoms (filled in arbitrary order by
// atomics) are put in ascending index order, which makes every later step
// deterministic, and each is staged at its slot.  Ranks come from all-pairs
// comparisons across the lanes; bins over 64 atoms are sorted by one lane.
__device__ inline void sort_stage_bin(int32_t *a, int64_t start, int c, int lane, const Stage &S, bool &wide,
                                      bool &bad) {
    if (c <= 0) return;
    if (c <= 64) {
        const int v = lane < c ? a[lane] : 0x7fffffff;
        int rank = 0;
        for (int k = 0; k < c; ++k) rank += __shfl(v, k, 64) < v ? 1 : 0;
        if (lane < c) {
            a[rank] = v;
            stage_atom(S, start + rank, v, wide, bad);
        }
    } else if (lane == 0) {
        for (int x = 1; x < c; ++x) {
            const int32_t v = a[x];
            int y = x - 1;
            while (y >= 0 && a[y] > v) {
                a[y + 1] = a[y];
                --y;
            }
            a[y + 1] = v;
        }
        for (int x = 0; x < c; ++x) stage_atom(S, start + x, a[x], wide, bad);
    }
}

__global__ __launch_bounds__(256) void sort_bins(int32_t *flags, BinStart start, const int32_t *count,
                                                 int32_t *bin_atoms, Stage S) {
    const int lane = threadIdx.x & 63;
    const int64_t nbins = flags[4];
    bool wide = false, bad = false;
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nbins; b += (int64_t)gridDim.x * 4) {
        const int32_t sb = start[b];
        sort_stage_bin(bin_atoms + sb, sb, count[b], lane, S, wide, bad);
    }
    const bool any_wide = __ballot(wide) != 0, any_bad = __ballot(bad) != 0;
    if (lane == 0 && (any_wide || any_bad)) atomicOr(&flags[3], (any_wide ? 2 : 0) | (any_bad ? 8 : 0));
}

__device__ inline int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// ---- pair search ------------------------------------------------------------
//
// One block of four wavefronts per bin.  The candidates of the bin (atoms of
// the surrounding bins, every periodic image that can be in range) are
// numbered by a wave-wide prefix sum over the bin offsets and staged in LDS,
// a window of PS_WIN at a time, each as y_j = x_j - w_j.H (atom j wrapped
// into the cell) and its bin offset, whose periodic wrap q gives the lattice
// vector q.H.  For an atom i of the bin r_ij = (y_j - y_i) + q.H, which is
// bitwise -r_ji (the opposite pair has offset -d and wrap -q), so the lists
// are exactly symmetric; the pair's shift is q - w_j + w_i.  Wave w builds the neighborhoods of the bin's atoms
// w, w + 4, ...: lanes test candidates 64 at a time, ballots per neighbor
// species give every accepted pair its place in the list (grouped by
// species, candidate order inside a group, clamped to max_nbrs), and the
// pairs are then written with consecutive lanes on consecutive slots.  When
// the candidates fit one window (the usual case) every distance is computed
// once; otherwise each atom takes a counting sweep and a writing sweep over
// the windows.
constexpr int PS_WIN = 512;
constexpr int PS_CC = PS_WIN / 64;

__device__ inline int field(int p, int k) { return ((p >> (10 * k)) & 1023) - 512; }

struct Around {   // the bins around one bin: this lane's bin offset
    int start, count, qp, excl, total;
};

__device__ inline Around around_bin(const CfgGeo &g, int bx, int by, int bz, int o, int n_off, int lane,
                                    const BinStart &bin_start, const int32_t *bin_count) {
    Around A{0, 0, pack_q(0, 0, 0), 0, 0};
    if (o < n_off) {
        const int ox = 2 * g.s[0] + 1, oy = 2 * g.s[1] + 1;
        const int dx = o % ox - g.s[0], dy = (o / ox) % oy - g.s[1], dz = o / (ox * oy) - g.s[2];
        int ux = bx + dx, uy = by + dy, uz = bz + dz, qx = 0, qy = 0, qz = 0;
        bool ok = true;
        if (g.pbc[0]) { qx = floordiv(ux, g.n[0]); ux -= qx * g.n[0]; } else ok = ok && ux >= 0 && ux < g.n[0];
        if (g.pbc[1]) { qy = floordiv(uy, g.n[1]); uy -= qy * g.n[1]; } else ok = ok && uy >= 0 && uy < g.n[1];
        if (g.pbc[2]) { qz = floordiv(uz, g.n[2]); uz -= qz * g.n[2]; } else ok = ok && uz >= 0 && uz < g.n[2];
        if (ok) {
            const long long nb = g.bin_off + ((long long)uz * g.n[1] + uy) * g.n[0] + ux;
            A.start = bin_start[nb];
            A.count = bin_count[nb];
            A.qp = pack_q(qx, qy, qz);
        }
    }
    int inc = A.count;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    A.excl = inc - A.count;
    A.total = __shfl(inc, 63, 64);
    return A;
}

struct Staged {
    const double *sx;
    const int32_t *sw, *st, *bin_atoms;
};

struct Window {   // LDS: one window of candidates
    double x[PS_WIN], y[PS_WIN], z[PS_WIN];
    int jq[PS_WIN];   // j if the bin offset has no periodic wrap, else ~j (never equal to an atom index)
    int qt[PS_WIN];   // pack_q(q - w_j) | species << 30
    unsigned char lo[PS_WIN];   // bin offset (lane of the offset group)
    double qh[64][3];           // q.H per bin offset of the group
};

// Candidates w0 .. w0 + PS_WIN - 1 of an offset group into LDS; every wave
// of the block holds the same offset group A, and each stages its quarter.
__device__ inline void stage_window(Window &W, const Around &A, int w0, int wave, int lane, const double (&H)[9],
                                    const Staged &S) {
    if (wave == 0) {
        const int qx = field(A.qp, 0), qy = field(A.qp, 1), qz = field(A.qp, 2);
#pragma unroll
        for (int k = 0; k < 3; ++k) W.qh[lane][k] = qx * H[k] + qy * H[3 + k] + qz * H[6 + k];
    }
    for (int e = wave * 64 + lane, e0 = wave * 64; e0 < PS_WIN && w0 + e0 < A.total; e += 256, e0 += 256) {
        const int v = w0 + e;
        int L = 0;   // last lane whose bins start at or before candidate v
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int ex = __shfl(A.excl, L + step, 64);
            if (ex <= v) L += step;
        }
        const int st = __shfl(A.start, L, 64), pe = __shfl(A.excl, L, 64), q = __shfl(A.qp, L, 64);
        if (v < A.total && e < PS_WIN) {
            const int64_t u = st + v - pe;
            const int qx = field(q, 0), qy = field(q, 1), qz = field(q, 2);
            W.x[e] = S.sx[3 * u];
            W.y[e] = S.sx[3 * u + 1];
            W.z[e] = S.sx[3 * u + 2];
            const int nw = S.sw[u];
            const int j = S.bin_atoms[u];
            W.jq[e] = (qx == 0 && qy == 0 && qz == 0) ? j : ~j;
            W.qt[e] = pack_q(qx + field(nw, 0), qy + field(nw, 1), qz + field(nw, 2)) | (S.st[u] << 30);
            W.lo[e] = (unsigned char)L;
        }
    }
}

struct Centre {   // the atom whose neighborhood is built (wave-uniform)
    int i, w0, w1, w2;
    double y0, y1, y2;   // y_i
};

struct Flags {
    bool overlap = false, wide = false;
};

// Tests the window's candidates against atom i: bit cc of the returned mask
// is candidate 64 cc + lane; *tb gets its species (2 bits each).  The test
// 0 < |r| < R_cut is made as r.r <= d2max, d2max being the largest double
// whose (correctly rounded) square root is below R_cut: the same decision as
// sqrt(r.r) < R_cut, without the square root.
__device__ inline unsigned test_window(const Window &W, int n, const Centre &c, int lane, double d2max, unsigned &tb,
                                       Flags &fl) {
    unsigned in = 0;
    tb = 0;
    for (int cc = 0; cc * 64 < n; ++cc) {
        const int e = cc * 64 + lane;
        if (e >= n) break;
        const int o = W.lo[e];
        const double r0 = (W.x[e] - c.y0) + W.qh[o][0], r1 = (W.y[e] - c.y1) + W.qh[o][1],
                     r2 = (W.z[e] - c.y2) + W.qh[o][2];
        const double d2 = r0 * r0 + r1 * r1 + r2 * r2;
        bool ok = d2 <= d2max;
        ok = ok && W.jq[e] != c.i;   // the atom itself (same image)
        if (ok) {
            in |= 1u << cc;
            tb |= ((unsigned)W.qt[e] >> 30) << (2 * cc);
            if (d2 < 1e-12) fl.overlap = true;
        }
    }
    return in;
}

// One-window form of the test: the candidates' chunks are unrolled and the
// per-species counts come from ballots (scalar popcounts), so no separate
// counting pass is needed.  in / tb as for test_window.
template <int NT>
__device__ inline unsigned test_count(const Window &W, int n, const Centre &c, int lane, double d2max, unsigned &tb,
                                      int (&cnt)[MAX_TYPES], Flags &fl) {
    unsigned in = 0;
    tb = 0;
#pragma unroll
    for (int cc = 0; cc < PS_CC; ++cc) {
        if (cc * 64 < n) {   // wave-uniform
            const int e = cc * 64 + lane;
            bool ok = false;
            unsigned t = 0;
            if (e < n) {
                const int o = W.lo[e];
                const double r0 = (W.x[e] - c.y0) + W.qh[o][0], r1 = (W.y[e] - c.y1) + W.qh[o][1],
                             r2 = (W.z[e] - c.y2) + W.qh[o][2];
                const double d2 = r0 * r0 + r1 * r1 + r2 * r2;
                t = (unsigned)W.qt[e] >> 30;
                ok = d2 <= d2max && W.jq[e] != c.i;   // not the atom itself (same image)
                if (ok && d2 < 1e-12) fl.overlap = true;
            }
            if (ok) {
                in |= 1u << cc;
                tb |= t << (2 * cc);
            }
#pragma unroll
            for (int s = 0; s < NT; ++s) cnt[s] += __popcll(__ballot(ok && t == (unsigned)s));
        }
    }
    return in;
}

// One-window neighborhoods: an accepted candidate of species t goes to list
// offset base[t] + (accepted candidates of species t before it), kept if
// below cap[t] (the rank within a chunk is mbcnt on the chunk's ballot of
// species t); the list offset is below PS_WIN, so perm is indexed by it
// directly (no compaction) and every offset below the capped total gets
// exactly one candidate, in candidate order within each species group.
// The same chunk ballots also give, for this lane's candidate index x (the
// first candidate of its bin offset), how many accepted candidates of each
// species come before x: pre[s], clamped to cap[s] on return (where that
// bin offset's run starts in the species group).
template <int NT>
__device__ inline void place_chunks(unsigned in, unsigned tb, int n, int lane, const int (&cap)[MAX_TYPES],
                                    const int (&base)[MAX_TYPES], short *perm, int x, int (&pre)[MAX_TYPES]) {
    int run[NT];
#pragma unroll
    for (int s = 0; s < NT; ++s) run[s] = 0;
    const int xc = x >> 6;
    const unsigned long long xbelow = (1ull << (x & 63)) - 1ull;
    bool xset = false;
#pragma unroll
    for (int cc = 0; cc < PS_CC; ++cc) {
        if (cc * 64 < n) {   // wave-uniform
            const bool a = (in >> cc) & 1u;
            const int t = (tb >> (2 * cc)) & 3;
            const bool here = xc == cc;
            unsigned long long mk = 0ull;
            int r = 0, cp = 0, bs = 0;
#pragma unroll
            for (int s = 0; s < NT; ++s) {
                const unsigned long long m = __ballot(a && t == s);
                if (t == s) {
                    mk = m;
                    r = run[s];
                    cp = cap[s];
                    bs = base[s];
                }
                if (here) pre[s] = run[s] + __popcll(m & xbelow);
                run[s] += __popcll(m);
            }
            xset = xset || here;
            const int k = r + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mk >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((unsigned)mk, 0u));
            if (a && k < cp) perm[bs + k] = (short)(cc * 64 + lane);
        }
    }
#pragma unroll
    for (int s = 0; s < NT; ++s) {
        const int v = xset ? pre[s] : run[s];   // x at or past the last candidate: all of them
        pre[s] = v < cap[s] ? v : cap[s];
    }
}

// per-species counts of the accepted candidates (wave-uniform)
__device__ inline void count_window(unsigned in, unsigned tb, int n, int n_types, int (&cnt)[MAX_TYPES]) {
    for (int cc = 0; cc * 64 < n; ++cc) {
        const bool a = (in >> cc) & 1u;
        const int t = (tb >> (2 * cc)) & 3;
#pragma unroll
        for (int s = 0; s < MAX_TYPES; ++s)
            if (s < n_types) cnt[s] += __popcll(__ballot(a && t == s));
    }
}

// Places the accepted candidates: list offset base[t] + run[t] + rank among
// this window's pairs of species t; kept if the rank is below cap[t] - run[t].
// perm_e / perm_k receive (candidate, list offset) for the kept ones; returns
// how many.  run[] advances by the window's counts.
__device__ inline int place_window(unsigned in, unsigned tb, int n, int n_types, int lane, int (&run)[MAX_TYPES],
                                   const int (&cap)[MAX_TYPES], const int (&base)[MAX_TYPES], short *perm_e,
                                   int *perm_k) {
    const unsigned long long below = (1ull << lane) - 1ull;
    int kept = 0;
    for (int cc = 0; cc * 64 < n; ++cc) {
        const bool a = (in >> cc) & 1u;
        const int t = (tb >> (2 * cc)) & 3;
#pragma unroll
        for (int s = 0; s < MAX_TYPES; ++s) {
            if (s >= n_types) continue;
            const unsigned long long mk = __ballot(a && t == s);
            const int k = run[s] + __popcll(mk & below);
            const bool keep = a && t == s && k < cap[s];
            const unsigned long long km = __ballot(keep);
            if (keep) {
                const int slot = kept + __popcll(km & below);
                perm_e[slot] = (short)(cc * 64 + lane);
                perm_k[slot] = base[s] + k;
            }
            kept += __popcll(km);
            run[s] += __popcll(mk);
        }
    }
    return kept;
}

// consecutive lanes write consecutive kept pairs (multi-window path: the
// opposite bin offset is not recorded, 0xff)
__device__ inline void write_kept(const Window &W, const short *perm_e, const int *perm_k, int kept,
                                  const Centre &c, int lane, int max_nbrs, double *rout, int32_t *jout,
                                  int32_t *shout, Flags &fl) {
    for (int a = lane; a < kept; a += 64) {
        const int e = perm_e[a];
        const int64_t slot = (int64_t)c.i * max_nbrs + perm_k[a];
        const int qt = W.qt[e], jq = W.jq[e];
        const int sh0 = field(qt, 0) + c.w0, sh1 = field(qt, 1) + c.w1, sh2 = field(qt, 2) + c.w2;
        const int o = W.lo[e];
        rout[3 * slot] = (W.x[e] - c.y0) + W.qh[o][0];
        rout[3 * slot + 1] = (W.y[e] - c.y1) + W.qh[o][1];
        rout[3 * slot + 2] = (W.z[e] - c.y2) + W.qh[o][2];
        jout[slot] = jq >= 0 ? jq : ~jq;
        if (sh0 < -127 || sh0 > 127 || sh1 < -127 || sh1 > 127 || sh2 < -127 || sh2 > 127) fl.wide = true;
        shout[slot] = (sh0 & 0xff) | ((sh1 & 0xff) << 8) | ((sh2 & 0xff) << 16) | (0xff << 24);
    }
}

// consecutive lanes write list slots 0 .. tot - 1 from perm
__device__ inline void write_direct(const Window &W, const short *perm, int tot, const Centre &c, int lane,
                                    int max_nbrs, int n_off, double *rout, int32_t *jout, int32_t *shout,
                                    Flags &fl) {
    for (int a = lane; a < tot; a += 64) {
        const int e = perm[a];
        const int64_t slot = (int64_t)c.i * max_nbrs + a;
        const int qt = W.qt[e], jq = W.jq[e];
        const int sh0 = field(qt, 0) + c.w0, sh1 = field(qt, 1) + c.w1, sh2 = field(qt, 2) + c.w2;
        const int o = W.lo[e];
        rout[3 * slot] = (W.x[e] - c.y0) + W.qh[o][0];
        rout[3 * slot + 1] = (W.y[e] - c.y1) + W.qh[o][1];
        rout[3 * slot + 2] = (W.z[e] - c.y2) + W.qh[o][2];
        jout[slot] = jq >= 0 ? jq : ~jq;
        if (sh0 < -127 || sh0 > 127 || sh1 < -127 || sh1 > 127 || sh2 < -127 || sh2 > 127) fl.wide = true;
        // top byte: the opposite bin offset (from j's bin to i's), for the reverse-pair search
        shout[slot] = (sh0 & 0xff) | ((sh1 & 0xff) << 8) | ((sh2 & 0xff) << 16) | ((n_off - 1 - o) << 24);
    }
}

// Per-species slots of one neighborhood: counts -> capacities (clamped to
// max_nbrs in species order) and list offsets.
__device__ inline void list_layout(const int (&cnt)[MAX_TYPES], int n_types, int max_nbrs, int (&cap)[MAX_TYPES],
                                   int (&base)[MAX_TYPES], int &tot) {
    int off = 0;
    tot = 0;
#pragma unroll
    for (int t = 0; t < MAX_TYPES; ++t) {
        cap[t] = 0;
        base[t] = off;
        if (t < n_types) {
            tot += cnt[t];
            const int room = max_nbrs - off;
            cap[t] = cnt[t] < room ? cnt[t] : room;
            off += cap[t];
        }
    }
}

__device__ inline int from_lane(int v, int k) { return __shfl(v, k, 64); }

// WIDE = false: every bin whose candidates fit one window; the others are
// appended to wide_list (count in flags[5]) for the WIDE = true launch.
template <bool WIDE, int NT>
__global__ __launch_bounds__(256) void pair_search(const int32_t *nbins_dev, int n_cfg, int n_types_arg, int max_nbrs,
                                                   double d2max, const CfgGeo *geo, Staged S, BinStart bin_start,
                                                   const int32_t *bin_count, int32_t *tcnt, double *rout,
                                                   int32_t *jout, int32_t *shout, int32_t *flags,
                                                   int32_t *wide_list, uint16_t *pre_out) {
    __shared__ Window W;
    __shared__ short perm_e[4][PS_WIN];
    __shared__ int perm_k[4][PS_WIN];
    __shared__ int s_max[4], s_bits[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int n_types = NT;   // species loops unroll to the actual count
    (void)n_types_arg;
    const int64_t nbins = WIDE ? flags[5] : *nbins_dev;
    Flags fl;
    int max_tot = 0;
    for (int64_t it = blockIdx.x; it < nbins; it += gridDim.x) {   // block-uniform
        const int64_t bin = WIDE ? wide_list[it] : it;
        const int my_cnt = bin_count[bin];
        if (my_cnt == 0) continue;
        int lo = 0, hi = n_cfg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (geo[mid].bin_off <= bin) lo = mid; else hi = mid - 1;
        }
        const CfgGeo &g = geo[lo];
        double H[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) H[k] = g.H[k];
        const int local = (int)(bin - g.bin_off);
        const int bx = local % g.n[0], by = (local / g.n[0]) % g.n[1], bz = local / (g.n[0] * g.n[1]);
        const int n_off = (2 * g.s[0] + 1) * (2 * g.s[1] + 1) * (2 * g.s[2] + 1);
        const int my_start = bin_start[bin];
        const Around A0 = around_bin(g, bx, by, bz, lane, n_off, lane, bin_start, bin_count);
        const bool one_window = n_off <= 64 && A0.total <= PS_WIN;
        if (!WIDE && !one_window) {
            if (threadIdx.x == 0) wide_list[atomicAdd(&flags[5], 1)] = (int32_t)bin;
            continue;
        }
        if (one_window) {
            __syncthreads();   // the previous bin's window is no longer read
            stage_window(W, A0, 0, wave, lane, H, S);
            __syncthreads();
        }
        for (int a_base = 0; a_base < my_cnt; a_base += 256) {   // block-uniform
            // lane k of wave w holds atom a_base + w + 4 k of the bin
            const int ak = a_base + wave + 4 * lane;
            int hold_i = 0, hold_w = pack_q(0, 0, 0);
            double hold_x = 0.0, hold_y = 0.0, hold_z = 0.0;
            if (ak < my_cnt) {
                const int64_t u = (int64_t)my_start + ak;
                hold_i = S.bin_atoms[u];
                hold_w = S.sw[u];
                hold_x = S.sx[3 * u];
                hold_y = S.sx[3 * u + 1];
                hold_z = S.sx[3 * u + 2];
            }
            const int left = (my_cnt - a_base - wave + 3) / 4;
            const int na = left < 0 ? 0 : (left < 64 ? left : 64);
            auto centre = [&](int k) {
                Centre c;
                c.i = from_lane(hold_i, k);
                const int nw = from_lane(hold_w, k);
                c.w0 = -field(nw, 0);
                c.w1 = -field(nw, 1);
                c.w2 = -field(nw, 2);
                c.y0 = __shfl(hold_x, k, 64);
                c.y1 = __shfl(hold_y, k, 64);
                c.y2 = __shfl(hold_z, k, 64);
                return c;
            };
            if (!WIDE) {
                for (int k = 0; k < na; ++k) {
                    const Centre c = centre(k);
                    unsigned tb;
                    int cnt[MAX_TYPES] = {0, 0, 0, 0}, cap[MAX_TYPES], base[MAX_TYPES];
                    const unsigned in = test_count<NT>(W, A0.total, c, lane, d2max, tb, cnt, fl);
                    int tot;
                    list_layout(cnt, n_types, max_nbrs, cap, base, tot);
                    int pre[MAX_TYPES] = {0, 0, 0, 0};
                    place_chunks<NT>(in, tb, A0.total, lane, cap, base, perm_e[wave], A0.excl, pre);
                    const int kept = tot < max_nbrs ? tot : max_nbrs;
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    // lane o: where the run of bin offset o starts in each species group
#pragma unroll
                    for (int t = 0; t < n_types; ++t)
                        pre_out[((int64_t)c.i * n_types + t) * 64 + lane] = (uint16_t)pre[t];
                    write_direct(W, perm_e[wave], kept, c, lane, max_nbrs, n_off, rout, jout, shout, fl);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    max_tot = tot > max_tot ? tot : max_tot;
                    if (lane < n_types) {
                        int v = 0;
#pragma unroll
                        for (int t = 0; t < MAX_TYPES; ++t)
                            if (t == lane) v = cap[t];
                        tcnt[(int64_t)c.i * n_types + lane] = v;
                    }
                }
            } else {
                // per held atom (lane k): counts, then capacities / offsets / placed so far
                int hc[MAX_TYPES] = {0, 0, 0, 0}, hcap[MAX_TYPES] = {0, 0, 0, 0}, hbase[MAX_TYPES] = {0, 0, 0, 0},
                    hrun[MAX_TYPES] = {0, 0, 0, 0};
                for (int pass = 0; pass < 2; ++pass) {
                    if (pass == 1) {
                        int tot;
                        list_layout(hc, n_types, max_nbrs, hcap, hbase, tot);
                        if (lane < na) max_tot = tot > max_tot ? tot : max_tot;
                    }
                    for (int og = 0; og < n_off; og += 64) {
                        const Around A = around_bin(g, bx, by, bz, og + lane, n_off, lane, bin_start, bin_count);
                        for (int w0 = 0; w0 < A.total; w0 += PS_WIN) {
                            const int n = A.total - w0 < PS_WIN ? A.total - w0 : PS_WIN;
                            __syncthreads();
                            stage_window(W, A, w0, wave, lane, H, S);
                            __syncthreads();
                            for (int k = 0; k < na; ++k) {
                                const Centre c = centre(k);
                                unsigned tb;
                                const unsigned in = test_window(W, n, c, lane, d2max, tb, fl);
                                int cnt[MAX_TYPES] = {0, 0, 0, 0};
                                count_window(in, tb, n, n_types, cnt);
                                if (pass == 0) {
                                    if (lane == k)
                                        for (int t = 0; t < MAX_TYPES; ++t) hc[t] += cnt[t];
                                    continue;
                                }
                                int run[MAX_TYPES], cap[MAX_TYPES], base[MAX_TYPES];
#pragma unroll
                                for (int t = 0; t < MAX_TYPES; ++t) {
                                    run[t] = from_lane(hrun[t], k);
                                    cap[t] = from_lane(hcap[t], k);
                                    base[t] = from_lane(hbase[t], k);
                                }
                                const int kept = place_window(in, tb, n, n_types, lane, run, cap, base, perm_e[wave],
                                                              perm_k[wave]);
                                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                                __builtin_amdgcn_wave_barrier();
                                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                                write_kept(W, perm_e[wave], perm_k[wave], kept, c, lane, max_nbrs, rout, jout, shout,
                                           fl);
                                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                                __builtin_amdgcn_wave_barrier();
                                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                                if (lane == k)
                                    for (int t = 0; t < MAX_TYPES; ++t) hrun[t] = run[t];
                            }
                        }
                    }
                }
                if (lane < na)
                    for (int t = 0; t < n_types; ++t) tcnt[(int64_t)hold_i * n_types + t] = hcap[t];
                for (int k = 0; k < na; ++k)   // no offset table for these atoms
                    for (int t = 0; t < n_types; ++t)
                        pre_out[((int64_t)from_lane(hold_i, k) * n_types + t) * 64 + lane] = (uint16_t)0xffff;
            }
        }
    }
    // Status words: one atomic per block (same-address atomics from every
    // atom would serialise in L2), and only when the stored value changes.
    const int bits = (__ballot(fl.overlap) ? 1 : 0) | (__ballot(fl.wide) ? 2 : 0);
    int wmax = max_tot;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) wmax = max(wmax, __shfl_xor(wmax, d, 64));
    if (lane == 0) {
        s_max[wave] = wmax;
        s_bits[wave] = bits;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int mt = max(max(s_max[0], s_max[1]), max(s_max[2], s_max[3]));
        const int b = s_bits[0] | s_bits[1] | s_bits[2] | s_bits[3];
        if (mt > max_nbrs) atomicOr(&flags[0], 1);
        if (mt > __hip_atomic_load(&flags[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(&flags[1], mt);
        if (b & 1) atomicOr(&flags[2], 1);
        if (b & 2) atomicOr(&flags[3], 2);
    }
}

__device__ inline int sx8(int v) { return (int)(signed char)(v & 0xff); }

// One thread per list slot: find the slot of (j, i, -n) in j's list.  The
// top byte of a slot's shift word is the index of the opposite bin offset
// (from j's bin to i's); j's offset table gives where that offset's run
// starts in j's species-z_i group, so only the run (ascending atom index) is
// scanned.  Without a table entry the whole group is scanned.
__global__ __launch_bounds__(256) void reverse_pairs(int64_t n, int n_types, int max_nbrs, const int32_t *type, const int32_t *tcnt,
                              const int32_t *jl, const int32_t *sh, const uint16_t *pre, int32_t *rev,
                              int32_t *flags) {
    const int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x;   // blocks of 256 threads
    if (slot >= n * max_nbrs) return;
    const int64_t i = slot / max_nbrs;
    const int p = (int)(slot % max_nbrs);
    // Each level of dependent loads is issued at once: the slot's own entry,
    // i's species and counts (the entry is stale and unused past the count) ...
    const int j = jl[slot];
    const int s = sh[slot];
    const int zi = type[i];
    int tot = 0;
#pragma unroll
    for (int t = 0; t < MAX_TYPES; ++t) tot += t < n_types ? tcnt[i * n_types + t] : 0;
    __asm__ volatile("" ::"v"(j), "v"(s), "v"(zi));   // keeps the loads above the branch
    if (p >= tot) return;
    if (zi < 0 || zi >= n_types) {   // flagged when the atom was staged; the slot names itself (in bounds)
        rev[slot] = (int)slot;
        return;
    }
    const int want = ((-sx8(s)) & 0xff) | ((-sx8(s >> 8)) & 0xff) << 8 | ((-sx8(s >> 16)) & 0xff) << 16;
    const int orev = (s >> 24) & 0xff;
    // ... then j's counts and both offset-table entries of the opposite bin offset ...
    int start = 0, cnt = 0;
#pragma unroll
    for (int t = 0; t < MAX_TYPES; ++t) {
        const int c = t < n_types ? tcnt[(int64_t)j * n_types + t] : 0;
        if (t < zi) start += c;
        if (t == zi) cnt = c;
    }
    const uint16_t *pj = pre + ((int64_t)j * n_types + zi) * 64;
    const int oa = orev != 0xff ? orev : 0;
    const int a = pj[oa], b = pj[oa + 1 < 64 ? oa + 1 : 63];
    int lo = 0, hi = cnt;
    if (orev != 0xff && a != 0xffff) {   // without a table entry the whole group is scanned
        lo = a < cnt ? a : cnt;
        if (orev + 1 < 64) hi = b < cnt ? b : cnt;
    }
    // ... then the run (usually one to three entries), both words of an entry together
    int found = -1;
    for (int q = start + lo; q < start + hi; ++q) {
        const int64_t s2 = (int64_t)j * max_nbrs + q;
        const int j2 = jl[s2], sh2 = sh[s2];
        if ((j2 == (int)i) & ((sh2 & 0xffffff) == want)) {
            found = (int)s2;
            break;
        }
    }
    if (found < 0) {
        atomicOr(&flags[3], 4);
        found = (int)slot;   // keeps the gather in bounds; the status call reports the fault
    }
    rev[slot] = found;
}

}  // namespace

void build_neighbors(const mtp_model *m, const mtp_system *s, int max_nbrs, mtp_nbrs *nb, hipStream_t st) {
    const int64_t n = s->n_atoms;
    const int nt = m->n_types;
    nb->device = m->device;
    nb->n_atoms = n;
    nb->n_cfg = s->n_cfg;
    nb->max_nbrs = max_nbrs;
    nb->n_types = nt;
    nb->r_cut = m->r_cut;
    const int64_t P = n * max_nbrs;
    nb->r.ensure(sizeof(double) * 3 * (P > 0 ? P : 1));
    nb->j.ensure(sizeof(int32_t) * (P > 0 ? P : 1));
    nb->shift.ensure(sizeof(int32_t) * (P > 0 ? P : 1));
    nb->rev.ensure(sizeof(int32_t) * (P > 0 ? P : 1));
    nb->tcnt.ensure(sizeof(int32_t) * (n * nt > 0 ? n * nt : 1));
    nb->atom_cfg.ensure(sizeof(int32_t) * (n > 0 ? n : 1));
    nb->atom_bin.ensure(sizeof(int32_t) * (n > 0 ? n : 1));
    nb->atom_wrap.ensure(sizeof(int32_t) * 3 * (n > 0 ? n : 1));
    nb->cfg_geo.ensure(sizeof(CfgGeo) * s->n_cfg);
    const int64_t bins = n + s->n_cfg;   // upper bound: each configuration has at most max(1, N_c) bins
    nb->bin_count.ensure(sizeof(int32_t) * bins);
    nb->bin_start.ensure(sizeof(int32_t) * bins);
    nb->bin_cursor.ensure(sizeof(int32_t) * bins);
    nb->bin_atoms.ensure(sizeof(int32_t) * (n > 0 ? n : 1));
    nb->stage_x.ensure(sizeof(double) * 3 * (n > 0 ? n : 1));
    nb->stage_w.ensure(sizeof(int32_t) * (n > 0 ? n : 1));
    nb->stage_t.ensure(sizeof(int32_t) * (n > 0 ? n : 1));
    nb->pre.ensure(sizeof(uint16_t) * 64 * (n * nt > 0 ? n * nt : 1));
    nb->flags.ensure(sizeof(int32_t) * 8);
    nb->bins_cap = bins;
    auto *geo = nb->cfg_geo.as<CfgGeo>();
    int32_t *flags = nb->flags.as<int32_t>();
    const int TB = 256;
    hipLaunchKernelGGL(nbr_prepare, dim3((unsigned)std::min<int64_t>((bins + TB - 1) / TB, 1024)), dim3(TB), 0, st,
                       s->n_cfg, s->cfg_off, s->cell, s->pbc, m->r_cut, geo, flags, nb->bin_count.as<int32_t>(),
                       nb->bin_cursor.as<int32_t>(), bins);
    if (n == 0) return;
    const dim3 ga((unsigned)((n + TB - 1) / TB));
    hipLaunchKernelGGL(bin_kernel, ga, dim3(TB), 0, st, n, s->n_cfg, s->cfg_off, s->pos, geo,
                       nb->atom_cfg.as<int32_t>(), nb->atom_bin.as<int32_t>(), nb->atom_wrap.as<int32_t>(),
                       nb->bin_count.as<int32_t>(), flags);
    hipLaunchKernelGGL(scan_bins, dim3(1), dim3(SCAN_T), 0, st, nb->bin_count.as<int32_t>(),
                       nb->bin_start.as<int32_t>(), flags + 4);
    const BinStart bstart{nb->bin_start.as<int32_t>()};
    hipLaunchKernelGGL(fill_bins, ga, dim3(TB), 0, st, n, nb->atom_bin.as<int32_t>(), bstart,
                       nb->bin_cursor.as<int32_t>(), nb->bin_atoms.as<int32_t>());
    Stage sg{s->pos, s->type, nb->atom_cfg.as<int32_t>(), nb->atom_wrap.as<int32_t>(), geo, nt,
             nb->stage_x.as<double>(), nb->stage_w.as<int32_t>(), nb->stage_t.as<int32_t>()};
    const unsigned gbins = (unsigned)std::min<int64_t>((bins + 3) / 4, 2048);
    hipLaunchKernelGGL(sort_bins, dim3(gbins), dim3(256), 0, st, flags, bstart,
                       nb->bin_count.as<int32_t>(), nb->bin_atoms.as<int32_t>(), sg);
    // largest d2 with sqrt(d2) < R_cut (IEEE square roots are correctly rounded, host and device alike)
    double d2max = m->r_cut * m->r_cut;
    while (d2max > 0 && std::sqrt(d2max) >= m->r_cut) d2max = std::nextafter(d2max, 0.0);
    while (std::sqrt(std::nextafter(d2max, INFINITY)) < m->r_cut) d2max = std::nextafter(d2max, INFINITY);
    // bin_cursor is free after fill_bins: it holds the list of bins for the WIDE launch
    const Staged staged{nb->stage_x.as<double>(), nb->stage_w.as<int32_t>(), nb->stage_t.as<int32_t>(),
                        nb->bin_atoms.as<int32_t>()};
    auto search = [&](auto wide, auto ntc) {
        constexpr bool W = decltype(wide)::value;
        constexpr int NTC = decltype(ntc)::value;
        hipLaunchKernelGGL((pair_search<W, NTC>), dim3((unsigned)std::min<int64_t>(bins, 2048)), dim3(256), 0, st,
                           flags + 4, s->n_cfg, nt, max_nbrs, d2max, geo, staged, bstart,
                           nb->bin_count.as<int32_t>(), nb->tcnt.as<int32_t>(), nb->r.as<double>(),
                           nb->j.as<int32_t>(), nb->shift.as<int32_t>(), flags, nb->bin_cursor.as<int32_t>(),
                           nb->pre.as<uint16_t>());
    };
    auto both = [&](auto ntc) {
        search(std::false_type{}, ntc);
        search(std::true_type{}, ntc);
    };
    switch (nt) {
        case 1: both(std::integral_constant<int, 1>{}); break;
        case 2: both(std::integral_constant<int, 2>{}); break;
        case 3: both(std::integral_constant<int, 3>{}); break;
        default: both(std::integral_constant<int, 4>{}); break;
    }
    hipLaunchKernelGGL(reverse_pairs, dim3((unsigned)((P + TB - 1) / TB)), dim3(TB), 0, st, n, nt, max_nbrs, s->type,
                       nb->tcnt.as<int32_t>(), nb->j.as<int32_t>(), nb->shift.as<int32_t>(), nb->pre.as<uint16_t>(),
                       nb->rev.as<int32_t>(), flags);
    MTP_HIP(hipGetLastError());
}

}  // namespace mtp
