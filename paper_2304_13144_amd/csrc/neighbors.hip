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
// a counting pass and a filling pass over the 27 (or more) nearby bins,
// grouped by neighbor species -> reverse-pair index for the atomic-free
// force gather.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// one thread walks all configurations (bin offsets are a running sum)
__global__ void geo_kernel(int n_cfg, const int64_t *cfg_off, const double *cell, const uint8_t *pbc, double rc,
                           CfgGeo *geo, int *flags) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
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

__global__ void bin_kernel(int64_t n, int n_cfg, const int64_t *cfg_off, const double *pos, const CfgGeo *geo,
                           int32_t *atom_cfg, int32_t *atom_bin, int32_t *atom_wrap, int32_t *bin_count) {
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

// exclusive scan, three kernels (block scan, scan of block sums, add)
constexpr int SCAN_B = 1024;

__global__ void scan_block(const int32_t *in, int32_t *out, int32_t *sums, const int32_t *n_dev) {
    __shared__ int32_t s[SCAN_B];
    const int64_t n = *n_dev;
    const int64_t i = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
    int32_t v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 1; d < SCAN_B; d <<= 1) {
        int32_t t = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = s[threadIdx.x] - v;
    if (threadIdx.x == SCAN_B - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void scan_sums(int32_t *sums, int64_t nb) {
    // single block; sequential carry over chunks of SCAN_B
    __shared__ int32_t s[SCAN_B];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += SCAN_B) {
        const int64_t i = base + threadIdx.x;
        int32_t v = i < nb ? sums[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < SCAN_B; d <<= 1) {
            int32_t t = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
            __syncthreads();
            s[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == SCAN_B - 1) carry += s[threadIdx.x];
        __syncthreads();
    }
}

__global__ void scan_add(int32_t *out, const int32_t *sums, const int32_t *n_dev, int32_t *copy) {
    const int64_t n = *n_dev;
    const int64_t i = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
    if (i < n) {
        const int32_t v = out[i] + sums[blockIdx.x];
        out[i] = v;
        copy[i] = v;
    }
}

__global__ void fill_bins(int64_t n, const int32_t *atom_bin, int32_t *cursor, int32_t *bin_atoms) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int slot = atomicAdd(&cursor[atom_bin[i]], 1);
    bin_atoms[slot] = (int32_t)i;
}

// One wavefront per bin: the bin's atoms (filled in arbitrary order by
// atomics) are put in ascending index order, which makes every later step
// deterministic.  Ranks come from all-pairs comparisons across the lanes.
__device__ inline void sort_one_bin(int32_t *a, int c, int lane) {
    if (c <= 1) return;
    if (c <= 64) {
        const int v = lane < c ? a[lane] : 0x7fffffff;
        int rank = 0;
        for (int k = 0; k < c; ++k) rank += __shfl(v, k, 64) < v ? 1 : 0;
        if (lane < c) a[rank] = v;
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
    }
}

__global__ __launch_bounds__(256) void sort_bins(const int32_t *flags, const int32_t *start, const int32_t *count,
                                                 int32_t *bin_atoms) {
    const int lane = threadIdx.x & 63;
    const int64_t nbins = flags[4];
    for (int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); b < nbins; b += (int64_t)gridDim.x * 4)
        sort_one_bin(bin_atoms + start[b], count[b], lane);
}

__device__ inline int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// One block per bin.  The atoms of the bins around it (all periodic images
// that can hold a neighbor) are staged in LDS in chunks, each as its image
// position x_j + (q - w_j).H, so that r_ij = staged + w_i.H - x_i.  Each
// wavefront then tests one of the bin's atoms against the chunk, 64
// candidates at a time; ballots per neighbor species give every accepted pair
// its slot, so the order (bin offset, then atom index in the bin) is
// deterministic.  Pass 0 counts per species, pass 1 writes the lists
// (clamped to max_nbrs).
constexpr int BS_T = 256, BS_CAP = 1024, BS_ATOMS = 64;

__device__ inline int pack_q(int x, int y, int z) { return (x + 512) | ((y + 512) << 10) | ((z + 512) << 20); }

__global__ __launch_bounds__(BS_T) void bin_search(const int32_t *nbins_dev, int n_cfg, int n_types, int max_nbrs, double rc,
                                                   const double *pos, const int32_t *type, const CfgGeo *geo,
                                                   const int32_t *atom_wrap, const int32_t *bin_start,
                                                   const int32_t *bin_count, const int32_t *bin_atoms, int32_t *tcnt,
                                                   double *rout, int32_t *jout, int32_t *shout, int32_t *flags) {
    __shared__ double cx[BS_CAP], cy[BS_CAP], cz[BS_CAP];
    __shared__ int cj[BS_CAP], cs[BS_CAP], ct[BS_CAP];
    __shared__ int o_start[BS_T], o_pre[BS_T + 1], o_q[BS_T];
    __shared__ int a_cnt[BS_ATOMS][MAX_TYPES], a_base[BS_ATOMS][MAX_TYPES], a_cap[BS_ATOMS][MAX_TYPES];
    __shared__ int a_idx[BS_ATOMS], a_w[BS_ATOMS][3];
    __shared__ double a_off[BS_ATOMS][3];   // w_i.H - x_i of the bin's atoms
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    bool overlap = false, wide = false, bad_type = false;
    const int64_t nbins = *nbins_dev;
    for (int64_t bin = blockIdx.x; bin < nbins; bin += gridDim.x) {
    const int my_cnt = bin_count[bin];
    if (my_cnt == 0) continue;   // uniform per block
    int lo = 0, hi = n_cfg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (geo[mid].bin_off <= bin) lo = mid; else hi = mid - 1;
    }
    const CfgGeo g = geo[lo];
    const int local = (int)(bin - g.bin_off);
    const int bx = local % g.n[0], by = (local / g.n[0]) % g.n[1], bz = local / (g.n[0] * g.n[1]);
    const int ox = 2 * g.s[0] + 1, oy = 2 * g.s[1] + 1, oz = 2 * g.s[2] + 1;
    const int n_off = ox * oy * oz;
    const int my_start = bin_start[bin];
    for (int a0 = 0; a0 < my_cnt; a0 += BS_ATOMS) {
        const int na = my_cnt - a0 < BS_ATOMS ? my_cnt - a0 : BS_ATOMS;
        for (int aa = tid; aa < na; aa += BS_T) {
            const int i = bin_atoms[my_start + a0 + aa];
            const int w0 = atom_wrap[3 * i], w1 = atom_wrap[3 * i + 1], w2 = atom_wrap[3 * i + 2];
            a_idx[aa] = i;
            a_w[aa][0] = w0;
            a_w[aa][1] = w1;
            a_w[aa][2] = w2;
            a_off[aa][0] = w0 * g.H[0] + w1 * g.H[3] + w2 * g.H[6] - pos[3 * i];
            a_off[aa][1] = w0 * g.H[1] + w1 * g.H[4] + w2 * g.H[7] - pos[3 * i + 1];
            a_off[aa][2] = w0 * g.H[2] + w1 * g.H[5] + w2 * g.H[8] - pos[3 * i + 2];
        }
        for (int pass = 0; pass < 2; ++pass) {
            if (pass == 0) {
                for (int k = tid; k < BS_ATOMS * MAX_TYPES; k += BS_T) a_cnt[k / MAX_TYPES][k % MAX_TYPES] = 0;
            } else {
                for (int aa = tid; aa < na; aa += BS_T) {
                    int off = 0, tot = 0;
                    for (int t = 0; t < n_types; ++t) {
                        const int c = a_cnt[aa][t];
                        tot += c;
                        const int room = max_nbrs - off;
                        a_cap[aa][t] = c < room ? c : room;
                        a_base[aa][t] = off;
                        off += a_cap[aa][t];
                        a_cnt[aa][t] = 0;
                    }
                    if (tot > max_nbrs) atomicOr(&flags[0], 1);
                    atomicMax(&flags[1], tot);
                }
            }
            __syncthreads();
            // the staged chunk of pass 0 is still in LDS when it held every candidate
            const bool reuse = pass == 1 && n_off <= BS_T && o_pre[BS_T] <= BS_CAP;
            for (int og = 0; og < n_off; og += BS_T) {
                if (!reuse) {
                    const int o = og + tid;
                    int start = 0, c = 0, qp = pack_q(0, 0, 0);
                    if (o < n_off) {
                        const int dx = o % ox - g.s[0], dy = (o / ox) % oy - g.s[1], dz = o / (ox * oy) - g.s[2];
                        int ux = bx + dx, uy = by + dy, uz = bz + dz, qx = 0, qy = 0, qz = 0;
                        bool ok = true;
                        if (g.pbc[0]) { qx = floordiv(ux, g.n[0]); ux -= qx * g.n[0]; } else ok = ok && ux >= 0 && ux < g.n[0];
                        if (g.pbc[1]) { qy = floordiv(uy, g.n[1]); uy -= qy * g.n[1]; } else ok = ok && uy >= 0 && uy < g.n[1];
                        if (g.pbc[2]) { qz = floordiv(uz, g.n[2]); uz -= qz * g.n[2]; } else ok = ok && uz >= 0 && uz < g.n[2];
                        if (ok) {
                            const long long nb = g.bin_off + ((long long)uz * g.n[1] + uy) * g.n[0] + ux;
                            start = bin_start[nb];
                            c = bin_count[nb];
                            qp = pack_q(qx, qy, qz);
                        }
                    }
                    o_start[tid] = start;
                    o_q[tid] = qp;
                    o_pre[tid + 1] = c;
                    if (tid == 0) o_pre[0] = 0;
                    __syncthreads();
                    for (int d = 1; d < BS_T; d <<= 1) {   // inclusive scan of o_pre[1..BS_T]
                        const int t = tid >= d ? o_pre[tid + 1 - d] : 0;
                        __syncthreads();
                        o_pre[tid + 1] += t;
                        __syncthreads();
                    }
                }
                const int total = o_pre[BS_T];
                for (int v0 = 0; v0 < total; v0 += BS_CAP) {
                    const int nchunk = total - v0 < BS_CAP ? total - v0 : BS_CAP;
                    for (int v = v0 + tid; !reuse && v < v0 + nchunk; v += BS_T) {
                        int L = 0;
                        for (int step = BS_T / 2; step >= 1; step >>= 1)
                            if (o_pre[L + step] <= v) L += step;
                        const int j = bin_atoms[o_start[L] + v - o_pre[L]];
                        const int q = o_q[L];
                        const int sx = ((q & 1023) - 512) - atom_wrap[3 * j];
                        const int sy = (((q >> 10) & 1023) - 512) - atom_wrap[3 * j + 1];
                        const int sz = (((q >> 20) & 1023) - 512) - atom_wrap[3 * j + 2];
                        const int e = v - v0;
                        cx[e] = pos[3 * j] + sx * g.H[0] + sy * g.H[3] + sz * g.H[6];
                        cy[e] = pos[3 * j + 1] + sx * g.H[1] + sy * g.H[4] + sz * g.H[7];
                        cz[e] = pos[3 * j + 2] + sx * g.H[2] + sy * g.H[5] + sz * g.H[8];
                        cj[e] = j;
                        cs[e] = pack_q(sx, sy, sz);
                        const int t = type[j];
                        ct[e] = (t < 0 || t >= n_types) ? -1 : t;
                    }
                    __syncthreads();
                    for (int aa = wave; aa < na; aa += BS_T / 64) {
                        const int i = a_idx[aa];
                        const int wi0 = a_w[aa][0], wi1 = a_w[aa][1], wi2 = a_w[aa][2];
                        // r_ij = staged + w_i.H - x_i
                        const double bx0 = a_off[aa][0], bx1 = a_off[aa][1], bx2 = a_off[aa][2];
                        int cnt_t[MAX_TYPES], cap_t[MAX_TYPES], base_t[MAX_TYPES];
#pragma unroll
                        for (int t = 0; t < MAX_TYPES; ++t) {
                            cnt_t[t] = a_cnt[aa][t];
                            cap_t[t] = pass ? a_cap[aa][t] : 0;
                            base_t[t] = pass ? a_base[aa][t] : 0;
                        }
                        for (int e0 = 0; e0 < nchunk; e0 += 64) {
                            const int e = e0 + lane;
                            bool ok = false;
                            int t = -1, sh0 = 0, sh1 = 0, sh2 = 0, j = 0;
                            double r0 = 0.0, r1 = 0.0, r2 = 0.0;
                            if (e < nchunk) {
                                j = cj[e];
                                const int q = cs[e];
                                sh0 = ((q & 1023) - 512) + wi0;
                                sh1 = (((q >> 10) & 1023) - 512) + wi1;
                                sh2 = (((q >> 20) & 1023) - 512) + wi2;
                                if (!(j == i && sh0 == 0 && sh1 == 0 && sh2 == 0)) {
                                    r0 = cx[e] + bx0;
                                    r1 = cy[e] + bx1;
                                    r2 = cz[e] + bx2;
                                    const double d = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
                                    if (d < rc) {
                                        t = ct[e];
                                        if (t < 0) {
                                            bad_type = true;
                                        } else {
                                            ok = true;
                                            if (d < 1e-6) overlap = true;
                                        }
                                    }
                                }
                            }
                            for (int tt = 0; tt < n_types; ++tt) {
                                const bool mine = ok && t == tt;
                                const unsigned long long mk = __ballot(mine);
                                if (pass == 1 && mine) {
                                    const int slot_in = cnt_t[tt] + __popcll(mk & ((1ull << lane) - 1ull));
                                    if (slot_in < cap_t[tt]) {
                                        const int64_t slot = (int64_t)i * max_nbrs + base_t[tt] + slot_in;
                                        rout[3 * slot] = r0;
                                        rout[3 * slot + 1] = r1;
                                        rout[3 * slot + 2] = r2;
                                        jout[slot] = j;
                                        if (sh0 < -127 || sh0 > 127 || sh1 < -127 || sh1 > 127 || sh2 < -127 ||
                                            sh2 > 127)
                                            wide = true;
                                        shout[slot] = (sh0 & 0xff) | ((sh1 & 0xff) << 8) | ((sh2 & 0xff) << 16);
                                    }
                                }
                                cnt_t[tt] += __popcll(mk);
                            }
                        }
                        if (lane == 0)
                            for (int t = 0; t < MAX_TYPES; ++t) a_cnt[aa][t] = cnt_t[t];
                    }
                    __syncthreads();
                }
            }
            __syncthreads();
        }
        for (int aa = tid; aa < na; aa += BS_T) {
            const int i = a_idx[aa];
            for (int t = 0; t < n_types; ++t) tcnt[(int64_t)i * n_types + t] = a_cap[aa][t];
        }
        __syncthreads();
    }
    }
    if (overlap) atomicOr(&flags[2], 1);
    if (wide) atomicOr(&flags[3], 2);
    if (bad_type) atomicOr(&flags[3], 8);
}

// One wavefront per bin, no block barriers.  Lanes take the surrounding bins
// (64 at a time) and a wave-wide prefix sum numbers their atoms; windows of
// up to 64 x SW_C candidates are held in registers, as their image
// positions x_j + (q - w_j).H.  The bin's atoms are then visited one after
// the other (their data broadcast from the lane that holds it) and tested
// against every candidate of the window; ballots per neighbor species give
// each accepted pair its slot.  Order: bin offset, then atom index in the
// bin -- deterministic.  Pass 0 counts per species, pass 1 writes (clamped
// to max_nbrs).
constexpr int SW_C = 8;

__global__ __launch_bounds__(256) void bin_search_wave(const int32_t *nbins_dev, int n_cfg, int n_types,
                                                        int max_nbrs, double rc, const double *pos,
                                                        const int32_t *type, const CfgGeo *geo,
                                                        const int32_t *atom_wrap, const int32_t *bin_start,
                                                        const int32_t *bin_count, const int32_t *bin_atoms,
                                                        int32_t *tcnt, double *rout, int32_t *jout, int32_t *shout,
                                                        int32_t *flags) {
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t nbins = *nbins_dev;
    bool overlap = false, wide = false, bad_type = false;
    for (int64_t bin = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); bin < nbins; bin += (int64_t)gridDim.x * 4) {
        const int my_cnt = bin_count[bin];
        if (my_cnt == 0) continue;   // uniform per wavefront
        int lo = 0, hi = n_cfg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (geo[mid].bin_off <= bin) lo = mid; else hi = mid - 1;
        }
        const CfgGeo &g = geo[lo];
        double H[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) H[k] = g.H[k];
        const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
        const int s0 = g.s[0], s1 = g.s[1], s2 = g.s[2];
        const int p0 = g.pbc[0], p1 = g.pbc[1], p2 = g.pbc[2];
        const long long boff = g.bin_off;
        const int local = (int)(bin - boff);
        const int bx = local % n0, by = (local / n0) % n1, bz = local / (n0 * n1);
        const int ox = 2 * s0 + 1, oy = 2 * s1 + 1, oz = 2 * s2 + 1;
        const int n_off = ox * oy * oz;
        const int my_start = bin_start[bin];
        for (int a0 = 0; a0 < my_cnt; a0 += 64) {
            const int na = my_cnt - a0 < 64 ? my_cnt - a0 : 64;
            // lane a holds atom a0 + a: index, wrap, w.H - x, and its counters
            int ai = 0, aw0 = 0, aw1 = 0, aw2 = 0;
            double ao0 = 0.0, ao1 = 0.0, ao2 = 0.0;
            if (lane < na) {
                ai = bin_atoms[my_start + a0 + lane];
                aw0 = atom_wrap[3 * ai];
                aw1 = atom_wrap[3 * ai + 1];
                aw2 = atom_wrap[3 * ai + 2];
                ao0 = aw0 * H[0] + aw1 * H[3] + aw2 * H[6] - pos[3 * ai];
                ao1 = aw0 * H[1] + aw1 * H[4] + aw2 * H[7] - pos[3 * ai + 1];
                ao2 = aw0 * H[2] + aw1 * H[5] + aw2 * H[8] - pos[3 * ai + 2];
            }
            int run[MAX_TYPES] = {0, 0, 0, 0}, cap[MAX_TYPES] = {0, 0, 0, 0}, base[MAX_TYPES] = {0, 0, 0, 0};
            for (int pass = 0; pass < 2; ++pass) {
                if (pass == 1 && lane < na) {
                    int off = 0, tot = 0;
                    for (int t = 0; t < n_types; ++t) {
                        tot += run[t];
                        const int room = max_nbrs - off;
                        cap[t] = run[t] < room ? run[t] : room;
                        base[t] = off;
                        off += cap[t];
                        run[t] = 0;
                    }
                    if (tot > max_nbrs) atomicOr(&flags[0], 1);
                    atomicMax(&flags[1], tot);
                }
                for (int og = 0; og < n_off; og += 64) {
                    const int o = og + lane;
                    int start = 0, c = 0, qp = pack_q(0, 0, 0);
                    if (o < n_off) {
                        const int dx = o % ox - s0, dy = (o / ox) % oy - s1, dz = o / (ox * oy) - s2;
                        int ux = bx + dx, uy = by + dy, uz = bz + dz, qx = 0, qy = 0, qz = 0;
                        bool ok = true;
                        if (p0) { qx = floordiv(ux, n0); ux -= qx * n0; } else ok = ok && ux >= 0 && ux < n0;
                        if (p1) { qy = floordiv(uy, n1); uy -= qy * n1; } else ok = ok && uy >= 0 && uy < n1;
                        if (p2) { qz = floordiv(uz, n2); uz -= qz * n2; } else ok = ok && uz >= 0 && uz < n2;
                        if (ok) {
                            const long long nb = boff + ((long long)uz * n1 + uy) * n0 + ux;
                            start = bin_start[nb];
                            c = bin_count[nb];
                            qp = pack_q(qx, qy, qz);
                        }
                    }
                    int inc = c;
#pragma unroll
                    for (int d = 1; d < 64; d <<= 1) {
                        const int t = __shfl_up(inc, d, 64);
                        if (lane >= d) inc += t;
                    }
                    const int excl = inc - c;
                    const int total = __shfl(inc, 63, 64);
                    for (int w0 = 0; w0 < total; w0 += 64 * SW_C) {
                        double cx[SW_C], cy[SW_C], cz[SW_C];
                        int cj[SW_C], cs[SW_C], ct[SW_C];
#pragma unroll
                        for (int cc = 0; cc < SW_C; ++cc) {
                            const int v = w0 + cc * 64 + lane;
                            int L = 0;
#pragma unroll
                            for (int step = 32; step >= 1; step >>= 1) {
                                const int e = __shfl(excl, L + step, 64);
                                if (e <= v) L += step;
                            }
                            const int st = __shfl(start, L, 64), pe = __shfl(excl, L, 64), q = __shfl(qp, L, 64);
                            cj[cc] = -1;
                            cx[cc] = cy[cc] = cz[cc] = 0.0;
                            cs[cc] = pack_q(0, 0, 0);
                            ct[cc] = -1;
                            if (v < total) {
                                const int j = bin_atoms[st + v - pe];
                                const int sx = ((q & 1023) - 512) - atom_wrap[3 * j];
                                const int sy = (((q >> 10) & 1023) - 512) - atom_wrap[3 * j + 1];
                                const int sz = (((q >> 20) & 1023) - 512) - atom_wrap[3 * j + 2];
                                cx[cc] = pos[3 * j] + sx * H[0] + sy * H[3] + sz * H[6];
                                cy[cc] = pos[3 * j + 1] + sx * H[1] + sy * H[4] + sz * H[7];
                                cz[cc] = pos[3 * j + 2] + sx * H[2] + sy * H[5] + sz * H[8];
                                cj[cc] = j;
                                cs[cc] = pack_q(sx, sy, sz);
                                const int t = type[j];
                                ct[cc] = (t < 0 || t >= n_types) ? -2 : t;
                            }
                        }
                        for (int a = 0; a < na; ++a) {
                            const int i = __shfl(ai, a, 64);
                            const int wi0 = __shfl(aw0, a, 64), wi1 = __shfl(aw1, a, 64), wi2 = __shfl(aw2, a, 64);
                            const double bx0 = __shfl(ao0, a, 64), bx1 = __shfl(ao1, a, 64), bx2 = __shfl(ao2, a, 64);
                            int cnt_t[MAX_TYPES], cap_t[MAX_TYPES], base_t[MAX_TYPES];
#pragma unroll
                            for (int t = 0; t < MAX_TYPES; ++t) {
                                cnt_t[t] = __shfl(run[t], a, 64);
                                cap_t[t] = __shfl(cap[t], a, 64);
                                base_t[t] = __shfl(base[t], a, 64);
                            }
#pragma unroll
                            for (int cc = 0; cc < SW_C; ++cc) {
                                if (w0 + cc * 64 >= total) break;   // uniform
                                bool ok = false;
                                int t = -1, sh0 = 0, sh1 = 0, sh2 = 0;
                                double r0 = 0.0, r1 = 0.0, r2 = 0.0;
                                if (cj[cc] >= 0) {
                                    const int q = cs[cc];
                                    sh0 = ((q & 1023) - 512) + wi0;
                                    sh1 = (((q >> 10) & 1023) - 512) + wi1;
                                    sh2 = (((q >> 20) & 1023) - 512) + wi2;
                                    if (!(cj[cc] == i && sh0 == 0 && sh1 == 0 && sh2 == 0)) {
                                        r0 = cx[cc] + bx0;
                                        r1 = cy[cc] + bx1;
                                        r2 = cz[cc] + bx2;
                                        const double d = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
                                        if (d < rc) {
                                            t = ct[cc];
                                            if (t == -2) {
                                                bad_type = true;
                                            } else {
                                                ok = true;
                                                if (d < 1e-6) overlap = true;
                                            }
                                        }
                                    }
                                }
                                for (int tt = 0; tt < n_types; ++tt) {
                                    const bool mine = ok && t == tt;
                                    const unsigned long long mk = __ballot(mine);
                                    if (pass == 1 && mine) {
                                        const int slot_in = cnt_t[tt] + __popcll(mk & below);
                                        if (slot_in < cap_t[tt]) {
                                            const int64_t slot = (int64_t)i * max_nbrs + base_t[tt] + slot_in;
                                            rout[3 * slot] = r0;
                                            rout[3 * slot + 1] = r1;
                                            rout[3 * slot + 2] = r2;
                                            jout[slot] = cj[cc];
                                            if (sh0 < -127 || sh0 > 127 || sh1 < -127 || sh1 > 127 || sh2 < -127 ||
                                                sh2 > 127)
                                                wide = true;
                                            shout[slot] = (sh0 & 0xff) | ((sh1 & 0xff) << 8) | ((sh2 & 0xff) << 16);
                                        }
                                    }
                                    cnt_t[tt] += __popcll(mk);
                                }
                            }
                            if (lane == a)
                                for (int t = 0; t < MAX_TYPES; ++t) run[t] = cnt_t[t];
                        }
                    }
                }
            }
            if (lane < na)
                for (int t = 0; t < n_types; ++t) tcnt[(int64_t)ai * n_types + t] = cap[t];
        }
    }
    if (overlap) atomicOr(&flags[2], 1);
    if (wide) atomicOr(&flags[3], 2);
    if (bad_type) atomicOr(&flags[3], 8);
}

__device__ inline int sx8(int v) { return (int)(signed char)(v & 0xff); }

// one thread per list slot: find the slot of (j, i, -n) in j's list
__global__ void reverse_pairs(int64_t n, int n_types, int max_nbrs, const int32_t *type, const int32_t *tcnt,
                              const int32_t *jl, const int32_t *sh, int32_t *rev, int32_t *flags) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= n * max_nbrs) return;
    const int64_t i = slot / max_nbrs;
    const int p = (int)(slot % max_nbrs);
    int tot = 0;
    for (int t = 0; t < n_types; ++t) tot += tcnt[i * n_types + t];
    if (p >= tot) return;
    const int zi = type[i];
    if (zi < 0 || zi >= n_types) return;
    const int j = jl[slot];
    const int s = sh[slot];
    const int want = ((-sx8(s)) & 0xff) | ((-sx8(s >> 8)) & 0xff) << 8 | ((-sx8(s >> 16)) & 0xff) << 16;
    int start = 0;
    for (int t = 0; t < zi; ++t) start += tcnt[(int64_t)j * n_types + t];
    const int cnt = tcnt[(int64_t)j * n_types + zi];
    int found = -1;
    for (int q = start; q < start + cnt; ++q) {
        const int64_t s2 = (int64_t)j * max_nbrs + q;
        if (jl[s2] == (int)i && sh[s2] == want) {
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
    const int64_t nscan = (bins + SCAN_B - 1) / SCAN_B;
    nb->work_sums.ensure(sizeof(int32_t) * (nscan > 0 ? nscan : 1));
    nb->bin_atoms.ensure(sizeof(int32_t) * (n > 0 ? n : 1));
    nb->flags.ensure(sizeof(int32_t) * 8);
    nb->bins_cap = bins;
    launch_zero(nb->flags.ptr, sizeof(int32_t) * 8, st);
    launch_zero(nb->bin_count.ptr, sizeof(int32_t) * bins, st);
    if (n == 0) return;
    auto *geo = nb->cfg_geo.as<CfgGeo>();
    int32_t *flags = nb->flags.as<int32_t>();
    hipLaunchKernelGGL(geo_kernel, dim3(1), dim3(64), 0, st, s->n_cfg, s->cfg_off, s->cell, s->pbc, m->r_cut, geo,
                       flags);
    const int TB = 256;
    const dim3 ga((unsigned)((n + TB - 1) / TB));
    hipLaunchKernelGGL(bin_kernel, ga, dim3(TB), 0, st, n, s->n_cfg, s->cfg_off, s->pos, geo,
                       nb->atom_cfg.as<int32_t>(), nb->atom_bin.as<int32_t>(), nb->atom_wrap.as<int32_t>(),
                       nb->bin_count.as<int32_t>());
    hipLaunchKernelGGL(scan_block, dim3((unsigned)nscan), dim3(SCAN_B), 0, st, nb->bin_count.as<int32_t>(),
                       nb->bin_start.as<int32_t>(), nb->work_sums.as<int32_t>(), flags + 4);
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(SCAN_B), 0, st, nb->work_sums.as<int32_t>(), nscan);
    hipLaunchKernelGGL(scan_add, dim3((unsigned)nscan), dim3(SCAN_B), 0, st, nb->bin_start.as<int32_t>(),
                       nb->work_sums.as<int32_t>(), flags + 4, nb->bin_cursor.as<int32_t>());
    hipLaunchKernelGGL(fill_bins, ga, dim3(TB), 0, st, n, nb->atom_bin.as<int32_t>(), nb->bin_cursor.as<int32_t>(),
                       nb->bin_atoms.as<int32_t>());
    const unsigned gbins = (unsigned)std::min<int64_t>((bins + 3) / 4, 2048);
    hipLaunchKernelGGL(sort_bins, dim3(gbins), dim3(256), 0, st, flags,
                       nb->bin_start.as<int32_t>(), nb->bin_count.as<int32_t>(), nb->bin_atoms.as<int32_t>());
    hipLaunchKernelGGL(bin_search, dim3((unsigned)std::min<int64_t>(bins, 2048)), dim3(BS_T), 0, st, flags + 4, s->n_cfg, nt, max_nbrs, m->r_cut,
                       s->pos, s->type, geo, nb->atom_wrap.as<int32_t>(), nb->bin_start.as<int32_t>(),
                       nb->bin_count.as<int32_t>(), nb->bin_atoms.as<int32_t>(), nb->tcnt.as<int32_t>(),
                       nb->r.as<double>(), nb->j.as<int32_t>(), nb->shift.as<int32_t>(), flags);
    hipLaunchKernelGGL(reverse_pairs, dim3((unsigned)((P + TB - 1) / TB)), dim3(TB), 0, st, n, nt, max_nbrs, s->type,
                       nb->tcnt.as<int32_t>(), nb->j.as<int32_t>(), nb->shift.as<int32_t>(), nb->rev.as<int32_t>(),
                       flags);
    MTP_HIP(hipGetLastError());
}

}  // namespace mtp
