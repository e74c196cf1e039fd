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

__global__ void scan_block(const int32_t *in, int32_t *out, int32_t *sums, int64_t n) {
    __shared__ int32_t s[SCAN_B];
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

__global__ void scan_add(int32_t *out, const int32_t *sums, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * SCAN_B + threadIdx.x;
    if (i < n) out[i] += sums[blockIdx.x];
}

__global__ void fill_bins(int64_t n, const int32_t *atom_bin, int32_t *cursor, int32_t *bin_atoms) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int slot = atomicAdd(&cursor[atom_bin[i]], 1);
    bin_atoms[slot] = (int32_t)i;
}

__global__ void sort_bins(int64_t nbins, const int32_t *start, const int32_t *count, int32_t *bin_atoms) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbins) return;
    int32_t *a = bin_atoms + start[b];
    const int c = count[b];
    for (int x = 1; x < c; ++x) {
        int32_t v = a[x];
        int y = x - 1;
        while (y >= 0 && a[y] > v) {
            a[y + 1] = a[y];
            --y;
        }
        a[y + 1] = v;
    }
}

__device__ inline int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// FILL = false: count per species; FILL = true: write the lists
template <bool FILL>
__global__ void search_kernel(int64_t n, int n_types, int max_nbrs, double rc, const double *pos, const int32_t *type,
                              const CfgGeo *geo, const int32_t *atom_cfg, const int32_t *atom_bin,
                              const int32_t *atom_wrap, const int32_t *bin_start, const int32_t *bin_count,
                              const int32_t *bin_atoms, int32_t *tcnt, double *rout, int32_t *jout,
                              int32_t *shout, int32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const CfgGeo &g = geo[atom_cfg[i]];
    const int local = (int)(atom_bin[i] - g.bin_off);
    const int bx = local % g.n[0], by = (local / g.n[0]) % g.n[1], bz = local / (g.n[0] * g.n[1]);
    const int wi[3] = {atom_wrap[3 * i], atom_wrap[3 * i + 1], atom_wrap[3 * i + 2]};
    const double xi[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    int cnt[MAX_TYPES] = {0, 0, 0, 0};
    int base[MAX_TYPES] = {0, 0, 0, 0}, cap[MAX_TYPES] = {0, 0, 0, 0};
    if (FILL) {
        int off = 0;
        for (int t = 0; t < n_types; ++t) {
            int want = tcnt[i * n_types + t];
            int room = max_nbrs - off;
            cap[t] = want < room ? want : room;
            base[t] = off;
            off += cap[t];
        }
    }
    bool overlap = false, wide = false, bad_type = false;
    for (int dz = -g.s[2]; dz <= g.s[2]; ++dz) {
        int uz = bz + dz, qz = 0;
        if (g.pbc[2]) { qz = floordiv(uz, g.n[2]); uz -= qz * g.n[2]; }
        else if (uz < 0 || uz >= g.n[2]) continue;
        for (int dy = -g.s[1]; dy <= g.s[1]; ++dy) {
            int uy = by + dy, qy = 0;
            if (g.pbc[1]) { qy = floordiv(uy, g.n[1]); uy -= qy * g.n[1]; }
            else if (uy < 0 || uy >= g.n[1]) continue;
            for (int dx = -g.s[0]; dx <= g.s[0]; ++dx) {
                int ux = bx + dx, qx = 0;
                if (g.pbc[0]) { qx = floordiv(ux, g.n[0]); ux -= qx * g.n[0]; }
                else if (ux < 0 || ux >= g.n[0]) continue;
                const long long bin = g.bin_off + ((long long)uz * g.n[1] + uy) * g.n[0] + ux;
                const int st = bin_start[bin], c = bin_count[bin];
                for (int q = 0; q < c; ++q) {
                    const int j = bin_atoms[st + q];
                    const int sh0 = qx - atom_wrap[3 * j] + wi[0];
                    const int sh1 = qy - atom_wrap[3 * j + 1] + wi[1];
                    const int sh2 = qz - atom_wrap[3 * j + 2] + wi[2];
                    if (j == i && sh0 == 0 && sh1 == 0 && sh2 == 0) continue;
                    double r[3];
                    for (int k = 0; k < 3; ++k)
                        r[k] = pos[3 * j + k] + sh0 * g.H[k] + sh1 * g.H[3 + k] + sh2 * g.H[6 + k] - xi[k];
                    const double d = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
                    if (!(d < rc)) continue;
                    if (d < 1e-6) overlap = true;
                    const int t = type[j];
                    if (t < 0 || t >= n_types) {
                        bad_type = true;
                        continue;
                    }
                    if (FILL) {
                        if (cnt[t] < cap[t]) {
                            const int64_t slot = i * max_nbrs + base[t] + cnt[t];
                            rout[3 * slot] = r[0];
                            rout[3 * slot + 1] = r[1];
                            rout[3 * slot + 2] = r[2];
                            jout[slot] = j;
                            if (sh0 < -127 || sh0 > 127 || sh1 < -127 || sh1 > 127 || sh2 < -127 || sh2 > 127)
                                wide = true;
                            shout[slot] = (sh0 & 0xff) | ((sh1 & 0xff) << 8) | ((sh2 & 0xff) << 16);
                        }
                    }
                    cnt[t]++;
                }
            }
        }
    }
    if (!FILL) {
        int tot = 0;
        for (int t = 0; t < n_types; ++t) {
            tcnt[i * n_types + t] = cnt[t];
            tot += cnt[t];
        }
        if (tot > max_nbrs) atomicOr(&flags[0], 1);
        atomicMax(&flags[1], tot);
        if (overlap) atomicOr(&flags[2], 1);
        if (bad_type) atomicOr(&flags[3], 8);
    } else {
        for (int t = 0; t < n_types; ++t) tcnt[i * n_types + t] = cap[t];
        if (wide) atomicOr(&flags[3], 2);
    }
}

__device__ inline int sx8(int v) { return (int)(signed char)(v & 0xff); }

__global__ void reverse_kernel(int64_t n, int n_types, int max_nbrs, const int32_t *type, const int32_t *tcnt,
                               const int32_t *jl, const int32_t *sh, int32_t *rev, int32_t *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int tot = 0;
    for (int t = 0; t < n_types; ++t) tot += tcnt[i * n_types + t];
    const int zi = type[i];
    if (zi < 0 || zi >= n_types) return;
    for (int p = 0; p < tot; ++p) {
        const int64_t slot = i * max_nbrs + p;
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
            found = (int)slot;   // keeps the gather in bounds; status reports the fault
        }
        rev[slot] = found;
    }
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
    nb->flags.ensure(sizeof(int32_t) * 4);
    nb->bins_cap = bins;
    launch_zero(nb->flags.ptr, sizeof(int32_t) * 4, st);
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
                       nb->bin_start.as<int32_t>(), nb->work_sums.as<int32_t>(), bins);
    hipLaunchKernelGGL(scan_sums, dim3(1), dim3(SCAN_B), 0, st, nb->work_sums.as<int32_t>(), nscan);
    hipLaunchKernelGGL(scan_add, dim3((unsigned)nscan), dim3(SCAN_B), 0, st, nb->bin_start.as<int32_t>(),
                       nb->work_sums.as<int32_t>(), bins);
    MTP_HIP(hipMemcpyAsync(nb->bin_cursor.ptr, nb->bin_start.ptr, sizeof(int32_t) * bins, hipMemcpyDeviceToDevice,
                           st));
    hipLaunchKernelGGL(fill_bins, ga, dim3(TB), 0, st, n, nb->atom_bin.as<int32_t>(), nb->bin_cursor.as<int32_t>(),
                       nb->bin_atoms.as<int32_t>());
    hipLaunchKernelGGL(sort_bins, dim3((unsigned)((bins + TB - 1) / TB)), dim3(TB), 0, st, bins,
                       nb->bin_start.as<int32_t>(), nb->bin_count.as<int32_t>(), nb->bin_atoms.as<int32_t>());
    hipLaunchKernelGGL(search_kernel<false>, ga, dim3(TB), 0, st, n, nt, max_nbrs, m->r_cut, s->pos, s->type, geo,
                       nb->atom_cfg.as<int32_t>(), nb->atom_bin.as<int32_t>(), nb->atom_wrap.as<int32_t>(),
                       nb->bin_start.as<int32_t>(), nb->bin_count.as<int32_t>(), nb->bin_atoms.as<int32_t>(),
                       nb->tcnt.as<int32_t>(), nullptr, nullptr, nullptr, flags);
    hipLaunchKernelGGL(search_kernel<true>, ga, dim3(TB), 0, st, n, nt, max_nbrs, m->r_cut, s->pos, s->type, geo,
                       nb->atom_cfg.as<int32_t>(), nb->atom_bin.as<int32_t>(), nb->atom_wrap.as<int32_t>(),
                       nb->bin_start.as<int32_t>(), nb->bin_count.as<int32_t>(), nb->bin_atoms.as<int32_t>(),
                       nb->tcnt.as<int32_t>(), nb->r.as<double>(), nb->j.as<int32_t>(), nb->shift.as<int32_t>(),
                       flags);
    hipLaunchKernelGGL(reverse_kernel, ga, dim3(TB), 0, st, n, nt, max_nbrs, s->type, nb->tcnt.as<int32_t>(),
                       nb->j.as<int32_t>(), nb->shift.as<int32_t>(), nb->rev.as<int32_t>(), flags);
    MTP_HIP(hipGetLastError());
}

}  // namespace mtp
