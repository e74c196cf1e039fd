// C ABI of libmtp: argument checks, model state, workspaces and the order
// of kernel launches.  Every entry point catches its own errors and turns
// them into an mtp_status (see include/mtp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"

namespace mtp {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

void DevBuf::ensure(size_t n) {
    if (n <= bytes && ptr) return;
    release();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        (void)hipGetLastError();
        throw Error{MTP_E_NOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed"};
    }
    bytes = n;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

namespace {

hipStream_t S(void *s) { return static_cast<hipStream_t>(s); }

// columns of the rows buffer: m padded with zeros to a multiple of 64 for the
// mixed form (the k step of its int8 product), of 32 for the FP64 form (the
// k chunk of the FP64 products, which never read further)
int ld_of(int m, int prec) { return prec == MTP_MIXED ? (m + 63) / 64 * 64 : (m + 31) / 32 * 32; }

// FULL-mode gauge: per mu drop mu+1 columns of block c_mu chosen as the
// first mu+1 pivots of a column-pivoted Gram-Schmidt (= QR with column
// pivoting) of the (mu+1) x (T^2 N_polyn) matrix [c_0; ...; c_mu].
void choose_gauge(mtp_model *m) {
    const int T = m->n_types, L = m->basis.n_lin(), R = m->basis.n_rad;
    const int blk = T * T * NPOLY;
    const int base = T + L;
    std::vector<int> drop;
    for (int mu = 0; mu < R; ++mu) {
        const int rows = mu + 1;
        // columns of the block as vectors of length rows
        std::vector<std::vector<double>> col(blk, std::vector<double>(rows));
        for (int c = 0; c < blk; ++c)
            for (int r = 0; r < rows; ++r) col[c][r] = m->theta_host[base + r * blk + c];
        std::vector<bool> used(blk, false);
        for (int step = 0; step < rows; ++step) {
            int best = -1;
            double bn = -1.0;
            for (int c = 0; c < blk; ++c) {
                if (used[c]) continue;
                double nn = 0.0;
                for (double v : col[c]) nn += v * v;
                if (nn > bn) {
                    bn = nn;
                    best = c;
                }
            }
            used[best] = true;
            drop.push_back(base + mu * blk + best);
            const double nrm = std::sqrt(bn);
            if (nrm == 0.0) continue;
            std::vector<double> q(rows);
            for (int r = 0; r < rows; ++r) q[r] = col[best][r] / nrm;
            for (int c = 0; c < blk; ++c) {
                if (used[c]) continue;
                double d = 0.0;
                for (int r = 0; r < rows; ++r) d += q[r] * col[c][r];
                for (int r = 0; r < rows; ++r) col[c][r] -= d * q[r];
            }
        }
    }
    std::sort(drop.begin(), drop.end());
    m->kept.clear();
    m->colmap_host.assign(m->n_theta, -1);
    size_t d = 0;
    for (int k = 0; k < m->n_theta; ++k) {
        if (d < drop.size() && drop[d] == k) {
            ++d;
            continue;
        }
        m->colmap_host[k] = (int)m->kept.size();
        m->kept.push_back(k);
    }
}

void upload_params(mtp_model *m) {
    MTP_HIP(hipSetDevice(m->device));
    m->theta64.ensure(sizeof(double) * m->n_theta);
    m->theta32.ensure(sizeof(float) * m->n_theta);
    std::vector<float> t32(m->theta_host.begin(), m->theta_host.end());
    MTP_HIP(hipMemcpy(m->theta64.ptr, m->theta_host.data(), sizeof(double) * m->n_theta, hipMemcpyHostToDevice));
    MTP_HIP(hipMemcpy(m->theta32.ptr, t32.data(), sizeof(float) * m->n_theta, hipMemcpyHostToDevice));
    m->colmap.ensure(sizeof(int32_t) * m->n_theta);
    MTP_HIP(hipMemcpy(m->colmap.ptr, m->colmap_host.data(), sizeof(int32_t) * m->n_theta, hipMemcpyHostToDevice));
}

mtp_model *new_model(int level, int n_types, double r_min, double r_cut, int device) {
    MTP_CHECK(n_types >= 1 && n_types <= MAX_TYPES, MTP_E_UNSUPPORTED, "n_types must be 1..4");
    MTP_CHECK(r_cut > r_min && r_min >= 0.0, MTP_E_INVAL, "need 0 <= r_min < r_cut");
    auto lv = compiled_levels();
    MTP_CHECK(std::find(lv.begin(), lv.end(), level) != lv.end(), MTP_E_UNSUPPORTED,
              "level " + std::to_string(level) + " is not compiled into this library");
    int ndev = 0;
    MTP_HIP(hipGetDeviceCount(&ndev));
    MTP_CHECK(device >= 0 && device < ndev, MTP_E_INVAL, "bad hip_device");
    auto *m = new mtp_model();
    m->device = device;
    m->level = level;
    m->n_types = n_types;
    m->r_min = r_min;
    m->r_cut = r_cut;
    m->basis = build_basis(level);
    m->n_theta = n_types + m->basis.n_lin() + m->basis.n_rad * n_types * n_types * NPOLY;
    m->theta_host.assign(m->n_theta, 0.0);
    return m;
}

void set_active(mtp_model *m, int mode, const double *A_dev, hipStream_t st) {
    ActiveSet &as = m->act[mode];
    as.m = m->m_of(mode);
    as.A.ensure(sizeof(double) * as.m * as.m);
    as.Ainv.ensure(sizeof(double) * as.m * as.m);
    MTP_HIP(hipMemcpyAsync(as.A.ptr, A_dev, sizeof(double) * as.m * as.m, hipMemcpyDeviceToDevice, st));
    int singular = 0;
    launch_invert(as, as.A.as<double>(), st, m->work, &singular);
    if (singular) {
        as.valid = false;
        throw Error{MTP_E_SINGULAR, "active-set matrix is singular (pivot below 1e-300)"};
    }
    prepare_split(as, st);
    as.valid = true;
}

void check_system(const mtp_model *m, const mtp_system *s) {
    MTP_CHECK(s, MTP_E_INVAL, "system is NULL");
    MTP_CHECK(s->n_cfg >= 1 && s->n_atoms >= 0, MTP_E_INVAL, "need n_cfg >= 1 and n_atoms >= 0");
    MTP_CHECK(s->cfg_off && s->cell, MTP_E_INVAL, "system arrays must not be NULL");
    MTP_CHECK(s->n_atoms == 0 || (s->pos && s->type), MTP_E_INVAL, "positions and types must not be NULL");
    MTP_CHECK(s->n_atoms < (int64_t)1 << 31, MTP_E_INVAL, "at most 2^31-1 atoms per call");
    (void)m;
}

void check_nbrs(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb) {
    MTP_CHECK(nb && nb->n_atoms == s->n_atoms && nb->n_types == m->n_types && nb->n_cfg == s->n_cfg,
              MTP_E_INVAL, "neighbor lists were not built for this system and model");
    MTP_CHECK(nb->r_cut == m->r_cut, MTP_E_INVAL, "neighbor lists were built with another cutoff");
}

int size_bucket(int64_t n) {
    int b = 0;
    while (b < 47 && (int64_t(1) << (b + 1)) <= n) ++b;
    return b;
}

// schedule = 16 x (moments / contraction lanes) + (pair-gradient lanes)
int lanes_for(const mtp_model *m, int64_t n, int prec) {
    if (m->force_lanes) return m->force_lanes;
    if (const char *e = std::getenv("MTP_LANES")) {
        int v = std::atoi(e);
        if (v == 2 || v == 4 || v == 8) return 17 * v;
    }
    if (int t = m->tuned_lanes[prec == MTP_FP64 ? 0 : 1][size_bucket(n)]) return t;
    // enough wavefronts for 256 CUs x 4 SIMDs, few lanes when the batch is large
    if (n >= (int64_t)1 << 20) return 17 * 2;
    if (n >= (int64_t)1 << 17) return 17 * 4;
    return 17 * 8;
}

// grade schedule: the tuner's choice for this size class, else GRADE_AUTO
int grade_sched_for(const mtp_model *m, int64_t n, int prec, int mode) {
    if (m->force_grade) return m->force_grade;
    if (const char *e = std::getenv("MTP_GRADE_FORM")) {   // 1 .. 6 (GRADE_*), where available
        const int v = std::atoi(e);
        if (v >= GRADE_F64_REG && v <= GRADE_F64_KOUTER2 && grade_sched_valid(m->act[mode & 1], prec, v)) return v;
    }
    const int t = m->tuned_grade[prec == MTP_FP64 ? 0 : 1][mode & 1][size_bucket(n)];
    return t && grade_sched_valid(m->act[mode & 1], prec, t) ? t : GRADE_AUTO;
}

struct EvalOut {
    double *energy = nullptr, *forces = nullptr, *stress = nullptr, *site_e = nullptr;
    double *gamma = nullptr;
    int32_t *argmax = nullptr;
    void *b_rows = nullptr;
    int mode = MTP_GRADE_FULL;
    // preselection fused into the grade (gamma > sel_thr), or sel_idx NULL
    double sel_thr = 0.0;
    int32_t *sel_idx = nullptr, *sel_count = nullptr;
    int32_t sel_cap = 0;
    bool keep_rows = false;   // leave the rows in m->brow (configuration mode)
};

// Where the evaluation's scratch comes from: the model's buffers, grown on
// demand (hipMalloc), or one fixed device region that is carved up in order
// (the no-allocation entry point; sizes past the region are rejected).
struct Workspace {
    char *base = nullptr;   // fixed region, or NULL for the model's buffers
    size_t cap = 0, used = 0;
    void *get(DevBuf &b, size_t bytes) {
        if (!base) {
            b.ensure(bytes);
            return b.ptr;
        }
        const size_t off = (used + 255) / 256 * 256;
        MTP_CHECK(off <= cap && bytes <= cap - off, MTP_E_CAPACITY,
                  "the evaluation needs more than the " + std::to_string(cap >> 20) +
                      " MiB of the fixed scratch region (fewer atoms or a smaller max_nbrs)");
        used = off + bytes;
        return base + off;
    }
};

void evaluate(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, int prec, const EvalOut &o,
              hipStream_t st, Workspace ws = Workspace{}) {
    check_system(m, s);
    check_nbrs(m, s, nb);
    MTP_CHECK(prec == MTP_FP64 || prec == MTP_MIXED, MTP_E_INVAL, "bad precision");
    MTP_CHECK(o.mode == MTP_GRADE_FULL || o.mode == MTP_GRADE_LINEAR, MTP_E_INVAL, "bad grade mode");
    const bool want_sel = o.sel_idx != nullptr;
    const bool want_grade = o.gamma || o.argmax || want_sel;
    const bool want_rows = want_grade || o.b_rows || o.keep_rows;
    if (want_grade) MTP_CHECK(m->act[o.mode].valid, MTP_E_INVAL, "no active set for this grade mode");
    MTP_HIP(hipSetDevice(m->device));
    const int64_t n = s->n_atoms;
    // tsz: the pair gradients' type; msz: the moments' and dE/dM's (FP64 in
    // the mixed form too when rows are wanted: rows are always FP64)
    const size_t tsz = prec == MTP_FP64 ? sizeof(double) : sizeof(float);
    const size_t msz = (prec == MTP_FP64 || want_rows) ? sizeof(double) : sizeof(float);
    const bool want_f = o.forces != nullptr;
    const bool want_v = o.stress != nullptr;
    const bool want_e = o.energy || o.site_e;
    const int mm = m->m_of(o.mode);
    const int ldb = ld_of(mm, prec);
    void *gbuf = want_f ? ws.get(m->gbuf, tsz * 3 * (size_t)std::max<int64_t>(1, n * nb->max_nbrs)) : nullptr;
    double *virial =
        want_v ? static_cast<double *>(ws.get(m->virial, sizeof(double) * 9 * (size_t)std::max<int64_t>(1, n))) : nullptr;
    double *site = o.site_e;
    if (want_e && !site) site = static_cast<double *>(ws.get(m->sitebuf, sizeof(double) * (size_t)std::max<int64_t>(1, n)));
    double *brow = want_rows ? static_cast<double *>(ws.get(m->brow, sizeof(double) * (size_t)ldb *
                                                                        (size_t)std::max<int64_t>(1, n)))
                             : nullptr;
    if (n == 0) {
        if (o.energy) launch_zero(o.energy, sizeof(double) * s->n_cfg, st);
        if (o.stress) launch_zero(o.stress, sizeof(double) * 9 * s->n_cfg, st);
        if (want_sel) launch_zero(o.sel_count, sizeof(int32_t), st);
        return;
    }
    EfsArgs a{};
    a.n_atoms = n;
    a.atom_list = nullptr;
    a.n_types = m->n_types;
    a.max_nbrs = nb->max_nbrs;
    a.r = nb->r.as<double>();
    a.tcnt = nb->tcnt.as<int32_t>();
    a.type = s->type;
    a.r_min = m->r_min;
    a.r_cut = m->r_cut;
    a.th64 = m->theta64.as<double>();
    a.th32 = m->theta32.as<float>();
    a.n_lin = m->basis.n_lin();
    a.site_e = want_e ? site : nullptr;
    a.gbuf = gbuf;
    a.rev = nb->rev.as<int32_t>();
    a.F = o.forces;
    a.virial = virial;
    a.brow = brow;
    a.ldn = n;
    a.ldb = ldb;
    a.grade_mode = o.mode;
    a.colmap = m->colmap.as<int32_t>();
    a.m = mm;
    a.precision = prec;
    const int sched = lanes_for(m, n, prec);
    a.lanes = sched & 15;
    a.lanes_mc = sched >> 4;
    a.stream = st;
    a.mbuf = ws.get(m->mbuf, msz * m->basis.n_comp() * (size_t)n);
    a.dmbuf = ws.get(m->dmbuf, msz * m->basis.n_comp() * (size_t)n);
    if (const int ngs = staged_graphs(m->level)) {   // tiles of 64 neighborhoods
        const size_t bytes = msz * ngs * (size_t)((n + 63) / 64 * 64);
        a.gval = ws.get(m->gval, bytes);
        a.dgval = ws.get(m->dgval, bytes);
    }
    // per-configuration sums: chunk partials, then one block per configuration.
    // With forces and a preselection the force gather runs as extra blocks of
    // the preselection's launch (one launch less per step) and the partials
    // come from the pair-gradient kernel; otherwise the gather (or a kernel of
    // their own) writes them.
    const bool want_sums = o.energy || want_v;
    const double *sum_e = o.energy ? site : nullptr;
    const double *sum_v = want_v ? virial : nullptr;
    double *sums = want_sums ? static_cast<double *>(ws.get(m->sums, cfg_partials_bytes(n))) : nullptr;
    const bool fuse_gather = want_f && want_sel;
    if (fuse_gather && want_sums) {
        a.part = sums;
        a.part_e = sum_e;
    }
    int e;
    {
        ProfScope ps("efs", st);
        e = launch_efs(m->level, a);
    }
    MTP_CHECK(e == 0, MTP_E_HIP, std::string("efs kernel launch: ") + hipGetErrorString((hipError_t)e));
    if (want_f && !fuse_gather) {
        ProfScope ps("force_gather", st);
        launch_force_gather(nb, gbuf, prec, o.forces, st, sum_e, sum_v, sums);
    } else if (want_sums && !fuse_gather) {
        launch_cfg_partials(n, sum_e, sum_v, sums, st);
    }
    // with a preselection the sums are finished by the preselection's launch
    const CfgSums csums{s, sum_e, sum_v, sums, o.energy, o.stress};
    if (want_sums && !want_sel) {
        ProfScope ps("cfg_sums", st);
        launch_cfg_final(s, sum_e, sum_v, sums, o.energy, o.stress, st);
    }
    if (want_grade) {
        double *gam = o.gamma ? o.gamma : static_cast<double *>(ws.get(m->gamma_ws, sizeof(double) * n));
        int32_t *blk = nullptr;
        const int sched = grade_sched_for(m, n, prec, o.mode);
        const int count_rows = grade_count_rows(m->act[o.mode], prec, sched);
        if (want_sel)
            blk = static_cast<int32_t *>(
                ws.get(m->selblk, sizeof(int32_t) * (size_t)((n + count_rows - 1) / count_rows + 1)));
        {
            ProfScope ps("grade", st);
            launch_grade(m->act[o.mode], prec, brow, ldb, n, n, gam, o.argmax, st, o.sel_thr, blk, sched);
        }
        if (want_sel) {
            ProfScope ps("select", st);
            const GatherArgs ga = fuse_gather ? gather_args(nb, gbuf, prec, o.forces) : GatherArgs{};
            launch_select_write(gam, n, o.sel_thr, blk, o.sel_idx, o.sel_cap, o.sel_count, st,
                                want_sums ? &csums : nullptr, fuse_gather ? &ga : nullptr, count_rows);
        }
    }
    if (o.b_rows) launch_copy_rows(brow, n, mm, n, static_cast<double *>(o.b_rows), st);
    MTP_HIP(hipGetLastError());
}

std::string read_file(const char *path) {
    std::ifstream f(path);
    MTP_CHECK(f.good(), MTP_E_IO, std::string("cannot open ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    return ss.str();
}

}  // namespace
}  // namespace mtp

using namespace mtp;

#define API_BEGIN try {
#define API_END                                                  \
    }                                                            \
    catch (const mtp::Error &e) {                                \
        mtp::set_error(e.msg);                                   \
        return e.code;                                           \
    }                                                            \
    catch (const std::bad_alloc &) {                             \
        mtp::set_error("host allocation failed");                \
        return MTP_E_NOMEM;                                      \
    }                                                            \
    catch (const std::exception &e) {                            \
        mtp::set_error(e.what());                                \
        return MTP_E_INVAL;                                      \
    }                                                            \
    return MTP_OK;

extern "C" {

const char *mtp_last_error(void) { return g_last_error.c_str(); }

int mtp_create(int32_t level, int32_t n_types, double r_min, double r_cut, int hip_device, mtp_model **out) {
    API_BEGIN
    MTP_CHECK(out, MTP_E_INVAL, "out is NULL");
    mtp_model *m = new_model(level, n_types, r_min, r_cut, hip_device);
    choose_gauge(m);
    upload_params(m);
    *out = m;
    API_END
}

int mtp_load(const char *path, int hip_device, mtp_model **out) {
    API_BEGIN
    MTP_CHECK(path && out, MTP_E_INVAL, "NULL argument");
    std::istringstream in(read_file(path));
    std::string key;
    int level = -1, nt = -1, npoly = NPOLY, fmt = -1;
    double rmin = NAN, rcut = NAN;
    std::vector<double> theta;
    std::vector<std::pair<int, std::vector<double>>> acts;
    while (in >> key) {
        if (key[0] == '#') {
            std::string rest;
            std::getline(in, rest);
            continue;
        }
        if (key == "format") in >> fmt;
        else if (key == "level") in >> level;
        else if (key == "n_types") in >> nt;
        else if (key == "r_min") in >> rmin;
        else if (key == "r_cut") in >> rcut;
        else if (key == "n_polyn") in >> npoly;
        else if (key == "theta") {
            long n = -1;
            in >> n;
            MTP_CHECK(n >= 0 && n < 100000000, MTP_E_PARSE, "bad theta length");
            theta.resize(n);
            for (long k = 0; k < n; ++k) MTP_CHECK(bool(in >> theta[k]), MTP_E_PARSE, "theta truncated");
        } else if (key == "active") {
            std::string mode;
            long mm = -1;
            in >> mode >> mm;
            const char *names[4] = {"full", "linear", "full_cfg", "linear_cfg"};
            int mi = -1;
            for (int k = 0; k < 4; ++k)
                if (mode == names[k]) mi = k;
            MTP_CHECK(mi >= 0, MTP_E_PARSE, "active mode must be full, linear, full_cfg or linear_cfg");
            MTP_CHECK(mm > 0 && mm < 100000, MTP_E_PARSE, "bad active-set size");
            std::vector<double> A(mm * mm);
            for (long k = 0; k < mm * mm; ++k) MTP_CHECK(bool(in >> A[k]), MTP_E_PARSE, "active set truncated");
            acts.push_back({mi, A});
        } else {
            throw Error{MTP_E_PARSE, "unknown key '" + key + "'"};
        }
        MTP_CHECK(!in.fail(), MTP_E_PARSE, "bad value after '" + key + "'");
    }
    MTP_CHECK(fmt == 1, MTP_E_PARSE, "missing or unsupported 'format'");
    MTP_CHECK(npoly == NPOLY, MTP_E_UNSUPPORTED, "only n_polyn 8 is compiled");
    MTP_CHECK(level > 0 && nt > 0 && std::isfinite(rmin) && std::isfinite(rcut), MTP_E_PARSE,
              "need level, n_types, r_min, r_cut");
    mtp_model *m = new_model(level, nt, rmin, rcut, hip_device);
    MTP_CHECK(theta.empty() || (int)theta.size() == m->n_theta,
              (delete m, MTP_E_PARSE), "theta length does not match level and n_types");
    if (!theta.empty()) m->theta_host = theta;
    choose_gauge(m);
    upload_params(m);
    for (auto &a : acts) {
        const int mm = m->m_of(a.first);
        if ((long)a.second.size() != (long)mm * mm) {
            delete m;
            throw Error{MTP_E_PARSE, "active-set size does not match the model"};
        }
        DevBuf tmp;
        tmp.ensure(sizeof(double) * mm * mm);
        MTP_HIP(hipMemcpy(tmp.ptr, a.second.data(), sizeof(double) * mm * mm, hipMemcpyHostToDevice));
        try {
            set_active(m, a.first, tmp.as<double>(), nullptr);
        } catch (...) {
            delete m;
            throw;
        }
    }
    *out = m;
    API_END
}

int mtp_save(const mtp_model *m, const char *path) {
    API_BEGIN
    MTP_CHECK(m && path, MTP_E_INVAL, "NULL argument");
    std::ofstream f(path);
    MTP_CHECK(f.good(), MTP_E_IO, std::string("cannot write ") + path);
    f.precision(17);
    f << "# MTP model (MI355X library text format)\nformat 1\nlevel " << m->level << "\nn_types " << m->n_types
      << "\nr_min " << m->r_min << "\nr_cut " << m->r_cut << "\nn_polyn " << NPOLY << "\ntheta " << m->n_theta << "\n";
    for (int k = 0; k < m->n_theta; ++k) f << m->theta_host[k] << (k % 8 == 7 ? "\n" : " ");
    f << "\n";
    const char *names[4] = {"full", "linear", "full_cfg", "linear_cfg"};
    for (int mode = 0; mode < 4; ++mode) {
        const ActiveSet &as = m->act[mode];
        if (!as.valid) continue;
        std::vector<double> A((size_t)as.m * as.m);
        MTP_HIP(hipSetDevice(m->device));
        MTP_HIP(hipMemcpy(A.data(), as.A.ptr, sizeof(double) * A.size(), hipMemcpyDeviceToHost));
        f << "active " << names[mode] << " " << as.m << "\n";
        for (size_t k = 0; k < A.size(); ++k) f << A[k] << ((k + 1) % as.m == 0 ? "\n" : " ");
    }
    MTP_CHECK(f.good(), MTP_E_IO, "write failed");
    API_END
}

int mtp_free(mtp_model *m) {
    API_BEGIN
    if (m) {
        (void)hipSetDevice(m->device);
        delete m;
    }
    API_END
}

int mtp_info(const mtp_model *m, mtp_model_info *info) {
    API_BEGIN
    MTP_CHECK(m && info, MTP_E_INVAL, "NULL argument");
    info->level = m->level;
    info->n_types = m->n_types;
    info->n_polyn = NPOLY;
    info->n_lin = m->basis.n_lin();
    info->n_rad = m->basis.n_rad;
    info->n_comp = m->basis.n_comp();
    info->n_theta = m->n_theta;
    info->m_full = m->m_of(MTP_GRADE_FULL);
    info->m_linear = m->m_of(MTP_GRADE_LINEAR);
    info->r_min = m->r_min;
    info->r_cut = m->r_cut;
    info->has_active_full = m->act[0].valid;
    info->has_active_linear = m->act[1].valid;
    info->contraction_flops = contraction_flops(m->level);
    API_END
}

int mtp_set_params(mtp_model *m, const double *theta, void *stream) {
    API_BEGIN
    MTP_CHECK(m && theta, MTP_E_INVAL, "NULL argument");
    MTP_HIP(hipSetDevice(m->device));
    std::vector<double> h(m->n_theta);
    MTP_HIP(hipMemcpyAsync(h.data(), theta, sizeof(double) * m->n_theta, hipMemcpyDeviceToHost, S(stream)));
    MTP_HIP(hipStreamSynchronize(S(stream)));
    for (double v : h) MTP_CHECK(std::isfinite(v), MTP_E_INVAL, "theta holds NaN or Inf");
    m->theta_host = h;
    choose_gauge(m);
    upload_params(m);
    m->act[MTP_GRADE_FULL].valid = false;   // FULL rows depend on theta
    m->act[MTP_GRADE_FULL_CFG].valid = false;
    API_END
}

int mtp_get_params(const mtp_model *m, double *theta) {
    API_BEGIN
    MTP_CHECK(m && theta, MTP_E_INVAL, "NULL argument");
    std::copy(m->theta_host.begin(), m->theta_host.end(), theta);
    API_END
}

int mtp_kept_columns(const mtp_model *m, int32_t *cols) {
    API_BEGIN
    MTP_CHECK(m && cols, MTP_E_INVAL, "NULL argument");
    for (size_t k = 0; k < m->kept.size(); ++k) cols[k] = m->kept[k];
    API_END
}

int mtp_set_active_set(mtp_model *m, mtp_grade_mode mode, const double *A, void *stream) {
    API_BEGIN
    MTP_CHECK(m && A, MTP_E_INVAL, "NULL argument");
    MTP_CHECK(mode >= MTP_GRADE_FULL && mode <= MTP_GRADE_LINEAR_CFG, MTP_E_INVAL, "bad grade mode");
    MTP_HIP(hipSetDevice(m->device));
    set_active(m, mode, A, S(stream));
    API_END
}

int mtp_get_active_set(const mtp_model *m, mtp_grade_mode mode, double *A_out, double *Ainv_out, void *stream) {
    API_BEGIN
    MTP_CHECK(m, MTP_E_INVAL, "NULL model");
    MTP_CHECK(mode >= MTP_GRADE_FULL && mode <= MTP_GRADE_LINEAR_CFG, MTP_E_INVAL, "bad grade mode");
    const ActiveSet &as = m->act[mode];
    MTP_CHECK(as.valid, MTP_E_INVAL, "no active set for this mode");
    MTP_HIP(hipSetDevice(m->device));
    const size_t b = sizeof(double) * as.m * as.m;
    if (A_out) MTP_HIP(hipMemcpyAsync(A_out, as.A.ptr, b, hipMemcpyDeviceToDevice, S(stream)));
    if (Ainv_out) MTP_HIP(hipMemcpyAsync(Ainv_out, as.Ainv.ptr, b, hipMemcpyDeviceToDevice, S(stream)));
    API_END
}

int mtp_nbrs_create(mtp_nbrs **out) {
    API_BEGIN
    MTP_CHECK(out, MTP_E_INVAL, "out is NULL");
    *out = new mtp_nbrs();
    API_END
}

int mtp_nbrs_free(mtp_nbrs *nb) {
    API_BEGIN
    if (nb) {
        if (nb->device >= 0) (void)hipSetDevice(nb->device);
        delete nb;
    }
    API_END
}

int mtp_build_neighbors(const mtp_model *m, const mtp_system *s, int32_t max_nbrs, mtp_nbrs *nb, void *stream) {
    API_BEGIN
    MTP_CHECK(m && nb, MTP_E_INVAL, "NULL argument");
    check_system(m, s);
    MTP_CHECK(max_nbrs >= 1 && max_nbrs <= 4096, MTP_E_INVAL, "max_nbrs must be 1..4096");
    MTP_CHECK(s->n_atoms * (int64_t)max_nbrs < ((int64_t)1 << 31), MTP_E_INVAL,
              "n_atoms * max_nbrs must stay below 2^31");
    MTP_HIP(hipSetDevice(m->device));
    ProfScope ps("neighbors", S(stream));
    build_neighbors(m, s, max_nbrs, nb, S(stream));
    API_END
}

int mtp_nbrs_status(const mtp_nbrs *nb, void *stream) {
    API_BEGIN
    MTP_CHECK(nb && nb->device >= 0, MTP_E_INVAL, "neighbor lists not built");
    MTP_HIP(hipSetDevice(nb->device));
    int32_t f[4] = {0, 0, 0, 0};
    MTP_HIP(hipMemcpyAsync(f, nb->flags.ptr, sizeof(f), hipMemcpyDeviceToHost, S(stream)));
    MTP_HIP(hipStreamSynchronize(S(stream)));
    MTP_CHECK(!(f[3] & 16), MTP_E_INVAL, "a position is not finite (NaN or Inf)");
    MTP_CHECK(!(f[3] & 1), MTP_E_INVAL, "a cell matrix is singular");
    MTP_CHECK(!(f[3] & 8), MTP_E_INVAL, "an atom type is outside 0..n_types-1");
    MTP_CHECK(!(f[3] & 2), MTP_E_INVAL, "an image shift exceeds +-127 cells (atoms far outside the cell)");
    MTP_CHECK(!f[0], MTP_E_CAPACITY,
              "a neighborhood has " + std::to_string(f[1]) + " atoms, more than max_nbrs = " +
                  std::to_string(nb->max_nbrs));
    MTP_CHECK(!(f[3] & 4), MTP_E_INVAL, "internal: a reverse pair was not found");
    MTP_CHECK(!f[2], MTP_E_OVERLAP, "two atoms are closer than 1e-6 Angstrom");
    API_END
}

int mtp_nbrs_export(const mtp_nbrs *nb, int32_t *count, int32_t *j, int32_t *shift, int32_t *stride, void *stream) {
    API_BEGIN
    MTP_CHECK(nb && nb->device >= 0, MTP_E_INVAL, "neighbor lists not built");
    MTP_HIP(hipSetDevice(nb->device));
    const int64_t n = nb->n_atoms, P = n * nb->max_nbrs;
    if (stride) *stride = nb->max_nbrs;
    if (count) {
        // per-atom totals from the per-species counts
        std::vector<int32_t> t((size_t)n * nb->n_types), c((size_t)n);
        MTP_HIP(hipMemcpyAsync(t.data(), nb->tcnt.ptr, sizeof(int32_t) * t.size(), hipMemcpyDeviceToHost, S(stream)));
        MTP_HIP(hipStreamSynchronize(S(stream)));
        for (int64_t i = 0; i < n; ++i) {
            int s = 0;
            for (int k = 0; k < nb->n_types; ++k) s += t[i * nb->n_types + k];
            c[i] = s;
        }
        MTP_HIP(hipMemcpyAsync(count, c.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, S(stream)));
        MTP_HIP(hipStreamSynchronize(S(stream)));
    }
    if (j) MTP_HIP(hipMemcpyAsync(j, nb->j.ptr, sizeof(int32_t) * P, hipMemcpyDeviceToDevice, S(stream)));
    if (shift) {
        std::vector<int32_t> p((size_t)P), o((size_t)P * 3);
        MTP_HIP(hipMemcpyAsync(p.data(), nb->shift.ptr, sizeof(int32_t) * P, hipMemcpyDeviceToHost, S(stream)));
        MTP_HIP(hipStreamSynchronize(S(stream)));
        for (int64_t k = 0; k < P; ++k)
            for (int a = 0; a < 3; ++a) o[3 * k + a] = (int32_t)(signed char)((p[k] >> (8 * a)) & 0xff);
        MTP_HIP(hipMemcpyAsync(shift, o.data(), sizeof(int32_t) * 3 * P, hipMemcpyHostToDevice, S(stream)));
        MTP_HIP(hipStreamSynchronize(S(stream)));
    }
    API_END
}

int mtp_energy_forces_stress(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p,
                             double *energy, double *forces, double *stress, double *site_e, void *stream) {
    API_BEGIN
    MTP_CHECK(m, MTP_E_INVAL, "NULL model");
    EvalOut o;
    o.energy = energy;
    o.forces = forces;
    o.stress = stress;
    o.site_e = site_e;
    evaluate(m, s, nb, p, o, S(stream));
    API_END
}

int mtp_energy_forces_stress_noalloc(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p,
                                     double *energy, double *forces, double *stress, double *site_e, void *stream) {
    API_BEGIN
    MTP_CHECK(m, MTP_E_INVAL, "NULL model");
    MTP_HIP(hipSetDevice(m->device));
    EvalOut o;
    o.energy = energy;
    o.forces = forces;
    o.stress = stress;
    o.site_e = site_e;
    Workspace ws;
    ws.base = static_cast<char *>(noalloc_scratch(m->device));
    ws.cap = NOALLOC_SCRATCH_BYTES;
    evaluate(m, s, nb, p, o, S(stream), ws);
    API_END
}

int mtp_grade(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, mtp_grade_mode g,
              double *gamma, int32_t *argmax, void *b_rows, void *stream) {
    API_BEGIN
    MTP_CHECK(m && gamma, MTP_E_INVAL, "NULL argument");
    EvalOut o;
    o.gamma = gamma;
    o.argmax = argmax;
    o.b_rows = b_rows;
    o.mode = g;
    evaluate(m, s, nb, p, o, S(stream));
    API_END
}

int mtp_grade_rows(const mtp_model *m, mtp_precision p, mtp_grade_mode g, const double *rows, int64_t n, int64_t ld,
                   int32_t ldb, double *gamma, int32_t *argmax, void *stream) {
    API_BEGIN
    MTP_CHECK(m && gamma && (rows || n == 0), MTP_E_INVAL, "NULL argument");
    MTP_CHECK(p == MTP_FP64 || p == MTP_MIXED, MTP_E_INVAL, "bad precision");
    MTP_CHECK(g == MTP_GRADE_FULL || g == MTP_GRADE_LINEAR, MTP_E_INVAL, "bad grade mode");
    MTP_CHECK(n >= 0 && ld >= n, MTP_E_INVAL, "need n >= 0 and ld >= n");
    MTP_CHECK(m->act[g].valid, MTP_E_INVAL, "no active set for this grade mode");
    const int mm = m->m_of(g);
    MTP_CHECK(ldb >= ld_of(mm, p), MTP_E_INVAL, "rows: fewer columns than the padded row length");
    if (n == 0) return MTP_OK;
    MTP_HIP(hipSetDevice(m->device));
    hipStream_t st = S(stream);
    const int sched = grade_sched_for(m, n, p, g);
    ProfScope ps("grade", st);
    launch_grade(m->act[g], p, rows, ldb, ld, n, gamma, argmax, st, 0.0, nullptr, sched);
    MTP_HIP(hipGetLastError());
    API_END
}

int mtp_grade_cfg(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, mtp_grade_mode g,
                  double *gamma, int32_t *argmax, double *b_cfg, void *stream) {
    API_BEGIN
    MTP_CHECK(m && (gamma || b_cfg), MTP_E_INVAL, "NULL argument");
    MTP_CHECK(g == MTP_GRADE_FULL_CFG || g == MTP_GRADE_LINEAR_CFG, MTP_E_INVAL,
              "configuration grades take MTP_GRADE_FULL_CFG or MTP_GRADE_LINEAR_CFG");
    check_system(m, s);
    const bool want_grade = gamma || argmax;
    if (want_grade) MTP_CHECK(m->act[g].valid, MTP_E_INVAL, "no active set for this grade mode");
    hipStream_t st = S(stream);
    // the neighborhood rows of every atom (FP64, column-major), left in m->brow
    EvalOut o;
    o.mode = g & 1;
    o.keep_rows = true;
    evaluate(m, s, nb, p, o, st);
    const int mm = m->m_of(g), ldb = ld_of(mm, p);   // as the evaluation above left the rows
    const int64_t n = s->n_atoms;
    m->cfgrows.ensure(sizeof(double) * (size_t)ldb * s->n_cfg);
    m->cfgpart.ensure(cfg_row_partials_bytes(n, ldb));
    if (n == 0) {
        launch_zero(m->cfgrows.ptr, sizeof(double) * (size_t)ldb * s->n_cfg, st);
    } else {
        ProfScope ps("cfg_rows", st);
        launch_cfg_rows(m->brow.as<double>(), ldb, n, s, m->cfgpart.as<double>(), m->cfgrows.as<double>(), st);
    }
    if (want_grade) {
        m->gamma_ws.ensure(sizeof(double) * s->n_cfg);
        ProfScope ps("grade", st);
        launch_grade(m->act[g], MTP_FP64, m->cfgrows.as<double>(), ldb, s->n_cfg, s->n_cfg,
                     gamma ? gamma : m->gamma_ws.as<double>(), argmax, st);
    }
    if (b_cfg) launch_copy_rows(m->cfgrows.as<double>(), s->n_cfg, mm, s->n_cfg, b_cfg, st);
    MTP_HIP(hipGetLastError());
    API_END
}

int mtp_evaluate(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, mtp_grade_mode g,
                 double *energy, double *forces, double *stress, double *site_e, double *gamma, int32_t *argmax,
                 void *stream) {
    API_BEGIN
    MTP_CHECK(m, MTP_E_INVAL, "NULL model");
    EvalOut o;
    o.energy = energy;
    o.forces = forces;
    o.stress = stress;
    o.site_e = site_e;
    o.gamma = gamma;
    o.argmax = argmax;
    o.mode = g;
    evaluate(m, s, nb, p, o, S(stream));
    API_END
}

int mtp_evaluate_select(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p,
                        mtp_grade_mode g, double *energy, double *forces, double *stress, double *site_e,
                        double *gamma, int32_t *argmax, double threshold, int32_t *idx, int32_t capacity,
                        int32_t *count, void *stream) {
    API_BEGIN
    MTP_CHECK(m && idx && count, MTP_E_INVAL, "NULL argument");
    MTP_CHECK(capacity >= 0, MTP_E_INVAL, "negative capacity");
    EvalOut o;
    o.energy = energy;
    o.forces = forces;
    o.stress = stress;
    o.site_e = site_e;
    o.gamma = gamma;
    o.argmax = argmax;
    o.mode = g;
    o.sel_thr = threshold;
    o.sel_idx = idx;
    o.sel_cap = capacity;
    o.sel_count = count;
    evaluate(m, s, nb, p, o, S(stream));
    API_END
}

int mtp_b_rows(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_grade_mode g, const int32_t *idx,
               int32_t n_idx, double *rows, void *stream) {
    API_BEGIN
    MTP_CHECK(m && idx && rows, MTP_E_INVAL, "NULL argument");
    MTP_CHECK(n_idx >= 0, MTP_E_INVAL, "n_idx < 0");
    MTP_CHECK(g == MTP_GRADE_FULL || g == MTP_GRADE_LINEAR, MTP_E_INVAL, "bad grade mode");
    check_system(m, s);
    check_nbrs(m, s, nb);
    if (n_idx == 0) return MTP_OK;
    MTP_HIP(hipSetDevice(m->device));
    const int mm = m->m_of(g);
    const int ldb = ld_of(mm, MTP_FP64);
    m->brow.ensure(sizeof(double) * (size_t)ldb * n_idx);
    EfsArgs a{};
    a.n_atoms = n_idx;
    a.atom_list = idx;
    a.n_types = m->n_types;
    a.max_nbrs = nb->max_nbrs;
    a.r = nb->r.as<double>();
    a.tcnt = nb->tcnt.as<int32_t>();
    a.type = s->type;
    a.r_min = m->r_min;
    a.r_cut = m->r_cut;
    a.th64 = m->theta64.as<double>();
    a.th32 = m->theta32.as<float>();
    a.n_lin = m->basis.n_lin();
    a.brow = m->brow.as<double>();
    a.ldn = n_idx;
    a.ldb = ldb;
    a.grade_mode = g;
    a.colmap = m->colmap.as<int32_t>();
    a.m = mm;
    a.precision = MTP_FP64;
    a.lanes = 4;
    a.lanes_mc = 4;
    a.stream = S(stream);
    m->mbuf.ensure(sizeof(double) * m->basis.n_comp() * (size_t)n_idx);
    m->dmbuf.ensure(sizeof(double) * m->basis.n_comp() * (size_t)n_idx);
    a.mbuf = m->mbuf.ptr;
    a.dmbuf = m->dmbuf.ptr;
    if (const int ngs = staged_graphs(m->level)) {
        const size_t bytes = sizeof(double) * ngs * (size_t)((n_idx + 63) / 64 * 64);
        m->gval.ensure(bytes);
        m->dgval.ensure(bytes);
        a.gval = m->gval.ptr;
        a.dgval = m->dgval.ptr;
    }
    int e = launch_efs(m->level, a);
    MTP_CHECK(e == 0, MTP_E_HIP, std::string("efs kernel launch: ") + hipGetErrorString((hipError_t)e));
    launch_copy_rows(m->brow.as<double>(), n_idx, mm, n_idx, rows, S(stream));
    API_END
}

int mtp_select(const double *gamma, int64_t n, double threshold, int32_t *idx, int32_t capacity, int32_t *count,
               void *stream) {
    API_BEGIN
    MTP_CHECK(gamma && idx && count, MTP_E_INVAL, "NULL argument");
    MTP_CHECK(n >= 0 && capacity >= 0, MTP_E_INVAL, "negative size");
    static thread_local DevBuf work;
    ProfScope ps("select", S(stream));
    launch_select(gamma, n, threshold, idx, capacity, count, S(stream), work);
    API_END
}

int mtp_cut_neighborhood(const mtp_system *s, const double *grades, double cutoff, int32_t capacity, double *pos_out,
                         int32_t *type_out, int32_t *src_out, int32_t *shift_out, int32_t *count, int32_t *center,
                         void *stream) {
    API_BEGIN
    MTP_CHECK(s && grades && count, MTP_E_INVAL, "NULL argument");
    MTP_CHECK(s->n_cfg == 1 && s->n_atoms >= 1, MTP_E_INVAL, "one configuration with at least one atom");
    MTP_CHECK(s->pos && s->type && s->cell, MTP_E_INVAL, "system arrays must not be NULL");
    MTP_CHECK(cutoff > 0 && std::isfinite(cutoff), MTP_E_INVAL, "cutoff must be positive");
    MTP_CHECK(capacity >= 0, MTP_E_INVAL, "negative capacity");
    hipStream_t st = S(stream);
    double H[9];
    uint8_t pb[3] = {1, 1, 1};
    MTP_HIP(hipMemcpyAsync(H, s->cell, sizeof(H), hipMemcpyDeviceToHost, st));
    if (s->pbc) MTP_HIP(hipMemcpyAsync(pb, s->pbc, sizeof(pb), hipMemcpyDeviceToHost, st));
    MTP_HIP(hipStreamSynchronize(st));
    const int per[3] = {pb[0] != 0, pb[1] != 0, pb[2] != 0};
    static thread_local DevBuf keys, idx, work, scal;
    scal.ensure(2 * sizeof(int32_t));
    int32_t *dev = scal.as<int32_t>();   // [0] count, [1] center
    ProfScope ps("cut", st);
    cut_fragment(s->pos, s->type, s->n_atoms, H, per, grades, cutoff, capacity, pos_out, type_out, src_out,
                 shift_out, dev, dev + 1, st, keys, idx, work);
    int32_t h[2] = {0, 0};
    MTP_HIP(hipMemcpyAsync(h, dev, sizeof(h), hipMemcpyDeviceToHost, st));
    MTP_HIP(hipStreamSynchronize(st));
    *count = h[0];
    if (center) *center = h[1];
    API_END
}

namespace mtp {
namespace {
// acceleration of 1 eV/A on 1 amu in A/fs^2: CODATA 2018 elementary charge
// (exact) over the atomic mass constant, m/s^2 -> A/fs^2
constexpr double EV_A_AMU = 1.602176634e-19 / 1e-10 / 1.66053906660e-27 * 1e-20;

void throw_nbr_flags(const int32_t *f, int max_nbrs) {
    MTP_CHECK(!(f[3] & 16), MTP_E_INVAL, "a position is not finite (NaN or Inf)");
    MTP_CHECK(!(f[3] & 1), MTP_E_INVAL, "a cell matrix is singular");
    MTP_CHECK(!(f[3] & 8), MTP_E_INVAL, "an atom type is outside 0..n_types-1");
    MTP_CHECK(!(f[3] & 2), MTP_E_INVAL, "an image shift exceeds +-127 cells (atoms far outside the cell)");
    MTP_CHECK(!f[0], MTP_E_CAPACITY,
              "a neighborhood has " + std::to_string(f[1]) + " atoms, more than max_nbrs = " + std::to_string(max_nbrs));
    MTP_CHECK(!(f[3] & 4), MTP_E_INVAL, "internal: a reverse pair was not found");
    MTP_CHECK(!f[2], MTP_E_OVERLAP, "two atoms are closer than 1e-6 Angstrom");
}
}  // namespace
}  // namespace mtp

int mtp_md_run(const mtp_model *m, const mtp_system *s, mtp_nbrs *nb, int32_t max_nbrs, double *pos, double *vel,
               const double *masses, double dt, int32_t n_steps, mtp_precision p, mtp_grade_mode g,
               double gamma_save, double gamma_break, double *gamma_hist, int32_t *saved, int32_t *n_saved,
               int32_t *steps_done, void *stream) {
    API_BEGIN
    MTP_CHECK(m && s && nb && pos && vel && masses && n_saved && steps_done, MTP_E_INVAL, "NULL argument");
    check_system(m, s);
    MTP_CHECK(s->n_cfg == 1, MTP_E_INVAL, "the MD driver runs one configuration");
    MTP_CHECK(pos == s->pos, MTP_E_INVAL, "pos must be the system's position array");
    MTP_CHECK(g == MTP_GRADE_FULL || g == MTP_GRADE_LINEAR, MTP_E_INVAL, "neighborhood grade mode expected");
    MTP_CHECK(m->act[g].valid, MTP_E_INVAL, "no active set for this grade mode");
    MTP_CHECK(n_steps >= 0 && dt > 0 && std::isfinite(dt), MTP_E_INVAL, "need n_steps >= 0 and dt > 0");
    for (int t = 0; t < m->n_types; ++t) MTP_CHECK(masses[t] > 0, MTP_E_INVAL, "masses must be positive");
    MTP_HIP(hipSetDevice(m->device));
    hipStream_t st = S(stream);
    const int64_t n = s->n_atoms;
    m->md_f.ensure(sizeof(double) * 3 * (size_t)std::max<int64_t>(1, n));
    m->md_g.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, n));
    m->md_invm.ensure(sizeof(double) * m->n_types);
    m->md_scal.ensure(64);
    std::vector<double> invm(m->n_types);
    for (int t = 0; t < m->n_types; ++t) invm[t] = 1.0 / masses[t];
    MTP_HIP(hipMemcpyAsync(m->md_invm.ptr, invm.data(), sizeof(double) * invm.size(), hipMemcpyHostToDevice, st));
    double *F = m->md_f.as<double>(), *gam = m->md_g.as<double>(), *gmax = m->md_scal.as<double>();
    const double h = 0.5 * dt * EV_A_AMU;
    // one step's grading: neighbor lists, forces and grades, gamma(cfg) = max_i gamma_i
    auto grade = [&]() -> double {
        build_neighbors(m, s, max_nbrs, nb, st);
        EvalOut o;
        o.forces = F;
        o.gamma = gam;
        o.mode = g;
        evaluate(m, s, nb, p, o, st);
        launch_argmax(gam, n, gmax, nullptr, st);
        int32_t f[4];
        double gm = 0.0;
        MTP_HIP(hipMemcpyAsync(f, nb->flags.ptr, sizeof(f), hipMemcpyDeviceToHost, st));
        MTP_HIP(hipMemcpyAsync(&gm, gmax, sizeof(double), hipMemcpyDeviceToHost, st));
        MTP_HIP(hipStreamSynchronize(st));
        throw_nbr_flags(f, max_nbrs);
        return gm;
    };
    *n_saved = 0;
    *steps_done = 0;
    auto record = [&](int step, double gm) -> bool {   // false: stop
        if (gamma_hist) gamma_hist[step] = gm;
        if (gm > gamma_break) return false;
        if (gm > gamma_save) {
            if (saved) saved[*n_saved] = step;
            ++*n_saved;
        }
        return true;
    };
    if (n == 0 || !record(0, grade())) return MTP_OK;
    for (int step = 1; step <= n_steps; ++step) {
        launch_md_step(0, n, pos, vel, F, s->type, m->md_invm.as<double>(), h, dt, st);
        if (!record(step, grade())) break;
        launch_md_step(1, n, pos, vel, F, s->type, m->md_invm.as<double>(), h, dt, st);
        *steps_done = step;
    }
    MTP_HIP(hipStreamSynchronize(st));
    API_END
}

int mtp_relax_fire(const mtp_model *m, const mtp_system *s, mtp_nbrs *nb, int32_t max_nbrs, double *pos,
                   const double *masses, double dt0, double dt_max, double fmax, int32_t max_steps, mtp_precision p,
                   mtp_grade_mode g, double gamma_save, double gamma_break, double *gamma_hist, int32_t *saved,
                   int32_t *n_saved, int32_t *steps_done, int32_t *converged, void *stream) {
    API_BEGIN
    MTP_CHECK(m && s && nb && pos && masses && n_saved && steps_done && converged, MTP_E_INVAL, "NULL argument");
    check_system(m, s);
    MTP_CHECK(s->n_cfg == 1, MTP_E_INVAL, "the relaxation runs one configuration");
    MTP_CHECK(pos == s->pos, MTP_E_INVAL, "pos must be the system's position array");
    MTP_CHECK(g == MTP_GRADE_FULL || g == MTP_GRADE_LINEAR, MTP_E_INVAL, "neighborhood grade mode expected");
    MTP_CHECK(m->act[g].valid, MTP_E_INVAL, "no active set for this grade mode");
    MTP_CHECK(max_steps >= 0 && dt0 > 0 && dt_max >= dt0 && std::isfinite(dt_max) && fmax >= 0, MTP_E_INVAL,
              "need max_steps >= 0, 0 < dt0 <= dt_max and fmax >= 0");
    for (int t = 0; t < m->n_types; ++t) MTP_CHECK(masses[t] > 0, MTP_E_INVAL, "masses must be positive");
    MTP_HIP(hipSetDevice(m->device));
    hipStream_t st = S(stream);
    const int64_t n = s->n_atoms;
    m->md_f.ensure(sizeof(double) * 3 * (size_t)std::max<int64_t>(1, n));
    m->md_v.ensure(sizeof(double) * 3 * (size_t)std::max<int64_t>(1, n));
    m->md_g.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, n));
    m->md_invm.ensure(sizeof(double) * m->n_types);
    m->md_scal.ensure(64);
    std::vector<double> invm(m->n_types);
    for (int t = 0; t < m->n_types; ++t) invm[t] = 1.0 / masses[t];
    MTP_HIP(hipMemcpyAsync(m->md_invm.ptr, invm.data(), sizeof(double) * invm.size(), hipMemcpyHostToDevice, st));
    double *F = m->md_f.as<double>(), *v = m->md_v.as<double>(), *gam = m->md_g.as<double>();
    double *scal = m->md_scal.as<double>();   // [0] gamma max, [1..4] FIRE norms
    launch_zero(v, sizeof(double) * 3 * (size_t)std::max<int64_t>(1, n), st);
    double nrm[4] = {0, 0, 0, 0};
    // grading of a configuration: neighbor lists, forces and grades, then
    // gamma(cfg) and the FIRE norms of (F, v) in one read-back
    auto grade = [&]() -> double {
        build_neighbors(m, s, max_nbrs, nb, st);
        EvalOut o;
        o.forces = F;
        o.gamma = gam;
        o.mode = g;
        evaluate(m, s, nb, p, o, st);
        launch_argmax(gam, n, scal, nullptr, st);
        launch_fire_norms(n, F, v, scal + 1, st);
        int32_t f[4];
        double h[5];
        MTP_HIP(hipMemcpyAsync(f, nb->flags.ptr, sizeof(f), hipMemcpyDeviceToHost, st));
        MTP_HIP(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, st));
        MTP_HIP(hipStreamSynchronize(st));
        throw_nbr_flags(f, max_nbrs);
        for (int k = 0; k < 4; ++k) nrm[k] = h[1 + k];
        return h[0];
    };
    *n_saved = 0;
    *steps_done = 0;
    *converged = 0;
    auto record = [&](int step, double gm) -> bool {   // false: stop
        if (gamma_hist) gamma_hist[step] = gm;
        if (gm > gamma_break) return false;
        if (gm > gamma_save) {
            if (saved) saved[*n_saved] = step;
            ++*n_saved;
        }
        return true;
    };
    if (n == 0) {
        *converged = 1;
        return MTP_OK;
    }
    if (!record(0, grade())) return MTP_OK;
    double dt = dt0, alpha = 0.1;
    int n_pos = 0;
    bool stopped = false;
    for (int step = 1; step <= max_steps; ++step) {
        if (std::sqrt(nrm[3]) < fmax) {
            *converged = 1;
            stopped = true;
            break;
        }
        if (nrm[0] > 0) {   // F.v > 0: turn v towards F
            launch_fire_mix(n, v, F, 1.0 - alpha, alpha * std::sqrt(nrm[2]) / std::sqrt(nrm[1]), st);
            if (++n_pos > 5) {
                dt = std::min(1.1 * dt, dt_max);
                alpha *= 0.99;
            }
        } else {
            launch_fire_mix(n, v, F, 0.0, 0.0, st);
            dt *= 0.5;
            alpha = 0.1;
            n_pos = 0;
        }
        launch_md_step(0, n, pos, v, F, s->type, m->md_invm.as<double>(), dt * EV_A_AMU, dt, st);
        if (!record(step, grade())) {
            stopped = true;
            break;
        }
        *steps_done = step;
    }
    if (!stopped) *converged = std::sqrt(nrm[3]) < fmax;
    MTP_HIP(hipStreamSynchronize(st));
    API_END
}

int mtp_fit_bfgs(mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, const double *E_t,
                 const double *F_t, const double *S_t, double w_e, double w_f, double w_s, int32_t max_iter,
                 double gtol, const double *scale, double *loss_hist, int32_t *iters, void *stream) {
    API_BEGIN
    MTP_CHECK(m && s && nb && iters, MTP_E_INVAL, "NULL argument");
    check_system(m, s);
    check_nbrs(m, s, nb);
    MTP_CHECK(p == MTP_FP64 || p == MTP_MIXED, MTP_E_INVAL, "bad precision");
    MTP_CHECK(w_e >= 0 && w_f >= 0 && w_s >= 0, MTP_E_INVAL, "weights must be non-negative");
    MTP_CHECK((w_e == 0 || E_t) && (w_f == 0 || F_t) && (w_s == 0 || S_t), MTP_E_INVAL,
              "a target with a positive weight is NULL");
    MTP_CHECK(max_iter >= 0, MTP_E_INVAL, "negative max_iter");
    MTP_HIP(hipSetDevice(m->device));
    hipStream_t st = S(stream);
    const int64_t nE = s->n_cfg, nF = 3 * s->n_atoms, nS = 9 * (int64_t)s->n_cfg;
    const int nth = m->n_theta;
    m->fit_y.ensure(sizeof(double) * (size_t)(nE + nF + nS));
    m->fit_g.ensure(sizeof(double) * (size_t)(nE + nF + nS));
    m->fit_part.ensure(sizeof(double) * (size_t)((nE + 255) / 256 + (nF + 255) / 256 + (nS + 255) / 256 + 3));
    m->fit_th.ensure(sizeof(double) * nth);
    double *y = m->fit_y.as<double>(), *gy = m->fit_g.as<double>(), *part = m->fit_part.as<double>();
    auto set_theta = [&](const std::vector<double> &th) {
        for (double v : th) MTP_CHECK(std::isfinite(v), MTP_E_INVAL, "theta became NaN or Inf");
        m->theta_host = th;
        choose_gauge(m);
        upload_params(m);
        m->act[MTP_GRADE_FULL].valid = false;   // FULL rows depend on theta
        m->act[MTP_GRADE_FULL_CFG].valid = false;
    };
    // eq. 7 at theta (forward only); leaves dL/dE, dL/dF, dL/dS on the device
    auto loss = [&](const std::vector<double> &th) -> double {
        set_theta(th);
        EvalOut o;
        o.energy = y;
        o.forces = y + nE;
        o.stress = y + nE + nF;
        evaluate(m, s, nb, p, o, st);
        int64_t np = 0;
        const double *tg[3] = {E_t, F_t, S_t};
        const double w[3] = {w_e, w_f, w_s};
        const int64_t off[3] = {0, nE, nE + nF}, len[3] = {nE, nF, nS};
        for (int k = 0; k < 3; ++k) {
            if (w[k] > 0)
                np += launch_fit_residual(len[k], y + off[k], tg[k], w[k], gy + off[k], part + np, st);
            else
                launch_zero(gy + off[k], sizeof(double) * (size_t)len[k], st);
        }
        std::vector<double> h((size_t)np);
        if (np) MTP_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * np, hipMemcpyDeviceToHost, st));
        MTP_HIP(hipStreamSynchronize(st));
        double f = 0.0;
        for (double v : h) f += v;
        return f;
    };
    auto grad = [&]() -> std::vector<double> {   // at the theta of the last loss()
        const int e = mtp_efs_backward(m, s, nb, p, gy, gy + nE, gy + nE + nF, m->fit_th.as<double>(), stream);
        MTP_CHECK(e == MTP_OK, e, std::string("backward: ") + mtp_last_error());
        std::vector<double> g(nth);
        MTP_HIP(hipMemcpyAsync(g.data(), m->fit_th.ptr, sizeof(double) * nth, hipMemcpyDeviceToHost, st));
        MTP_HIP(hipStreamSynchronize(st));
        return g;
    };
    auto dot = [](const std::vector<double> &a, const std::vector<double> &b) {
        double r = 0.0;
        for (size_t k = 0; k < a.size(); ++k) r += a[k] * b[k];
        return r;
    };
    auto amax = [](const std::vector<double> &a) {
        double r = 0.0;
        for (double v : a) r = std::max(r, std::fabs(v));
        return r;
    };
    // BFGS on the inverse Hessian with Armijo backtracking (the steps are
    // described in include/mtp.h)
    std::vector<double> x = m->theta_host;
    double f = loss(x);
    std::vector<double> g = grad();
    if (loss_hist) loss_hist[0] = f;
    std::vector<double> H((size_t)nth * nth, 0.0), d(nth), xn(nth), sv(nth), yv(nth), Hy(nth), D(nth, 1.0);
    if (scale)
        for (int k = 0; k < nth; ++k) {
            MTP_CHECK(scale[k] > 0 && std::isfinite(scale[k]), MTP_E_INVAL, "scale entries must be positive");
            D[k] = scale[k];
        }
    for (int k = 0; k < nth; ++k) H[(size_t)k * nth + k] = D[k] * D[k];
    bool first = true;
    int it = 0;
    for (; it < max_iter; ++it) {
        if (amax(g) <= gtol) break;
        for (int r = 0; r < nth; ++r) {
            double acc = 0.0;
            for (int c = 0; c < nth; ++c) acc += H[(size_t)r * nth + c] * g[c];
            d[r] = -acc;
        }
        const double slope = dot(g, d);
        double t = 1.0, fn = 0.0;
        if (first) {
            double dg = 0.0;
            for (int k = 0; k < nth; ++k) dg = std::max(dg, std::fabs(D[k] * g[k]));
            t = std::min(1.0, 0.1 / dg);
        }
        bool ok = false;
        for (int h = 0; h < 40; ++h) {
            for (int k = 0; k < nth; ++k) xn[k] = x[k] + t * d[k];
            fn = loss(xn);
            if (fn <= f + 1e-4 * t * slope) {
                ok = true;
                break;
            }
            t *= 0.5;
        }
        if (!ok) break;
        std::vector<double> gn = grad();
        for (int k = 0; k < nth; ++k) {
            sv[k] = xn[k] - x[k];
            yv[k] = gn[k] - g[k];
        }
        const double ys = dot(yv, sv);
        if (ys > 0) {
            auto hy = [&]() {
                for (int r = 0; r < nth; ++r) {
                    double acc = 0.0;
                    for (int c = 0; c < nth; ++c) acc += H[(size_t)r * nth + c] * yv[c];
                    Hy[r] = acc;
                }
            };
            hy();
            if (first) {   // the initial inverse Hessian rescaled by y.s / y.H.y
                const double sc = ys / dot(yv, Hy);
                for (double &v : H) v *= sc;
                hy();
            }
            // H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T
            //    = H - rho (s (H y)^T + (H y) s^T) + (rho^2 y.H.y + rho) s s^T   (H symmetric)
            const double rho = 1.0 / ys;
            const double yHy = dot(yv, Hy);
            const double cs = rho * rho * yHy + rho;
            for (int r = 0; r < nth; ++r)
                for (int c = 0; c < nth; ++c)
                    H[(size_t)r * nth + c] += cs * sv[r] * sv[c] - rho * (sv[r] * Hy[c] + Hy[r] * sv[c]);
            first = false;
        }
        x = xn;
        f = fn;
        g = gn;
        if (loss_hist) loss_hist[it + 1] = f;
    }
    // the model keeps the last accepted theta
    if (m->theta_host != x) set_theta(x);
    *iters = it;
    API_END
}

int mtp_maxvol_update(mtp_model *m, mtp_grade_mode g, double *cand, int64_t n_cand, double threshold,
                      int32_t max_swaps, int32_t *swap_cand, int32_t *swap_col, int32_t *n_swaps, void *stream) {
    API_BEGIN
    MTP_CHECK(m && n_swaps, MTP_E_INVAL, "NULL argument");
    MTP_CHECK(g >= MTP_GRADE_FULL && g <= MTP_GRADE_LINEAR_CFG, MTP_E_INVAL, "bad grade mode");
    MTP_CHECK(threshold > 1.0, MTP_E_INVAL, "threshold must exceed 1");
    MTP_CHECK(n_cand >= 0 && max_swaps >= 0, MTP_E_INVAL, "negative size");
    MTP_CHECK(n_cand == 0 || cand, MTP_E_INVAL, "cand is NULL");
    MTP_CHECK(max_swaps == 0 || (swap_cand && swap_col), MTP_E_INVAL, "swap log is NULL");
    ActiveSet &as = m->act[g];
    MTP_CHECK(as.valid, MTP_E_INVAL, "no active set for this mode");
    MTP_HIP(hipSetDevice(m->device));
    *n_swaps = 0;
    if (n_cand == 0 || max_swaps == 0) return MTP_OK;
    {
        ProfScope ps("maxvol", S(stream));
        run_maxvol(as, cand, n_cand, threshold, max_swaps, swap_cand, swap_col, n_swaps, S(stream), m->work);
    }
    API_END
}

int mtp_efs_backward(const mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, const double *gE,
                     const double *gF, const double *gS, double *g_theta, void *stream) {
    API_BEGIN
    MTP_CHECK(m && g_theta, MTP_E_INVAL, "NULL argument");
    check_system(m, s);
    check_nbrs(m, s, nb);
    MTP_CHECK(p == MTP_FP64 || p == MTP_MIXED, MTP_E_INVAL, "bad precision");
    MTP_CHECK(!staged_graphs(m->level), MTP_E_UNSUPPORTED,
              "level " + std::to_string(m->level) + " is compiled as a staged program, which evaluates energies, "
              "forces, stresses and rows; its backward pass is not built");
    MTP_HIP(hipSetDevice(m->device));
    hipStream_t st = S(stream);
    const int64_t n = s->n_atoms;
    if (n == 0) {
        launch_zero(g_theta, sizeof(double) * m->n_theta, st);
        return MTP_OK;
    }
    const size_t tsz = p == MTP_FP64 ? sizeof(double) : sizeof(float);
    const size_t nc = m->basis.n_comp();
    m->mbuf.ensure(tsz * nc * n);
    m->dmbuf.ensure(tsz * nc * n);
    m->tbuf.ensure(tsz * nc * n);
    m->dtbuf.ensure(tsz * nc * n);
    m->rows.ensure(tsz * (size_t)m->n_theta * n);
    BwdArgs b{};
    EfsArgs &a = b.e;
    a.n_atoms = n;
    a.atom_list = nullptr;
    a.n_types = m->n_types;
    a.max_nbrs = nb->max_nbrs;
    a.r = nb->r.as<double>();
    a.tcnt = nb->tcnt.as<int32_t>();
    a.type = s->type;
    a.r_min = m->r_min;
    a.r_cut = m->r_cut;
    a.th64 = m->theta64.as<double>();
    a.th32 = m->theta32.as<float>();
    a.n_lin = m->basis.n_lin();
    a.precision = p;
    a.lanes = 4;
    a.lanes_mc = 4;
    a.stream = st;
    a.mbuf = m->mbuf.ptr;
    a.dmbuf = m->dmbuf.ptr;
    b.gE = gE;
    b.gF = gF;
    b.gS = gS;
    b.atom_cfg = nb->atom_cfg.as<int32_t>();
    b.nbr_j = nb->j.as<int32_t>();
    b.tbuf = m->tbuf.ptr;
    b.dtbuf = m->dtbuf.ptr;
    b.rows = m->rows.ptr;
    b.n_theta = m->n_theta;
    int e;
    {
        ProfScope ps("backward", st);
        e = launch_backward(m->level, b);
    }
    MTP_CHECK(e == 0, MTP_E_HIP, std::string("backward kernel launch: ") + hipGetErrorString((hipError_t)e));
    {
        ProfScope ps("backward_sum", st);
        launch_column_sums(m->rows.ptr, p, n, m->n_theta, g_theta, st, m->sums);
    }
    MTP_HIP(hipGetLastError());
    API_END
}

int mtp_tune(mtp_model *m, const mtp_system *s, const mtp_nbrs *nb, mtp_precision p, mtp_grade_mode g,
             int32_t *lanes_out, int32_t *grade_out, void *stream) {
    API_BEGIN
    MTP_CHECK(m && lanes_out, MTP_E_INVAL, "NULL argument");
    check_system(m, s);
    check_nbrs(m, s, nb);
    MTP_CHECK(p == MTP_FP64 || p == MTP_MIXED, MTP_E_INVAL, "bad precision");
    MTP_CHECK(g == MTP_GRADE_FULL || g == MTP_GRADE_LINEAR, MTP_E_INVAL, "bad grade mode");
    MTP_HIP(hipSetDevice(m->device));
    hipStream_t st = S(stream);
    const int64_t n = s->n_atoms;
    DevBuf out;
    out.ensure(sizeof(double) * (3 * (size_t)n + 2 * (size_t)n + 10 * (size_t)s->n_cfg + 16));
    double *base = out.as<double>();
    EvalOut o;
    o.energy = base;
    o.stress = base + s->n_cfg;
    o.forces = base + 10 * (size_t)s->n_cfg;
    o.site_e = o.forces + 3 * (size_t)n;
    if (m->act[g].valid) o.gamma = o.site_e + n;
    o.mode = g;
    hipEvent_t e0, e1;
    MTP_HIP(hipEventCreate(&e0));
    MTP_HIP(hipEventCreate(&e1));
    // Schedules whose times differ by a few percent are told apart by
    // interleaved rounds (clock and cache drift hit every schedule alike) and
    // the minimum of each schedule over the rounds (a stray slow round is
    // dropped); ties go to the earlier schedule of the list.
    constexpr int SCHED[9] = {17 * 2, 17 * 4, 17 * 8, 16 * 4 + 2, 16 * 4 + 8, 16 * 2 + 4, 16 * 8 + 4, 16 * 2 + 8,
                              16 * 8 + 2};
    constexpr int ROUNDS = 5, REPS = 3;
    float tmin[9];
    int best = 0;
    try {
        for (int k = 0; k < 9; ++k) {   // warm-up (workspaces, caches)
            m->force_lanes = SCHED[k];
            evaluate(m, s, nb, p, o, st);
        }
        for (int rd = 0; rd < ROUNDS; ++rd)
            for (int k = 0; k < 9; ++k) {
                m->force_lanes = SCHED[k];
                MTP_HIP(hipEventRecord(e0, st));
                for (int r = 0; r < REPS; ++r) evaluate(m, s, nb, p, o, st);
                MTP_HIP(hipEventRecord(e1, st));
                MTP_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                MTP_HIP(hipEventElapsedTime(&ms, e0, e1));
                tmin[k] = rd == 0 ? ms : std::min(tmin[k], ms);
            }
        for (int k = 1; k < 9; ++k)
            if (tmin[k] < tmin[best]) best = k;
        best = SCHED[best];
    } catch (...) {
        m->force_lanes = 0;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    m->force_lanes = 0;
    m->tuned_lanes[p == MTP_FP64 ? 0 : 1][size_bucket(n)] = best;
    // the grade's kernel form: each form's launch alone, on the rows the
    // evaluations above left in the model's row buffer, with the
    // preselection count the evaluation asks of it (the forms differ by about
    // a microsecond, within the spread of whole evaluations)
    int gbest = GRADE_AUTO;
    if (o.gamma) {
        std::vector<int> cand;
        for (int sc : {GRADE_F64_REG, GRADE_F64_LDS, GRADE_I8, GRADE_F64_PAIR, GRADE_F64_KOUTER, GRADE_F64_KOUTER2})
            if (grade_sched_valid(m->act[g], p, sc)) cand.push_back(sc);
        std::vector<float> gmin(cand.size());
        const int ldb = ld_of(m->m_of(g), p);
        const double *rows = m->brow.as<double>();
        int cr = GRADE_ROWS;   // the finest preselection count among the forms
        for (int sc : cand) cr = std::min(cr, grade_count_rows(m->act[g], p, sc));
        DevBuf blk;
        blk.ensure(sizeof(int32_t) * (size_t)((n + cr - 1) / cr + 1));
        constexpr int GREPS = 10;
        try {
            for (int sc : cand)
                launch_grade(m->act[g], p, rows, ldb, n, n, o.gamma, nullptr, st, 2.0, blk.as<int32_t>(), sc);
            for (int rd = 0; rd < ROUNDS; ++rd)
                for (size_t k = 0; k < cand.size(); ++k) {
                    MTP_HIP(hipEventRecord(e0, st));
                    for (int r = 0; r < GREPS; ++r)
                        launch_grade(m->act[g], p, rows, ldb, n, n, o.gamma, nullptr, st, 2.0, blk.as<int32_t>(),
                                     cand[k]);
                    MTP_HIP(hipEventRecord(e1, st));
                    MTP_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    MTP_HIP(hipEventElapsedTime(&ms, e0, e1));
                    gmin[k] = rd == 0 ? ms : std::min(gmin[k], ms);
                }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            throw;
        }
        size_t kb = 0;
        for (size_t k = 1; k < cand.size(); ++k)
            if (gmin[k] < gmin[kb]) kb = k;
        gbest = cand[kb];
        m->tuned_grade[p == MTP_FP64 ? 0 : 1][g][size_bucket(n)] = gbest;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *lanes_out = best;
    if (grade_out) *grade_out = gbest;
    API_END
}

int mtp_mfma_rate(int kind, int32_t iters, double *tflops, void *stream) {
    API_BEGIN
    MTP_CHECK(tflops, MTP_E_INVAL, "NULL argument");
    *tflops = mfma_rate(kind, iters, S(stream));
    API_END
}

int mtp_basis_describe(int32_t level, char *buf, size_t len, int32_t *n_lin) {
    API_BEGIN
    Basis b = build_basis(level);
    std::string d = b.describe();
    if (n_lin) *n_lin = b.n_lin();
    if (buf && len) {
        const size_t k = std::min(len - 1, d.size());
        std::memcpy(buf, d.data(), k);
        buf[k] = 0;
        MTP_CHECK(d.size() < len, MTP_E_INVAL, "buffer too small: need " + std::to_string(d.size() + 1));
    }
    API_END
}

int mtp_compiled_levels(int32_t *levels, int32_t cap) {
    auto lv = compiled_levels();
    for (int k = 0; k < (int)lv.size() && k < cap; ++k) levels[k] = lv[k];
    return (int)lv.size();
}

}  // extern "C"
