// Host runtime behind the tdks C ABI (include/tdks.h): instance set-up (geometry,
// local potential, projector support tables, k tables), device layout, work lists,
// per-step HIP graphs, and read-out.
//
// Set-up arithmetic follows the model stated in tdks.h: grid r(i) = sum_d (i_d/N_d) a_d,
// reciprocal rows b_d with a_d . b_e = 2 pi delta_de, gradient = sum_d c_d d/ds_d with
// c_d = N_d b_d / (2 pi), metric g_de = c_d . c_e; Gaussian local potential summed over all
// lattice images within 15 widths; s + p Kleinman-Bylander projectors
// f_s = N_s g, f_p = N_p d g, g = max(0, exp(-d^2/2rc^2) - exp(-Rc^2/2rc^2)).
#include "tdks_internal.h"

#include "../../include/tdks.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace tdks;

// Partial sums of the allocation-free step (tdks_step_noalloc): a static device array instead
// of the context's buffers.  Every GPU the library runs on holds its own copy until the process
// ends.  In host code the name is only a stand-in: the device address comes from
// hipGetSymbolAddress (scratch_address below), once per device.
constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

// device address of the static scratch array on device dev (the current device), resolved
// with hipGetSymbolAddress the first time a context is created on that device
int scratch_address(int dev, void **out);

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
bool g_scratch_set[kMaxDevices];

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(TDKS_E_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                              \
    } while (0)

int scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(TDKS_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_set[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(TDKS_E_HIP, "hipGetSymbolAddress of the scratch array failed on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
        g_scratch_set[dev] = true;
    }
    *out = g_scratch_ptr[dev];
    return TDKS_OK;
}

struct TableSet {
    std::vector<int> col_atom, col_j01;
    std::vector<uint32_t> pt_pack;
    std::vector<double> pt_g;
    std::vector<float> pt_gf;
    std::vector<int> pt_ptr, atom_task;
    std::vector<uint32_t> chunk_pack;
    std::vector<double> chunk_g;   // [nchunk][4]
    std::vector<float> chunk_gf;
    std::vector<int> atom_chunk;   // [nat+1] first chunk of each atom
    std::vector<uint16_t> pt_ptr16;
    std::vector<uint32_t> pt_rec32;  // interleaved FP32 entry records (words)
    std::vector<int2> task;
    std::vector<double> atom_tau, atom_par;
    int nat = 0;
    int cls = -1;
    // sum over atoms of |E_s| ||f_s||^2 + |E_p| sum_i ||f_p,i||^2 (with |d| <= Rc): a bound of
    // the operator norm of V_NL (each channel is the rank-one E |P><P|)
    double nl_bound = 0.0;
    // device copies
    int *d_col_atom = nullptr, *d_col_j01 = nullptr;
    uint32_t *d_pt_pack = nullptr;
    double *d_pt_g = nullptr, *d_atom_tau = nullptr, *d_atom_par = nullptr;
    float *d_pt_gf = nullptr;
    int *d_pt_ptr = nullptr, *d_atom_task = nullptr;
    uint16_t *d_pt_ptr16 = nullptr;
    uint32_t *d_pt_rec = nullptr;
    uint32_t *d_chunk_pack = nullptr;
    double *d_chunk_g = nullptr;
    float *d_chunk_gf = nullptr;
    int2 *d_task = nullptr;
};

struct InstHost {
    int N[3];
    int ng;
    int nk, nb, nat;
    int group;
    bool nonorth;
    double lat[3][3], B[3][3], c[3][3], g[3][3], hv[3][3];
    double omega, dV;
    std::vector<double> kcart, kw, occ, vloc, vhxc_frozen;
    // |lambda| bound of h_kappa for the health check: lam0 + |A| lamA + |A|^2 / 2
    double lam0 = 0.0, lamA = 0.0;
    int table = -1;
    int cls = -1;
    int wbeg = 0, wend = 0;  // work items (global indices) of this instance
    int nslot = 0;
    size_t norm0_off = 0;    // first of this instance's reference norms in d_norm0
    void *d_u = nullptr;
    double *d_kcart = nullptr, *d_kw = nullptr, *d_occ = nullptr;
    double *d_rho_part = nullptr, *d_j_part = nullptr;
    bool loaded = false;
};

struct ShapeClass {
    int N[3];
    bool nonorth;
    int zl = 0, block = 0, minw = 0, sl = 0, rho_lds = 0, ragged = 0, mixt = 0;
    int gc = 0;                 // FP64 column tables in global memory (grids beyond the LDS otherwise)
    int ptpl = 0;               // no LDS records: the CSR pointers alone staged in LDS
    char *gcol = nullptr;       // their buffer, one slice of gstride bytes per work item of the class
    size_t gstride = 0;
    int wbeg = 0, wend = 0;
    int ng_max = 0, ncol_max = 0, nent_max = 0, nmaxd = 0, nat_max = 0, ntask_max = 0;
};

}  // namespace

struct tdks_ctx {
    tdks_options opt;
    int fp64 = 1;
    int device = 0;
    // allocation-free step: the device address of the static scratch array, the bytes this
    // context's partial sums need there, and the instance table pointing into it
    void *scratch = nullptr;
    size_t scratch_need = 0;
    DevInst *d_insts_scr = nullptr;
    bool noalloc_steps = false;  // steps since the load whose currents went to a caller's buffer
    int n_inst = 0;
    std::vector<InstHost> inst;
    std::vector<TableSet> tables;
    std::vector<ShapeClass> classes;
    std::vector<WorkItem> work;
    std::vector<int> groups;  // sorted distinct group ids
    int ng_max = 0;
    hipStream_t stream = nullptr;
    hipStream_t caller = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_acopy = nullptr;
    // with several shape classes: side streams (default priority) that the classes after the
    // first run on, forked from and joined back to `stream` every time
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev_join;
    hipEvent_t ev_fork = nullptr;
    std::vector<int> class_order;  // launch order: the class with the longest work items first
    // device buffers
    DevInst *d_insts = nullptr;
    WorkItem *d_work = nullptr;
    double *d_rho = nullptr, *d_vloc = nullptr, *d_vhxc = nullptr;
    double *d_vhxc_pred = nullptr;  // predictor-corrector: v_Hxc of the predicted density
    void *d_vtot = nullptr;
    double *d_trace = nullptr;
    size_t trace_cap = 0;  // records per instance
    double *d_A = nullptr;
    size_t A_cap = 0;
    double *h_A = nullptr;  // pinned staging
    int *d_ctrs = nullptr;  // [0] A row, [1] steps since the load, [2] always 0
    int rstride = 1;        // a current is recorded every rstride-th step
    // numeric health check (per instance): charge at load, accumulated log of the per-step norm
    // bound, first violation; per-step log bound per A row (host staging + device copy); norms
    // of every orbital at load when the per-orbital check is on
    double *d_q0 = nullptr, *d_lcum = nullptr;
    unsigned long long *d_health = nullptr, *h_health = nullptr;
    hipEvent_t ev_health = nullptr;
    bool health_pending = false;
    double *d_logF = nullptr, *h_logF = nullptr;
    double *d_norm0 = nullptr;
    double *d_jpre = nullptr, *d_jobs = nullptr, *d_Aobs = nullptr;
    std::vector<double> jpre;
    // ground-state preparation (allocated on first use): input density of the mixing,
    // residual per instance, (instance, k) list of the orthonormalisation, status flag
    double *d_rho_in = nullptr, *d_resid = nullptr;
    int2 *d_pairs = nullptr;
    int n_pairs = 0;
    int *d_status = nullptr;
    double *d_rho_k = nullptr;   // ground state: per-(instance, k) density partials [n_pairs][ng_max]
    int *d_pair_first = nullptr; // first pair of each instance [n_inst + 1]
    int steps_done = 0;
    hipGraphExec_t g_chunk = nullptr, g_one = nullptr;
    int chunk = 16;
    std::vector<void *> allocs;

    void *alloc(size_t bytes) {
        if (bytes == 0) bytes = 16;
        void *p = nullptr;
        if (opt.alloc) {
            p = opt.alloc(bytes, opt.alloc_user);
        } else if (hipMalloc(&p, bytes) != hipSuccess) {
            p = nullptr;
        }
        if (p) allocs.push_back(p);
        return p;
    }
    void release(void *p) {
        if (!p) return;
        auto it = std::find(allocs.begin(), allocs.end(), p);
        if (it != allocs.end()) allocs.erase(it);
        if (opt.free)
            opt.free(p, opt.alloc_user);
        else
            (void)hipFree(p);
    }
    HealthArgs health(bool check) const {
        HealthArgs h;
        h.q0 = d_q0;
        h.lcum = d_lcum;
        h.logF = d_logF;
        h.arow = d_ctrs;
        h.health = check ? d_health : nullptr;
        h.set_ref = 0;
        h.rstride = rstride;
        h.row_ctr = nullptr;
        h.logF_floor = std::log(0.25);
        h.tol = fp64 ? 1e-9 : 1e-4;
        return h;
    }
    void drop_graphs() {
        if (g_chunk) (void)hipGraphExecDestroy(g_chunk);
        if (g_one) (void)hipGraphExecDestroy(g_one);
        g_chunk = g_one = nullptr;
    }
};

namespace {

void inv3(const double a[3][3], double out[3][3], double &det) {
    det = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) -
          a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
          a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
    const double id = 1.0 / det;
    out[0][0] = (a[1][1] * a[2][2] - a[1][2] * a[2][1]) * id;
    out[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) * id;
    out[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) * id;
    out[1][0] = (a[1][2] * a[2][0] - a[1][0] * a[2][2]) * id;
    out[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) * id;
    out[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) * id;
    out[2][0] = (a[1][0] * a[2][1] - a[1][1] * a[2][0]) * id;
    out[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) * id;
    out[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) * id;
}

const double kPi = 3.14159265358979323846;

// grid point r(i) = sum_d (i_d / N_d) a_d for flat index p = i0 + N0 (i1 + N1 i2)
void point(const InstHost &I, int p, double r[3]) {
    const int i0 = p % I.N[0], i1 = (p / I.N[0]) % I.N[1], i2 = p / (I.N[0] * I.N[1]);
    for (int q = 0; q < 3; ++q)
        r[q] = double(i0) / I.N[0] * I.lat[0][q] + double(i1) / I.N[1] * I.lat[1][q] +
               double(i2) / I.N[2] * I.lat[2][q];
}

int build_geometry(InstHost &I, const tdks_instance_desc &d) {
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) I.lat[a][b] = d.lattice[a][b];
    for (int q = 0; q < 3; ++q) I.N[q] = d.grid[q];
    for (int q = 0; q < 3; ++q)
        if (I.N[q] < 4 || I.N[q] > kMaxGridDim)
            return fail(TDKS_E_UNSUPPORTED, "grid dimension %d = %d outside [4, %d]", q, I.N[q], kMaxGridDim);
    I.ng = I.N[0] * I.N[1] * I.N[2];
    if (I.ng > kMaxPoints) return fail(TDKS_E_UNSUPPORTED, "grid of %d points exceeds %d", I.ng, kMaxPoints);
    double inv[3][3], det;
    inv3(I.lat, inv, det);
    if (!(std::fabs(det) > 1e-12)) return fail(TDKS_E_ARG, "singular lattice");
    I.omega = std::fabs(det);
    I.dV = I.omega / I.ng;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) I.B[a][b] = 2.0 * kPi * inv[b][a];  // rows b_a
    for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 3; ++q) {
            I.c[a][q] = I.N[a] * I.B[a][q] / (2.0 * kPi);
            I.hv[a][q] = I.lat[a][q] / I.N[a];
        }
    I.nonorth = false;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            I.g[a][b] = I.c[a][0] * I.c[b][0] + I.c[a][1] * I.c[b][1] + I.c[a][2] * I.c[b][2];
            if (a != b && I.g[a][b] != 0.0) I.nonorth = true;
        }
    return TDKS_OK;
}

int build_potential_and_tables(InstHost &I, const tdks_instance_desc &d, TableSet &T) {
    const int nat = d.n_atoms;
    T.nat = nat;
    T.atom_tau.assign(3 * nat, 0.0);
    T.atom_par.assign(4 * nat, 0.0);
    for (int a = 0; a < nat; ++a) {
        for (int q = 0; q < 3; ++q)
            T.atom_tau[3 * a + q] = d.atom_frac[3 * a + 0] * I.lat[0][q] +
                                    d.atom_frac[3 * a + 1] * I.lat[1][q] +
                                    d.atom_frac[3 * a + 2] * I.lat[2][q];
        const tdks_species &sp = d.species[d.atom_species[a]];
        T.atom_par[4 * a + 0] = sp.Es;
        T.atom_par[4 * a + 1] = sp.Ep;
        T.atom_par[4 * a + 2] = std::pow(std::pow(kPi, 1.5) * sp.rc * sp.rc * sp.rc, -0.5);
        T.atom_par[4 * a + 3] = std::pow(std::pow(kPi, 1.5) * std::pow(sp.rc, 5) / 2.0, -0.5);
    }
    // local potential: every image within 15 widths
    I.vloc.assign(I.ng, 0.0);
    std::vector<double> r(3 * I.ng);
    for (int p = 0; p < I.ng; ++p) point(I, p, &r[3 * p]);
    for (int a = 0; a < nat; ++a) {
        const tdks_species &sp = d.species[d.atom_species[a]];
        const double rcut = 15.0 * sp.w;
        int nmax[3];
        for (int q = 0; q < 3; ++q) {
            const double bn = std::sqrt(I.B[q][0] * I.B[q][0] + I.B[q][1] * I.B[q][1] + I.B[q][2] * I.B[q][2]);
            nmax[q] = int(std::ceil(rcut * bn / (2.0 * kPi))) + 1;
        }
        const double inv2w2 = 1.0 / (2.0 * sp.w * sp.w);
        for (int n0 = -nmax[0]; n0 <= nmax[0]; ++n0)
            for (int n1 = -nmax[1]; n1 <= nmax[1]; ++n1)
                for (int n2 = -nmax[2]; n2 <= nmax[2]; ++n2) {
                    double c[3];
                    for (int q = 0; q < 3; ++q)
                        c[q] = T.atom_tau[3 * a + q] + n0 * I.lat[0][q] + n1 * I.lat[1][q] + n2 * I.lat[2][q];
                    for (int p = 0; p < I.ng; ++p) {
                        const double x = r[3 * p] - c[0], y = r[3 * p + 1] - c[1], z = r[3 * p + 2] - c[2];
                        const double d2 = x * x + y * y + z * z;
                        if (d2 < rcut * rcut) I.vloc[p] += sp.D * std::exp(-d2 * inv2w2);
                    }
                }
    }
    // projector support: points within Rc of exactly one image of each atom, grouped by
    // column image (atom, unwrapped j0, j1) and ordered by (column image, j2)
    struct Ent { int col; int j2u; int p; double g; };
    std::vector<Ent> ents;
    T.col_atom.clear();
    T.col_j01.clear();
    T.chunk_pack.clear();
    T.chunk_g.clear();
    T.atom_chunk.clear();
    for (int a = 0; a < nat; ++a) {
        const tdks_species &sp = d.species[d.atom_species[a]];
        if (!(sp.Rc > 0.0) || !(sp.rc > 0.0)) return fail(TDKS_E_ARG, "species radii must be positive");
        const double gcut = std::exp(-sp.Rc * sp.Rc / (2.0 * sp.rc * sp.rc));
        double sg2 = 0.0;  // sum of g^2 over the support
        std::vector<int> hits(I.ng, 0);
        std::map<int, std::vector<std::pair<int, std::pair<int, double>>>> bycol;  // j01 -> (j2u, (p, g))
        for (int n0 = -2; n0 <= 2; ++n0)
            for (int n1 = -2; n1 <= 2; ++n1)
                for (int n2 = -2; n2 <= 2; ++n2) {
                    double c[3];
                    for (int q = 0; q < 3; ++q)
                        c[q] = T.atom_tau[3 * a + q] + n0 * I.lat[0][q] + n1 * I.lat[1][q] + n2 * I.lat[2][q];
                    for (int p = 0; p < I.ng; ++p) {
                        const double x = r[3 * p] - c[0], y = r[3 * p + 1] - c[1], z = r[3 * p + 2] - c[2];
                        const double d2 = x * x + y * y + z * z;
                        if (!(d2 < sp.Rc * sp.Rc)) continue;
                        if (++hits[p] > 1)
                            return fail(TDKS_E_ARG, "atom %d: projector radius %.3f reaches two images of the "
                                        "same atom (must be below half the shortest lattice translation)", a, sp.Rc);
                        const int i0 = p % I.N[0], i1 = (p / I.N[0]) % I.N[1], i2 = p / (I.N[0] * I.N[1]);
                        const int u0 = i0 - n0 * I.N[0] + I.N[0], u1 = i1 - n1 * I.N[1] + I.N[1];
                        const int u2 = i2 - n2 * I.N[2] + I.N[2];
                        if (u0 < 0 || u0 >= 3 * I.N[0] || u1 < 0 || u1 >= 3 * I.N[1] || u2 < 0 || u2 >= 3 * I.N[2])
                            return fail(TDKS_E_ARG, "atom %d: projector support outside the neighbouring cells", a);
                        const double g = std::max(0.0, std::exp(-d2 / (2.0 * sp.rc * sp.rc)) - gcut);
                        sg2 += g * g;
                        bycol[u0 | (u1 << 8)].push_back({u2, {p, g}});
                    }
                }
        if (bycol.empty()) return fail(TDKS_E_ARG, "atom %d has no projector support points", a);
        {
            const double ns = T.atom_par[4 * a + 2], np = T.atom_par[4 * a + 3];
            T.nl_bound += (std::fabs(sp.Es) * ns * ns + std::fabs(sp.Ep) * np * np * sp.Rc * sp.Rc) * sg2 * I.dV;
        }
        // reference step r of each column image: the a_3 offset that brings its points
        // closest to the atom (d_ref = dcol + r a_3/N3); entries store j2 - r, so that
        // every offset the kernels form from tables stays small
        std::map<int, int> colref;
        {
            const double *h2 = I.hv[2];
            const double hh = h2[0] * h2[0] + h2[1] * h2[1] + h2[2] * h2[2];
            for (auto &kv : bycol) {
                const double j0 = double((kv.first & 255) - I.N[0]), j1 = double((kv.first >> 8) - I.N[1]);
                double dd = 0.0;
                for (int q = 0; q < 3; ++q)
                    dd += (j0 * I.hv[0][q] + j1 * I.hv[1][q] - T.atom_tau[3 * a + q]) * h2[q];
                const int r = int(std::lround(-dd / hh));
                if (r < -127 || r > 127) return fail(TDKS_E_UNSUPPORTED, "atom %d: column reference out of range", a);
                colref[kv.first] = r;
                for (auto &e : kv.second) {
                    const int f = e.first - r;  // (j2 - r) + N3 with j2 = u2 - N3; stored + 3
                    if (f < 0 || f >= 2 * I.N[2])
                        return fail(TDKS_E_ARG, "atom %d: projector support spans more than the cell along a_3", a);
                }
            }
        }
        // chunks of this atom: runs of up to 4 consecutive j2 on one column image, cut where
        // the grid index wraps; ordered by (first j2, j1, j0) so that the lanes of a wave
        // start on neighbouring grid points
        T.atom_chunk.push_back(int(T.chunk_pack.size()));
        {
            struct Ch { long long key; uint32_t pack; double g[4]; };
            std::vector<Ch> chs;
            int col = int(T.col_atom.size());
            for (auto &kv : bycol) {
                auto pts = kv.second;
                std::sort(pts.begin(), pts.end(), [](const std::pair<int, std::pair<int, double>> &x,
                                                     const std::pair<int, std::pair<int, double>> &y) {
                    return x.first < y.first;
                });
                size_t i = 0;
                while (i < pts.size()) {
                    Ch c{};
                    const int u2 = pts[i].first, p = pts[i].second.first;
                    c.key = (static_cast<long long>(u2) << 16) | ((kv.first >> 8) << 8) | (kv.first & 255);
                    double g[4] = {0.0, 0.0, 0.0, 0.0};
                    int n = 0;
                    while (n < 4 && i < pts.size() && pts[i].first == u2 + n &&
                           (n == 0 || pts[i].second.first == p + n * I.N[0] * I.N[1])) {
                        g[n] = pts[i].second.second;
                        ++n;
                        ++i;
                    }
                    // a chunk reads 4 consecutive grid planes: one that would run past the last
                    // plane starts lower, with g = 0 on the points ahead of its own
                    const int plane = I.N[0] * I.N[1];
                    const int sh = std::max(0, p / plane + 4 - I.N[2]);
                    for (int q = 0; q < 4; ++q) c.g[q] = (q >= sh) ? g[q - sh] : 0.0;
                    c.pack = uint32_t(p - sh * plane) | (uint32_t(u2 - sh - colref[kv.first] + 3) << 13) |
                             (uint32_t(col) << 20);
                    chs.push_back(c);
                }
                ++col;
            }
            std::sort(chs.begin(), chs.end(), [](const Ch &x, const Ch &y) { return x.key < y.key; });
            for (const Ch &c : chs) {
                T.chunk_pack.push_back(c.pack);
                for (int q = 0; q < 4; ++q) T.chunk_g.push_back(c.g[q]);
            }
        }
        // entries of one atom in plane-major order (j2, then j1, j0): lanes that walk
        // consecutive entries read consecutive grid points, i.e. distinct LDS banks
        std::vector<std::pair<long long, Ent>> order;
        for (auto &kv : bycol) {
            const int col = int(T.col_atom.size());
            T.col_atom.push_back(a);
            T.col_j01.push_back(kv.first | ((colref[kv.first] + 128) << 16));
            for (auto &e : kv.second) {
                const long long key = (static_cast<long long>(e.first) << 16) | ((kv.first >> 8) << 8) | (kv.first & 255);
                order.push_back({key, Ent{col, e.first - colref[kv.first] + 3, e.second.first, e.second.second}});
            }
        }
        std::sort(order.begin(), order.end(), [](const std::pair<long long, Ent> &x,
                                                 const std::pair<long long, Ent> &y) { return x.first < y.first; });
        for (auto &o : order) ents.push_back(o.second);
    }
    T.atom_chunk.push_back(int(T.chunk_pack.size()));
    T.chunk_gf.assign(T.chunk_g.begin(), T.chunk_g.end());
    if (T.col_atom.size() >= 4096)
        return fail(TDKS_E_UNSUPPORTED, "%zu projector column images exceed 4095", T.col_atom.size());
    std::vector<std::vector<std::pair<uint32_t, double>>> per_point(I.ng);
    for (const Ent &e : ents) {
        const uint32_t pack = uint32_t(e.col) | (uint32_t(e.j2u) << 16);  // scatter: column image, a_3 step
        per_point[e.p].push_back({pack, e.g});
    }
    T.pt_ptr.assign(I.ng + 1, 0);
    T.pt_pack.clear();
    T.pt_g.clear();
    for (int p = 0; p < I.ng; ++p) {
        T.pt_ptr[p] = int(T.pt_pack.size());
        for (auto &e : per_point[p]) {
            T.pt_pack.push_back(e.first);
            T.pt_g.push_back(e.second);
        }
    }
    T.pt_ptr[I.ng] = int(T.pt_pack.size());
    if (T.pt_pack.size() > 65535) return fail(TDKS_E_UNSUPPORTED, "more than 65535 projector entries");
    T.pt_ptr16.assign(T.pt_ptr.begin(), T.pt_ptr.end());
    T.pt_gf.assign(T.pt_g.begin(), T.pt_g.end());
    // records for the FP32 scatter from global memory: {byte offset of the column image's 16-byte
    // coefficients | a_3 step << 16, g}
    T.pt_rec32.resize(2 * T.pt_pack.size());
    for (size_t e = 0; e < T.pt_pack.size(); ++e) {
        const uint32_t pk = T.pt_pack[e];
        const float gf = float(T.pt_g[e]);
        uint32_t gb;
        std::memcpy(&gb, &gf, 4);
        T.pt_rec32[2 * e] = ((pk & 0xffffu) * 16u) | (pk & 0xffff0000u);
        T.pt_rec32[2 * e + 1] = gb;
    }
    return TDKS_OK;
}

// projection tasks: contiguous chunk ranges of one atom (one wave reduction each), taken by the
// block's waves in turn (task t by wave t mod NW). The split minimises the busiest wave's work,
// counted as 64-chunk passes plus 0.4 of a pass for each task's reduction, over two families:
// every atom cut into m equal ranges, and ranges of 64 j chunks; ties go to fewer tasks (LDS).
// E.g. 8 atoms on 13 waves (a 20^3 block of 832 threads, before blocks were padded to 16
// waves): two tasks per atom left three waves with two tasks each, twice the others' work.
// len_mode 0: every atom cut into arg equal ranges; 1: ranges of 64 arg chunks
std::vector<int2> split_tasks(const std::vector<int> &atom_chunk, int nat, int len_mode, int arg) {
    std::vector<int2> task;
    for (int a = 0; a < nat; ++a) {
        const int b0 = atom_chunk[a], cnt = atom_chunk[a + 1] - b0;
        if (cnt <= 0) continue;
        const int len = len_mode ? 64 * arg : (cnt + arg - 1) / arg;
        for (int s = 0; s < cnt; s += len) task.push_back(make_int2(b0 + s, a | (std::min(len, cnt - s) << 8)));
    }
    return task;
}

double tasks_cost(const std::vector<int2> &task, int nwaves) {
    std::vector<double> w(nwaves, 0.0);
    for (size_t t = 0; t < task.size(); ++t) w[t % nwaves] += double(((task[t].y >> 8) + 63) / 64) + 0.4;
    return *std::max_element(w.begin(), w.end());
}

void build_tasks(TableSet &T, int block) {
    const int nwaves = std::max(1, block / 64);
    const int max_tasks = std::max(4 * nwaves, T.nat);
    std::vector<int2> best;
    double best_cost = 0.0;
    for (int mode = 0; mode < 2; ++mode)
        for (int arg = 1; arg <= 32; ++arg) {
            std::vector<int2> cand = split_tasks(T.atom_chunk, T.nat, mode, arg);
            if (cand.empty() || (int(cand.size()) > max_tasks && !best.empty())) continue;
            const double c = tasks_cost(cand, nwaves);
            if (best.empty() || c < best_cost - 1e-9 || (c < best_cost + 1e-9 && cand.size() < best.size())) {
                best = std::move(cand);
                best_cost = c;
            }
        }
    T.task = best;
    T.atom_task.assign(T.nat + 1, 0);
    size_t t = 0;
    for (int a = 0; a < T.nat; ++a) {
        T.atom_task[a] = int(t);
        while (t < T.task.size() && (T.task[t].y & 255) == a) ++t;
    }
    T.atom_task[T.nat] = int(T.task.size());
}

std::string table_key(const tdks_instance_desc &d) {
    std::string k;
    auto add = [&](const void *p, size_t n) { k.append(reinterpret_cast<const char *>(p), n); };
    add(d.lattice, sizeof(d.lattice));
    add(d.grid, sizeof(d.grid));
    add(&d.n_atoms, sizeof(int));
    add(d.atom_frac, sizeof(double) * 3 * d.n_atoms);
    for (int a = 0; a < d.n_atoms; ++a) add(&d.species[d.atom_species[a]], sizeof(tdks_species));
    return k;
}

template <typename T>
int upload(tdks_ctx *c, T **dst, const std::vector<T> &src) {
    *dst = static_cast<T *>(c->alloc(sizeof(T) * std::max<size_t>(src.size(), 1)));
    if (!*dst) return fail(TDKS_E_OOM, "device allocation of %zu bytes failed", sizeof(T) * src.size());
    if (!src.empty()) HIPCHK(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return TDKS_OK;
}

#define CHK(expr)                     \
    do {                              \
        int r_ = (expr);              \
        if (r_ != TDKS_OK) return r_; \
    } while (0)

// the first tiling rule that applies to an instance, or null
const tdks_tiling_rule *rule_for(const tdks_options *opt, const InstHost &I) {
    for (int r = 0; r < opt->n_tiling_rules; ++r) {
        const tdks_tiling_rule &R = opt->tiling_rules[r];
        if (R.grid[0] == I.N[0] && R.grid[1] == I.N[1] && R.grid[2] == I.N[2] &&
            (R.nonorth < 0 || (R.nonorth != 0) == I.nonorth) && (R.n_bands == 0 || R.n_bands == I.nb))
            return &R;
    }
    return nullptr;
}

// choose the column-segment length, block and occupancy target for one grid shape
bool choose_tiling(const int N[3], int fp64, int want_block, int want_w, int &zl, int &block, int &minw,
                   int &ragged) {
    static const int zls[] = {2, 3, 4, 6, 8, 10, 12, 16};
    // measured on MI355X: FP32 runs best with short segments and 4 waves per SIMD,
    // FP64 with 512-thread blocks at 2 waves per SIMD (see the autotuner for other shapes)
    const int target = fp64 ? 8 : 4;
    int best_cost = 1 << 30;
    bool found = false;
    for (int z : zls) {
        // segments of z points along a_3; if z does not divide N3 the last one of each column
        // is shorter (only some tilings are built for that)
        const int rg = (N[2] % z) ? 1 : 0;
        const int nseg = (N[2] + z - 1) / z;
        int b = N[0] * N[1] * nseg;
        b = (b + 63) / 64 * 64;
        // a block of more than 8 waves runs alone on its CU (4 waves per SIMD, and its LDS):
        // padded to the 16 waves the CU then holds, its wave-parallel phases (projection tasks,
        // scatter coefficients, the current's chunk tasks) spread over all of them (20^3: 13 ->
        // 16 waves, HHG step 17.16 -> 15.89 ms); a requested block size at least the one the
        // segments need is taken as given
        if (want_block >= b && want_block <= 1024 && want_block % 64 == 0)
            b = want_block;
        else if (want_block <= 0 && b > 512 && b < 1024)
            b = 1024;
        // more than 512 threads need 4 waves per SIMD; otherwise short FP32 segments fit the
        // 128-register budget of 4 waves, longer ones (and FP64) run at 2
        int w = (b > 512) ? 4 : (want_w > 0 ? want_w : ((!fp64 && z <= 4) ? 4 : 2));
        if (!propagate_config_ok(b, z, w, rg)) w = (w == 4) ? 2 : 4;
        if (!propagate_config_ok(b, z, w, rg)) continue;
        int cost = std::abs(z - target) * 4 + (b < 128 ? 2 : 0) + rg * 16;
        if (want_block > 0) cost = std::abs(b - want_block) * 16 + std::abs(z - target) + rg * 16;
        if (cost < best_cost) {
            best_cost = cost;
            zl = z;
            block = b;
            minw = w;
            ragged = rg;
            found = true;
        }
    }
    return found;
}

int sync_in(tdks_ctx *c) {
    if (c->caller != c->stream) {
        HIPCHK(hipEventRecord(c->ev_in, c->caller));
        HIPCHK(hipStreamWaitEvent(c->stream, c->ev_in, 0));
    }
    return TDKS_OK;
}
int sync_out(tdks_ctx *c) {
    if (c->caller != c->stream) {
        HIPCHK(hipEventRecord(c->ev_out, c->stream));
        HIPCHK(hipStreamWaitEvent(c->caller, c->ev_out, 0));
    }
    return TDKS_OK;
}

// the launch covers the class's work items from wb on: their instance table, work list and
// global column-table slices
void set_work(tdks_ctx *c, const ShapeClass &S, int wb, PropArgs &a) {
    a.work = c->d_work + wb;
    if (a.gcol) a.gcol = S.gcol + size_t(wb - S.wbeg) * S.gstride;
}

PropArgs class_args(tdks_ctx *c, const ShapeClass &S, int mode, const double *A, const int *ctr) {
    PropArgs a;
    a.insts = c->d_insts;
    a.work = c->d_work;
    a.A_tab = A;
    a.step_ctr = ctr;
    a.dt = c->opt.dt;
    a.mode = mode;
    a.ng_max = S.ng_max;
    a.ncol_max = S.ncol_max;
    a.nent_max = S.nent_max;
    a.nmaxd = S.nmaxd;
    a.rho_lds = S.rho_lds;
    a.mixt = S.mixt;
    a.gcol = S.gcol;
    a.ptp_lds = S.ptpl;
    a.nat_max = S.nat_max;
    a.ntask_max = S.ntask_max;
    a.apply_in = nullptr;
    a.apply_out = nullptr;
    return a;
}

// Runs launch(S, stream) for every shape class.  With several classes, the first stays on the
// context's stream and the others go to the side streams, forked from it and joined back, so
// that the last workgroups of one class overlap another class instead of leaving compute
// units idle (the classes touch disjoint instances).  Graph-capturable: the fork and join
// become parallel branches of the graph.
template <typename F>
int for_classes(tdks_ctx *c, F &&launch) {
    const int nc = int(c->classes.size()), ns = int(c->side.size());
    if (nc <= 1 || ns == 0) {
        for (const ShapeClass &S : c->classes) CHK(launch(S, c->stream));
        return TDKS_OK;
    }
    HIPCHK(hipEventRecord(c->ev_fork, c->stream));
    for (int q = 0; q < ns; ++q) HIPCHK(hipStreamWaitEvent(c->side[q], c->ev_fork, 0));
    for (int r = 0; r < nc; ++r)
        CHK(launch(c->classes[c->class_order[r]], r == 0 ? c->stream : c->side[(r - 1) % ns]));
    for (int q = 0; q < ns; ++q) {
        HIPCHK(hipEventRecord(c->ev_join[q], c->side[q]));
        HIPCHK(hipStreamWaitEvent(c->stream, c->ev_join[q], 0));
    }
    return TDKS_OK;
}

// Where a step reads its A table and puts its per-work-item partial sums and its recorded
// currents: the context's own buffers (tdks_step), or the caller's A table and current buffer
// with the partials in the static scratch array (tdks_step_noalloc).
struct StepTarget {
    const DevInst *insts;  // instance table whose rho_part / j_part receive the partials
    const double *A;       // A table [rows][2][3]
    const double *logF;    // per-row log norm bound, or null
    double *trace;         // recorded currents [n_inst][jstride][3]
    int jstride;
    const int *row_ctr;    // record row (every step), or null: steps since the load / rstride
};

StepTarget own_target(const tdks_ctx *c) {
    return StepTarget{c->d_insts, c->d_A, c->d_logF, c->d_trace, int(c->trace_cap), nullptr};
}

// the propagation launches of one step of every instance (mode STEP or PREDICT)
int enqueue_propagation(tdks_ctx *c, int mode, const StepTarget &t) {
    return for_classes(c, [&](const ShapeClass &S, hipStream_t st) {
        PropArgs a = class_args(c, S, mode, t.A, c->d_ctrs);
        a.insts = t.insts;
        set_work(c, S, S.wbeg, a);
        HIPCHK(launch_propagate(c->fp64, a, S.wend - S.wbeg, S.block, S.zl, S.minw, S.nonorth, S.sl, S.ragged, st));
        return TDKS_OK;
    });
}

bool predictor_corrector(const tdks_ctx *c) {
    return c->opt.propagator == TDKS_PROP_PC && c->opt.hxc_mode == TDKS_HXC_SCF;
}

// after the predictor: its density, v~ = v_Hxc[rho~] (kept apart), and the mid-step potential
// v_loc + (v_Hxc[rho(t_n)] + v~) / 2 for the corrector; the predictor's current is discarded
int enqueue_predictor_tail(tdks_ctx *c, const StepTarget &t) {
    HealthArgs none = c->health(false);
    none.q0 = nullptr;
    HIPCHK(launch_reduce(t.insts, 0, c->n_inst, c->ng_max, c->d_rho, c->d_jobs, 1, nullptr, none, c->stream));
    HIPCHK(launch_hxc(c->d_insts, 0, c->n_inst, c->ng_max, c->d_rho, c->d_vloc, c->d_vhxc_pred, c->d_vtot,
                      c->fp64, c->stream));
    HIPCHK(launch_vmid(c->d_insts, c->n_inst, c->ng_max, c->d_vloc, c->d_vhxc, c->d_vhxc_pred, c->d_vtot, c->fp64,
                       c->stream));
    return TDKS_OK;
}

// after the step: the per-orbital norm check when due, density, recorded current and the
// charge check, v_Hxc[rho(t_{n+1})], counters
int enqueue_step_tail(tdks_ctx *c, const StepTarget &t) {
    HealthArgs h = c->health(true);
    h.logF = t.logF;
    h.row_ctr = t.row_ctr;
    if (c->opt.norm_stride > 0)
        HIPCHK(launch_health_norms(c->d_insts, c->d_work, int(c->work.size()), c->d_ctrs + 1, c->opt.norm_stride, h,
                                   c->fp64, c->stream));
    HIPCHK(launch_reduce(t.insts, 0, c->n_inst, c->ng_max, c->d_rho, t.trace, t.jstride, c->d_ctrs + 1, h,
                         c->stream));
    if (c->opt.hxc_mode == TDKS_HXC_SCF)
        HIPCHK(launch_hxc(c->d_insts, 0, c->n_inst, c->ng_max, c->d_rho, c->d_vloc, c->d_vhxc, c->d_vtot,
                          c->fp64, c->stream));
    HIPCHK(launch_advance(c->d_ctrs, 2, c->stream));
    return TDKS_OK;
}

// enqueue one time step of every instance (graph-capturable; allocates nothing)
int enqueue_step(tdks_ctx *c, const StepTarget &t) {
    if (predictor_corrector(c)) {
        CHK(enqueue_propagation(c, MODE_PREDICT, t));
        CHK(enqueue_predictor_tail(c, t));
    }
    CHK(enqueue_propagation(c, MODE_STEP, t));
    return enqueue_step_tail(c, t);
}
int enqueue_step(tdks_ctx *c) { return enqueue_step(c, own_target(c)); }

int build_graph(tdks_ctx *c, int nsteps, hipGraphExec_t *out) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = TDKS_OK;
    for (int s = 0; s < nsteps && rc == TDKS_OK; ++s) rc = enqueue_step(c);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc != TDKS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(TDKS_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(TDKS_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    return TDKS_OK;
}

// room for `need` recorded currents per instance
int ensure_trace(tdks_ctx *c, size_t need) {
    if (need <= c->trace_cap) return TDKS_OK;
    size_t cap = std::max<size_t>(need, std::max<size_t>(2 * c->trace_cap, 1024));
    double *nt = static_cast<double *>(c->alloc(sizeof(double) * 3 * cap * c->n_inst));
    if (!nt) return fail(TDKS_E_OOM, "trace allocation failed");
    const size_t rec = size_t(c->steps_done / c->rstride);
    if (c->d_trace && rec > 0) {
        HIPCHK(hipMemcpy2DAsync(nt, sizeof(double) * 3 * cap, c->d_trace, sizeof(double) * 3 * c->trace_cap,
                                sizeof(double) * 3 * rec, c->n_inst, hipMemcpyDeviceToDevice, c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    c->release(c->d_trace);
    c->d_trace = nt;
    c->trace_cap = cap;
    c->drop_graphs();
    return TDKS_OK;
}

int ensure_A(tdks_ctx *c, size_t n) {
    if (n <= c->A_cap) return TDKS_OK;
    HIPCHK(hipStreamSynchronize(c->stream));
    size_t cap = std::max<size_t>(n, std::max<size_t>(2 * c->A_cap, 1024));
    // both new buffers first: on failure the old pair stays in place, consistent with A_cap
    // rows of 6 A components, then one log norm bound per row (d_logF follows d_A)
    double *hn = nullptr;
    if (hipHostMalloc(reinterpret_cast<void **>(&hn), sizeof(double) * 7 * cap, hipHostMallocDefault) != hipSuccess)
        return fail(TDKS_E_OOM, "pinned A table allocation failed");
    double *na = static_cast<double *>(c->alloc(sizeof(double) * 7 * cap));
    if (!na) {
        (void)hipHostFree(hn);
        return fail(TDKS_E_OOM, "A table allocation failed");
    }
    c->release(c->d_A);
    c->d_A = na;
    c->d_logF = na + 6 * cap;
    if (c->h_A) (void)hipHostFree(c->h_A);
    c->h_A = hn;
    c->h_logF = hn + 6 * cap;
    c->A_cap = cap;
    c->drop_graphs();
    return TDKS_OK;
}

int check_inst(tdks_ctx *c, int i) {
    if (!c) return fail(TDKS_E_ARG, "null context");
    if (i < 0 || i >= c->n_inst) return fail(TDKS_E_ARG, "instance %d out of range [0, %d)", i, c->n_inst);
    return TDKS_OK;
}

size_t orb_bytes(const tdks_ctx *c, const InstHost &I) {
    return size_t(I.nk) * I.nb * I.ng * (c->fp64 ? 16 : 8);
}

// observe: current (and density) of instance range for given A; writes d_jobs or d_jpre.
// enqueue_observe leaves the work on the stream; d_Aobs must already hold A.  With set_ref the
// charge becomes the instances' reference of the health check.
int enqueue_observe(tdks_ctx *c, int i_first, int i_last, double *jdst, int set_ref = 0) {
    const int mode = MODE_OBSERVE;
    CHK(for_classes(c, [&](const ShapeClass &S, hipStream_t st) {
        int wb = S.wend, we = S.wbeg;
        for (int i = i_first; i <= i_last; ++i) {
            const InstHost &I = c->inst[i];
            if (I.cls != int(&S - &c->classes[0])) continue;
            wb = std::min(wb, I.wbeg);
            we = std::max(we, I.wend);
        }
        if (we <= wb) return TDKS_OK;
        PropArgs a = class_args(c, S, mode, c->d_Aobs, c->d_ctrs + 2);
        set_work(c, S, wb, a);
        HIPCHK(launch_propagate(c->fp64, a, we - wb, S.block, S.zl, S.minw, S.nonorth, S.sl, S.ragged, st));
        return TDKS_OK;
    }));
    HealthArgs h = c->health(false);
    h.set_ref = set_ref;
    HIPCHK(launch_reduce(c->d_insts, i_first, i_last - i_first + 1, c->ng_max, c->d_rho, jdst, 1, nullptr, h,
                         c->stream));
    return TDKS_OK;
}

int observe(tdks_ctx *c, int i_first, int i_last, const double A[3], double *jdst, int set_ref = 0) {
    double h[6] = {A[0], A[1], A[2], A[0], A[1], A[2]};
    HIPCHK(hipMemcpyAsync(c->d_Aobs, h, sizeof(h), hipMemcpyHostToDevice, c->stream));
    CHK(enqueue_observe(c, i_first, i_last, jdst, set_ref));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TDKS_OK;
}

// Upper bound of the kinetic part of h_k over the instance's k-set: per axis the 4th-order
// second difference reaches 16/3 at the zone edge, the first difference at most
// max |8 sin t - sin 2t| / 6 < 1.3722; |k|^2 / 2 on top.
double kinetic_bound(const InstHost &I) {
    const double s1 = 1.3722;
    double b = 0.0;
    for (int d = 0; d < 3; ++d) {
        b += 0.5 * (16.0 / 3.0) * I.g[d][d];
        for (int e = 0; e < 3; ++e)
            if (e != d) b += 0.5 * std::fabs(I.g[d][e]) * s1 * s1;
    }
    double kmax = 0.0;
    for (int k = 0; k < I.nk; ++k) {
        const double *kc = &I.kcart[3 * k];
        double t = 0.5 * (kc[0] * kc[0] + kc[1] * kc[1] + kc[2] * kc[2]);
        for (int d = 0; d < 3; ++d)
            t += std::fabs(kc[0] * I.c[d][0] + kc[1] * I.c[d][1] + kc[2] * I.c[d][2]) * s1;
        kmax = std::max(kmax, t);
    }
    return b + kmax;
}

// log of the closed-form norm bound of one Taylor-4 step with A(t_n + dt/2) = Amid, for the
// health check: F = min over |x| <= x_max of |T4(-i x)|^2 = 1 - x^6/72 + x^8/576, which is
// f(x_max) while x_max < sqrt 6 and 0.25 beyond; x_max = |dt| max over instances of
// lam0 + |A| lamA + |A|^2 / 2 (a bound of |lambda| of h_kappa, kappa = k + A).
double step_log_bound(const tdks_ctx *c, const double *Amid) {
    const double a = std::sqrt(Amid[0] * Amid[0] + Amid[1] * Amid[1] + Amid[2] * Amid[2]);
    double lam = 0.0;
    for (const InstHost &I : c->inst) lam = std::max(lam, I.lam0 + a * I.lamA + 0.5 * a * a);
    const double x = std::fabs(c->opt.dt) * lam;
    if (!(x < std::sqrt(6.0))) return std::log(0.25);
    const double x2 = x * x, x6 = x2 * x2 * x2;
    return std::log(1.0 - x6 / 72.0 + x6 * x2 / 576.0);
}

// copies an A table (HOST [n][2][3]) and its per-step norm bounds to the device (the A-table
// row counter restarts at 0)
int upload_A(tdks_ctx *c, int n_steps, const double *A_tab) {
    CHK(ensure_A(c, size_t(n_steps)));
    HIPCHK(hipEventSynchronize(c->ev_acopy));  // previous copy out of the staging buffer is done
    std::memcpy(c->h_A, A_tab, sizeof(double) * 6 * n_steps);
    for (int n = 0; n < n_steps; ++n) c->h_logF[n] = step_log_bound(c, A_tab + 6 * n);
    HIPCHK(hipMemcpyAsync(c->d_A, c->h_A, sizeof(double) * 6 * n_steps, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_logF, c->h_logF, sizeof(double) * n_steps, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipEventRecord(c->ev_acopy, c->stream));
    HIPCHK(launch_fill_int(c->d_ctrs, 0, 1, c->stream));
    return TDKS_OK;
}

// clears the health record of instances [i0, i1] and, with the per-orbital check on, takes
// their present norms as the reference (the charge reference is set by the observation)
int health_reset(tdks_ctx *c, int i0, int i1) {
    if (c->health_pending) {  // a copy still in flight would bring the old record back
        HIPCHK(hipEventSynchronize(c->ev_health));
        c->health_pending = false;
    }
    std::fill(c->h_health + i0, c->h_health + i1 + 1, 0ull);
    HIPCHK(launch_fill_int(reinterpret_cast<int *>(c->d_health + i0), 0, 2 * (i1 - i0 + 1), c->stream));
    if (c->opt.norm_stride > 0)
        for (int i = i0; i <= i1; ++i) {
            const InstHost &I = c->inst[i];
            HIPCHK(launch_norms(I.d_u, I.nk * I.nb, I.ng, I.dV, c->fp64, c->d_norm0 + I.norm0_off, c->stream));
        }
    return TDKS_OK;
}

// E_NUMERIC naming the first instance with a recorded violation, else OK
int health_report(const tdks_ctx *c, const unsigned long long *h) {
    static const char *what[] = {"", "non-finite current or charge", "charge above its value at the load",
                                 "charge below the Taylor-4 norm bound", "orbital norm above its value at the load",
                                 "orbital norm below the Taylor-4 norm bound"};
    for (int i = 0; i < c->n_inst; ++i) {
        if (!h[i]) continue;
        const int code = int(h[i] & 15u), step = int(h[i] >> 32);
        const long long orb = static_cast<long long>((h[i] >> 4) & 0xfffffffull) - 1;
        const InstHost &I = c->inst[i];
        if (orb >= 0)
            return fail(TDKS_E_NUMERIC, "instance %d, step %d after the load: %s (k %lld, band %lld)", i, step,
                        what[code < 6 ? code : 0], orb / I.nb, orb % I.nb);
        return fail(TDKS_E_NUMERIC, "instance %d, step %d after the load: %s", i, step, what[code < 6 ? code : 0]);
    }
    return TDKS_OK;
}

// the health record as of the last synchronisation point: waits for the stream
int health_sync(tdks_ctx *c) {
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(c->h_health, c->d_health, sizeof(unsigned long long) * c->n_inst, hipMemcpyDeviceToHost));
    c->health_pending = false;
    return health_report(c, c->h_health);
}

}  // namespace

extern "C" {

void tdks_default_options(tdks_options *opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = TDKS_FP64;
    opt->dt = 0.02;
    opt->taylor_order = 4;
    opt->hxc_mode = TDKS_HXC_SCF;
    opt->graph_steps = 16;
}

const char *tdks_last_error(void) { return g_last_error.c_str(); }

void tdks_destroy(tdks_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    c->drop_graphs();
    std::vector<void *> all = c->allocs;
    for (void *p : all) c->release(p);
    if (c->h_A) (void)hipHostFree(c->h_A);
    if (c->h_health) (void)hipHostFree(c->h_health);
    if (c->ev_health) (void)hipEventDestroy(c->ev_health);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->ev_acopy) (void)hipEventDestroy(c->ev_acopy);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    for (hipEvent_t e : c->ev_join) (void)hipEventDestroy(e);
    for (hipStream_t st : c->side) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

static int create_impl(const tdks_instance_desc *desc, int n_inst, const tdks_options *opt, tdks_ctx *c) {
    c->opt = *opt;
    if (opt->precision != TDKS_FP64 && opt->precision != TDKS_FP32_MIXED)
        return fail(TDKS_E_ARG, "unknown precision %d", opt->precision);
    if (opt->taylor_order != 4) return fail(TDKS_E_UNSUPPORTED, "taylor_order must be 4");
    if (!(opt->dt != 0.0) || !std::isfinite(opt->dt)) return fail(TDKS_E_ARG, "dt must be finite and non-zero");
    if (opt->hxc_mode < TDKS_HXC_SCF || opt->hxc_mode > TDKS_HXC_NONE)
        return fail(TDKS_E_ARG, "unknown hxc_mode %d", opt->hxc_mode);
    if (opt->propagator != TDKS_PROP_TAYLOR && opt->propagator != TDKS_PROP_PC)
        return fail(TDKS_E_ARG, "unknown propagator %d", opt->propagator);
    if (opt->norm_stride < 0) return fail(TDKS_E_ARG, "norm_stride must be >= 0");
    if (opt->record_stride < 0) return fail(TDKS_E_ARG, "record_stride must be >= 0");
    if (opt->n_tiling_rules < 0 || (opt->n_tiling_rules > 0 && !opt->tiling_rules))
        return fail(TDKS_E_ARG, "bad tiling rules");
    c->opt.tiling_rules = nullptr;  // borrowed for this call only
    c->opt.n_tiling_rules = 0;
    c->rstride = opt->record_stride > 0 ? opt->record_stride : 1;
    c->fp64 = opt->precision == TDKS_FP64;
    c->n_inst = n_inst;
    c->chunk = opt->graph_steps == 0 ? 16 : opt->graph_steps;
    c->caller = static_cast<hipStream_t>(opt->stream);
    c->inst.resize(n_inst);
    std::map<std::string, int> table_of;
    for (int i = 0; i < n_inst; ++i) {
        const tdks_instance_desc &d = desc[i];
        InstHost &I = c->inst[i];
        CHK(build_geometry(I, d));
        if (d.n_atoms < 0 || d.n_atoms > kMaxAtoms) return fail(TDKS_E_UNSUPPORTED, "n_atoms %d outside [0, %d]", d.n_atoms, kMaxAtoms);
        if (d.n_atoms > 0 && (!d.atom_frac || !d.atom_species || !d.species))
            return fail(TDKS_E_ARG, "instance %d: atom arrays missing", i);
        for (int a = 0; a < d.n_atoms; ++a)
            if (d.atom_species[a] < 0 || d.atom_species[a] >= d.n_species)
                return fail(TDKS_E_ARG, "instance %d atom %d: species index out of range", i, a);
        if (d.n_k <= 0 || !d.k_frac) return fail(TDKS_E_ARG, "instance %d: no k-points", i);
        if (d.n_bands <= 0) return fail(TDKS_E_ARG, "instance %d: no bands", i);
        I.nk = d.n_k;
        I.nb = d.n_bands;
        I.nat = d.n_atoms;
        I.group = d.group;
        I.kcart.resize(3 * I.nk);
        I.kw.resize(I.nk);
        for (int k = 0; k < I.nk; ++k) {
            for (int q = 0; q < 3; ++q)
                I.kcart[3 * k + q] = d.k_frac[3 * k + 0] * I.B[0][q] + d.k_frac[3 * k + 1] * I.B[1][q] +
                                     d.k_frac[3 * k + 2] * I.B[2][q];
            I.kw[k] = d.k_weight ? d.k_weight[k] : 1.0 / I.nk;
        }
        I.occ.resize(I.nb);
        for (int b = 0; b < I.nb; ++b) I.occ[b] = d.occ ? d.occ[b] : 2.0;
        if (opt->hxc_mode == TDKS_HXC_FROZEN) {
            if (!d.v_hxc_frozen) return fail(TDKS_E_ARG, "instance %d: FROZEN mode needs v_hxc_frozen", i);
            I.vhxc_frozen.assign(d.v_hxc_frozen, d.v_hxc_frozen + I.ng);
        }
        const std::string key = table_key(d);
        auto it = table_of.find(key);
        if (it == table_of.end()) {
            TableSet T;
            CHK(build_potential_and_tables(I, d, T));
            c->tables.push_back(std::move(T));
            I.table = int(c->tables.size()) - 1;
            table_of[key] = I.table;
        } else {
            I.table = it->second;
            for (int j = 0; j < i; ++j)
                if (c->inst[j].table == it->second) {
                    I.vloc = c->inst[j].vloc;
                    break;
                }
        }
        c->ng_max = std::max(c->ng_max, I.ng);
    }
    // |lambda| bound of each instance's h_kappa for the health check: kinetic bound at A = 0,
    // |v_loc| and the V_NL bound, plus an allowance of 5 Ha for |v_Hxc|; with a field,
    // |k + A|^2 / 2 + sum_d |(k + A).c_d| s1 grows by at most |A| (|k|max + s1 sum_d |c_d|) + |A|^2 / 2
    for (InstHost &I : c->inst) {
        double vmax = 0.0, kmax = 0.0, cs = 0.0;
        for (double v : I.vloc) vmax = std::max(vmax, std::fabs(v));
        for (int k = 0; k < I.nk; ++k) {
            const double *kc = &I.kcart[3 * k];
            kmax = std::max(kmax, std::sqrt(kc[0] * kc[0] + kc[1] * kc[1] + kc[2] * kc[2]));
        }
        for (int d = 0; d < 3; ++d) cs += 1.3722 * std::sqrt(I.g[d][d]);
        I.lam0 = kinetic_bound(I) + vmax + c->tables[I.table].nl_bound + 5.0;
        I.lamA = kmax + cs;
    }
    // shape classes and tiling (per-shape rules override the context's options)
    std::vector<int> class_block(0), class_waves(0);
    for (int i = 0; i < n_inst; ++i) {
        InstHost &I = c->inst[i];
        const tdks_tiling_rule *R = rule_for(opt, I);
        const int want_b = (R && R->block_size > 0) ? R->block_size : opt->block_size;
        const int want_w = (R && R->waves_per_simd > 0) ? R->waves_per_simd : opt->waves_per_simd;
        int cls = -1;
        for (size_t s = 0; s < c->classes.size(); ++s) {
            const ShapeClass &S = c->classes[s];
            if (S.N[0] == I.N[0] && S.N[1] == I.N[1] && S.N[2] == I.N[2] && S.nonorth == I.nonorth) cls = int(s);
        }
        if (cls >= 0 && (class_block[cls] != want_b || class_waves[cls] != want_w))
            return fail(TDKS_E_ARG, "instance %d: its tiling rule gives grid %dx%dx%d another block size or "
                        "occupancy than an earlier instance of that shape", i, I.N[0], I.N[1], I.N[2]);
        if (cls < 0) {
            ShapeClass S;
            for (int q = 0; q < 3; ++q) S.N[q] = I.N[q];
            S.nonorth = I.nonorth;
            if (!choose_tiling(S.N, c->fp64, want_b, want_w, S.zl, S.block, S.minw, S.ragged))
                return fail(TDKS_E_UNSUPPORTED, "no built propagation tiling for grid %dx%dx%d", S.N[0], S.N[1], S.N[2]);
            c->classes.push_back(S);
            class_block.push_back(want_b);
            class_waves.push_back(want_w);
            cls = int(c->classes.size()) - 1;
        }
        I.cls = cls;
        ShapeClass &S = c->classes[cls];
        TableSet &T = c->tables[I.table];
        if (T.cls < 0) {
            T.cls = cls;
            build_tasks(T, S.block);
        }
        S.ng_max = std::max(S.ng_max, I.ng);
        S.ncol_max = std::max(S.ncol_max, int(T.col_atom.size()));
        S.nent_max = std::max(S.nent_max, int(T.pt_pack.size()));
        S.nmaxd = std::max(S.nmaxd, std::max(I.N[0], std::max(I.N[1], I.N[2])));
        S.nat_max = std::max(S.nat_max, T.nat);
        S.ntask_max = std::max(S.ntask_max, int(T.task.size()));
    }
    for (ShapeClass &S : c->classes) {
        PropArgs a = class_args(c, S, MODE_STEP, nullptr, nullptr);
        auto fits = [&](int sl, int rho, int mixt, int gc = 0, int ptpl = 0) {
            a.rho_lds = rho;
            a.mixt = mixt;
            a.gcol = gc ? reinterpret_cast<char *>(256) : nullptr;  // only its presence counts here
            a.ptp_lds = ptpl;
            return propagate_lds_bytes(c->fp64, sl, a, S.block) <= 160 * 1024;
        };
        // non-orthogonal cells: the mixed-derivative intermediate when it fits beside the
        // orbital and the LDS-staged projector records (FP32), at the expense of the density
        // partial if need be; FP32: stage the point-major projector tables in LDS when they
        // fit; then keep the density partial in LDS too if there is room (in the global slot,
        // every band's update of it would leave L2)
        S.mixt = (S.nonorth && fits(c->fp64 ? 0 : 1, 0, 1)) ? 1 : 0;
        if (S.nonorth && !S.mixt && !c->fp64 && fits(0, 0, 1)) S.mixt = 1;
        S.sl = (!c->fp64 && fits(1, 0, S.mixt)) ? 1 : 0;
        S.rho_lds = (!c->fp64 && fits(S.sl, 1, S.mixt)) ? 1 : 0;
        // FP64 grids whose orbital and column tables exceed the LDS (20^3, 16x16x32): the
        // column tables go to a per-work-item global buffer
        S.gc = (c->fp64 && !fits(0, 0, S.mixt) && fits(0, 0, 0, 1)) ? 1 : 0;
        if (S.gc) S.mixt = 0;
        // without LDS records the FP32 scatter reads its records from global memory: its CSR
        // pointers (2 bytes per point) from LDS when they fit (FP64 reads both from global
        // memory: 5 % faster than its 16-byte records with the pointers in LDS)
        S.ptpl = (!c->fp64 && !S.sl && fits(0, S.rho_lds, S.mixt, S.gc, 1)) ? 1 : 0;
        a.rho_lds = S.rho_lds;
        a.mixt = S.mixt;
        a.gcol = S.gc ? reinterpret_cast<char *>(256) : nullptr;
        a.ptp_lds = S.ptpl;
        S.gstride = S.gc ? propagate_gcol_stride(c->fp64, S.ncol_max) : 0;
        const size_t lds = propagate_lds_bytes(c->fp64, S.sl, a, S.block);
        if (lds > 160 * 1024)
            return fail(TDKS_E_UNSUPPORTED, "grid %dx%dx%d needs %zu bytes of LDS per workgroup", S.N[0], S.N[1],
                        S.N[2], lds);
    }
    // work list: class-major, instance-major, then k groups and band groups
    long long items1 = 0;  // work items with one k-point per workgroup
    for (int i = 0; i < n_inst; ++i) {
        const InstHost &I = c->inst[i];
        const tdks_tiling_rule *R = rule_for(opt, I);
        const int want = (R && R->bands_per_group > 0) ? R->bands_per_group : opt->bands_per_group;
        const int bpg = (want > 0 && want < I.nb) ? want : I.nb;
        items1 += (long long)I.nk * ((I.nb + bpg - 1) / bpg);
    }
    const bool big = items1 >= 16384;
    // work items of each shape class with every band in one workgroup
    std::vector<long long> class_items(c->classes.size(), 0);
    for (int i = 0; i < n_inst; ++i) {
        const InstHost &I = c->inst[i];
        const tdks_tiling_rule *R = rule_for(opt, I);
        const int want = (R && R->bands_per_group > 0) ? R->bands_per_group : opt->bands_per_group;
        const int bpg = (want > 0 && want < I.nb) ? want : I.nb;
        class_items[I.cls] += (long long)I.nk * ((I.nb + bpg - 1) / bpg);
    }
    for (size_t s = 0; s < c->classes.size(); ++s) {
        ShapeClass &S = c->classes[s];
        S.wbeg = int(c->work.size());
        for (int i = 0; i < n_inst; ++i) {
            InstHost &I = c->inst[i];
            if (I.cls != int(s)) continue;
            const tdks_tiling_rule *R = rule_for(opt, I);
            const int want = (R && R->bands_per_group > 0) ? R->bands_per_group : opt->bands_per_group;
            int bpg = (want > 0 && want < I.nb) ? want : I.nb;
            // a class with fewer work items than compute units (a lone small-k instance, the
            // 13 supercells of the uneven batch) splits its bands, down to 8 per workgroup, until
            // its items cover the 256 CUs (the supercell class alone: 1.84 -> 1.06 ms)
            if (want <= 0) {
                int f = 1;
                while (class_items[s] * f < 256 && (I.nb + 2 * f - 1) / (2 * f) >= 8) f *= 2;
                bpg = (I.nb + f - 1) / f;
            }
            const int want_k = (R && R->k_per_group > 0) ? R->k_per_group : opt->k_per_group;
            // k-points per workgroup: by default 4 for instances with at least 256 k-points in
            // a context of at least 16384 single-k work items (64 per CU: fewer table stagings
            // and density slots, 2.5 % faster per step on the two-step workload), else 1 (a
            // lone 512-k instance needs its 512 workgroups to fill the GPU)
            const int kpg = want_k > 0 ? want_k : (I.nk >= 256 && big ? 4 : 1);
            I.wbeg = int(c->work.size());
            int slot = 0;
            for (int k0 = 0; k0 < I.nk; k0 += kpg)
                for (int b0 = 0; b0 < I.nb; b0 += bpg) {
                    WorkItem w;
                    w.inst = i;
                    w.k0 = k0;
                    w.nk = std::min(kpg, I.nk - k0);
                    w.b0 = b0;
                    w.nb = std::min(bpg, I.nb - b0);
                    w.slot = slot++;
                    c->work.push_back(w);
                }
            I.wend = int(c->work.size());
            I.nslot = slot;
        }
        S.wend = int(c->work.size());
    }
    // classes in decreasing work per item (grid points x k-points x bands of its largest item),
    // so that the longest workgroups start first and do not end up as a step's tail
    {
        std::vector<double> cost(c->classes.size(), 0.0);
        for (const WorkItem &w : c->work) {
            const InstHost &I = c->inst[w.inst];
            cost[I.cls] = std::max(cost[I.cls], double(I.ng) * w.nk * w.nb);
        }
        c->class_order.resize(c->classes.size());
        for (size_t s = 0; s < c->classes.size(); ++s) c->class_order[s] = int(s);
        std::stable_sort(c->class_order.begin(), c->class_order.end(),
                         [&](int x, int y) { return cost[x] > cost[y]; });
    }
    for (const InstHost &I : c->inst) {
        if (std::find(c->groups.begin(), c->groups.end(), I.group) == c->groups.end()) c->groups.push_back(I.group);
    }
    std::sort(c->groups.begin(), c->groups.end());
    // device side: stream, events, memory; the scratch array's address on this device
    HIPCHK(hipGetDevice(&c->device));
    CHK(scratch_address(c->device, &c->scratch));
    HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&c->ev_acopy, hipEventDisableTiming));
    // side streams for the shape classes after the first (at most 3: with the context's own
    // stream, the 4 hardware queues a process gets by default)
    const int n_side = std::min(int(c->classes.size()) - 1, 3);
    for (int q = 0; q < n_side; ++q) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        c->side.push_back(st);
        HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        c->ev_join.push_back(ev);
    }
    if (n_side > 0) HIPCHK(hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    for (TableSet &T : c->tables) {
        CHK(upload(c, &T.d_col_atom, T.col_atom));
        CHK(upload(c, &T.d_col_j01, T.col_j01));
        CHK(upload(c, &T.d_pt_ptr, T.pt_ptr));
        CHK(upload(c, &T.d_pt_ptr16, T.pt_ptr16));
        if (!c->fp64) CHK(upload(c, &T.d_pt_rec, T.pt_rec32));
        CHK(upload(c, &T.d_pt_pack, T.pt_pack));
        CHK(upload(c, &T.d_pt_g, T.pt_g));
        CHK(upload(c, &T.d_pt_gf, T.pt_gf));
        CHK(upload(c, &T.d_task, T.task));
        CHK(upload(c, &T.d_atom_task, T.atom_task));
        CHK(upload(c, &T.d_chunk_pack, T.chunk_pack));
        CHK(upload(c, &T.d_chunk_g, T.chunk_g));
        CHK(upload(c, &T.d_chunk_gf, T.chunk_gf));
        CHK(upload(c, &T.d_atom_tau, T.atom_tau));
        CHK(upload(c, &T.d_atom_par, T.atom_par));
    }
    const size_t ngm = size_t(c->ng_max) * n_inst;
    std::vector<double> vloc_all(ngm, 0.0), vhxc_all(ngm, 0.0);
    for (int i = 0; i < n_inst; ++i) {
        const InstHost &I = c->inst[i];
        std::copy(I.vloc.begin(), I.vloc.end(), vloc_all.begin() + size_t(i) * c->ng_max);
        if (!I.vhxc_frozen.empty())
            std::copy(I.vhxc_frozen.begin(), I.vhxc_frozen.end(), vhxc_all.begin() + size_t(i) * c->ng_max);
    }
    CHK(upload(c, &c->d_vloc, vloc_all));
    CHK(upload(c, &c->d_vhxc, vhxc_all));
    if (opt->propagator == TDKS_PROP_PC && opt->hxc_mode == TDKS_HXC_SCF)
        CHK(upload(c, &c->d_vhxc_pred, vhxc_all));
    c->d_rho = static_cast<double *>(c->alloc(sizeof(double) * ngm));
    c->d_vtot = c->alloc((c->fp64 ? 8 : 4) * ngm);
    c->d_ctrs = static_cast<int *>(c->alloc(sizeof(int) * 4));
    c->d_jpre = static_cast<double *>(c->alloc(sizeof(double) * 3 * n_inst));
    c->d_jobs = static_cast<double *>(c->alloc(sizeof(double) * 3 * n_inst));
    c->d_Aobs = static_cast<double *>(c->alloc(sizeof(double) * 6));
    c->d_q0 = static_cast<double *>(c->alloc(sizeof(double) * n_inst));
    c->d_lcum = static_cast<double *>(c->alloc(sizeof(double) * n_inst));
    c->d_health = static_cast<unsigned long long *>(c->alloc(sizeof(unsigned long long) * n_inst));
    if (!c->d_rho || !c->d_vtot || !c->d_ctrs || !c->d_jpre || !c->d_jobs || !c->d_Aobs || !c->d_q0 ||
        !c->d_lcum || !c->d_health)
        return fail(TDKS_E_OOM, "device allocation failed");
    if (hipHostMalloc(reinterpret_cast<void **>(&c->h_health), sizeof(unsigned long long) * n_inst,
                      hipHostMallocDefault) != hipSuccess)
        return fail(TDKS_E_OOM, "pinned health record allocation failed");
    std::fill(c->h_health, c->h_health + n_inst, 0ull);
    HIPCHK(hipEventCreateWithFlags(&c->ev_health, hipEventDisableTiming));
    HIPCHK(hipMemset(c->d_health, 0, sizeof(unsigned long long) * n_inst));
    HIPCHK(hipMemset(c->d_q0, 0, sizeof(double) * n_inst));
    HIPCHK(hipMemset(c->d_lcum, 0, sizeof(double) * n_inst));
    if (opt->norm_stride > 0) {
        size_t norb = 0;
        for (InstHost &I : c->inst) {
            I.norm0_off = norb;
            norb += size_t(I.nk) * I.nb;
        }
        c->d_norm0 = static_cast<double *>(c->alloc(sizeof(double) * norb));
        if (!c->d_norm0) return fail(TDKS_E_OOM, "reference norm allocation failed");
    }
    HIPCHK(hipMemset(c->d_ctrs, 0, sizeof(int) * 4));
    HIPCHK(hipMemset(c->d_rho, 0, sizeof(double) * ngm));
    std::vector<DevInst> dinst(n_inst);
    for (int i = 0; i < n_inst; ++i) {
        InstHost &I = c->inst[i];
        const TableSet &T = c->tables[I.table];
        I.d_u = c->alloc(orb_bytes(c, I));
        if (!I.d_u) return fail(TDKS_E_OOM, "orbital allocation of %zu bytes failed (instance %d)", orb_bytes(c, I), i);
        CHK(upload(c, &I.d_kcart, I.kcart));
        CHK(upload(c, &I.d_kw, I.kw));
        CHK(upload(c, &I.d_occ, I.occ));
        I.d_rho_part = static_cast<double *>(c->alloc(sizeof(double) * size_t(I.nslot) * I.ng));
        I.d_j_part = static_cast<double *>(c->alloc(sizeof(double) * 4 * size_t(I.nslot)));
        if (!I.d_rho_part || !I.d_j_part) return fail(TDKS_E_OOM, "partial-sum allocation failed");
        DevInst &D = dinst[i];
        std::memset(&D, 0, sizeof(D));
        for (int q = 0; q < 3; ++q) D.N[q] = I.N[q];
        D.ng = I.ng;
        D.nk = I.nk;
        D.nb = I.nb;
        D.nat = T.nat;
        D.nonorth = I.nonorth;
        D.ntask = int(T.task.size());
        D.dV = I.dV;
        D.omega = I.omega;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                D.lat[a][b] = I.lat[a][b];
                D.hv[a][b] = I.hv[a][b];
                D.c[a][b] = I.c[a][b];
                D.g[a][b] = I.g[a][b];
            }
        D.u = I.d_u;
        D.vtot = static_cast<char *>(c->d_vtot) + size_t(i) * c->ng_max * (c->fp64 ? 8 : 4);
        D.kcart = I.d_kcart;
        D.kw = I.d_kw;
        D.occ = I.d_occ;
        D.ncol = int(T.col_atom.size());
        D.col_atom = T.d_col_atom;
        D.col_j01 = T.d_col_j01;
        D.pt_ptr = T.d_pt_ptr;
        D.pt_ptr16 = T.d_pt_ptr16;
        D.pt_rec = T.d_pt_rec;
        D.nent = int(T.pt_pack.size());
        D.pt_pack = T.d_pt_pack;
        D.pt_gf = T.d_pt_gf;
        D.pt_gd = T.d_pt_g;
        D.task = T.d_task;
        D.atom_task = T.d_atom_task;
        D.chunk_pack = T.d_chunk_pack;
        D.chunk_gf = T.d_chunk_gf;
        D.chunk_gd = T.d_chunk_g;
        D.atom_tau = T.d_atom_tau;
        D.atom_par = T.d_atom_par;
        D.rho_part = I.d_rho_part;
        D.j_part = I.d_j_part;
        D.nslot = I.nslot;
        D.norm0 = c->d_norm0 ? c->d_norm0 + I.norm0_off : nullptr;
    }
    {
        std::vector<DevInst> tmp = dinst;
        CHK(upload(c, &c->d_insts, tmp));
    }
    // the same table with the partial sums in the static scratch array (allocation-free step),
    // when they fit: per instance [nslot][ng] densities, then [nslot][4] currents, 256-aligned
    {
        std::vector<DevInst> scr = dinst;
        size_t off = 0;
        auto al256 = [](size_t x) { return (x + 255) & ~size_t(255); };
        for (int i = 0; i < n_inst; ++i) {
            const InstHost &I = c->inst[i];
            scr[i].rho_part = reinterpret_cast<double *>(static_cast<char *>(c->scratch) + off);
            off = al256(off + sizeof(double) * size_t(I.nslot) * I.ng);
            scr[i].j_part = reinterpret_cast<double *>(static_cast<char *>(c->scratch) + off);
            off = al256(off + sizeof(double) * 4 * size_t(I.nslot));
        }
        c->scratch_need = off;
        if (off <= kScratchBytes) CHK(upload(c, &c->d_insts_scr, scr));
    }
    CHK(upload(c, &c->d_work, c->work));
    for (ShapeClass &S : c->classes) {
        if (!S.gc) continue;
        const size_t bytes = S.gstride * size_t(S.wend - S.wbeg);
        S.gcol = static_cast<char *>(c->alloc(bytes));
        if (!S.gcol) return fail(TDKS_E_OOM, "column-table allocation of %zu bytes failed", bytes);
    }
    HIPCHK(launch_vtot(c->d_insts, 0, n_inst, c->ng_max, c->d_vloc, c->d_vhxc, c->d_vtot, c->fp64, c->stream));
    c->jpre.assign(3 * n_inst, 0.0);
    CHK(ensure_A(c, 64));
    CHK(ensure_trace(c, 1024));
    HIPCHK(hipStreamSynchronize(c->stream));
    return TDKS_OK;
}

int tdks_create(const tdks_instance_desc *inst, int n_inst, const tdks_options *opt, tdks_ctx **out) {
    if (!out) return fail(TDKS_E_ARG, "out is null");
    *out = nullptr;
    if (!inst || n_inst <= 0) return fail(TDKS_E_ARG, "no instances");
    tdks_options def;
    tdks_default_options(&def);
    if (!opt) opt = &def;
    tdks_ctx *c = new tdks_ctx();
    int rc = create_impl(inst, n_inst, opt, c);
    if (rc != TDKS_OK) {
        std::string msg = g_last_error;
        tdks_destroy(c);
        g_last_error = msg;
        return rc;
    }
    *out = c;
    g_last_error.clear();
    return TDKS_OK;
}

int tdks_load_orbitals(tdks_ctx *c, int i, const void *u, int where) {
    CHK(check_inst(c, i));
    if (!u) return fail(TDKS_E_ARG, "null orbital pointer");
    if (where != TDKS_HOST && where != TDKS_DEVICE) return fail(TDKS_E_ARG, "bad where flag");
    InstHost &I = c->inst[i];
    CHK(sync_in(c));
    const size_t n = size_t(I.nk) * I.nb * I.ng;
    if (c->fp64) {
        HIPCHK(hipMemcpyAsync(I.d_u, u, 16 * n, where == TDKS_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                              c->stream));
    } else {
        const double *src = static_cast<const double *>(u);
        double *stage = nullptr;
        if (where == TDKS_HOST) {
            stage = static_cast<double *>(c->alloc(16 * n));
            if (!stage) return fail(TDKS_E_OOM, "staging allocation failed");
            HIPCHK(hipMemcpyAsync(stage, u, 16 * n, hipMemcpyHostToDevice, c->stream));
            src = stage;
        }
        HIPCHK(launch_convert_in(src, I.d_u, n, 0, c->stream));
        if (stage) {
            HIPCHK(hipStreamSynchronize(c->stream));
            c->release(stage);
        }
    }
    // density, v_Hxc and the current before the field (A = 0); the charge and the norms of the
    // new orbitals become the health check's references
    const double zero[3] = {0.0, 0.0, 0.0};
    CHK(health_reset(c, i, i));
    CHK(observe(c, i, i, zero, c->d_jpre, 1));
    if (c->opt.hxc_mode == TDKS_HXC_SCF) {
        HIPCHK(launch_hxc(c->d_insts, i, 1, c->ng_max, c->d_rho, c->d_vloc, c->d_vhxc, c->d_vtot, c->fp64, c->stream));
    }
    HIPCHK(hipMemcpyAsync(c->jpre.data() + 3 * i, c->d_jpre + 3 * i, 3 * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(launch_fill_int(c->d_ctrs, 0, 3, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    I.loaded = true;
    c->steps_done = 0;
    c->noalloc_steps = false;
    CHK(sync_out(c));
    return TDKS_OK;
}

int tdks_step(tdks_ctx *c, int n_steps, const double *A_tab) {
    if (!c) return fail(TDKS_E_ARG, "null context");
    if (n_steps < 0) return fail(TDKS_E_ARG, "n_steps < 0");
    if (n_steps == 0) return TDKS_OK;
    if (!A_tab) return fail(TDKS_E_ARG, "null A table");
    for (int i = 0; i < c->n_inst; ++i)
        if (!c->inst[i].loaded) return fail(TDKS_E_STATE, "instance %d has no orbitals loaded", i);
    // the health record copied after an earlier call, if it has arrived (no wait)
    if (c->health_pending && hipEventQuery(c->ev_health) == hipSuccess) c->health_pending = false;
    if (!c->health_pending) CHK(health_report(c, c->h_health));
    CHK(sync_in(c));
    CHK(ensure_trace(c, size_t(c->steps_done + n_steps) / c->rstride));
    // A row counter restarts for this call; the step counter continues
    CHK(upload_A(c, n_steps, A_tab));
    int done = 0;
    if (c->chunk > 0) {
        if (!c->g_one) CHK(build_graph(c, 1, &c->g_one));
        if (c->chunk > 1 && n_steps >= c->chunk && !c->g_chunk) CHK(build_graph(c, c->chunk, &c->g_chunk));
        while (c->chunk > 1 && n_steps - done >= c->chunk) {
            HIPCHK(hipGraphLaunch(c->g_chunk, c->stream));
            done += c->chunk;
        }
        while (done < n_steps) {
            HIPCHK(hipGraphLaunch(c->g_one, c->stream));
            ++done;
        }
    } else {
        for (; done < n_steps; ++done) CHK(enqueue_step(c));
    }
    c->steps_done += n_steps;
    HIPCHK(hipMemcpyAsync(c->h_health, c->d_health, sizeof(unsigned long long) * c->n_inst, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipEventRecord(c->ev_health, c->stream));
    c->health_pending = true;
    CHK(sync_out(c));
    return TDKS_OK;
}

int tdks_step_noalloc(tdks_ctx *c, int n_steps, const double *A_dev, double *j_dev) {
    if (!c) return fail(TDKS_E_ARG, "null context");
    if (n_steps < 0) return fail(TDKS_E_ARG, "n_steps < 0");
    if (c->scratch_need > kScratchBytes)
        return fail(TDKS_E_UNSUPPORTED, "the partial sums of this context need %zu bytes; the static scratch array "
                    "holds %zu (use tdks_step)", c->scratch_need, kScratchBytes);
    for (const ShapeClass &S : c->classes)
        if (S.gc)
            return fail(TDKS_E_UNSUPPORTED, "grid %dx%dx%d keeps its FP64 column tables in context memory outside "
                        "the scratch array (use tdks_step)", S.N[0], S.N[1], S.N[2]);
    if (n_steps == 0) return TDKS_OK;
    if (!A_dev || !j_dev) return fail(TDKS_E_ARG, "null A table or current buffer");
    for (int i = 0; i < c->n_inst; ++i)
        if (!c->inst[i].loaded) return fail(TDKS_E_STATE, "instance %d has no orbitals loaded", i);
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != c->device)
        return fail(TDKS_E_ARG, "the context lives on device %d but device %d is current", c->device, dev);
    CHK(sync_in(c));
    // the A-table row counter (also the record row) restarts; the step counter continues
    HIPCHK(launch_fill_int(c->d_ctrs, 0, 1, c->stream));
    const StepTarget t{c->d_insts_scr, A_dev, nullptr, j_dev, n_steps, c->d_ctrs};
    for (int s = 0; s < n_steps; ++s) CHK(enqueue_step(c, t));
    c->steps_done += n_steps;
    c->noalloc_steps = true;
    CHK(sync_out(c));
    return TDKS_OK;
}

int tdks_check(tdks_ctx *c, unsigned long long *info) {
    if (!c) return fail(TDKS_E_ARG, "null context");
    const int rc = health_sync(c);
    if (info) std::copy(c->h_health, c->h_health + c->n_inst, info);
    return rc;
}

int tdks_steps_done(tdks_ctx *c) { return c ? c->steps_done : 0; }

int tdks_ground_state(tdks_ctx *c, int n_iter, double tau, double mix, double *residual) {
    if (!c) return fail(TDKS_E_ARG, "null context");
    if (n_iter < 0) return fail(TDKS_E_ARG, "n_iter < 0");
    if (!(tau > 0.0) || !std::isfinite(tau)) return fail(TDKS_E_ARG, "tau must be positive and finite");
    if (!(mix > 0.0 && mix <= 1.0)) return fail(TDKS_E_ARG, "mix must lie in (0, 1]");
    for (int i = 0; i < c->n_inst; ++i) {
        const InstHost &I = c->inst[i];
        if (!I.loaded) return fail(TDKS_E_STATE, "instance %d has no orbitals loaded", i);
        if (I.nb > kOrthMaxBands)
            return fail(TDKS_E_UNSUPPORTED, "instance %d: %d bands; the orthonormalisation holds at most %d",
                        i, I.nb, kOrthMaxBands);
        const double lam = kinetic_bound(I);
        if (tau * lam > 2.5)
            return fail(TDKS_E_ARG, "instance %d: tau %.4g too large for the Taylor-4 filter (kinetic bound %.4g Ha;"
                        " need tau * bound <= 2.5)", i, tau, lam);
    }
    CHK(sync_in(c));
    if (c->n_pairs == 0) {  // first call: its buffers (n_pairs is set only once all exist)
        std::vector<int2> pairs;
        for (int i = 0; i < c->n_inst; ++i)
            for (int k = 0; k < c->inst[i].nk; ++k) pairs.push_back(make_int2(i, k));
        std::vector<int> first(1, 0);
        for (int i = 0; i < c->n_inst; ++i) first.push_back(first.back() + c->inst[i].nk);
        auto drop = [c]() {  // a failed set-up leaves nothing behind, so the next call starts over
            c->release(c->d_pairs);
            c->release(c->d_pair_first);
            c->release(c->d_rho_k);
            c->release(c->d_rho_in);
            c->release(c->d_resid);
            c->release(c->d_status);
            c->d_pairs = nullptr;
            c->d_pair_first = nullptr;
            c->d_rho_k = c->d_rho_in = c->d_resid = nullptr;
            c->d_status = nullptr;
        };
        int rc = upload(c, &c->d_pairs, pairs);
        if (rc == TDKS_OK) rc = upload(c, &c->d_pair_first, first);
        if (rc == TDKS_OK) {
            c->d_rho_k = static_cast<double *>(c->alloc(sizeof(double) * size_t(c->ng_max) * pairs.size()));
            c->d_rho_in = static_cast<double *>(c->alloc(sizeof(double) * size_t(c->ng_max) * c->n_inst));
            c->d_resid = static_cast<double *>(c->alloc(sizeof(double) * c->n_inst));
            c->d_status = static_cast<int *>(c->alloc(sizeof(int)));
            if (!c->d_rho_in || !c->d_resid || !c->d_status || !c->d_rho_k)
                rc = fail(TDKS_E_OOM, "ground-state buffers (%zu bytes of density partials)",
                          sizeof(double) * size_t(c->ng_max) * pairs.size());
        }
        if (rc != TDKS_OK) {
            drop();
            return rc;
        }
        c->n_pairs = int(pairs.size());
    }
    const bool scf = (c->opt.hxc_mode == TDKS_HXC_SCF);
    int nb_max = 1;
    for (int i = 0; i < c->n_inst; ++i) nb_max = std::max(nb_max, c->inst[i].nb);
    const double zero6[6] = {0, 0, 0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(c->d_Aobs, zero6, sizeof(zero6), hipMemcpyHostToDevice, c->stream));
    HIPCHK(launch_fill_int(c->d_ctrs, 0, 3, c->stream));
    HIPCHK(launch_fill_int(c->d_status, 0, 1, c->stream));
    // the mixing starts from the density of the current orbitals (what v_Hxc was built from)
    HIPCHK(hipMemcpyAsync(c->d_rho_in, c->d_rho, sizeof(double) * size_t(c->ng_max) * c->n_inst,
                          hipMemcpyDeviceToDevice, c->stream));
    for (int it = 0; it < n_iter; ++it) {
        CHK(for_classes(c, [&](const ShapeClass &S, hipStream_t st) {
            PropArgs a = class_args(c, S, MODE_ITIME, c->d_Aobs, c->d_ctrs + 2);
            a.dt = tau;
            set_work(c, S, S.wbeg, a);
            HIPCHK(launch_propagate(c->fp64, a, S.wend - S.wbeg, S.block, S.zl, S.minw, S.nonorth, S.sl, S.ragged,
                                    st));
            return TDKS_OK;
        }));
        HIPCHK(launch_orth(c->d_insts, c->d_pairs, c->n_pairs, nb_max, c->fp64, c->d_status, c->d_rho_k, c->ng_max,
                           c->stream));
        HIPCHK(launch_reduce_k(c->d_insts, c->n_inst, c->d_pair_first, c->d_rho_k, c->ng_max, c->d_rho, c->stream));
        HIPCHK(launch_mix(c->d_insts, c->n_inst, c->ng_max, c->d_rho, c->d_rho_in, scf ? mix : 1.0, c->d_resid,
                          c->stream));
        if (scf)
            HIPCHK(launch_hxc(c->d_insts, 0, c->n_inst, c->ng_max, c->d_rho, c->d_vloc, c->d_vhxc, c->d_vtot,
                              c->fp64, c->stream));
    }
    // the prepared state: density, v_Hxc and the current before the field of the final orbitals
    // (and the health check's references)
    CHK(health_reset(c, 0, c->n_inst - 1));
    CHK(enqueue_observe(c, 0, c->n_inst - 1, c->d_jpre, 1));
    if (scf)
        HIPCHK(launch_hxc(c->d_insts, 0, c->n_inst, c->ng_max, c->d_rho, c->d_vloc, c->d_vhxc, c->d_vtot, c->fp64,
                          c->stream));
    int status = 0;
    HIPCHK(hipMemcpyAsync(c->jpre.data(), c->d_jpre, sizeof(double) * 3 * c->n_inst, hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipMemcpyAsync(&status, c->d_status, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    if (residual && n_iter > 0)  // every iteration writes every instance's residual
        HIPCHK(hipMemcpyAsync(residual, c->d_resid, sizeof(double) * c->n_inst, hipMemcpyDeviceToHost, c->stream));
    else if (residual)
        std::fill(residual, residual + c->n_inst, 0.0);
    HIPCHK(launch_fill_int(c->d_ctrs, 0, 3, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->steps_done = 0;
    c->noalloc_steps = false;
    CHK(sync_out(c));
    if (status) return fail(TDKS_E_NUMERIC, "orthonormalisation met linearly dependent bands");
    return TDKS_OK;
}

int tdks_current(tdks_ctx *c, int mode, double *out, size_t cap, size_t *n_written) {
    if (!c || !out) return fail(TDKS_E_ARG, "null argument");
    const size_t ns = size_t(c->steps_done / c->rstride);  // recorded currents
    const size_t rows = (mode == TDKS_PER_GROUP) ? c->groups.size() : size_t(c->n_inst);
    if (mode != TDKS_PER_GROUP && mode != TDKS_PER_INSTANCE) return fail(TDKS_E_ARG, "bad mode");
    if (c->noalloc_steps)
        return fail(TDKS_E_STATE, "steps since the load ran through tdks_step_noalloc, whose currents went to the "
                    "caller's buffer; load again to record");
    if (cap < rows * ns * 3) return fail(TDKS_E_ARG, "capacity %zu < %zu", cap, rows * ns * 3);
    // trace row r of instance i holds J^{(r+1) rstride}
    std::vector<double> tr(size_t(c->n_inst) * 3 * std::max<size_t>(ns, 1));
    CHK(health_sync(c));
    if (ns > 0)
        HIPCHK(hipMemcpy2D(tr.data(), sizeof(double) * 3 * ns, c->d_trace, sizeof(double) * 3 * c->trace_cap,
                           sizeof(double) * 3 * ns, c->n_inst, hipMemcpyDeviceToHost));
    for (int i = 0; i < c->n_inst; ++i)
        for (size_t n = 0; n < ns; ++n)
            for (int q = 0; q < 3; ++q)
                if (!std::isfinite(tr[(size_t(i) * ns + n) * 3 + q]))
                    return fail(TDKS_E_NUMERIC, "non-finite current in instance %d at step %zu", i,
                                (n + 1) * c->rstride);
    if (mode == TDKS_PER_INSTANCE) {
        for (int i = 0; i < c->n_inst; ++i)
            for (size_t n = 0; n < ns; ++n)
                for (int q = 0; q < 3; ++q)
                    out[(size_t(i) * ns + n) * 3 + q] = tr[(size_t(i) * ns + n) * 3 + q] - c->jpre[3 * i + q];
    } else {
        for (size_t gi = 0; gi < c->groups.size(); ++gi) {
            int cnt = 0;
            std::vector<double> acc(3 * ns, 0.0);
            for (int i = 0; i < c->n_inst; ++i) {
                if (c->inst[i].group != c->groups[gi]) continue;
                ++cnt;
                for (size_t n = 0; n < ns; ++n)
                    for (int q = 0; q < 3; ++q)
                        acc[3 * n + q] += tr[(size_t(i) * ns + n) * 3 + q] - c->jpre[3 * i + q];
            }
            for (size_t n = 0; n < 3 * ns; ++n) out[gi * 3 * ns + n] = acc[n] / cnt;
        }
    }
    if (n_written) *n_written = rows * ns * 3;
    return TDKS_OK;
}

int tdks_current_pre(tdks_ctx *c, double *out) {
    if (!c || !out) return fail(TDKS_E_ARG, "null argument");
    std::copy(c->jpre.begin(), c->jpre.end(), out);
    return TDKS_OK;
}

int tdks_current_at(tdks_ctx *c, const double *A, double *out) {
    if (!c || !A || !out) return fail(TDKS_E_ARG, "null argument");
    for (int i = 0; i < c->n_inst; ++i)
        if (!c->inst[i].loaded) return fail(TDKS_E_STATE, "instance %d has no orbitals loaded", i);
    CHK(sync_in(c));
    CHK(observe(c, 0, c->n_inst - 1, A, c->d_jobs));
    HIPCHK(hipMemcpy(out, c->d_jobs, sizeof(double) * 3 * c->n_inst, hipMemcpyDeviceToHost));
    CHK(sync_out(c));
    return TDKS_OK;
}

int tdks_density(tdks_ctx *c, int i, double *rho_out) {
    CHK(check_inst(c, i));
    if (!rho_out) return fail(TDKS_E_ARG, "null output");
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(rho_out, c->d_rho + size_t(i) * c->ng_max, sizeof(double) * c->inst[i].ng, hipMemcpyDeviceToHost));
    return TDKS_OK;
}

int tdks_vhxc(tdks_ctx *c, int i, double *out) {
    CHK(check_inst(c, i));
    if (!out) return fail(TDKS_E_ARG, "null output");
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(out, c->d_vhxc + size_t(i) * c->ng_max, sizeof(double) * c->inst[i].ng, hipMemcpyDeviceToHost));
    return TDKS_OK;
}

int tdks_vloc(tdks_ctx *c, int i, double *out) {
    CHK(check_inst(c, i));
    if (!out) return fail(TDKS_E_ARG, "null output");
    std::copy(c->inst[i].vloc.begin(), c->inst[i].vloc.end(), out);
    return TDKS_OK;
}

int tdks_get_orbitals(tdks_ctx *c, int i, void *u_out, int where) {
    CHK(check_inst(c, i));
    if (!u_out) return fail(TDKS_E_ARG, "null output");
    const InstHost &I = c->inst[i];
    const size_t n = size_t(I.nk) * I.nb * I.ng;
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->fp64) {
        HIPCHK(hipMemcpy(u_out, I.d_u, 16 * n, where == TDKS_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice));
        return TDKS_OK;
    }
    double *dst = static_cast<double *>(u_out);
    double *stage = nullptr;
    if (where == TDKS_HOST) {
        stage = static_cast<double *>(c->alloc(16 * n));
        if (!stage) return fail(TDKS_E_OOM, "staging allocation failed");
        dst = stage;
    }
    HIPCHK(launch_convert_out(I.d_u, dst, n, 0, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (stage) {
        HIPCHK(hipMemcpy(u_out, stage, 16 * n, hipMemcpyDeviceToHost));
        c->release(stage);
    }
    return TDKS_OK;
}

int tdks_norms(tdks_ctx *c, int i, double *out) {
    CHK(check_inst(c, i));
    if (!out) return fail(TDKS_E_ARG, "null output");
    const InstHost &I = c->inst[i];
    double *d = static_cast<double *>(c->alloc(sizeof(double) * I.nk * I.nb));
    if (!d) return fail(TDKS_E_OOM, "allocation failed");
    HIPCHK(launch_norms(I.d_u, I.nk * I.nb, I.ng, I.dV, c->fp64, d, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(out, d, sizeof(double) * I.nk * I.nb, hipMemcpyDeviceToHost));
    c->release(d);
    return TDKS_OK;
}

int tdks_apply_h(tdks_ctx *c, int i, const void *w, void *hw, const double *A, int where) {
    CHK(check_inst(c, i));
    if (!w || !hw || !A) return fail(TDKS_E_ARG, "null argument");
    const InstHost &I = c->inst[i];
    const size_t n = size_t(I.nk) * I.nb * I.ng;
    const size_t cb = c->fp64 ? 16 : 8;
    CHK(sync_in(c));
    double *stage = static_cast<double *>(c->alloc(16 * n));
    void *win = c->alloc(cb * n);
    void *wout = c->alloc(cb * n);
    if (!stage || !win || !wout) return fail(TDKS_E_OOM, "scratch allocation failed");
    HIPCHK(hipMemcpyAsync(stage, w, 16 * n, where == TDKS_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                          c->stream));
    HIPCHK(launch_convert_in(stage, win, n, c->fp64, c->stream));
    double h[6] = {A[0], A[1], A[2], A[0], A[1], A[2]};
    HIPCHK(hipMemcpyAsync(c->d_Aobs, h, sizeof(h), hipMemcpyHostToDevice, c->stream));
    const ShapeClass &S = c->classes[I.cls];
    PropArgs a = class_args(c, S, MODE_APPLY, c->d_Aobs, c->d_ctrs + 2);
    set_work(c, S, I.wbeg, a);
    a.apply_in = win;
    a.apply_out = wout;
    HIPCHK(launch_propagate(c->fp64, a, I.wend - I.wbeg, S.block, S.zl, S.minw, S.nonorth, S.sl, S.ragged,
                            c->stream));
    HIPCHK(launch_convert_out(wout, stage, n, c->fp64, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(hw, stage, 16 * n, where == TDKS_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice));
    c->release(stage);
    c->release(win);
    c->release(wout);
    CHK(sync_out(c));
    return TDKS_OK;
}

int tdks_time_kernels(tdks_ctx *c, int n_steps, const double *A_tab, double *out) {
    if (!c || !out) return fail(TDKS_E_ARG, "null argument");
    if (n_steps <= 0) return fail(TDKS_E_ARG, "n_steps must be positive");
    if (!A_tab) return fail(TDKS_E_ARG, "null A table");
    for (int i = 0; i < c->n_inst; ++i)
        if (!c->inst[i].loaded) return fail(TDKS_E_STATE, "instance %d has no orbitals loaded", i);
    CHK(sync_in(c));
    CHK(ensure_trace(c, size_t(c->steps_done + n_steps) / c->rstride));
    CHK(upload_A(c, n_steps, A_tab));
    // per step: [0] start, [1] after the predictor's propagation, [2] after its tail (PC only),
    // [3] after the step's propagation, [4] end
    std::vector<hipEvent_t> ev(5 * n_steps);
    for (auto &e : ev) HIPCHK(hipEventCreate(&e));
    const bool pc = predictor_corrector(c);
    int rc = TDKS_OK;
    for (int s = 0; s < n_steps && rc == TDKS_OK; ++s) {
        HIPCHK(hipEventRecord(ev[5 * s], c->stream));
        const StepTarget t = own_target(c);
        if (pc) CHK(enqueue_propagation(c, MODE_PREDICT, t));
        HIPCHK(hipEventRecord(ev[5 * s + 1], c->stream));
        if (pc) CHK(enqueue_predictor_tail(c, t));
        HIPCHK(hipEventRecord(ev[5 * s + 2], c->stream));
        CHK(enqueue_propagation(c, MODE_STEP, t));
        HIPCHK(hipEventRecord(ev[5 * s + 3], c->stream));
        CHK(enqueue_step_tail(c, t));
        HIPCHK(hipEventRecord(ev[5 * s + 4], c->stream));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    double tp = 0.0, tr = 0.0;
    for (int s = 0; s < n_steps; ++s) {
        float t[4] = {0.f, 0.f, 0.f, 0.f};
        for (int q = 0; q < 4; ++q) HIPCHK(hipEventElapsedTime(&t[q], ev[5 * s + q], ev[5 * s + q + 1]));
        tp += t[0] + t[2];
        tr += t[1] + t[3];
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    out[0] = tp / n_steps;
    out[1] = tr / n_steps;
    out[2] = (tp + tr) / n_steps;
    c->steps_done += n_steps;
    CHK(sync_out(c));
    return rc;
}

int tdks_tiling(tdks_ctx *c, int *block, int *zl, int *waves_per_simd, int *bands_per_group, int *k_per_group,
                int *n_groups) {
    if (!c) return fail(TDKS_E_ARG, "null context");
    if (waves_per_simd) *waves_per_simd = c->classes.empty() ? 0 : c->classes[0].minw;
    if (block) *block = c->classes.empty() ? 0 : c->classes[0].block;
    if (zl) *zl = c->classes.empty() ? 0 : c->classes[0].zl;
    if (bands_per_group) *bands_per_group = c->work.empty() ? 0 : c->work[0].nb;
    if (k_per_group) *k_per_group = c->work.empty() ? 0 : c->work[0].nk;
    if (n_groups) *n_groups = int(c->work.size());
    return TDKS_OK;
}

}  // extern "C"
