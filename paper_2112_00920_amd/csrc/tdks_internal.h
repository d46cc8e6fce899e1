// Internal structures shared by the host runtime (tdks_runtime.cpp) and the
// device kernels (tdks_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdks {

constexpr int kMaxAtoms = 64;
constexpr int kMaxGridDim = 32;   // N_d <= 32 (DFT lines held in registers; packed j_d + N_d < 256)
constexpr int kMaxPoints = 8192;  // N1 N2 N3 <= 8192 (one orbital per workgroup in LDS)

// Per-instance data visible to the kernels (lives in device memory).
struct DevInst {
    int N[3];
    int ng;
    int nk, nb, nat;
    int nonorth;        // lattice not orthogonal: mixed second derivatives present
    int ntask;          // projection tasks (chunk ranges of one atom)
    double dV, omega;
    double lat[3][3];   // rows a_d
    double hv[3][3];    // rows a_d / N_d (grid step vectors)
    double c[3][3];     // rows c_d = N_d b_d / (2 pi): grad = sum_d c_d d/ds_d
    double g[3][3];     // metric g_de = c_d . c_e
    void *u;            // orbitals [nk][nb][ng], complex R (float2 / double2)
    const void *vtot;   // v_loc + v_Hxc in R precision [ng]
    const double *kcart;  // [nk][3]
    const double *kw;     // [nk]
    const double *occ;    // [nb]
    // projectors (k-independent tables, shared between identical cells).  Support
    // points are grouped by "column image" (atom a, unwrapped in-plane grid offsets
    // j0, j1, reference step r along a_3): d = d_ref + (j2 - r) a_3/N3 with
    // d_ref = j0 a_1/N1 + j1 a_2/N2 + r a_3/N3 - tau_a; r is chosen so that |d_ref|
    // is small, and tables store the relative step j2 - r.
    int ncol;                  // column images
    const int *col_atom;       // [ncol] atom of each column image
    const int *col_j01;        // [ncol] (j0 + N1) | (j1 + N2) << 8 | (r + 128) << 16
    // entries (support points of the column images), point-major: each packs
    // col | (j2 - r + N3 + 3) << 16, with its radial factor g(|d|)
    const int *pt_ptr;         // [ng+1] CSR: entries touching each grid point
    const uint16_t *pt_ptr16;  // same, 16-bit copy (staged into LDS by the FP32 kernel)
    int nent;                  // projector entries
    const uint32_t *pt_pack;   // [nent] packed entries
    const float *pt_gf;        // [nent] radial factors, FP32 copy
    const double *pt_gd;       // [nent] ... FP64 copy
    const void *pt_rec;        // [nent] FP32 only: the same entries interleaved with their radial
                               // factors, {byte offset of the column image's scatter coefficients |
                               // a_3 step << 16, g}
    // chunks: up to 4 consecutive support points of one column image (consecutive j2,
    // no periodic wrap inside), each packed as its first point's grid index p |
    // (j2 - r + N3 + 3) << 13 | col << 20; radial factors g of the 4 points, zero-padded
    const uint32_t *chunk_pack;
    const float *chunk_gf;     // [nchunk][4]
    const double *chunk_gd;    // [nchunk][4]
    const int2 *task;          // [ntask] {first chunk, atom | count << 8}
    const int *atom_task;      // [nat+1] first task of each atom
    const double *atom_tau;    // [nat][3] Cartesian positions
    const double *atom_par;    // [nat][4] Es, Ep, Ns, Np
    // per-step outputs of the propagation kernel
    double *rho_part;   // [nslot][ng] partial densities (one slot per work item)
    double *j_part;     // [nslot][4] partial currents (x, y, z) and charge sum_k w_k sum_b f_b ||u||^2
    int nslot;
    int pad_;
    double *norm0;      // [nk][nb] norms at load (per-orbital health check), or null
};

// Numeric health check of a step (per instance).  The charge Q = sum_k w_k sum_b f_b ||u_bk||^2
// is summed with the current every step; the Taylor-4 step multiplies the squared norm of an
// eigencomponent of the (Hermitian) h by |T4(-i x)|^2 = 1 - x^6/72 + x^8/576, x = dt lambda,
// which is <= 1 for |x| <= 2 sqrt 2 and, below sqrt 6, decreasing in |x|.  With a bound
// lambda_max of |lambda| a step therefore keeps Q within [Q F, Q], F = |T4(-i dt lambda_max)|^2
// (0.25 beyond sqrt 6).  logF holds log F per step (A-table row), lcum its running sum since the
// load.  A violation records (step << 32) | (orbital + 1) << 4 | code in health[inst] (first
// one only): code 1 non-finite current or charge, 2 charge above Q0 (1 + tol), 3 charge below
// Q0 (e^lcum - tol), 4 / 5 an orbital's norm above / below the same bounds.
struct HealthArgs {
    double *q0;                     // [n_inst] charge at load (written when set_ref)
    double *lcum;                   // [n_inst] accumulated log F since load
    const double *logF;             // [A rows] log F of each step, or null: logF_floor every step
    double logF_floor;              // log 0.25, the least |T4(-i x)|^2 over |x| <= 2 sqrt 2
    const int *arow;                // A-table row of the step
    unsigned long long *health;     // [n_inst] first violation, 0 if none (null: no check)
    const int *row_ctr;             // record row of every step instead (or null)
    int set_ref;                    // observe: store Q as Q0 and reset lcum
    int rstride;                    // record every rstride-th current
    double tol;                     // relative tolerance (rounding of the propagation precision)
};

// One workgroup's share: bands [b0, b0+nb) of k-points [k0, k0+nk) of an instance.
struct WorkItem {
    int inst, k0, nk, b0, nb, slot;
};

// Built (column-segment length ZL, max threads per workgroup, min waves per SIMD) triples
// of the propagation kernel.  N3 must be a multiple of ZL (or a ragged tiling is used); the
// block is N1 N2 (N3 / ZL) threads rounded up to whole waves, and a block of more than 8
// waves is padded to 16.
#define TDKS_PROPAGATE_CONFIGS(X) \
    X(2, 512, 2) X(3, 512, 2) X(4, 512, 2) X(6, 512, 2) X(8, 512, 2) X(12, 512, 2) X(16, 512, 2) \
    X(4, 512, 4) X(6, 512, 4) X(8, 512, 4) X(4, 1024, 4) X(8, 1024, 4) X(10, 1024, 4)
// tilings whose last z-segment of a column may be shorter (N3 not a multiple of ZL)
#define TDKS_PROPAGATE_RAGGED_CONFIGS(X) \
    X(4, 512, 4) X(4, 1024, 4) X(8, 512, 2) X(8, 1024, 4) X(10, 1024, 4)

// STEP: real-time Taylor-4 step + density/current partials; OBSERVE: partials only;
// APPLY: one h application; ITIME: imaginary-time Taylor-4 step exp(-tau h) (dt holds tau),
// orbitals stored, no partials; PREDICT: real-time step whose orbitals are not stored, density
// partials only (the predictor of the predictor-corrector step)
enum Mode : int { MODE_STEP = 0, MODE_OBSERVE = 1, MODE_APPLY = 2, MODE_ITIME = 3, MODE_PREDICT = 4 };

constexpr int kOrthMaxBands = 32;  // bands per k the orthonormalisation kernel holds in LDS

struct PropArgs {
    const DevInst *insts;
    const WorkItem *work;
    const double *A_tab;   // [*][2][3]
    const int *step_ctr;   // A_tab row to use
    double dt;
    int mode;
    int ng_max;            // largest grid of the launch (sizes the LDS orbital buffer)
    int ncol_max;          // most projector column images of an instance in the launch
    int nent_max;          // most projector entries of an instance in the launch
    int nmaxd;             // largest N_d of the launch (phase tables)
    int rho_lds;           // accumulate the FP64 density partial in LDS (else in the global slot)
    int nat_max;           // most atoms of an instance in the launch
    int ntask_max;         // most projection tasks of an instance in the launch
    int mixt;              // non-orthogonal cells: mixed derivatives through the LDS intermediate
    char *gcol;            // per-work-item global column tables of the launch (FP64 grids whose tables
                           // do not fit the LDS beside the orbital), or null
    int ptp_lds;           // without LDS-staged records: stage the 16-bit CSR pointers in LDS
    const void *apply_in;  // MODE_APPLY: input orbitals [nk][nb][ng] complex R of instance
    void *apply_out;       // MODE_APPLY: output
};

// Host-side launchers implemented in tdks_kernels.hip.
hipError_t launch_propagate(int fp64, const PropArgs &a, int n_items, int block, int zl, int minw,
                            int nonorth, int sl, int ragged, hipStream_t s);
size_t propagate_lds_bytes(int fp64, int sl, const PropArgs &a, int block);
size_t propagate_gcol_stride(int fp64, int ncol_max);  // bytes of one work item's global column tables
bool propagate_config_ok(int block, int zl, int minw, int ragged);
hipError_t launch_reduce(const DevInst *insts, int inst0, int n, int ng_max, double *rho,
                         double *jout, int jstride, const int *step_ctr, const HealthArgs &h, hipStream_t s);
hipError_t launch_health_norms(const DevInst *insts, const WorkItem *work, int n_items, const int *step_ctr,
                               int stride, const HealthArgs &h, int fp64, hipStream_t s);
hipError_t launch_hxc(const DevInst *insts, int inst0, int n, int ng_max, const double *rho,
                      const double *vloc, double *vhxc, void *vtot, int fp64, hipStream_t s);
hipError_t launch_vtot(const DevInst *insts, int inst0, int n, int ng_max, const double *vloc,
                       const double *vhxc, void *vtot, int fp64, hipStream_t s);
hipError_t launch_vmid(const DevInst *insts, int n, int ng_max, const double *vloc, const double *va,
                       const double *vb, void *vtot, int fp64, hipStream_t s);
hipError_t launch_advance(int *ctrs, int n, hipStream_t s);
hipError_t launch_fill_int(int *p, int v, int n, hipStream_t s);
hipError_t launch_convert_in(const double *src, void *dst, size_t n_complex, int fp64, hipStream_t s);
hipError_t launch_convert_out(const void *src, double *dst, size_t n_complex, int fp64, hipStream_t s);
hipError_t launch_norms(const void *u, int n_orb, int ng, double dV, int fp64, double *out, hipStream_t s);
hipError_t launch_orth(const DevInst *insts, const int2 *pairs, int n_pairs, int nb_max, int fp64, int *status,
                       double *rho_k, int ng_max, hipStream_t s);
hipError_t launch_reduce_k(const DevInst *insts, int n_inst, const int *first, const double *rho_k, int ng_max,
                           double *rho, hipStream_t s);
hipError_t launch_mix(const DevInst *insts, int n_inst, int ng_max, double *rho, double *rho_in, double alpha,
                      double *resid, hipStream_t s);

}  // namespace tdks
