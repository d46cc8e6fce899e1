// Device code of the propagation kernel for CDNA4 (gfx950): real-time TDKS
// propagation of Bloch orbitals (Sato, arXiv:2112.00920, Sec. II.A, Eqs. 1-6) on
// a real-space grid.
//
// k_propagate: one workgroup owns bands [b0, b0+nb) of k-points [k0, k0+nk) of
//   one instance.  Each orbital lives in LDS for the whole Taylor-4 step and the
//   running Taylor sum stays in registers, so HBM sees one read and one write of
//   every orbital per step.  Thread t owns the column (i0, i1) of the grid over a
//   z-segment of ZL points; z neighbours come from registers, in-plane ones from
//   LDS.  Per application of h (Eq. 2):
//     1. projections c_{a,lm} = dV sum_p f_lm(d) e^{i kappa.d} w(p) over the
//        atom-major support list (fixed-length tasks, one wave each);
//     2. 4th-order FD kinetic stencil (13 points; 61 for non-orthogonal cells)
//        + (v_loc + v_Hxc) w + sum_a e^{-i kappa.d} sum_lm f_lm E_l c_{a,lm}
//        (point-major support list);
//     3. w <- (-i dt / m) h w, acc += w.
//   Projector geometry is stored per "column image" (atom a, unwrapped in-plane
//   offsets j0, j1, reference step r along a_3): d = dcol + j2 a_3/N3 with
//   dcol = j0 a_1/N1 + j1 a_2/N2 + r a_3/N3 - tau_a and j2 counted from r, and
//   e^{i kappa.d} = colphase * e^{i j2 kappa.a_3/N3}; both factors are rebuilt in
//   LDS once per k-point.  After the step the new orbital yields FP64
//   partials of the density (Eq. 3) and of the current (Eqs. 5-6) with
//   kappa = k + A(t_{n+1}).
#pragma once
#include "tdks_internal.h"

#include <math.h>

namespace tdks {

template <typename R> struct CT;
template <> struct CT<float> { using T = float2; using Q = float4; };
template <> struct CT<double> { using T = double2; using Q = double4; };

template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
    T r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename T> __device__ __forceinline__ T cmulc(T a, T b) {  // conj(a) * b
    T r;
    r.x = a.x * b.x + a.y * b.y;
    r.y = a.x * b.y - a.y * b.x;
    return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the 64 lanes of a wave with DPP moves (VALU latency, no LDS round trips):
// quad all-reduce, half-row and row mirrors give every lane its row sum; row_bcast:15
// and row_bcast:31 then fold the rows so that lane 63 holds the total, which is
// broadcast with readlane.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_f(float v) {
    return __builtin_bit_cast(float, dpp_i<CTRL, ROWMASK>(__builtin_bit_cast(int, v)));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_i<CTRL, ROWMASK>(int(b & 0xffffffffll));
    const int hi = dpp_i<CTRL, ROWMASK>(int(b >> 32));
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ float wave_total(float v) {
    v += dpp_f<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += dpp_f<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += dpp_f<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_f<0x140, 0xF>(v);  // row_mirror
    v += dpp_f<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ double wave_total(double v) {
    v += dpp_d<0xB1, 0xF>(v);
    v += dpp_d<0x4E, 0xF>(v);
    v += dpp_d<0x141, 0xF>(v);
    v += dpp_d<0x140, 0xF>(v);
    v += dpp_d<0x142, 0xA>(v);
    v += dpp_d<0x143, 0xC>(v);
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), 63);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Wave total of FP32 values with an FP64 result: each row of 16 lanes is summed in
// FP32 (as the per-lane partials are), the four row sums in FP64.
__device__ __forceinline__ double wave_total_wide(float v) {
    v += dpp_f<0xB1, 0xF>(v);
    v += dpp_f<0x4E, 0xF>(v);
    v += dpp_f<0x141, 0xF>(v);
    v += dpp_f<0x140, 0xF>(v);
    double d = double(v);
    d += dpp_d<0x142, 0xA>(d);
    d += dpp_d<0x143, 0xC>(d);
    const long long b = __builtin_bit_cast(long long, d);
    const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), 63);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
__device__ __forceinline__ double wave_total_wide(double v) { return wave_total(v); }

// Wave totals of four values at once.  v_permlane32_swap exchanges rows 2-3 of its first
// operand with rows 0-1 of its second and v_permlane16_swap the odd rows of the first with
// the even rows of the second (rows of 16 lanes), so adding a swapped pair folds the rows
// of two values into one register.  Two folds leave v0..v3 in rows 0..3 of one register,
// each summed lane by lane over the four rows; DPP then sums each row, and every lane of
// row r holds the total of v_r.
__device__ __forceinline__ unsigned fbits(float x) { return __builtin_bit_cast(unsigned, x); }
__device__ __forceinline__ float bitsf(unsigned x) { return __builtin_bit_cast(float, x); }
__device__ __forceinline__ float fold32(float x, float y) {
    const auto r = __builtin_amdgcn_permlane32_swap(fbits(x), fbits(y), false, false);
    return bitsf(r[0]) + bitsf(r[1]);  // rows: x r0+r2, x r1+r3, y r0+r2, y r1+r3
}
__device__ __forceinline__ float fold16(float x, float y) {
    const auto r = __builtin_amdgcn_permlane16_swap(fbits(x), fbits(y), false, false);
    return bitsf(r[0]) + bitsf(r[1]);  // rows: x r0+r1, y r0+r1, x r2+r3, y r2+r3
}
__device__ __forceinline__ double fold32(double x, double y) {
    const long long bx = __builtin_bit_cast(long long, x), by = __builtin_bit_cast(long long, y);
    const auto lo = __builtin_amdgcn_permlane32_swap(unsigned(bx), unsigned(by), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(unsigned(bx >> 32), unsigned(by >> 32), false, false);
    const double x2 = __builtin_bit_cast(double, (static_cast<long long>(hi[0]) << 32) | lo[0]);
    const double y2 = __builtin_bit_cast(double, (static_cast<long long>(hi[1]) << 32) | lo[1]);
    return x2 + y2;
}
__device__ __forceinline__ double fold16(double x, double y) {
    const long long bx = __builtin_bit_cast(long long, x), by = __builtin_bit_cast(long long, y);
    const auto lo = __builtin_amdgcn_permlane16_swap(unsigned(bx), unsigned(by), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(unsigned(bx >> 32), unsigned(by >> 32), false, false);
    const double x2 = __builtin_bit_cast(double, (static_cast<long long>(hi[0]) << 32) | lo[0]);
    const double y2 = __builtin_bit_cast(double, (static_cast<long long>(hi[1]) << 32) | lo[1]);
    return x2 + y2;
}
__device__ __forceinline__ float row_total(float v) {
    v += dpp_f<0xB1, 0xF>(v);
    v += dpp_f<0x4E, 0xF>(v);
    v += dpp_f<0x141, 0xF>(v);
    v += dpp_f<0x140, 0xF>(v);
    return v;
}
__device__ __forceinline__ double row_total(double v) {
    v += dpp_d<0xB1, 0xF>(v);
    v += dpp_d<0x4E, 0xF>(v);
    v += dpp_d<0x141, 0xF>(v);
    v += dpp_d<0x140, 0xF>(v);
    return v;
}
template <typename R> __device__ __forceinline__ R totals4(R v0, R v1, R v2, R v3) {
    return row_total(fold16(fold32(v0, v2), fold32(v1, v3)));
}
// the same with the four-row folds in the input precision and the row sums in FP64
__device__ __forceinline__ double totals4_wide(float v0, float v1, float v2, float v3) {
    return row_total(double(fold16(fold32(v0, v2), fold32(v1, v3))));
}
__device__ __forceinline__ double totals4_wide(double v0, double v1, double v2, double v3) {
    return totals4(v0, v1, v2, v3);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane(int(b >> 32), l);
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// 4th-order central differences (+-2 neighbours)
#define D1C1 (2.0 / 3.0)
#define D1C2 (-1.0 / 12.0)
#define D2C0 (-5.0 / 2.0)
#define D2C1 (4.0 / 3.0)
#define D2C2 (-1.0 / 12.0)

// scatter entry staged in LDS by the FP32 kernel: the byte offset of its column image's
// coefficients (low half) and its stored a_3 step (bits 16-23), with the radial factor
template <typename R> struct PtRec;
template <> struct PtRec<float> {
    uint32_t pk;
    float g;
};
template <> struct PtRec<double> {
    uint32_t pk, pad;
    double g;
};

// Shared-memory layout of k_propagate (bytes, 16-aligned), identical on host and device.
struct PropLds {
    size_t W, cold, colm, cole, t2m, t2e, apar, part, tsk, atk, ab, wacc, nlm, ptp, ptk, rho, tmix, total;
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

// With gcol the per-column-image tables (geometry, the two phase tables, the scatter
// coefficients) live in a per-workgroup global buffer instead (prop_gcol), so that FP64
// orbitals of grids up to 8192 points fit the LDS.
__host__ __device__ inline PropLds prop_lds(int fp64, int sl, int ng_max, int ncol_max, int nent_max,
                                            int nmaxd, int nat_max, int ntask_max, int block,
                                            int rho_lds, int mixt, int gcol = 0, int ptpl = 0) {
    const size_t c = fp64 ? 16 : 8;  // complex
    const size_t r = fp64 ? 8 : 4;   // real
    const int na = nat_max > 0 ? nat_max : 1;
    const int nc = gcol ? 0 : (ncol_max > 0 ? ncol_max : 1);
    PropLds L;
    size_t o = 0;
    L.W = o; o = al16(o + c * size_t(ng_max));
    L.cold = o; o = al16(o + 4 * r * nc);
    L.colm = o; o = al16(o + c * nc);
    L.cole = o; o = al16(o + c * nc);
    L.t2m = o; o = al16(o + c * (3 * nmaxd + 6));
    L.t2e = o; o = al16(o + c * (3 * nmaxd + 6));
    L.apar = o; o = al16(o + 4 * r * na);
    L.part = o; o = al16(o + c * 4 * (ntask_max > 0 ? ntask_max : 1));
    L.tsk = o; o = al16(o + 8 * size_t(ntask_max > 0 ? ntask_max : 1));  // task list
    L.atk = o; o = al16(o + 4 * size_t(na + 1));                        // first task of each atom
    L.ab = o; o = al16(o + 2 * c * nc);                  // scatter coefficients per column image
    L.wacc = o; o = al16(o + 8 * 4 * size_t(block / 64));  // FP64 current partial per wave
    L.nlm = o; o = al16(o + 8 * 20 * size_t(ntask_max > 0 ? ntask_max : 1));  // current moments per task
    // point-major projector tables staged in LDS (sl): 16-bit CSR, packed entries, radial factors
    L.ptp = o; o = al16(o + ((sl || ptpl) ? 2 * size_t(ng_max + 1) : 0));
    L.ptk = o; o = al16(o + (sl ? (fp64 ? 16 : 8) * size_t(nent_max) : 0));  // PtRec records
    L.rho = o; o = al16(o + (rho_lds ? 8 * size_t(ng_max) : 0));  // FP64 density partial
    L.tmix = o; o = al16(o + (mixt ? c * size_t(ng_max) : 0));      // mixed-derivative intermediate
    L.total = o;
    return L;
}

inline size_t propagate_lds_bytes_inl(int fp64, int sl, const PropArgs &a, int block) {
    return prop_lds(fp64, sl, a.ng_max, a.ncol_max, a.nent_max, a.nmaxd, a.nat_max, a.ntask_max,
                    block, a.rho_lds, a.mixt, a.gcol != nullptr, a.ptp_lds).total;
}

// Layout of one workgroup's global column tables (bytes, 256-aligned stride): geometry, phase
// at the mid-step, phase at the step's end, scatter coefficients.
struct PropGcol {
    size_t cold, colm, cole, ab, stride;
};
__host__ __device__ inline PropGcol prop_gcol(int fp64, int ncol_max) {
    const size_t c = fp64 ? 16 : 8, r = fp64 ? 8 : 4;
    const size_t nc = ncol_max > 0 ? size_t(ncol_max) : 1;
    PropGcol G;
    size_t o = 0;
    G.cold = o; o = al16(o + 4 * r * nc);
    G.colm = o; o = al16(o + c * nc);
    G.cole = o; o = al16(o + c * nc);
    G.ab = o; o = al16(o + 2 * c * nc);
    G.stride = (o + 255) & ~size_t(255);
    return G;
}

// Uniform real value forced into a scalar register (VALU instructions then read it as
// their scalar operand instead of holding a copy per lane).
__device__ __forceinline__ float uni(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ double uni(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readfirstlane(int(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane(int(b >> 32));
    return __builtin_bit_cast(double, (static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Opaque copy of a value: stops loop-invariant code motion from hoisting address
// arithmetic derived from it out of the band / Taylor loops (which would keep one
// register per neighbour address alive for the whole kernel).
__device__ __forceinline__ int opq(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Global-address-space view of a pointer read from device memory: lets the compiler
// emit global (not flat) loads with a scalar base.
#define TDKS_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ const TDKS_GLOBAL T *gview(const T *p) {
    return (const TDKS_GLOBAL T *)p;
}
template <typename T> __device__ __forceinline__ TDKS_GLOBAL T *gview_w(T *p) { return (TDKS_GLOBAL T *)p; }
// two-component vector types go through clang native vectors for global loads/stores
template <typename T> struct NV2;
template <> struct NV2<float2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct NV2<double2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct NV2<int2> { typedef int type __attribute__((ext_vector_type(2))); };
template <typename T> __device__ __forceinline__ T gld(const T *p) {
    const auto v = *(const TDKS_GLOBAL typename NV2<T>::type *)p;
    T r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
template <typename T> __device__ __forceinline__ void gst(T *p, T x) {
    typename NV2<T>::type v;
    v.x = x.x;
    v.y = x.y;
    *(TDKS_GLOBAL typename NV2<T>::type *)p = v;
}

// four-component global load (chunk radial factors)
template <typename Q> struct NV4;
template <> struct NV4<float4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct NV4<double4> { typedef double type __attribute__((ext_vector_type(4))); };
template <typename Q> __device__ __forceinline__ Q gld4(const Q *p) {
    const auto v = *(const TDKS_GLOBAL typename NV4<Q>::type *)p;
    Q r;
    r.x = v.x;
    r.y = v.y;
    r.z = v.z;
    r.w = v.w;
    return r;
}

template <typename R> __device__ __forceinline__ const R *chunktab(const DevInst &I);
template <> __device__ __forceinline__ const float *chunktab<float>(const DevInst &I) { return I.chunk_gf; }
template <> __device__ __forceinline__ const double *chunktab<double>(const DevInst &I) { return I.chunk_gd; }
template <typename R> __device__ __forceinline__ const R *ptgtab(const DevInst &I);
template <> __device__ __forceinline__ const float *ptgtab<float>(const DevInst &I) { return I.pt_gf; }
template <> __device__ __forceinline__ const double *ptgtab<double>(const DevInst &I) { return I.pt_gd; }


// Non-local current of one atom from the 20 totals m (re, im) of its moments over one orbital,
// M0 = sum g x, M1_a = sum g d_a x, M2_ab = sum g d_a d_b x (ab = 00 11 22 01 02 12), x the
// orbital times the conjugate Bloch phase, g the radial factor and d the offset from the atom.
// With c = <P|u> and c_d = <d P|u> the commutator term is sum_lm 2 E_l Im(conj(c_d,lm) c_lm);
// for f_s = N_s g and f_p,i = N_p g d_i that is, per axis a,
//   E_s N_s^2 Im(conj(M1_a) M0) + E_p N_p^2 sum_i Im(conj(M2_ia) M1_i).
// Adds scale times it to j.
__device__ __forceinline__ void nl_current(const double *m, double Es, double Ep, double ns, double np,
                                           double scale, double *j) {
    const int qi[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    const double ws = Es * ns * ns, wp = Ep * np * np;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double px = m[2 + 2 * d], py = m[3 + 2 * d];
        double v = ws * (px * m[1] - py * m[0]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int q = qi[i][d];
            v += wp * (m[8 + 2 * q] * m[3 + 2 * i] - m[9 + 2 * q] * m[2 + 2 * i]);
        }
        j[d] += scale * v;
    }
}

// NONORTH: 0 orthogonal cell (13-point stencil); 1 non-orthogonal, mixed derivatives
// -sum_{d<e} g_de D1_d D1_e w formed directly (16 neighbours per pair); 2 non-orthogonal with the
// pairs (0,1) and (0,2) factorised through an LDS intermediate,
//   -g_01 D1_0 D1_1 w - g_02 D1_0 D1_2 w = D1_0 T,  T = -g_01 D1_1 w - g_02 D1_2 w,
// formed while the projections run (before their barrier), and the pair (1,2) direct.
// GC: the per-column-image tables in the work item's part of a.gcol (global memory, read and
// written only by this workgroup, ordered by its barriers) instead of LDS.
// SL: 1 the point-major projector records and their CSR pointers staged in LDS; 2 the CSR
// pointers only (records read from global memory); 0 both from global memory.
template <typename R, int ZL, int NONORTH, int MAXT, int MINW, int SL, bool RAGGED, bool ITIME, bool GC = false>
__global__ __launch_bounds__(MAXT) __attribute__((amdgpu_waves_per_eu(MINW, 8)))
void k_propagate(PropArgs a) {
    using C = typename CT<R>::T;
    using Q4 = typename CT<R>::Q;
    extern __shared__ __align__(16) char smem[];
    // the work item is uniform over the workgroup: keep it (and the instance) in scalar registers
    const WorkItem *wp = a.work + blockIdx.x;
    const int w_inst = __builtin_amdgcn_readfirstlane(wp->inst);
    const int w_k0 = __builtin_amdgcn_readfirstlane(wp->k0);
    const int w_nk = __builtin_amdgcn_readfirstlane(wp->nk);
    const int w_b0 = __builtin_amdgcn_readfirstlane(wp->b0);
    const int w_nb = __builtin_amdgcn_readfirstlane(wp->nb);
    const int w_slot = __builtin_amdgcn_readfirstlane(wp->slot);
    const DevInst &I = a.insts[w_inst];
    const int ng = I.ng;
    const int N0 = I.N[0], N1 = I.N[1], N2 = I.N[2];
    const int BS = blockDim.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int NW = BS >> 6;

    const PropLds L = prop_lds(sizeof(R) == 8, SL == 1, a.ng_max, a.ncol_max, a.nent_max, a.nmaxd,
                               a.nat_max, a.ntask_max, BS, a.rho_lds, NONORTH == 2, GC, SL == 2);
    constexpr bool ptpl = SL == 2;
    const PropGcol G = prop_gcol(sizeof(R) == 8, a.ncol_max);
    char *gcb = GC ? a.gcol + size_t(blockIdx.x) * G.stride : nullptr;
    C *W = reinterpret_cast<C *>(smem + L.W);
    Q4 *cold = reinterpret_cast<Q4 *>(GC ? gcb + G.cold : smem + L.cold);  // dcol.xyz, atom index
    C *colm = reinterpret_cast<C *>(GC ? gcb + G.colm : smem + L.colm);    // column phase, kappa(t_n + dt/2)
    C *cole = reinterpret_cast<C *>(GC ? gcb + G.cole : smem + L.cole);    // column phase, kappa(t_{n+1})
    C *t2m = reinterpret_cast<C *>(smem + L.t2m);           // e^{i j2 kappa.a_3/N3}, mid
    C *t2e = reinterpret_cast<C *>(smem + L.t2e);           // same, kappa(t_{n+1})
    Q4 *apar = reinterpret_cast<Q4 *>(smem + L.apar);       // Es dV, Ep dV, Ns, Np per atom
    C *part = reinterpret_cast<C *>(smem + L.part);
    int2 *task_l = reinterpret_cast<int2 *>(smem + L.tsk);
    int *atk_l = reinterpret_cast<int *>(smem + L.atk);
    Q4 *AB = reinterpret_cast<Q4 *>(GC ? gcb + G.ab : smem + L.ab);  // scatter coefficients A, B per column image
    double *wacc = reinterpret_cast<double *>(smem + L.wacc);  // current partial per wave (x, y, z, -)
    double *nlm = reinterpret_cast<double *>(smem + L.nlm);    // non-local current moments per task
    uint16_t *ptp_l = reinterpret_cast<uint16_t *>(smem + L.ptp);
    PtRec<R> *ptk_l = reinterpret_cast<PtRec<R> *>(smem + L.ptk);
    double *RHO = reinterpret_cast<double *>(smem + L.rho);
    C *TM = reinterpret_cast<C *>(smem + L.tmix);
    const bool rho_lds = sizeof(R) == 4 && a.rho_lds != 0;  // the FP64 kernels keep it in HBM

    const auto *vtot = gview(reinterpret_cast<const R *>(I.vtot));
    const auto *pgt = gview(ptgtab<R>(I));
    const auto *chunk_pack = gview(I.chunk_pack);
    const Q4 *chunk_g = reinterpret_cast<const Q4 *>(chunktab<R>(I));
    const auto *pt_ptr = gview(I.pt_ptr);
    const auto *pt_pack = gview(I.pt_pack);
    // FP32 scatter records in device memory (read here once: the instance table is global
    // memory, which the kernel's stores could alias, so a read inside the loops is repeated)
    const TDKS_GLOBAL PtRec<R> *pt_recs =
        (SL != 1 && sizeof(R) == 4) ? gview(reinterpret_cast<const PtRec<R> *>(I.pt_rec)) : nullptr;
    const int2 *task = I.task;
    const auto *atom_task = gview(I.atom_task);
    const auto *kcart = gview(I.kcart);
    const int plane = N0 * N1;
    const int j2off = N2 + 3;  // stored a_3 steps are j2 + N3 + 3 (j2 counted from the reference step)
    // z-segments of ZL points; with RAGGED the last one of a column is shorter (N3 % ZL)
    const int nseg = RAGGED ? (N2 + ZL - 1) / ZL : N2 / ZL;
    const bool active = tid < plane * nseg;
    const int i0 = tid % N0, i1 = (tid / N0) % N1, seg = tid / plane;
    const int z0 = seg * ZL;
    const int zlen = RAGGED ? min(ZL, N2 - z0) : ZL;  // points of this thread's segment
#define TDKS_ZOK(z) (!RAGGED || (z) < zlen)
    const int pbase = i0 + N0 * i1;  // p(z) = pbase + plane * z
    // in-plane neighbour offsets: +1, -1, +2, -2 along a_1 and a_2 (periodic)
    int ox[4], oy[4];
    ox[0] = (i0 + 1 < N0) ? 1 : 1 - N0;
    ox[1] = (i0 >= 1) ? -1 : N0 - 1;
    ox[2] = (i0 + 2 < N0) ? 2 : 2 - N0;
    ox[3] = (i0 >= 2) ? -2 : N0 - 2;
    oy[0] = ((i1 + 1 < N1) ? 1 : 1 - N1) * N0;
    oy[1] = ((i1 >= 1) ? -1 : N1 - 1) * N0;
    oy[2] = ((i1 + 2 < N1) ? 2 : 2 - N1) * N0;
    oy[3] = ((i1 >= 2) ? -2 : N1 - 2) * N0;

    const double *Am = a.A_tab + 6 * (*a.step_ctr);
    for (int i = tid; i < 4 * NW; i += BS) wacc[i] = 0.0;
    const double dV = I.dV;
    const int nat = I.nat;
    const int ntask = I.ntask;
    const int ncol = I.ncol;
    const R h2x = uni(R(I.hv[2][0])), h2y = uni(R(I.hv[2][1])), h2z = uni(R(I.hv[2][2]));

    // k-independent projector geometry of this instance into LDS
    for (int c = tid; c < ncol; c += BS) {
        const int at = I.col_atom[c];
        const int j01 = I.col_j01[c];
        const double j0 = double((j01 & 255) - N0), j1 = double(((j01 >> 8) & 255) - N1);
        const double jr = double(((j01 >> 16) & 255) - 128);
        const double *tau = I.atom_tau + 3 * at;
        Q4 q;
        q.x = R(j0 * I.hv[0][0] + j1 * I.hv[1][0] + jr * I.hv[2][0] - tau[0]);
        q.y = R(j0 * I.hv[0][1] + j1 * I.hv[1][1] + jr * I.hv[2][1] - tau[1]);
        q.z = R(j0 * I.hv[0][2] + j1 * I.hv[1][2] + jr * I.hv[2][2] - tau[2]);
        q.w = R(at);
        cold[c] = q;
    }
    for (int at = tid; at < nat; at += BS) {
        const double *par = I.atom_par + 4 * at;
        Q4 q;
        q.x = R(par[0] * dV);
        q.y = R(par[1] * dV);
        q.z = R(par[2]);
        q.w = R(par[3]);
        apar[at] = q;
    }
    for (int i = tid; i <= nat; i += BS) atk_l[i] = I.atom_task[i];
    for (int i = tid; i < ntask; i += BS) task_l[i] = gld(task + i);

    if (SL != 0) {
        const auto *p16 = gview(I.pt_ptr16);
        for (int i = tid; i <= ng; i += BS) ptp_l[i] = p16[i];
    }
    if (SL == 1) {
        for (int e = tid; e < I.nent; e += BS) {
            const uint32_t pk = pt_pack[e];  // column image | stored a_3 step << 16
            PtRec<R> rec;
            rec.pk = (sizeof(R) == 4) ? ((pk & 0xffffu) * uint32_t(sizeof(Q4))) | (pk & 0xffff0000u) : pk;
            rec.g = pgt[e];
            ptk_l[e] = rec;
        }
    }

    // v_loc + v_Hxc of the owned points: kept in registers for short segments and FP64, read
    // from global memory (cache-resident) in every h application for long FP32 segments, whose
    // 128-register budget it would otherwise push into spills (20^3: 14 % faster)
    constexpr bool VREG = ZL <= 4 || sizeof(R) == 8;
    R vz[VREG ? ZL : 1];
#pragma unroll
    for (int z = 0; z < (VREG ? ZL : 0); ++z) {
        vz[z] = (active && TDKS_ZOK(z)) ? vtot[pbase + plane * (z0 + z)] : R(0);
    }

    // Laplacian coefficients (metric only)
    R a1[3], a2[3], cx[3];
    double c0l = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a1[d] = uni(R(-0.5 * I.g[d][d] * D2C1));
        a2[d] = uni(R(-0.5 * I.g[d][d] * D2C2));
        c0l += -0.5 * I.g[d][d] * D2C0;
    }
    cx[0] = uni(R(-I.g[0][1]));  // -(1/2) * 2 g_de for d < e
    cx[1] = uni(R(-I.g[0][2]));
    cx[2] = uni(R(-I.g[1][2]));
    const int norder = (a.mode == MODE_STEP || a.mode == MODE_PREDICT || ITIME) ? 4 : (a.mode == MODE_APPLY ? 1 : 0);
    // non-local current of a band: its per-task moment totals are combined per atom (in task
    // order) after the next barrier, with the band's weight kept in fo_prev
    double fo_prev = 0.0;
    bool nl_pending = false;
    auto nl_combine = [&]() {
#pragma unroll 1
        for (int at = wave; at < nat; at += NW) {
            // lane c < 20 adds up component c over the atom's tasks; the totals are then read
            // out as wave-uniform values
            const int c = (lane < 20) ? lane : 0;
            double s = 0.0;
            for (int tt = atk_l[at]; tt < atk_l[at + 1]; ++tt) s += nlm[20 * tt + c];
            double m[20];
#pragma unroll
            for (int q = 0; q < 20; ++q) m[q] = readlane_d(s, q);
            const double *par = I.atom_par + 4 * at;
            double j[3] = {0.0, 0.0, 0.0};
            nl_current(m, par[0], par[1], par[2], par[3], 2.0 * dV * dV, j);
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < 3; ++q) wacc[4 * wave + q] += fo_prev * j[q];
            }
        }
    };

#pragma unroll 1
    for (int kk = 0; kk < w_nk; ++kk) {
        const int k = w_k0 + kk;
        // kappa-dependent coefficients: -i kappa.grad_FD and |kappa|^2 / 2, kappa = k + A(t_n + dt/2)
        R b1[3], b2[3];
        R c0;
        {
            double km[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) km[d] = kcart[3 * k + d] + Am[d];
            const double kk2 = km[0] * km[0] + km[1] * km[1] + km[2] * km[2];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double kc = km[0] * I.c[d][0] + km[1] * I.c[d][1] + km[2] * I.c[d][2];
                b1[d] = uni(R(kc * D1C1));
                b2[d] = uni(R(kc * D1C2));
            }
            c0 = uni(R(c0l + 0.5 * kk2));
        }

        // phases: column images and the a_3 factor, for kappa(t_n + dt/2) and kappa(t_{n+1})
        __syncthreads();
        const double inv_pi = 0.3183098861837907;
        double km[3], ke[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            km[d] = kcart[3 * k + d] + Am[d];
            ke[d] = kcart[3 * k + d] + Am[3 + d];
        }
        for (int c = tid; c < ncol; c += BS) {
            const int at = I.col_atom[c];
            const int j01 = I.col_j01[c];
            const double j0 = double((j01 & 255) - N0), j1 = double(((j01 >> 8) & 255) - N1);
            const double jr = double(((j01 >> 16) & 255) - 128);
            const double *tau = I.atom_tau + 3 * at;
            double dcx = j0 * I.hv[0][0] + j1 * I.hv[1][0] + jr * I.hv[2][0] - tau[0];
            double dcy = j0 * I.hv[0][1] + j1 * I.hv[1][1] + jr * I.hv[2][1] - tau[1];
            double dcz = j0 * I.hv[0][2] + j1 * I.hv[1][2] + jr * I.hv[2][2] - tau[2];
            double sm, cm, se, ce;
            sincospi((km[0] * dcx + km[1] * dcy + km[2] * dcz) * inv_pi, &sm, &cm);
            sincospi((ke[0] * dcx + ke[1] * dcy + ke[2] * dcz) * inv_pi, &se, &ce);
            C t;
            t.x = R(cm);
            t.y = R(sm);
            colm[c] = t;
            t.x = R(ce);
            t.y = R(se);
            cole[c] = t;
        }
        {
            const double thm = (km[0] * I.hv[2][0] + km[1] * I.hv[2][1] + km[2] * I.hv[2][2]) * inv_pi;
            const double the = (ke[0] * I.hv[2][0] + ke[1] * I.hv[2][1] + ke[2] * I.hv[2][2]) * inv_pi;
            for (int j = tid; j < 3 * N2 + 6; j += BS) {
                double sm, cm, se, ce;
                sincospi(double(j - j2off) * thm, &sm, &cm);
                sincospi(double(j - j2off) * the, &se, &ce);
                C t;
                t.x = R(cm);
                t.y = R(sm);
                t2m[j] = t;
                t.x = R(ce);
                t.y = R(se);
                t2e[j] = t;
            }
        }

#pragma unroll 1
        for (int bb = 0; bb < w_nb; ++bb) {
            const int b = w_b0 + bb;
            const size_t orb = (size_t(k) * I.nb + b) * size_t(ng);
            C *ug = reinterpret_cast<C *>(I.u) + orb;
            const C *src = (a.mode == MODE_APPLY) ? reinterpret_cast<const C *>(a.apply_in) + orb : ug;
            // Taylor sum: for short segments the terms are summed in registers,
            //   acc = sum_m w_m, w_m = (-i dt/m) h w_{m-1};
            // long FP32 segments, short of registers, evaluate the same polynomial by Horner's
            // rule, v <- u + (-i dt/m) h v for m = 4, 3, 2, 1 (v = u first), re-reading u from
            // global memory (cache-resident) and keeping v in LDS only (W), not in registers
            constexpr bool HORNER = !VREG;
            C acc[ZL];
            const int pl = opq(pbase + plane * z0);
            // the orbital's loads are issued before the barrier, so their latency overlaps
            // the wait for the other waves
#pragma unroll
            for (int z = 0; z < ZL; ++z) {
                C v;
                v.x = R(0);
                v.y = R(0);
                if (active && TDKS_ZOK(z)) v = gld(src + pl + plane * z);
                acc[z] = v;
            }
            __syncthreads();  // previous users of W (and the phase tables) are done
            if (nl_pending) {  // the previous band's split non-local current
                nl_combine();
                nl_pending = false;
            }
            if (active) {
#pragma unroll
                for (int z = 0; z < ZL; ++z)
                    if (TDKS_ZOK(z)) W[pl + plane * z] = acc[z];
            }

#pragma unroll 1
            for (int m = 1; m <= norder; ++m) {
                __syncthreads();  // W holds w_{m-1}
                // ---- 1. projections c = <P|w> (tasks of chunks of one atom, one wave each).
                // On a chunk (points j2_0 + i, i < 4, of one column image) with x_i = t2(j2_i) w_i g_i:
                //   sum g d e^{i kappa.d} w = colphase (d_0 X0 + (a_3/N3) X1),
                //   d_0 = dcol + j2_0 a_3/N3 (the first point's offset), X0 = sum x_i, X1 = sum i x_i.
                for (int t = wave; t < ntask; t += NW) {
                    const int2 tk = task_l[t];
                    const int c0 = tk.x, cnt = tk.y >> 8, at = tk.y & 255;
                    C s[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) { s[l].x = R(0); s[l].y = R(0); }
                    for (int ci = lane; ci < cnt; ci += 64) {
                        const uint32_t cp = chunk_pack[c0 + ci];
                        const Q4 g4 = gld4(chunk_g + c0 + ci);
                        const int p0 = int(cp & 8191u), j2u0 = int((cp >> 13) & 127u), col = int(cp >> 20);
                        const R gg[4] = {g4.x, g4.y, g4.z, g4.w};
                        C y0, y1;
                        y0.x = R(0); y0.y = R(0); y1.x = R(0); y1.y = R(0);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            C x = cmul(t2m[j2u0 + i], W[p0 + plane * i]);
                            x.x *= gg[i];
                            x.y *= gg[i];
                            y0.x += x.x;
                            y0.y += x.y;
                            if (i > 0) {
                                y1.x += R(i) * x.x;
                                y1.y += R(i) * x.y;
                            }
                        }
                        const C ph = colm[col];
                        const Q4 cd = cold[col];
                        const C X0 = cmul(ph, y0), X1 = cmul(ph, y1);
                        const R j20 = R(j2u0 - j2off);
                        const R d0x = cd.x + j20 * h2x, d0y = cd.y + j20 * h2y, d0z = cd.z + j20 * h2z;
                        s[0].x += X0.x;
                        s[0].y += X0.y;
                        s[1].x += d0x * X0.x + h2x * X1.x;
                        s[1].y += d0x * X0.y + h2x * X1.y;
                        s[2].x += d0y * X0.x + h2y * X1.x;
                        s[2].y += d0y * X0.y + h2y * X1.y;
                        s[3].x += d0z * X0.x + h2z * X1.x;
                        s[3].y += d0z * X0.y + h2z * X1.y;
                    }
                    // row l of (re, im) holds channel l's totals; the first lane of each row stores it
                    const R re = totals4(s[0].x, s[1].x, s[2].x, s[3].x);
                    const R im = totals4(s[0].y, s[1].y, s[2].y, s[3].y);
                    if ((lane & 15) == 0) {
                        const int l = lane >> 4;
                        const Q4 ap = apar[at];  // N_s, N_p in .z, .w
                        const R f = (l == 0) ? ap.z : ap.w;
                        C v;
                        v.x = f * re;
                        v.y = f * im;
                        part[4 * t + l] = v;
                    }
                }
                // Non-orthogonal cells: everything of h w at the owned points that needs no
                // in-plane a_1 neighbour is formed here, from the column w(z0 - 2 .. z0 + ZL + 1)
                // and its D1_1 w, which this phase reads anyway for the intermediate T: the a_2
                // and a_3 parts of the stencil, the mixed pair (1, 2) = cx2 D1_2 D1_1 w, and the
                // potential when it sits in registers. The sum is kept in registers until the
                // stencil, which then adds only the a_1 part, D1_0 T and the non-local term.
                C hpre[NONORTH == 2 ? ZL : 1];
                if (NONORTH == 2 && active) {
                    // mixed-derivative intermediate of the owned points, T = cx0 D1_1 w + cx1 D1_2 w
                    const int pt = opq(pbase);
                    int oyt[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) oyt[q] = opq(oy[q]);
                    C gyh[ZL + 4];  // D1_1 w at z0 - 2 + j
                    C wcol[ZL + 4];  // w itself there
                    C hy[ZL];        // a_2 part of the stencil at the owned points
#pragma unroll
                    for (int j = 0; j < ZL + 4; ++j) {
                        gyh[j].x = R(0);
                        gyh[j].y = R(0);
                        wcol[j] = gyh[j];
                        if (j >= 2 && j < ZL + 2) hy[j - 2] = gyh[j];
                        if (!TDKS_ZOK(j - 4)) continue;
                        int zw = z0 + j - 2;
                        zw = zw < 0 ? zw + N2 : (zw >= N2 ? zw - N2 : zw);
                        const int p = pt + plane * zw;
                        const C y1 = W[p + oyt[0]], y2 = W[p + oyt[1]], y3 = W[p + oyt[2]], y4 = W[p + oyt[3]];
                        wcol[j] = W[p];
                        C d1, d2;
                        d1.x = y1.x - y2.x;
                        d1.y = y1.y - y2.y;
                        d2.x = y3.x - y4.x;
                        d2.y = y3.y - y4.y;
                        gyh[j].x = R(D1C1) * d1.x + R(D1C2) * d2.x;
                        gyh[j].y = R(D1C1) * d1.y + R(D1C2) * d2.y;
                        if (j >= 2 && j < ZL + 2) {
                            C e;
                            e.x = fma(a1[1], y1.x + y2.x, R(0));
                            e.x = fma(a2[1], y3.x + y4.x, e.x);
                            e.x = fma(b1[1], d1.y, e.x);
                            e.x = fma(b2[1], d2.y, e.x);
                            e.y = fma(a1[1], y1.y + y2.y, R(0));
                            e.y = fma(a2[1], y3.y + y4.y, e.y);
                            e.y = fma(-b1[1], d1.x, e.y);
                            e.y = fma(-b2[1], d2.x, e.y);
                            hy[j - 2] = e;
                        }
                    }
#pragma unroll
                    for (int z = 0; z < ZL; ++z) {
                        hpre[NONORTH == 2 ? z : 0].x = R(0);
                        hpre[NONORTH == 2 ? z : 0].y = R(0);
                        if (!TDKS_ZOK(z)) continue;
                        const int zg = z0 + z;
                        const int p = pt + plane * zg;
                        const C gy = gyh[z + 2];  // D1_1 w
                        const C z1p = wcol[z + 3], z1m = wcol[z + 1], z2p = wcol[z + 4], z2m = wcol[z];
                        C gz;                     // D1_2 w
                        gz.x = R(D1C1) * (z1p.x - z1m.x) + R(D1C2) * (z2p.x - z2m.x);
                        gz.y = R(D1C1) * (z1p.y - z1m.y) + R(D1C2) * (z2p.y - z2m.y);
                        C tv;
                        tv.x = cx[0] * gy.x + cx[1] * gz.x;
                        tv.y = cx[0] * gy.y + cx[1] * gz.y;
                        TM[p] = tv;
                        // h so far: potential (from registers), a_2 and a_3 parts, pair (1, 2)
                        C hv;
                        if (VREG) {
                            const R cv = c0 + vz[VREG ? z : 0];
                            const C cen = wcol[z + 2];
                            hv.x = cv * cen.x;
                            hv.y = cv * cen.y;
                        } else {
                            hv.x = R(0);
                            hv.y = R(0);
                        }
                        hv.x += hy[z].x;
                        hv.y += hy[z].y;
                        hv.x = fma(a1[2], z1p.x + z1m.x, hv.x);
                        hv.x = fma(a2[2], z2p.x + z2m.x, hv.x);
                        hv.x = fma(b1[2], z1p.y - z1m.y, hv.x);
                        hv.x = fma(b2[2], z2p.y - z2m.y, hv.x);
                        hv.y = fma(a1[2], z1p.y + z1m.y, hv.y);
                        hv.y = fma(a2[2], z2p.y + z2m.y, hv.y);
                        hv.y = fma(-b1[2], z1p.x - z1m.x, hv.y);
                        hv.y = fma(-b2[2], z2p.x - z2m.x, hv.y);
                        const C a1p = gyh[z + 3], a1m = gyh[z + 1], a2p = gyh[z + 4], a2m = gyh[z];
                        hv.x += cx[2] * (R(D1C1) * (a1p.x - a1m.x) + R(D1C2) * (a2p.x - a2m.x));
                        hv.y += cx[2] * (R(D1C1) * (a1p.y - a1m.y) + R(D1C2) * (a2p.y - a2m.y));
                        hpre[NONORTH == 2 ? z : 0] = hv;
                    }
                }
                __syncthreads();
                // scatter coefficients per column image: on the column the non-local term is
                //   e^{-i kappa.d} sum_lm f_lm(d) E_l c_lm = g conj(t2(j2)) (A + j2 B),
                //   A = conj(colphase) (N_s e_s + N_p dcol.e_p),  B = conj(colphase) N_p (a_3/N3).e_p,
                // with e_lm = E_l dV c_lm and d = dcol + j2 a_3/N3.
                for (int c = tid; c < ncol; c += BS) {
                    const Q4 cd = cold[c];
                    const int at = int(cd.w);
                    const Q4 ap = apar[at];
                    C e[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) { e[l].x = R(0); e[l].y = R(0); }
                    for (int t = atk_l[at]; t < atk_l[at + 1]; ++t) {
#pragma unroll
                        for (int l = 0; l < 4; ++l) {
                            const C v = part[4 * t + l];
                            e[l].x += v.x;
                            e[l].y += v.y;
                        }
                    }
                    C k1, k2;
                    k1.x = ap.z * ap.x * e[0].x + ap.w * ap.y * (cd.x * e[1].x + cd.y * e[2].x + cd.z * e[3].x);
                    k1.y = ap.z * ap.x * e[0].y + ap.w * ap.y * (cd.x * e[1].y + cd.y * e[2].y + cd.z * e[3].y);
                    k2.x = ap.w * ap.y * (h2x * e[1].x + h2y * e[2].x + h2z * e[3].x);
                    k2.y = ap.w * ap.y * (h2x * e[1].y + h2y * e[2].y + h2z * e[3].y);
                    const C ph = colm[c];
                    const C A = cmulc(ph, k1), B = cmulc(ph, k2);
                    Q4 q;
                    q.x = A.x;
                    q.y = A.y;
                    q.z = B.x;
                    q.w = B.y;
                    AB[c] = q;
                }
                __syncthreads();
                // ---- 2. h w along the owned column segment
                // (opaque copies keep the compiler from hoisting every neighbour address
                // out of the band and Taylor loops, which would pin them in registers; the
                // orthogonal kernels, with fewer neighbours, run faster with the in-plane
                // offsets hoisted: 16^3 step launch -1.1 %, 20^3 -1.3 %)
                const int pb = opq(pbase);
                int oxl[4], oyl[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    oxl[s] = NONORTH ? opq(ox[s]) : ox[s];
                    oyl[s] = NONORTH ? opq(oy[s]) : oy[s];
                }
                C hz[ZL];
                // long FP32 segments and the FP64 kernels of orthogonal cells walk the column
                // with a window of five values (z - 2 .. z + 2) in registers, one LDS read per
                // point for the centre and the a_3 neighbours (20^3 FP32: spills 18 -> 9, step
                // -3.8 %; FP64 -0.4 %); the 4-point FP32 segments read them like the in-plane ones
                // (with the window: 0.6 % slower), and a copy of a whole long segment spilled
                constexpr bool WIN = NONORTH == 0 && (!VREG || sizeof(R) == 8);
                C win[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) {
                    win[q].x = R(0);
                    win[q].y = R(0);
                }
                if (WIN && active) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        int zw = z0 - 2 + q;
                        zw = zw < 0 ? zw + N2 : (zw >= N2 ? zw - N2 : zw);
                        win[q] = W[pb + plane * zw];
                    }
                }
#pragma unroll
                for (int z = 0; z < ZL; ++z) {
                    hz[z].x = R(0);
                    hz[z].y = R(0);
                    if (!active || !TDKS_ZOK(z)) continue;
                    const int zg = z0 + z;
                    const int p = pb + plane * zg;
                    if (WIN) {  // a ring: position zg + d sits in win[(z + d + 2) % 5]
                        int zw = zg + 2;
                        zw = zw >= N2 ? zw - N2 : zw;
                        win[(z + 4) % 5] = W[pb + plane * zw];
                    }
                    C zn[4];  // +1, -1, +2, -2
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        zn[s].x = R(0);
                        zn[s].y = R(0);
                        if (NONORTH == 2) continue;  // the a_3 part came with hpre
                        if (WIN) {
                            zn[s] = win[(z + ((s == 0) ? 3 : (s == 1) ? 1 : (s == 2) ? 4 : 0)) % 5];
                            continue;
                        }
                        const int dz = (s == 0) ? 1 : (s == 1) ? -1 : (s == 2) ? 2 : -2;
                        int zw = zg + dz;
                        zw = zw < 0 ? zw + N2 : (zw >= N2 ? zw - N2 : zw);
                        zn[s] = W[pb + plane * zw];
                    }
                    // FP32 records in device memory: this point's range and first record are
                    // requested before the stencil arithmetic, which covers their latency
                    int se0 = 0, se1 = 0;
                    PtRec<R> rfirst;
                    rfirst.pk = 0u;
                    rfirst.g = R(0);
                    if (SL != 1 && sizeof(R) == 4) {
                        se0 = ptpl ? int(ptp_l[p]) : pt_ptr[p];
                        se1 = ptpl ? int(ptp_l[p + 1]) : pt_ptr[p + 1];
                        if (se0 < se1) {
                            rfirst.pk = pt_recs[se0].pk;
                            rfirst.g = pt_recs[se0].g;
                        }
                    }
                    C cen;
                    cen.x = R(0);
                    cen.y = R(0);
                    if (WIN) cen = win[(z + 2) % 5];
                    else if (NONORTH != 2 || !VREG) cen = W[p];
                    // a potential read from memory (long FP32 segments) enters after the
                    // kinetic sums, so that the arithmetic before it covers the load's latency
                    const R vmem = VREG ? R(0) : vtot[p];
                    C h;
                    if (NONORTH == 2) {
                        h = hpre[NONORTH == 2 ? z : 0];
                    } else if (VREG) {
                        const R cv = c0 + vz[VREG ? z : 0];
                        h.x = cv * cen.x;
                        h.y = cv * cen.y;
                    } else {
                        h.x = R(0);
                        h.y = R(0);
                    }
#pragma unroll
                    for (int d = 0; d < (NONORTH == 2 ? 1 : 3); ++d) {
                        C p1, m1, p2, m2;
                        if (d == 0) {
                            p1 = W[p + oxl[0]]; m1 = W[p + oxl[1]]; p2 = W[p + oxl[2]]; m2 = W[p + oxl[3]];
                        } else if (d == 1) {
                            p1 = W[p + oyl[0]]; m1 = W[p + oyl[1]]; p2 = W[p + oyl[2]]; m2 = W[p + oyl[3]];
                        } else {
                            p1 = zn[0]; m1 = zn[1]; p2 = zn[2]; m2 = zn[3];
                        }
                        // a1 (p1 + m1) + a2 (p2 + m2) - i (b1 (p1 - m1) + b2 (p2 - m2)), one
                        // multiply-add per neighbour pair and component
                        h.x = fma(a1[d], p1.x + m1.x, h.x);
                        h.x = fma(a2[d], p2.x + m2.x, h.x);
                        h.x = fma(b1[d], p1.y - m1.y, h.x);
                        h.x = fma(b2[d], p2.y - m2.y, h.x);
                        h.y = fma(a1[d], p1.y + m1.y, h.y);
                        h.y = fma(a2[d], p2.y + m2.y, h.y);
                        h.y = fma(-b1[d], p1.x - m1.x, h.y);
                        h.y = fma(-b2[d], p2.x - m2.x, h.y);
                    }
                    if (!VREG) {
                        const R cv = c0 + vmem;
                        h.x = fma(cv, cen.x, h.x);
                        h.y = fma(cv, cen.y, h.y);
                    }
                    if (NONORTH == 2) {
                        // pairs (0, 1) and (0, 2): D1_0 T (the pair (1, 2) came with hpre)
                        const C tp1 = TM[p + oxl[0]], tm1 = TM[p + oxl[1]];
                        const C tp2 = TM[p + oxl[2]], tm2 = TM[p + oxl[3]];
                        h.x += R(D1C1) * (tp1.x - tm1.x) + R(D1C2) * (tp2.x - tm2.x);
                        h.y += R(D1C1) * (tp1.y - tm1.y) + R(D1C2) * (tp2.y - tm2.y);
                    }
                    if (NONORTH == 1) {
                        // - sum_{d<e} g_de D1_d D1_e w, all from LDS
                        int oz[4];
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            const int dz = (s == 0) ? 1 : (s == 1) ? -1 : (s == 2) ? 2 : -2;
                            int zw = zg + dz;
                            zw = zw < 0 ? zw + N2 : (zw >= N2 ? zw - N2 : zw);
                            oz[s] = plane * (zw - zg);
                        }
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            if (cx[q] == R(0)) continue;
                            C tot;
                            tot.x = R(0);
                            tot.y = R(0);
#pragma unroll
                            for (int t = 0; t < 4; ++t) {
                                const int oe = (q == 0) ? oyl[t] : oz[t];
                                const int o0 = (q == 2) ? oyl[0] : oxl[0], o1 = (q == 2) ? oyl[1] : oxl[1];
                                const int o2 = (q == 2) ? oyl[2] : oxl[2], o3 = (q == 2) ? oyl[3] : oxl[3];
                                const C pp1 = W[p + oe + o0], mm1 = W[p + oe + o1];
                                const C pp2 = W[p + oe + o2], mm2 = W[p + oe + o3];
                                const R ix = R(D1C1) * (pp1.x - mm1.x) + R(D1C2) * (pp2.x - mm2.x);
                                const R iy = R(D1C1) * (pp1.y - mm1.y) + R(D1C2) * (pp2.y - mm2.y);
                                const R ct = (t == 0) ? R(D1C1) : (t == 1) ? R(-D1C1)
                                           : (t == 2) ? R(D1C2) : R(-D1C2);
                                tot.x += ct * ix;
                                tot.y += ct * iy;
                            }
                            h.x += cx[q] * tot.x;
                            h.y += cx[q] * tot.y;
                        }
                    }
                    // non-local part: projector entries touching p,
                    //   h += g conj(t2(j2)) (A + j2 B) of the entry's column image
                    auto scatter_one = [&](uint32_t pk, R gv, const Q4 &q) {
                        const int j2u = int((pk >> 16) & 255u);
                        const C t2 = t2m[j2u];
                        const R j2 = R(j2u - j2off);
                        C s;
                        s.x = (q.x + j2 * q.z) * gv;
                        s.y = (q.y + j2 * q.w) * gv;
                        h.x = fma(t2.x, s.x, h.x);  // h += conj(t2) * s
                        h.x = fma(t2.y, s.y, h.x);
                        h.y = fma(t2.x, s.y, h.y);
                        h.y = fma(-t2.y, s.x, h.y);
                    };
                    if (SL == 1) {  // LDS records; FP32 records hold the byte offset of the coefficients
                        const PtRec<R> *r1 = ptk_l + int(ptp_l[p + 1]);
                        for (const PtRec<R> *r = ptk_l + int(ptp_l[p]); r != r1; ++r) {
                            const PtRec<R> rec = *r;
                            const Q4 q = (sizeof(R) == 4)
                                ? *reinterpret_cast<const Q4 *>(reinterpret_cast<const char *>(AB) + (rec.pk & 0xffffu))
                                : AB[rec.pk & 0xffffu];
                            scatter_one(rec.pk, rec.g, q);
                        }
                    } else if (sizeof(R) == 4) {  // FP32: the same records in global memory, one load each
                        PtRec<R> rec = rfirst;
                        for (int e = se0; e < se1; ++e) {
                            PtRec<R> nx = rec;  // the next record is requested before this one is used
                            if (e + 1 < se1) {
                                nx.pk = pt_recs[e + 1].pk;
                                nx.g = pt_recs[e + 1].g;
                            }
                            const Q4 q = *reinterpret_cast<const Q4 *>(reinterpret_cast<const char *>(AB) + (rec.pk & 0xffffu));
                            scatter_one(rec.pk, rec.g, q);
                            rec = nx;
                        }
                    } else {  // FP64: packed entries and radial factors from their own arrays
                        const int e1 = pt_ptr[p + 1];
                        for (int e = pt_ptr[p]; e < e1; ++e) {
                            const uint32_t pk = pt_pack[e];
                            scatter_one(pk, pgt[e], AB[pk & 0xffffu]);
                        }
                    }
                    hz[z] = h;
                }
                __syncthreads();  // all reads of W done
                const int pw = opq(pbase + plane * z0);
                if (a.mode == MODE_APPLY) {
                    C *out = reinterpret_cast<C *>(a.apply_out) + orb;
                    if (active) {
#pragma unroll
                        for (int z = 0; z < ZL; ++z)
                            if (TDKS_ZOK(z)) gst(out + pw + plane * z, hz[z]);
                    }
                }
                if (!HORNER || a.mode != MODE_APPLY) {
                    // the Taylor update; the register-sum form runs it in MODE_APPLY too (one
                    // order: the sum is discarded, nothing is written to W), which spares the
                    // step's loop a merge of the sums at every order
                    // dt/m through a reciprocal of the (wave-uniform) order: one multiply
                    // instead of a double-precision division per thread
                    const int mo = HORNER ? norder + 1 - m : m;  // Horner runs the orders backwards
                    const double rm = (mo == 1) ? 1.0 : (mo == 2) ? 0.5 : (mo == 3) ? (1.0 / 3.0) : 0.25;
                    const R cm = R(a.dt * rm);
                    // Horner: u of the owned points, requested together so that their latencies
                    // overlap (one at a time, the loads wait for each other)
                    C uh[HORNER ? ZL : 1];
                    if (HORNER) {
#pragma unroll
                        for (int z = 0; z < (HORNER ? ZL : 0); ++z) {
                            uh[z].x = R(0);
                            uh[z].y = R(0);
                            if (active && TDKS_ZOK(z)) uh[z] = gld(src + pw + plane * z);
                        }
                    }
#pragma unroll
                    for (int z = 0; z < ZL; ++z) {
                        C wn;  // (-i dt/m) h w, or (-tau/m) h w in imaginary time (dt holds tau)
                        if (ITIME) {
                            wn.x = -cm * hz[z].x;
                            wn.y = -cm * hz[z].y;
                        } else {
                            wn.x = cm * hz[z].y;
                            wn.y = -cm * hz[z].x;
                        }
                        if (HORNER) {  // v <- u + wn, into W also after the last order
                            const C u0 = uh[HORNER ? z : 0];
                            wn.x += u0.x;
                            wn.y += u0.y;
                            if (active && TDKS_ZOK(z)) W[pw + plane * z] = wn;
                        } else {
                            acc[z].x += wn.x;
                            acc[z].y += wn.y;
                            // the last term is only summed: the next writer of W is the store below
                            if (active && TDKS_ZOK(z) && m < norder) W[pw + plane * z] = wn;
                        }
                    }
                }
            }
            if (a.mode == MODE_APPLY) continue;

            // ---- new orbital: store; FP64 partials of density (in LDS or in this work item's
            // global slot; only this thread touches these points) and current.  No barrier is
            // needed before the LDS store: after the last h application every read of W has
            // passed the barrier that precedes the Taylor update, and each thread stores only
            // its own points (with no Taylor terms W already holds the same values).
            const double fo = I.kw[k] * I.occ[b];
            const int ps = opq(pbase + plane * z0);
            if (active) {
                auto *rp = gview_w(I.rho_part + size_t(w_slot) * ng);
                const bool first = (kk == 0) && (bb == 0);
#pragma unroll
                for (int z = 0; z < ZL; ++z) {
                    if (!TDKS_ZOK(z)) continue;
                    const int p = ps + plane * z;
                    C fin;  // the new orbital (Horner: already in W, written by this thread)
                    if (HORNER) {
                        fin = W[p];
                    } else {
                        fin = acc[z];
                        W[p] = fin;
                    }
                    if (a.mode == MODE_STEP || ITIME) gst(ug + p, fin);
                    const double ux = double(fin.x), uy = double(fin.y);
                    const double r = fo * (ux * ux + uy * uy);
                    if (rho_lds)
                        RHO[p] = first ? r : RHO[p] + r;
                    else
                        rp[p] = first ? r : rp[p] + r;
                }
            }
            // no current: imaginary time, predictor
            if (ITIME || a.mode == MODE_PREDICT) continue;
            __syncthreads();
            // per-thread sums over the owned points in the orbital precision, FP64 beyond.
            // Summed over the whole periodic grid, sum_p Im(conj(u_p) (u_{p+s} - u_{p-s}))
            // = 2 sum_p Im(conj(u_p) u_{p+s}), so only forward neighbours are needed:
            // Q_d = sum Im(conj(u) D1_d u) = 2 (D1C1 q1_d + D1C2 q2_d).
            R q1[3] = {R(0), R(0), R(0)}, q2[3] = {R(0), R(0), R(0)};
            R qn[4] = {R(0), R(0), R(0), R(0)};
            const int pk0 = opq(pbase);
            const int oxk1 = opq(ox[0]), oxk2 = opq(ox[2]), oyk1 = opq(oy[0]), oyk2 = opq(oy[2]);
            if (active) {
#pragma unroll
                for (int z = 0; z < ZL; ++z) {
                    if (!TDKS_ZOK(z)) continue;
                    const int zg = z0 + z;
                    const int p = pk0 + plane * zg;
                    // FP64: the register sums still hold this thread's new values, and the centre
                    // and the a_3 neighbours inside the segment come from them, the rest from LDS
                    // (two-step FP64 -0.5 %; the FP32 16^3 kernel ran 0.7 % slower with it)
                    constexpr bool ACCU = !HORNER && sizeof(R) == 8;
                    const C u = ACCU ? acc[ACCU ? z : 0] : W[p];
                    qn[3] += u.x * u.x + u.y * u.y;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        C u1, u2;
                        if (d == 0) {
                            u1 = W[p + oxk1];
                            u2 = W[p + oxk2];
                        } else if (d == 1) {
                            u1 = W[p + oyk1];
                            u2 = W[p + oyk2];
                        } else {
#pragma unroll
                            for (int s = 1; s <= 2; ++s) {
                                C v;
                                if (ACCU && z + s < ZL && TDKS_ZOK(z + s)) {
                                    v = acc[ACCU ? (z + s < ZL ? z + s : 0) : 0];
                                } else {
                                    const int zw = (zg + s >= N2) ? zg + s - N2 : zg + s;
                                    v = W[pk0 + plane * zw];
                                }
                                if (s == 1) u1 = v; else u2 = v;
                            }
                        }
                        q1[d] = fma(u.x, u1.y, q1[d]);
                        q1[d] = fma(-u.y, u1.x, q1[d]);
                        q2[d] = fma(u.x, u2.y, q2[d]);
                        q2[d] = fma(-u.y, u2.x, q2[d]);
                    }
                }
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) qn[d] = R(2) * (R(D1C1) * q1[d] + R(D1C2) * q2[d]);
            // non-local current moments of the orbital over the projector chunks (the tasks of
            // the projections).  On a chunk with x_i = t2(j2_i) u_i g_i and d_i = d_0 + i a_3/N3:
            //   M0 = ph Y0, M1 = ph (d_0 Y0 + h Y1), M2_ab = ph (d0_a d0_b Y0 + (d0_a h_b + d0_b h_a) Y1
            //   + h_a h_b Y2), Y_n = sum i^n x_i, h = a_3/N3.  Per-lane sums in the orbital
            // precision, cross-lane totals in FP64, one row of 20 per task.
            const R hh[3] = {h2x, h2y, h2z};
#pragma unroll 1
            for (int t = wave; t < ntask; t += NW) {
                const int2 tk = task_l[t];
                const int c0 = tk.x, cnt = tk.y >> 8;
                C m0, m1[3], m2[6];
                m0.x = R(0);
                m0.y = R(0);
#pragma unroll
                for (int i = 0; i < 3; ++i) { m1[i].x = R(0); m1[i].y = R(0); }
#pragma unroll
                for (int i = 0; i < 6; ++i) { m2[i].x = R(0); m2[i].y = R(0); }
                for (int ci = lane; ci < cnt; ci += 64) {
                    const uint32_t cp = chunk_pack[c0 + ci];
                    const Q4 g4 = gld4(chunk_g + c0 + ci);
                    const int p0 = int(cp & 8191u), j2u0 = int((cp >> 13) & 127u), col = int(cp >> 20);
                    const R gg[4] = {g4.x, g4.y, g4.z, g4.w};
                    C y0, y1, y2;
                    y0.x = R(0); y0.y = R(0); y1.x = R(0); y1.y = R(0); y2.x = R(0); y2.y = R(0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        C x = cmul(t2e[j2u0 + i], W[p0 + plane * i]);
                        x.x *= gg[i];
                        x.y *= gg[i];
                        y0.x += x.x;
                        y0.y += x.y;
                        if (i > 0) {
                            y1.x += R(i) * x.x;
                            y1.y += R(i) * x.y;
                            y2.x += R(i * i) * x.x;
                            y2.y += R(i * i) * x.y;
                        }
                    }
                    const C ph = cole[col];
                    const Q4 cd = cold[col];
                    const C X0 = cmul(ph, y0), X1 = cmul(ph, y1), X2 = cmul(ph, y2);
                    const R j20 = R(j2u0 - j2off);
                    const R d0[3] = {cd.x + j20 * h2x, cd.y + j20 * h2y, cd.z + j20 * h2z};
                    m0.x += X0.x;
                    m0.y += X0.y;
#pragma unroll
                    for (int a2 = 0; a2 < 3; ++a2) {
                        m1[a2].x += d0[a2] * X0.x + hh[a2] * X1.x;
                        m1[a2].y += d0[a2] * X0.y + hh[a2] * X1.y;
                    }
                    const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
                    for (int q = 0; q < 6; ++q) {
                        const int i = pa[q], k = pb[q];
                        const R f0 = d0[i] * d0[k], f1 = d0[i] * hh[k] + d0[k] * hh[i], f2 = hh[i] * hh[k];
                        m2[q].x += f0 * X0.x + f1 * X1.x + f2 * X2.x;
                        m2[q].y += f0 * X0.y + f1 * X1.y + f2 * X2.y;
                    }
                }
                // totals of the 20 components, four per register: row r of g[i] holds component
                // 4 i + r; the rows' first lanes store them
                double g[5];
                g[0] = totals4_wide(m0.x, m0.y, m1[0].x, m1[0].y);
                g[1] = totals4_wide(m1[1].x, m1[1].y, m1[2].x, m1[2].y);
                g[2] = totals4_wide(m2[0].x, m2[0].y, m2[1].x, m2[1].y);
                g[3] = totals4_wide(m2[2].x, m2[2].y, m2[3].x, m2[3].y);
                g[4] = totals4_wide(m2[4].x, m2[4].y, m2[5].x, m2[5].y);
                if ((lane & 15) == 0) {
#pragma unroll
                    for (int i = 0; i < 5; ++i) nlm[20 * t + 4 * i + (lane >> 4)] = g[i];
                }
            }
            if (nat > 0) {
                fo_prev = fo;
                nl_pending = true;
            }
            // wave totals of the kinetic sums; each wave adds its share of this band's
            // current into its own FP64 slot (a fixed order, no atomics)
            double qt[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) qt[d] = wave_total_wide(qn[d]);
            if (lane == 0) {
                const double nrm = qt[3] * dV;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const double kin = dV * (I.c[0][q] * qt[0] + I.c[1][q] * qt[1] + I.c[2][q] * qt[2]);
                    const double keq = kcart[3 * k + q] + Am[3 + q];
                    wacc[4 * wave + q] += fo * (kin + keq * nrm);
                }
                wacc[4 * wave + 3] += fo * nrm;  // charge, for the numeric health check
            }
        }
    }
    if (a.mode == MODE_APPLY || ITIME) return;
    if (rho_lds && active) {
        auto *rp = gview_w(I.rho_part + size_t(w_slot) * ng);
        const int pr = opq(pbase + plane * z0);
#pragma unroll
        for (int z = 0; z < ZL; ++z)
            if (TDKS_ZOK(z)) rp[pr + plane * z] = RHO[pr + plane * z];
    }
    __syncthreads();
    if (nl_pending) {  // the last band's split non-local current
        nl_combine();
        __syncthreads();
    }
    if (tid < 4) {  // current (x, y, z) and charge of this work item
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += wacc[4 * w + tid];
        auto *jp = gview_w(I.j_part + 4 * w_slot);
        jp[tid] = s;
    }
#undef TDKS_ZOK
}

}  // namespace tdks
