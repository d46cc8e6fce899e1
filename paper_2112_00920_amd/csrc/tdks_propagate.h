// Device code of the propagation kernel for CDNA4 (gfx950): real-time TDKS propagation of Bloch orbitals
// (Sato, arXiv:2112.00920, Sec. II.A Eqs. 1-6) on a real-space grid.
//
// k_propagate: one workgroup owns bands [b0, b0+nb) of k-points [k0, k0+nk) of
//   one instance.  Each orbital lives in LDS for the whole Taylor-4 step; the
//   running Taylor sum stays in registers, so HBM sees one read and one write
//   of every orbital per step.  Per application of h (Eq. 2):
//     1. projection c_{a,lm} = sum_p f_lm(d) e^{i kappa.d} w(p) dV over the
//        atom-major support list, split into fixed-length tasks per wave;
//     2. 4th-order FD kinetic stencil (13 points, 61 for non-orthogonal cells)
//        read from LDS, + (v_loc + v_Hxc) w, + sum_e e^{-i kappa.d} f E c
//        (point-major list);
//     3. w <- (-i dt / m) h w, acc += w.
//   After the step the new orbital gives FP64 partials of the density (Eq. 3)
//   and of the current (Eqs. 5-6) with kappa = k + A(t_{n+1}).
// k_reduce: deterministic FP64 sum of the per-workgroup partials.
// k_hxc: one workgroup per instance: Poisson by separable DFT in LDS, Slater
//   exchange + PZ81 correlation, new v_Hxc and v_loc + v_Hxc.
#pragma once
#include "tdks_internal.h"

#include <math.h>

namespace tdks {

template <typename R> struct CT;
template <> struct CT<float> { using T = float2; };
template <> struct CT<double> { using T = double2; };

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

// 4th-order central differences (+-2 neighbours)
#define D1C1 (2.0 / 3.0)
#define D1C2 (-1.0 / 12.0)
#define D2C0 (-5.0 / 2.0)
#define D2C1 (4.0 / 3.0)
#define D2C2 (-1.0 / 12.0)

// Shared-memory layout of k_propagate (bytes, 16-aligned), identical on host and device.
struct PropLds {
    size_t W, tab_mid, tab_end, aph_mid, aph_end, part, ec, red, total;
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline PropLds prop_lds(int fp64, int ng_max, int nmaxd, int nat_max,
                                            int ntask_max, int block) {
    size_t c = fp64 ? 16 : 8;
    PropLds L;
    size_t o = 0;
    L.W = o; o = al16(o + c * ng_max);
    L.tab_mid = o; o = al16(o + c * 9 * nmaxd);
    L.tab_end = o; o = al16(o + 16 * 9 * nmaxd);
    L.aph_mid = o; o = al16(o + c * nat_max);
    L.aph_end = o; o = al16(o + 16 * nat_max);
    L.part = o; o = al16(o + c * 4 * (ntask_max > 0 ? ntask_max : 1));
    L.ec = o; o = al16(o + c * 4 * (nat_max > 0 ? nat_max : 1));
    L.red = o; o = al16(o + 8 * 8 * (block / 64 + 1));
    L.total = o;
    return L;
}

inline size_t propagate_lds_bytes_inl(int fp64, const PropArgs &a, int block) {
    return prop_lds(fp64, a.ng_max, a.nmaxd, a.nat_max, a.ntask_max, block).total;
}

// Block-wide sum of K <= 8 doubles held by every thread; every thread receives the sums.
// red must hold (nwaves + 1) * K doubles.
template <int K>
__device__ __forceinline__ void block_sum(double *v, double *red, int nwaves) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] = wave_sum(v[i]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < K; ++i) red[wave * K + i] = v[i];
    }
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
        for (int w = 0; w < nwaves; ++w) s += red[w * K + threadIdx.x];
        red[nwaves * K + threadIdx.x] = s;  // staging slot after the per-wave area
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) v[i] = red[nwaves * K + i];
    __syncthreads();
}

// unwrapped grid offsets j_d (relative to the home cell) of a packed entry
__device__ __forceinline__ void unpack(uint32_t pk, const int *N, int &j0, int &j1, int &j2, int &a) {
    j0 = int(pk & 255u) - N[0];
    j1 = int((pk >> 8) & 255u) - N[1];
    j2 = int((pk >> 16) & 255u) - N[2];
    a = int(pk >> 24);
}

// Opaque copy of a value: stops loop-invariant code motion from hoisting address
// arithmetic derived from it out of the band / Taylor loops (which would keep one
// register per neighbour address alive for the whole kernel).
__device__ __forceinline__ int opq(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ int wrapi(int j, int n) { return j < 0 ? j + n : (j >= n ? j - n : j); }

// Phase e^{i kappa.d} of a packed projector entry from the separable tables
// T_d[j_d + N_d] = e^{i j_d kappa.a_d / N_d} and the atom factor e^{-i kappa.tau_a};
// also returns the wrapped grid index p and the displacement d = sum_d j_d a_d/N_d - tau_a.
template <typename R, typename C, typename TC>
__device__ __forceinline__ TC entry_geom(uint32_t pk, const int N0, const int N1, const int N2,
                                         int ntab, const TC *tab, const TC *aph, const R (&hv)[3][3],
                                         const double *atom_tau, int &p, int &at, R (&dv)[3]) {
    const int j0 = int(pk & 255u) - N0;
    const int j1 = int((pk >> 8) & 255u) - N1;
    const int j2 = int((pk >> 16) & 255u) - N2;
    at = int(pk >> 24);
    p = wrapi(j0, N0) + N0 * (wrapi(j1, N1) + N1 * wrapi(j2, N2));
    const double *tau = atom_tau + 3 * at;
#pragma unroll
    for (int q = 0; q < 3; ++q) dv[q] = R(j0) * hv[0][q] + R(j1) * hv[1][q] + R(j2) * hv[2][q] - R(tau[q]);
    return cmul(cmul(tab[j0 + N0], tab[ntab + j1 + N1]), cmul(tab[2 * ntab + j2 + N2], aph[at]));
}

// Column ownership: thread t owns grid column (i0, i1) = (t mod N0, (t / N0) mod N1) and the
// z-segment [seg*ZL, seg*ZL + ZL), seg = t / (N0 N1); BS = N0 N1 (N2 / ZL) threads are active.
template <typename R, int ZL, bool NONORTH, int MAXT>
__global__ __launch_bounds__(MAXT) void k_propagate(PropArgs a) {
    using C = typename CT<R>::T;
    extern __shared__ __align__(16) char smem[];
    const WorkItem wi = a.work[blockIdx.x];
    const DevInst &I = a.insts[wi.inst];
    const int ng = I.ng;
    const int N0 = I.N[0], N1 = I.N[1], N2 = I.N[2];
    const int BS = blockDim.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int NW = BS >> 6;

    const PropLds L = prop_lds(sizeof(R) == 8, a.ng_max, a.nmaxd, a.nat_max, a.ntask_max, BS);
    C *W = reinterpret_cast<C *>(smem + L.W);
    C *tabm = reinterpret_cast<C *>(smem + L.tab_mid);
    double2 *tabe = reinterpret_cast<double2 *>(smem + L.tab_end);
    C *aphm = reinterpret_cast<C *>(smem + L.aph_mid);
    double2 *aphe = reinterpret_cast<double2 *>(smem + L.aph_end);
    C *part = reinterpret_cast<C *>(smem + L.part);
    C *EC = reinterpret_cast<C *>(smem + L.ec);
    double *red = reinterpret_cast<double *>(smem + L.red);

    const int ntab = 3 * a.nmaxd;  // per-dimension stride in the phase tables
    const R *vtot = reinterpret_cast<const R *>(I.vtot);
    const int plane = N0 * N1;
    const int nseg = N2 / ZL;
    const bool active = tid < plane * nseg;
    const int i0 = tid % N0, i1 = (tid / N0) % N1, seg = tid / plane;
    const int z0 = seg * ZL;
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
    double jacc[3] = {0.0, 0.0, 0.0};
    const double dV = I.dV;
    const int nat = I.nat;
    const int ntask = I.ntask;
    R hvr[3][3];
    double hvd[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            hvd[d][q] = I.hv[d][q];
            hvr[d][q] = R(I.hv[d][q]);
        }

    R vz[ZL];
    double rho[ZL];
#pragma unroll
    for (int z = 0; z < ZL; ++z) {
        vz[z] = active ? vtot[pbase + plane * (z0 + z)] : R(0);
        rho[z] = 0.0;
    }

    // Laplacian coefficients (metric only)
    R a1[3], a2[3], cx[3];
    double c0l = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a1[d] = R(-0.5 * I.g[d][d] * D2C1);
        a2[d] = R(-0.5 * I.g[d][d] * D2C2);
        c0l += -0.5 * I.g[d][d] * D2C0;
    }
    cx[0] = R(-I.g[0][1]);  // -(1/2) * 2 g_de for d < e
    cx[1] = R(-I.g[0][2]);
    cx[2] = R(-I.g[1][2]);
    const int norder = (a.mode == MODE_STEP) ? 4 : (a.mode == MODE_APPLY ? 1 : 0);

#pragma unroll 1
    for (int kk = 0; kk < wi.nk; ++kk) {
        const int k = wi.k0 + kk;
        double km[3], ke[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            km[d] = I.kcart[3 * k + d] + Am[d];
            ke[d] = I.kcart[3 * k + d] + Am[3 + d];
        }
        const double wk = I.kw[k];
        // kappa-dependent coefficients: -i kappa.grad_FD and |kappa|^2 / 2
        R b1[3], b2[3];
        const double kk2 = km[0] * km[0] + km[1] * km[1] + km[2] * km[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double kc = km[0] * I.c[d][0] + km[1] * I.c[d][1] + km[2] * I.c[d][2];
            b1[d] = R(kc * D1C1);
            b2[d] = R(kc * D1C2);
        }
        const R c0 = R(c0l + 0.5 * kk2);

        // phase tables for kappa(t_n + dt/2) (propagation precision) and kappa(t_{n+1}) (FP64)
        __syncthreads();
        for (int idx = tid; idx < 3 * ntab; idx += BS) {
            const int d = idx / ntab, jj = idx - d * ntab;
            const int n = I.N[d];
            if (jj < 3 * n) {
                const double j = double(jj - n);
                const double inv_pi_n = 0.3183098861837907 / n;
                const double thm = (km[0] * I.lat[d][0] + km[1] * I.lat[d][1] + km[2] * I.lat[d][2]) * inv_pi_n;
                const double the = (ke[0] * I.lat[d][0] + ke[1] * I.lat[d][1] + ke[2] * I.lat[d][2]) * inv_pi_n;
                double sm, cm, se, ce;
                sincospi(j * thm, &sm, &cm);
                sincospi(j * the, &se, &ce);
                C t;
                t.x = R(cm);
                t.y = R(sm);
                tabm[idx] = t;
                tabe[idx] = make_double2(ce, se);
            }
        }
        for (int at = tid; at < nat; at += BS) {
            const double *tau = I.atom_tau + 3 * at;
            const double pm = (km[0] * tau[0] + km[1] * tau[1] + km[2] * tau[2]) * 0.3183098861837907;
            const double pe = (ke[0] * tau[0] + ke[1] * tau[1] + ke[2] * tau[2]) * 0.3183098861837907;
            double sm, cm, se, ce;
            sincospi(pm, &sm, &cm);
            sincospi(pe, &se, &ce);
            C t;
            t.x = R(cm);
            t.y = R(-sm);
            aphm[at] = t;
            aphe[at] = make_double2(ce, -se);
        }

#pragma unroll 1
        for (int bb = 0; bb < wi.nb; ++bb) {
            const int b = wi.b0 + bb;
            const size_t orb = (size_t(k) * I.nb + b) * size_t(ng);
            C *ug = reinterpret_cast<C *>(I.u) + orb;
            const C *src = (a.mode == MODE_APPLY) ? reinterpret_cast<const C *>(a.apply_in) + orb : ug;
            C acc[ZL], wc[ZL];
            __syncthreads();  // previous users of W are done
            const int pl = opq(pbase + plane * z0);
#pragma unroll
            for (int z = 0; z < ZL; ++z) {
                C v;
                v.x = R(0);
                v.y = R(0);
                if (active) {
                    const int p = pl + plane * z;
                    v = src[p];
                    W[p] = v;
                }
                acc[z] = v;
                wc[z] = v;
            }

#pragma unroll 1
            for (int m = 1; m <= norder; ++m) {
                __syncthreads();  // W holds w_{m-1}
                // ---- 1. projections c = <P|w> (atom-major tasks, one wave each)
                for (int t = wave; t < ntask; t += NW) {
                    const int2 tk = I.task[t];
                    const int e0 = tk.x, cnt = tk.y >> 8;
                    C s[4];
#pragma unroll
                    for (int l = 0; l < 4; ++l) { s[l].x = R(0); s[l].y = R(0); }
                    for (int e = e0 + lane; e < e0 + cnt; e += 64) {
                        int p, at;
                        R dv[3];
                        const C ph = entry_geom<R, C, C>(I.ent_pack[e], N0, N1, N2, ntab, tabm, aphm,
                                                         hvr, I.atom_tau, p, at, dv);
                        const C x = cmul(ph, W[p]);
                        const R gv = R(I.ent_g[e]);
                        const double *par = I.atom_par + 4 * at;
                        const R fs = R(par[2]) * gv, fp = R(par[3]) * gv;
                        s[0].x += fs * x.x;
                        s[0].y += fs * x.y;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            const R f = fp * dv[q];
                            s[1 + q].x += f * x.x;
                            s[1 + q].y += f * x.y;
                        }
                    }
#pragma unroll
                    for (int l = 0; l < 4; ++l) {
                        s[l].x = wave_sum(s[l].x);
                        s[l].y = wave_sum(s[l].y);
                    }
                    if (lane == 0) {
#pragma unroll
                        for (int l = 0; l < 4; ++l) part[4 * t + l] = s[l];
                    }
                }
                __syncthreads();
                for (int idx = tid; idx < 4 * nat; idx += BS) {
                    const int at = idx >> 2, l = idx & 3;
                    C s;
                    s.x = R(0);
                    s.y = R(0);
                    for (int t = I.atom_task[at]; t < I.atom_task[at + 1]; ++t) {
                        const C v = part[4 * t + l];
                        s.x += v.x;
                        s.y += v.y;
                    }
                    const R e = R(I.atom_par[4 * at + (l == 0 ? 0 : 1)] * dV);
                    s.x *= e;
                    s.y *= e;
                    EC[idx] = s;
                }
                __syncthreads();
                // ---- 2. h w along the owned column segment
                // (opaque copies keep the compiler from hoisting every neighbour address
                // out of the band and Taylor loops, which would pin them in registers)
                int pb = pbase;
                int oxl[4], oyl[4];
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    oxl[s] = ox[s];
                    oyl[s] = oy[s];
                }
                asm volatile("" : "+v"(pb), "+v"(oxl[0]), "+v"(oxl[1]), "+v"(oxl[2]), "+v"(oxl[3]));
                asm volatile("" : "+v"(oyl[0]), "+v"(oyl[1]), "+v"(oyl[2]), "+v"(oyl[3]));
                C hz[ZL];
#pragma unroll
                for (int z = 0; z < ZL; ++z) {
                    hz[z].x = R(0);
                    hz[z].y = R(0);
                    if (!active) continue;
                    const int zg = z0 + z;
                    const int p = pb + plane * zg;
                    // z neighbours: registers inside the segment, LDS across segment ends
                    C zn[4];  // +1, -1, +2, -2
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int dz = (s == 0) ? 1 : (s == 1) ? -1 : (s == 2) ? 2 : -2;
                        const int zz = z + dz;
                        if (zz >= 0 && zz < ZL) {
                            zn[s] = wc[zz];
                        } else if (nseg == 1) {
                            zn[s] = wc[(zz + ZL) % ZL];
                        } else {
                            int zw = zg + dz;
                            zw = zw < 0 ? zw + N2 : (zw >= N2 ? zw - N2 : zw);
                            zn[s] = W[pb + plane * zw];
                        }
                    }
                    const C cen = wc[z];
                    const R cv = c0 + vz[z];
                    C h;
                    h.x = cv * cen.x;
                    h.y = cv * cen.y;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        C p1, m1, p2, m2;
                        if (d == 0) {
                            p1 = W[p + oxl[0]]; m1 = W[p + oxl[1]]; p2 = W[p + oxl[2]]; m2 = W[p + oxl[3]];
                        } else if (d == 1) {
                            p1 = W[p + oyl[0]]; m1 = W[p + oyl[1]]; p2 = W[p + oyl[2]]; m2 = W[p + oyl[3]];
                        } else {
                            p1 = zn[0]; m1 = zn[1]; p2 = zn[2]; m2 = zn[3];
                        }
                        h.x += a1[d] * (p1.x + m1.x) + a2[d] * (p2.x + m2.x);
                        h.y += a1[d] * (p1.y + m1.y) + a2[d] * (p2.y + m2.y);
                        // -i (b1 (p1 - m1) + b2 (p2 - m2))
                        const R qx = b1[d] * (p1.x - m1.x) + b2[d] * (p2.x - m2.x);
                        const R qy = b1[d] * (p1.y - m1.y) + b2[d] * (p2.y - m2.y);
                        h.x += qy;
                        h.y -= qx;
                    }
                    if (NONORTH) {
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
                    // non-local: sum over the projector entries touching p
                    const int e1 = I.pt_ptr[p + 1];
                    for (int e = I.pt_ptr[p]; e < e1; ++e) {
                        int pp, at;
                        R dv[3];
                        const C ph = entry_geom<R, C, C>(I.pt_pack[e], N0, N1, N2, ntab, tabm, aphm,
                                                         hvr, I.atom_tau, pp, at, dv);
                        const R gv = R(I.pt_g[e]);
                        const double *par = I.atom_par + 4 * at;
                        const R fs = R(par[2]) * gv, fp = R(par[3]) * gv;
                        const C *ec = EC + 4 * at;
                        C sum;
                        sum.x = fs * ec[0].x;
                        sum.y = fs * ec[0].y;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            const R f = fp * dv[q];
                            sum.x += f * ec[1 + q].x;
                            sum.y += f * ec[1 + q].y;
                        }
                        const C v = cmulc(ph, sum);  // e^{-i kappa.d} * sum
                        h.x += v.x;
                        h.y += v.y;
                    }
                    hz[z] = h;
                }
                __syncthreads();  // all reads of W done
                const int pw = opq(pbase + plane * z0);
                if (a.mode == MODE_APPLY) {
                    C *out = reinterpret_cast<C *>(a.apply_out) + orb;
                    if (active) {
#pragma unroll
                        for (int z = 0; z < ZL; ++z) out[pw + plane * z] = hz[z];
                    }
                } else {
                    const R cm = R(a.dt / m);
#pragma unroll
                    for (int z = 0; z < ZL; ++z) {
                        C wn;  // (-i dt/m) h w
                        wn.x = cm * hz[z].y;
                        wn.y = -cm * hz[z].x;
                        acc[z].x += wn.x;
                        acc[z].y += wn.y;
                        wc[z] = wn;
                        if (active) W[pw + plane * z] = wn;
                    }
                }
            }
            if (a.mode == MODE_APPLY) continue;

            // ---- new orbital: store; FP64 partials of density and current
            __syncthreads();
            const int ps = opq(pbase + plane * z0);
            if (active) {
#pragma unroll
                for (int z = 0; z < ZL; ++z) {
                    const int p = ps + plane * z;
                    W[p] = acc[z];
                    if (a.mode == MODE_STEP) ug[p] = acc[z];
                }
            }
            __syncthreads();
            const double fo = wk * I.occ[b];
            double qn[4] = {0.0, 0.0, 0.0, 0.0};  // Q_d = sum Im(conj(u) D1_d u), and sum |u|^2
            const int pk0 = opq(pbase);
            int oxk[4], oyk[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                oxk[s] = opq(ox[s]);
                oyk[s] = opq(oy[s]);
            }
            if (active) {
#pragma unroll
                for (int z = 0; z < ZL; ++z) {
                    const int zg = z0 + z;
                    const int p = pk0 + plane * zg;
                    const double ux = double(acc[z].x), uy = double(acc[z].y);
                    const double n2 = ux * ux + uy * uy;
                    rho[z] += fo * n2;
                    qn[3] += n2;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        int o[4];
                        if (d == 0) {
                            o[0] = oxk[0]; o[1] = oxk[1]; o[2] = oxk[2]; o[3] = oxk[3];
                        } else if (d == 1) {
                            o[0] = oyk[0]; o[1] = oyk[1]; o[2] = oyk[2]; o[3] = oyk[3];
                        } else {
#pragma unroll
                            for (int s = 0; s < 4; ++s) {
                                const int dz = (s == 0) ? 1 : (s == 1) ? -1 : (s == 2) ? 2 : -2;
                                int zw = zg + dz;
                                zw = zw < 0 ? zw + N2 : (zw >= N2 ? zw - N2 : zw);
                                o[s] = plane * (zw - zg);
                            }
                        }
                        const C p1 = W[p + o[0]], m1 = W[p + o[1]];
                        const C p2 = W[p + o[2]], m2 = W[p + o[3]];
                        const double dx = D1C1 * (double(p1.x) - double(m1.x)) + D1C2 * (double(p2.x) - double(m2.x));
                        const double dy = D1C1 * (double(p1.y) - double(m1.y)) + D1C2 * (double(p2.y) - double(m2.y));
                        qn[d] += ux * dy - uy * dx;
                    }
                }
            }
            // non-local current 2 E_l Im(conj(c_d) c): one wave per atom, one channel at a time
            double jnl[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
            for (int at = wave; at < nat; at += NW) {
                const int e_beg = I.task[I.atom_task[at]].x;
                const int tl = I.atom_task[at + 1] - 1;
                const int e_end = I.task[tl].x + (I.task[tl].y >> 8);
                const double *par = I.atom_par + 4 * at;
#pragma unroll 1
                for (int l = 0; l < 4; ++l) {
                    double2 cs = make_double2(0.0, 0.0);
                    double2 cd[3];
#pragma unroll
                    for (int q = 0; q < 3; ++q) cd[q] = make_double2(0.0, 0.0);
                    for (int e = e_beg + lane; e < e_end; e += 64) {
                        int p, at2;
                        double dv[3];
                        const double2 ph = entry_geom<double, double2, double2>(
                            I.ent_pack[e], N0, N1, N2, ntab, tabe, aphe, hvd, I.atom_tau, p, at2, dv);
                        const C wv = W[p];
                        const double2 x = cmul(ph, make_double2(double(wv.x), double(wv.y)));
                        const double gv = I.ent_g[e];
                        const double f = (l == 0) ? par[2] * gv : par[3] * gv * dv[l - 1];
                        cs.x += f * x.x;
                        cs.y += f * x.y;
#pragma unroll
                        for (int q = 0; q < 3; ++q) {
                            cd[q].x += dv[q] * f * x.x;
                            cd[q].y += dv[q] * f * x.y;
                        }
                    }
                    cs.x = wave_sum(cs.x);
                    cs.y = wave_sum(cs.y);
                    const double El = par[l == 0 ? 0 : 1];
#pragma unroll
                    for (int q = 0; q < 3; ++q) {
                        cd[q].x = wave_sum(cd[q].x);
                        cd[q].y = wave_sum(cd[q].y);
                        jnl[q] += 2.0 * El * dV * dV * (cd[q].x * cs.y - cd[q].y * cs.x);
                    }
                }
            }
            if (lane != 0) {
                jnl[0] = jnl[1] = jnl[2] = 0.0;
            }
            double v7[7] = {qn[0], qn[1], qn[2], qn[3], jnl[0], jnl[1], jnl[2]};
            block_sum<7>(v7, red, NW);
            if (tid == 0) {
                const double nrm = v7[3] * dV;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const double kin = dV * (I.c[0][q] * v7[0] + I.c[1][q] * v7[1] + I.c[2][q] * v7[2]);
                    jacc[q] += fo * (kin + ke[q] * nrm + v7[4 + q]);
                }
            }
        }
    }
    if (a.mode == MODE_APPLY) return;
    double *rp = I.rho_part + size_t(wi.slot) * ng;
    const int pr = opq(pbase + plane * z0);
    if (active) {
#pragma unroll
        for (int z = 0; z < ZL; ++z) rp[pr + plane * z] = rho[z];
    }
    if (tid == 0) {
        double *jp = I.j_part + 4 * wi.slot;
        jp[0] = jacc[0];
        jp[1] = jacc[1];
        jp[2] = jacc[2];
        jp[3] = 0.0;
    }
}

}  // namespace tdks
