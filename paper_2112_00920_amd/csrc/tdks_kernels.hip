// HIP kernels for CDNA4 (gfx950) around the propagation kernel: dispatch of the
// propagation variants, deterministic FP64 reductions, Hartree + LDA, utilities.
#include "tdks_propagate.h"

namespace tdks {

hipError_t launch_propagate_f32_orth(const PropArgs &, int, int, int, int, int, int, hipStream_t);
hipError_t launch_propagate_f32_nonorth(const PropArgs &, int, int, int, int, int, int, hipStream_t);
hipError_t launch_propagate_f64_orth(const PropArgs &, int, int, int, int, int, int, hipStream_t);
hipError_t launch_propagate_f64_nonorth(const PropArgs &, int, int, int, int, int, int, hipStream_t);
hipError_t launch_itime_f32_orth(const PropArgs &, int, int, int, int, int, int, hipStream_t);
hipError_t launch_itime_f32_nonorth(const PropArgs &, int, int, int, int, int, int, hipStream_t);
hipError_t launch_itime_f64_orth(const PropArgs &, int, int, int, int, int, int, hipStream_t);
hipError_t launch_itime_f64_nonorth(const PropArgs &, int, int, int, int, int, int, hipStream_t);

size_t propagate_lds_bytes(int fp64, int sl, const PropArgs &a, int block) {
    return propagate_lds_bytes_inl(fp64, sl, a, block);
}

size_t propagate_gcol_stride(int fp64, int ncol_max) { return prop_gcol(fp64, ncol_max).stride; }

bool propagate_config_ok(int block, int zl, int minw, int ragged) {
    if (block < 64 || block > 1024 || (block & 63)) return false;
#define TDKS_OK_CASE(Z, M, O) if (zl == Z && block <= M && minw == O) return true;
    if (ragged) {
        TDKS_PROPAGATE_RAGGED_CONFIGS(TDKS_OK_CASE)
    } else {
        TDKS_PROPAGATE_CONFIGS(TDKS_OK_CASE)
    }
#undef TDKS_OK_CASE
    return false;
}

hipError_t launch_propagate(int fp64, const PropArgs &a, int n_items, int block, int zl, int minw,
                            int nonorth, int sl, int ragged, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (a.mode == MODE_ITIME) {
        if (fp64) return nonorth ? launch_itime_f64_nonorth(a, n_items, block, zl, minw, sl, ragged, s)
                                 : launch_itime_f64_orth(a, n_items, block, zl, minw, sl, ragged, s);
        return nonorth ? launch_itime_f32_nonorth(a, n_items, block, zl, minw, sl, ragged, s)
                       : launch_itime_f32_orth(a, n_items, block, zl, minw, sl, ragged, s);
    }
    if (fp64) return nonorth ? launch_propagate_f64_nonorth(a, n_items, block, zl, minw, sl, ragged, s)
                             : launch_propagate_f64_orth(a, n_items, block, zl, minw, sl, ragged, s);
    return nonorth ? launch_propagate_f32_nonorth(a, n_items, block, zl, minw, sl, ragged, s)
                   : launch_propagate_f32_orth(a, n_items, block, zl, minw, sl, ragged, s);
}

// ---------------------------------------------------------------------------
// Deterministic FP64 reduction of the per-workgroup partials (a fixed order, independent of
// timing).  Density: 64 points per workgroup; wave w sums the slots w, w + 4, ... of each
// point (coalesced rows) and the four wave sums are added in wave order.  Current and charge
// (the first workgroup of the instance): lane l sums the slots l, l + 64, ..., then a fixed
// butterfly over the wave.  After a step (step_ctr given: steps since the load before this
// one) the current J^{n} is recorded at row n / rstride - 1 when rstride divides n, and the
// charge is checked against the bounds of HealthArgs; an observation (step_ctr null) writes
// row 0 and, with set_ref, takes the charge as the instance's reference.
__global__ __launch_bounds__(256) void k_reduce(const DevInst *insts, int inst0, int ng_max,
                                                double *rho, double *jout, int jstride,
                                                const int *step_ctr, HealthArgs h) {
    __shared__ double part[3][64];
    const int inst = inst0 + blockIdx.y;
    const DevInst &I = insts[inst];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (p < I.ng)
        for (int q = w; q < I.nslot; q += 4) s += I.rho_part[size_t(q) * I.ng + p];
    if (w > 0) part[w - 1][lane] = s;
    __syncthreads();
    if (w == 0 && p < I.ng)
        rho[size_t(inst) * ng_max + p] = ((s + part[0][lane]) + part[1][lane]) + part[2][lane];
    if (blockIdx.x == 0 && w == 1) {
        double j0 = 0.0, j1 = 0.0, j2 = 0.0, q = 0.0;
        for (int t = lane; t < I.nslot; t += 64) {
            j0 += I.j_part[4 * t];
            j1 += I.j_part[4 * t + 1];
            j2 += I.j_part[4 * t + 2];
            q += I.j_part[4 * t + 3];
        }
        j0 = wave_sum(j0);
        j1 = wave_sum(j1);
        j2 = wave_sum(j2);
        q = wave_sum(q);
        const int n = step_ctr ? *step_ctr + 1 : 0;  // steps since the load after this one
        const int rs = h.rstride > 0 ? h.rstride : 1;
        if (lane < 3 && (!step_ctr || h.row_ctr || n % rs == 0)) {
            const int row = h.row_ctr ? *h.row_ctr : step_ctr ? n / rs - 1 : 0;
            const double j = lane == 0 ? j0 : lane == 1 ? j1 : j2;
            jout[(size_t(inst) * jstride + row) * 3 + lane] = -j / I.omega;
        }
        if (lane == 0 && h.set_ref && h.q0) {
            h.q0[inst] = q;
            h.lcum[inst] = 0.0;
        }
        if (lane == 0 && step_ctr && h.health) {
            const double lc = h.lcum[inst] + (h.logF ? h.logF[*h.arow] : h.logF_floor);
            h.lcum[inst] = lc;
            const double q0 = h.q0[inst];
            int code = 0;
            if (!(isfinite(j0) && isfinite(j1) && isfinite(j2) && isfinite(q)))
                code = 1;
            else if (q > q0 * (1.0 + h.tol))
                code = 2;
            else if (q < q0 * (exp(lc) - h.tol))
                code = 3;
            if (code)
                atomicCAS(h.health + inst, 0ull, (static_cast<unsigned long long>(n) << 32) | unsigned(code));
        }
    }
}

hipError_t launch_reduce(const DevInst *insts, int inst0, int n, int ng_max, double *rho,
                         double *jout, int jstride, const int *step_ctr, const HealthArgs &h, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid((ng_max + 63) / 64, n);
    hipLaunchKernelGGL(k_reduce, grid, dim3(256), 0, s, insts, inst0, ng_max, rho, jout, jstride,
                       step_ctr, h);
    return hipGetLastError();
}

// Per-orbital part of the health check, every `stride` steps (the step counter is read on the
// device, so the launch sits in every captured step and returns at once when not due): one
// workgroup per work item, each wave sums sum_r |u|^2 dV of one orbital at a time in FP64 and
// compares it with the orbital's norm at the load times the bounds of the charge check.
template <typename C>
__global__ __launch_bounds__(256) void k_health_norms(const DevInst *insts, const WorkItem *work,
                                                      const int *step_ctr, int stride, HealthArgs h) {
    const int n = *step_ctr + 1;
    if (n % stride) return;
    const WorkItem wi = work[blockIdx.x];
    const DevInst &I = insts[wi.inst];
    if (!I.norm0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double lc = h.lcum[wi.inst] + (h.logF ? h.logF[*h.arow] : h.logF_floor);
    const int norb = wi.nk * wi.nb;
    for (int o = wave; o < norb; o += 4) {
        const int k = wi.k0 + o / wi.nb, b = wi.b0 + o % wi.nb;
        const size_t orb = size_t(k) * I.nb + b;
        const C *u = reinterpret_cast<const C *>(I.u) + orb * I.ng;
        double sq = 0.0;
        for (int p = lane; p < I.ng; p += 64) {
            const C v = u[p];
            sq += double(v.x) * double(v.x) + double(v.y) * double(v.y);
        }
        sq = wave_sum(sq) * I.dV;
        if (lane == 0) {
            const double n0 = I.norm0[orb];
            int code = 0;
            if (!isfinite(sq))
                code = 1;
            else if (sq > n0 * (1.0 + h.tol))
                code = 4;
            else if (sq < n0 * (exp(lc) - h.tol))
                code = 5;
            if (code)
                atomicCAS(h.health + wi.inst, 0ull,
                          (static_cast<unsigned long long>(n) << 32) | (static_cast<unsigned long long>(orb + 1) << 4) |
                              unsigned(code));
        }
    }
}

hipError_t launch_health_norms(const DevInst *insts, const WorkItem *work, int n_items, const int *step_ctr,
                               int stride, const HealthArgs &h, int fp64, hipStream_t s) {
    if (n_items <= 0 || stride <= 0 || !h.health) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_health_norms<double2>, dim3(n_items), dim3(256), 0, s, insts, work, step_ctr, stride, h);
    else
        hipLaunchKernelGGL(k_health_norms<float2>, dim3(n_items), dim3(256), 0, s, insts, work, step_ctr, stride, h);
    return hipGetLastError();
}

// Density of each instance from per-k partials rho_k[pair][r] (pairs of instance i are
// first[i] .. first[i+1]-1), summed in k order: the ground-state iteration's density.
__global__ __launch_bounds__(256) void k_reduce_k(const DevInst *insts, const int *first, const double *rho_k,
                                                  int ng_max, double *rho) {
    const int inst = blockIdx.y;
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= insts[inst].ng) return;
    double s = 0.0;
#pragma unroll 8
    for (int q = first[inst]; q < first[inst + 1]; ++q) s += rho_k[size_t(q) * ng_max + p];
    rho[size_t(inst) * ng_max + p] = s;
}

hipError_t launch_reduce_k(const DevInst *insts, int n_inst, const int *first, const double *rho_k, int ng_max,
                           double *rho, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_k, dim3((ng_max + 255) / 256, n_inst), dim3(256), 0, s, insts, first, rho_k,
                       ng_max, rho);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Hartree + LDA, one workgroup per instance.  Poisson: rho(G) by a separable
// discrete Fourier transform (each line of N_d <= 32 points held in registers, each
// output by Horner's rule in its twiddle, twiddles from sincospi), v_H(G) =
// 4 pi rho(G) / |G|^2 with G = 0 and the Nyquist planes zeroed, inverse transform.
// Exchange: Slater; correlation: Perdew-Zunger 81 (unpolarised).
__device__ double lda_vxc(double rho) {
    if (!(rho > 1e-30)) return 0.0;
    const double pi = 3.141592653589793;
    const double vx = -cbrt(3.0 * rho / pi);
    const double rs = cbrt(3.0 / (4.0 * pi * rho));
    double vc;
    if (rs >= 1.0) {
        const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
        const double sq = sqrt(rs);
        const double den = 1.0 + b1 * sq + b2 * rs;
        vc = g / den * (1.0 + 7.0 / 6.0 * b1 * sq + 4.0 / 3.0 * b2 * rs) / den;
    } else {
        const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
        const double l = log(rs);
        vc = A * l + (B - A / 3.0) + 2.0 / 3.0 * C * rs * l + (2.0 * D - C) / 3.0 * rs;
    }
    return vx + vc;
}

__device__ void dft_pass(double2 *X, const double2 *tw, int n, int stride, int nlines,
                         int inner, int ninner_stride, bool inverse) {
    // lines: start = (l % inner) + (l / inner) * ninner_stride, element i at start + i*stride
    for (int l = threadIdx.x; l < nlines; l += blockDim.x) {
        const int start = (l % inner) + (l / inner) * ninner_stride;
        double2 line[kMaxGridDim];
#pragma unroll
        for (int i = 0; i < kMaxGridDim; ++i)
            if (i < n) line[i] = X[start + i * stride];
        // X_m = sum_i x_i z^i with z = e^{-+2 pi i m / n}, by Horner's rule (|z| = 1: the
        // rounding stays at the direct sum's level; one twiddle read per output), two outputs
        // at a time so that their chains of multiply-adds overlap
        for (int m = 0; m < n; m += 2) {
            const int m1 = (m + 1 < n) ? m + 1 : m;
            const double2 t0 = tw[m], t1 = tw[m1];
            const double z0x = t0.x, z0y = inverse ? -t0.y : t0.y;
            const double z1x = t1.x, z1y = inverse ? -t1.y : t1.y;
            double s0x = 0.0, s0y = 0.0, s1x = 0.0, s1y = 0.0;
#pragma unroll
            for (int i = kMaxGridDim - 1; i >= 0; --i) {
                if (i < n) {
                    const double a0 = fma(s0x, z0x, fma(-s0y, z0y, line[i].x));
                    s0y = fma(s0x, z0y, fma(s0y, z0x, line[i].y));
                    s0x = a0;
                    const double a1 = fma(s1x, z1x, fma(-s1y, z1y, line[i].x));
                    s1y = fma(s1x, z1y, fma(s1y, z1x, line[i].y));
                    s1x = a1;
                }
            }
            X[start + m * stride] = make_double2(s0x, s0y);
            if (m + 1 < n) X[start + m1 * stride] = make_double2(s1x, s1y);
        }
    }
}

constexpr int kHxcThreads = 512;  // 2 waves per SIMD: a line of 32 points stays in registers

template <typename R>
__global__ __launch_bounds__(kHxcThreads) void k_hxc(const DevInst *insts, int inst0, int ng_max,
                                             const double *rho, const double *vloc, double *vhxc,
                                             R *vtot) {
    extern __shared__ __align__(16) char smem[];
    const int inst = inst0 + blockIdx.x;
    const DevInst &I = insts[inst];
    const int ng = I.ng, N0 = I.N[0], N1 = I.N[1], N2 = I.N[2];
    double2 *X = reinterpret_cast<double2 *>(smem);
    double2 *tw = X + ng_max;  // [3][kMaxGridDim] e^{-2 pi i q / N_d}
    const size_t base = size_t(inst) * ng_max;
    for (int p = threadIdx.x; p < ng; p += blockDim.x) X[p] = make_double2(rho[base + p], 0.0);
    for (int idx = threadIdx.x; idx < 3 * kMaxGridDim; idx += blockDim.x) {
        int d = idx / kMaxGridDim, q = idx % kMaxGridDim;
        int n = I.N[d];
        double s, c;
        sincospi(2.0 * q / n, &s, &c);
        tw[idx] = make_double2(c, -s);
    }
    __syncthreads();
    // forward transform along i1, i2, i3
    dft_pass(X, tw, N0, 1, N1 * N2, 1, N0, false);
    __syncthreads();
    dft_pass(X, tw + kMaxGridDim, N1, N0, N0 * N2, N0, N0 * N1, false);
    __syncthreads();
    dft_pass(X, tw + 2 * kMaxGridDim, N2, N0 * N1, N0 * N1, N0 * N1, 0, false);
    __syncthreads();
    const double two_pi = 6.283185307179586;
    for (int p = threadIdx.x; p < ng; p += blockDim.x) {
        const int m0 = p % N0, m1 = (p / N0) % N1, m2 = p / (N0 * N1);
        const int s0 = m0 < (N0 + 1) / 2 ? m0 : m0 - N0;
        const int s1 = m1 < (N1 + 1) / 2 ? m1 : m1 - N1;
        const int s2 = m2 < (N2 + 1) / 2 ? m2 : m2 - N2;
        const bool nyq = ((N0 % 2 == 0) && s0 == -N0 / 2) || ((N1 % 2 == 0) && s1 == -N1 / 2) ||
                         ((N2 % 2 == 0) && s2 == -N2 / 2);
        double G[3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
            G[q] = two_pi * (s0 * I.c[0][q] / N0 + s1 * I.c[1][q] / N1 + s2 * I.c[2][q] / N2);
        const double g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
        double2 v = X[p];
        if (nyq || (s0 == 0 && s1 == 0 && s2 == 0)) {
            v = make_double2(0.0, 0.0);
        } else {
            const double f = 4.0 * 3.141592653589793 / g2;
            v.x *= f;
            v.y *= f;
        }
        X[p] = v;
    }
    __syncthreads();
    dft_pass(X, tw, N0, 1, N1 * N2, 1, N0, true);
    __syncthreads();
    dft_pass(X, tw + kMaxGridDim, N1, N0, N0 * N2, N0, N0 * N1, true);
    __syncthreads();
    dft_pass(X, tw + 2 * kMaxGridDim, N2, N0 * N1, N0 * N1, N0 * N1, 0, true);
    __syncthreads();
    for (int p = threadIdx.x; p < ng; p += blockDim.x) {
        const double vh = X[p].x / ng;
        const double v = vh + lda_vxc(rho[base + p]);
        vhxc[base + p] = v;
        vtot[base + p] = R(vloc[base + p] + v);
    }
}

hipError_t launch_hxc(const DevInst *insts, int inst0, int n, int ng_max, const double *rho,
                      const double *vloc, double *vhxc, void *vtot, int fp64, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const size_t lds = 16 * size_t(ng_max) + 16 * 3 * kMaxGridDim;
    if (fp64) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_hxc<double>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_hxc<double>, dim3(n), dim3(kHxcThreads), lds, s, insts, inst0, ng_max, rho,
                           vloc, vhxc, reinterpret_cast<double *>(vtot));
    } else {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_hxc<float>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_hxc<float>, dim3(n), dim3(kHxcThreads), lds, s, insts, inst0, ng_max, rho,
                           vloc, vhxc, reinterpret_cast<float *>(vtot));
    }
    return hipGetLastError();
}

template <typename R>
__global__ void k_vtot(const DevInst *insts, int inst0, int ng_max, const double *vloc,
                       const double *vhxc, R *vtot) {
    const int inst = inst0 + blockIdx.y;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < insts[inst].ng) {
        const size_t o = size_t(inst) * ng_max + p;
        vtot[o] = R(vloc[o] + vhxc[o]);
    }
}

hipError_t launch_vtot(const DevInst *insts, int inst0, int n, int ng_max, const double *vloc,
                       const double *vhxc, void *vtot, int fp64, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid((ng_max + 255) / 256, n);
    if (fp64)
        hipLaunchKernelGGL(k_vtot<double>, grid, dim3(256), 0, s, insts, inst0, ng_max, vloc, vhxc,
                           reinterpret_cast<double *>(vtot));
    else
        hipLaunchKernelGGL(k_vtot<float>, grid, dim3(256), 0, s, insts, inst0, ng_max, vloc, vhxc,
                           reinterpret_cast<float *>(vtot));
    return hipGetLastError();
}

// Mid-step potential of the predictor-corrector step: vtot = v_loc + (v_a + v_b) / 2.
template <typename R>
__global__ void k_vmid(const DevInst *insts, int ng_max, const double *vloc, const double *va,
                       const double *vb, R *vtot) {
    const int inst = blockIdx.y;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < insts[inst].ng) {
        const size_t o = size_t(inst) * ng_max + p;
        vtot[o] = R(vloc[o] + 0.5 * (va[o] + vb[o]));
    }
}

hipError_t launch_vmid(const DevInst *insts, int n, int ng_max, const double *vloc, const double *va,
                       const double *vb, void *vtot, int fp64, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid((ng_max + 255) / 256, n);
    if (fp64)
        hipLaunchKernelGGL(k_vmid<double>, grid, dim3(256), 0, s, insts, ng_max, vloc, va, vb,
                           reinterpret_cast<double *>(vtot));
    else
        hipLaunchKernelGGL(k_vmid<float>, grid, dim3(256), 0, s, insts, ng_max, vloc, va, vb,
                           reinterpret_cast<float *>(vtot));
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// small utility kernels (graph-capturable: no memset nodes)
__global__ void k_advance(int *ctrs, int n) {
    if (threadIdx.x < n) ctrs[threadIdx.x] += 1;
}
hipError_t launch_advance(int *ctrs, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ctrs, n);
    return hipGetLastError();
}

__global__ void k_fill_int(int *p, int v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
hipError_t launch_fill_int(int *p, int v, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

template <typename C>
__global__ void k_convert_in(const double2 *src, C *dst, size_t n) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
         i += size_t(gridDim.x) * blockDim.x) {
        double2 v = src[i];
        C o;
        o.x = decltype(o.x)(v.x);
        o.y = decltype(o.y)(v.y);
        dst[i] = o;
    }
}
template <typename C>
__global__ void k_convert_out(const C *src, double2 *dst, size_t n) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n;
         i += size_t(gridDim.x) * blockDim.x) {
        C v = src[i];
        dst[i] = make_double2(double(v.x), double(v.y));
    }
}
hipError_t launch_convert_in(const double *src, void *dst, size_t n, int fp64, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int blocks = int((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (fp64)
        hipLaunchKernelGGL(k_convert_in<double2>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const double2 *>(src), reinterpret_cast<double2 *>(dst), n);
    else
        hipLaunchKernelGGL(k_convert_in<float2>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const double2 *>(src), reinterpret_cast<float2 *>(dst), n);
    return hipGetLastError();
}
hipError_t launch_convert_out(const void *src, double *dst, size_t n, int fp64, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const int blocks = int((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    if (fp64)
        hipLaunchKernelGGL(k_convert_out<double2>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const double2 *>(src), reinterpret_cast<double2 *>(dst), n);
    else
        hipLaunchKernelGGL(k_convert_out<float2>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const float2 *>(src), reinterpret_cast<double2 *>(dst), n);
    return hipGetLastError();
}

template <typename C>
__global__ __launch_bounds__(256) void k_norms(const C *u, int ng, double dV, double *out) {
    __shared__ double red[4];
    const C *o = u + size_t(blockIdx.x) * ng;
    double s = 0.0;
    for (int p = threadIdx.x; p < ng; p += 256) {
        C v = o[p];
        s += double(v.x) * double(v.x) + double(v.y) * double(v.y);
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * dV;
}
hipError_t launch_norms(const void *u, int n_orb, int ng, double dV, int fp64, double *out,
                        hipStream_t s) {
    if (n_orb <= 0) return hipSuccess;
    if (fp64)
        hipLaunchKernelGGL(k_norms<double2>, dim3(n_orb), dim3(256), 0, s,
                           reinterpret_cast<const double2 *>(u), ng, dV, out);
    else
        hipLaunchKernelGGL(k_norms<float2>, dim3(n_orb), dim3(256), 0, s,
                           reinterpret_cast<const float2 *>(u), ng, dV, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ground-state preparation: Cholesky orthonormalisation of the bands of one k-point,
// S = U^H U dV = L L^H, U <- U L^{-H} (the first band keeps its direction).  One
// workgroup per (instance, k); FP64 throughout, orbitals read twice and written once.
// The orbitals stream through LDS in tiles of TP points of all bands (TP as large as
// the tile buffer allows, so a tile is 8 elements per thread); the next tile is loaded
// into registers while the current one is used.  Both dense products run on the FP64
// matrix cores (v_mfma_f64_16x16x4: A 16 x 4, B 4 x 16, D 16 x 16; lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 r + l / 16][l % 16] in its
// register r):
//  - Gram matrix: with V = [Re U, Im U] (points x bands), S = Re^T Re + Im^T Im +
//    i (Re^T Im - (Re^T Im)^T), three real products over 4-point slices; each of the
//    4 waves sums every 4th slice and the wave sums are added in wave order, so the
//    result does not depend on timing;
//  - transform: U L^{-H} over 16-point blocks, four real products per 4 bands, with
//    the L^{-1} operands kept in registers for the whole pass.
// With rho_k given, the kernel also writes this k-point's FP64 density partial
// w_k sum_b f_b |u_b(r)|^2 of the stored (rounded) new orbitals to rho_k[pair][r]
// (bands summed by a fixed butterfly), so that no pass re-reads the orbitals for it.
constexpr int kOrthTileCap = 2080;  // tile elements (nb (TP + 1) <= cap), double2 slots
constexpr int kOrthPer = 8;         // tile elements per thread (nb TP <= 2048)

typedef double orth_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ orth_d4 mfma64(double a, double b, orth_d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename C>
__device__ __forceinline__ void orth_fetch(const C *u, int ng, int nb, int lt, int p0, C *pre) {
    const int tm = (1 << lt) - 1;
#pragma unroll
    for (int q = 0; q < kOrthPer; ++q) {
        const int idx = threadIdx.x + 256 * q;
        const int b = idx >> lt, pp = idx & tm;
        C x;
        x.x = 0;
        x.y = 0;
        if (b < nb && p0 + pp < ng) x = u[size_t(b) * ng + p0 + pp];
        pre[q] = x;
    }
}

// stores the prefetched elements as FP64; points past the grid end are zero
template <typename C>
__device__ __forceinline__ void orth_stage(const C *pre, int nb, int lt, double2 *T) {
    const int tm = (1 << lt) - 1;
#pragma unroll
    for (int q = 0; q < kOrthPer; ++q) {
        const int idx = threadIdx.x + 256 * q;
        const int b = idx >> lt, pp = idx & tm;
        if (b < nb) T[b * (tm + 2) + pp] = make_double2(double(pre[q].x), double(pre[q].y));
    }
}

// NBB: 16-band blocks (1: nb <= 16, 2: nb <= 32; the latter needs the larger register budget).
// With one block, L^{-1} takes 4 KB of LDS, so 4 workgroups fit a CU (FP32 orbitals: within
// the 128 registers that 4 waves per SIMD leave).
template <typename C, int NBB>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(NBB == 2 ? 2 : (sizeof(C) == 8 ? 4 : 3), 8)))
void k_orth(const DevInst *insts, const int2 *pairs, int *status, double *rho_k, int ng_max) {
    constexpr int NB = kOrthMaxBands;
    static_assert(NB * NB <= kOrthTileCap, "the Gram matrix shares the tile buffer");
    static_assert(16 * NBB <= NB, "band blocks");
    // tile [band][point] in FP64 (rows padded by one); the Gram matrix reuses its bytes
    // between the two passes over the tiles
    __shared__ double2 T[kOrthTileCap];
    __shared__ double2 Li[(16 * NBB) * (16 * NBB)];  // L^{-1} (lower triangle), row stride nb
    __shared__ int bad;
    double2 *S = T;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lm = lane & 15, lk = lane >> 4;
    const int2 pr = pairs[blockIdx.x];
    const DevInst &I = insts[pr.x];
    const int nb = I.nb, ng = I.ng;
    C *u = reinterpret_cast<C *>(I.u) + size_t(pr.y) * nb * ng;
    int lt = 4;  // tiles of 2^lt points
    while (lt < 9 && (nb << (lt + 1)) <= 256 * kOrthPer && nb * ((2 << lt) + 1) <= kOrthTileCap) ++lt;
    const int tp = 1 << lt, ld = tp + 1;
    if (tid == 0) bad = 0;
    C pre[kOrthPer];
    // ---- Gram matrix: per wave, blocks (I, J) of Re^T Re, Im^T Im and Re^T Im
    orth_d4 rr[NBB][NBB], ii[NBB][NBB], ri[NBB][NBB];
#pragma unroll
    for (int x = 0; x < NBB; ++x)
#pragma unroll
        for (int y = 0; y < NBB; ++y) rr[x][y] = ii[x][y] = ri[x][y] = orth_d4{0.0, 0.0, 0.0, 0.0};
    orth_fetch(u, ng, nb, lt, 0, pre);
    for (int p0 = 0; p0 < ng; p0 += tp) {
        const int np = (ng - p0 < tp) ? ng - p0 : tp;
        __syncthreads();  // previous tile consumed
        orth_stage(pre, nb, lt, T);
        __syncthreads();
        if (p0 + tp < ng) orth_fetch(u, ng, nb, lt, p0 + tp, pre);
        const int nsl = (np + 3) >> 2;  // 4-point slices holding grid points
        for (int sl = wave; sl < nsl; sl += 4) {
            const int pp = 4 * sl + lk;
            double2 v[NBB];
#pragma unroll
            for (int x = 0; x < NBB; ++x) {
                const int band = 16 * x + lm;
                v[x] = band < nb ? T[band * ld + pp] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int x = 0; x < NBB; ++x)
#pragma unroll
                for (int y = 0; y < NBB; ++y) {
                    rr[x][y] = mfma64(v[x].x, v[y].x, rr[x][y]);
                    ii[x][y] = mfma64(v[x].y, v[y].y, ii[x][y]);
                    ri[x][y] = mfma64(v[x].x, v[y].y, ri[x][y]);
                }
        }
    }
    // wave sums in wave order: S.x <- sum (Re^T Re + Im^T Im), S.y <- sum Re^T Im
    for (int w = 0; w < 4; ++w) {
        __syncthreads();  // last tile consumed / previous wave's sums written
        if (wave == w) {
#pragma unroll
            for (int x = 0; x < NBB; ++x)
#pragma unroll
                for (int y = 0; y < NBB; ++y)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int i = 16 * x + 4 * r + lk, j = 16 * y + lm;
                        if (i < nb && j < nb) {
                            double2 t = make_double2(rr[x][y][r] + ii[x][y][r], ri[x][y][r]);
                            if (w > 0) {
                                const double2 o = S[i * nb + j];
                                t = make_double2(o.x + t.x, o.y + t.y);
                            }
                            S[i * nb + j] = t;
                        }
                    }
        }
    }
    __syncthreads();
    const int ne = nb * nb;
    double2 sv[(NB * NB) / 256];
#pragma unroll
    for (int q = 0; q < (NB * NB) / 256; ++q) {  // Im S_ij = (Re^T Im)_ij - (Re^T Im)_ji
        const int e = tid + 256 * q;
        if (e < ne) {
            const int i = e / nb, j = e - i * nb;
            sv[q] = make_double2(S[e].x * I.dV, (S[e].y - S[j * nb + i].y) * I.dV);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (NB * NB) / 256; ++q) {
        const int e = tid + 256 * q;
        if (e < ne) S[e] = sv[q];
    }
    __syncthreads();
    // ---- Cholesky S = L L^H in place, one column per round (rows in parallel)
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            double d = S[j * nb + j].x;
            for (int k = 0; k < j; ++k) {
                const double2 l = S[j * nb + k];
                d -= l.x * l.x + l.y * l.y;
            }
            if (!(d > 0.0)) {
                bad = 1;
                d = 1.0;
            }
            S[j * nb + j] = make_double2(sqrt(d), 0.0);
        }
        __syncthreads();
        if (tid > j && tid < nb) {
            double2 v = S[tid * nb + j];
            for (int k = 0; k < j; ++k) {  // - L_ik conj(L_jk)
                const double2 a = S[tid * nb + k], b = S[j * nb + k];
                v.x -= a.x * b.x + a.y * b.y;
                v.y -= a.y * b.x - a.x * b.y;
            }
            const double r = 1.0 / S[j * nb + j].x;
            S[tid * nb + j] = make_double2(v.x * r, v.y * r);
        }
        __syncthreads();
    }
    if (bad) {  // S not positive definite: the bands are linearly dependent
        if (tid == 0) status[0] = 1;
        return;
    }
    // ---- L^{-1}, one column per thread: Li_cc = 1 / L_cc, Li_ic = -(sum_{c<=k<i} L_ik Li_kc) / L_ii
    if (tid < nb) {
        const int c = tid;
        for (int i = 0; i < nb; ++i) Li[i * nb + c] = make_double2(0.0, 0.0);
        Li[c * nb + c] = make_double2(1.0 / S[c * nb + c].x, 0.0);
        for (int i = c + 1; i < nb; ++i) {
            double2 v = make_double2(0.0, 0.0);
            for (int k = c; k < i; ++k) {
                const double2 a = S[i * nb + k], b = Li[k * nb + c];
                v.x += a.x * b.x - a.y * b.y;
                v.y += a.x * b.y + a.y * b.x;
            }
            const double r = -1.0 / S[i * nb + i].x;
            Li[i * nb + c] = make_double2(v.x * r, v.y * r);
        }
    }
    __syncthreads();
    // ---- U <- U L^{-H}: D[p][b] = sum_k U[p][k] conj(Li[b][k]) with B operand
    // B[k][b] = Li[b][k] per 4-band step k4 and 16-band output block y (lane: b = 16 y + l % 16,
    // k = 4 k4 + l / 16; zero outside the bands, and above the diagonal by construction).
    // Re D = Re U Re Li^T + Im U Im Li^T, Im D = Im U Re Li^T - Re U Im Li^T.
    constexpr int NK4 = 4 * NBB;
    double bx[NK4][NBB], by[NK4][NBB];
#pragma unroll
    for (int k4 = 0; k4 < NK4; ++k4)
#pragma unroll
        for (int y = 0; y < NBB; ++y) {
            const int b = 16 * y + lm, k = 4 * k4 + lk;
            const double2 l = (b < nb && k < nb) ? Li[b * nb + k] : make_double2(0.0, 0.0);
            bx[k4][y] = l.x;
            by[k4][y] = l.y;
        }
    const int nk4 = (nb + 3) >> 2;
    double fo[NBB];  // w_k f_b of the lane's output bands (zero past the last band)
#pragma unroll
    for (int y = 0; y < NBB; ++y) fo[y] = (16 * y + lm < nb) ? I.kw[pr.y] * I.occ[16 * y + lm] : 0.0;
    double *rk = rho_k ? rho_k + size_t(blockIdx.x) * ng_max : nullptr;
    // a tile is written only after it was read into LDS; the prefetch reads the next,
    // untouched tile
    orth_fetch(u, ng, nb, lt, 0, pre);
    for (int p0 = 0; p0 < ng; p0 += tp) {
        const int np = (ng - p0 < tp) ? ng - p0 : tp;
        __syncthreads();  // previous tile consumed
        orth_stage(pre, nb, lt, T);
        __syncthreads();
        if (p0 + tp < ng) orth_fetch(u, ng, nb, lt, p0 + tp, pre);
        const int npb = (np + 15) >> 4;  // 16-point blocks holding grid points
        for (int pb = wave; pb < npb; pb += 4) {
            orth_d4 dr[NBB], di[NBB];
#pragma unroll
            for (int y = 0; y < NBB; ++y) dr[y] = di[y] = orth_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k4 = 0; k4 < NK4; ++k4) {
                if (k4 < nk4) {
                    const int band = 4 * k4 + lk;
                    const double2 a = band < nb ? T[band * ld + 16 * pb + lm] : make_double2(0.0, 0.0);
                    const double nax = -a.x;
#pragma unroll
                    for (int y = 0; y < NBB; ++y) {
                        if (4 * k4 <= 16 * y + 15) {  // bands k contribute to outputs b >= k only
                            dr[y] = mfma64(a.x, bx[k4][y], dr[y]);
                            dr[y] = mfma64(a.y, by[k4][y], dr[y]);
                            di[y] = mfma64(a.y, bx[k4][y], di[y]);
                            di[y] = mfma64(nax, by[k4][y], di[y]);
                        }
                    }
                }
            }
            double rs[4] = {0.0, 0.0, 0.0, 0.0};  // density at the points 16 pb + 4 r + l / 16
#pragma unroll
            for (int y = 0; y < NBB; ++y)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int b = 16 * y + lm, pp = 16 * pb + 4 * r + lk;
                    C out;
                    out.x = decltype(out.x)(dr[y][r]);
                    out.y = decltype(out.y)(di[y][r]);
                    if (b < nb && pp < np) u[size_t(b) * ng + p0 + pp] = out;
                    const double ox = double(out.x), oy = double(out.y);
                    rs[r] = fma(fo[y], ox * ox + oy * oy, rs[r]);
                }
            if (rk) {
#pragma unroll
                for (int off = 1; off < 16; off <<= 1)  // sum over the 16 bands of a row
#pragma unroll
                    for (int r = 0; r < 4; ++r) rs[r] += __shfl_xor(rs[r], off);
                const int pp = 16 * pb + 4 * lm + lk;  // lane l % 16 = r < 4 writes row r
                const double v = lm == 0 ? rs[0] : lm == 1 ? rs[1] : lm == 2 ? rs[2] : rs[3];
                if (lm < 4 && pp < np) rk[p0 + pp] = v;
            }
        }
    }
}

hipError_t launch_orth(const DevInst *insts, const int2 *pairs, int n_pairs, int nb_max, int fp64, int *status,
                       double *rho_k, int ng_max, hipStream_t s) {
    if (n_pairs <= 0) return hipSuccess;
    if (nb_max < 1 || nb_max > kOrthMaxBands) return hipErrorInvalidValue;
    const bool two = nb_max > 16;
    if (fp64) {
        if (two)
            hipLaunchKernelGGL((k_orth<double2, 2>), dim3(n_pairs), dim3(256), 0, s, insts, pairs, status, rho_k, ng_max);
        else
            hipLaunchKernelGGL((k_orth<double2, 1>), dim3(n_pairs), dim3(256), 0, s, insts, pairs, status, rho_k, ng_max);
    } else {
        if (two)
            hipLaunchKernelGGL((k_orth<float2, 2>), dim3(n_pairs), dim3(256), 0, s, insts, pairs, status, rho_k, ng_max);
        else
            hipLaunchKernelGGL((k_orth<float2, 1>), dim3(n_pairs), dim3(256), 0, s, insts, pairs, status, rho_k, ng_max);
    }
    return hipGetLastError();
}

// Linear density mixing of the ground-state iteration, one workgroup per instance:
// resid = sum |rho_out - rho_in| dV, rho_in <- (1 - alpha) rho_in + alpha rho_out, and the
// mixed density replaces rho_out (v_Hxc is built from it next).
__global__ __launch_bounds__(256) void k_mix(const DevInst *insts, int ng_max, double *rho, double *rho_in,
                                             double alpha, double *resid) {
    __shared__ double red[4];
    const int inst = blockIdx.x;
    const DevInst &I = insts[inst];
    double *ro = rho + size_t(inst) * ng_max;
    double *ri = rho_in + size_t(inst) * ng_max;
    double s = 0.0;
    for (int p = threadIdx.x; p < I.ng; p += 256) {
        const double o = ro[p], i = ri[p];
        s += fabs(o - i);
        const double m = (1.0 - alpha) * i + alpha * o;
        ri[p] = m;
        ro[p] = m;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) resid[inst] = (red[0] + red[1] + red[2] + red[3]) * I.dV;
}

hipError_t launch_mix(const DevInst *insts, int n_inst, int ng_max, double *rho, double *rho_in, double alpha,
                      double *resid, hipStream_t s) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mix, dim3(n_inst), dim3(256), 0, s, insts, ng_max, rho, rho_in, alpha, resid);
    return hipGetLastError();
}

}  // namespace tdks
