// Coefficient construction (App. A), layout conversions, the FP64 residual,
// the misfit gradient and the reductions of the GMRES driver.
#include "hz_common.h"

namespace hz {

__device__ inline double model_m(const double* model, int kind, int n, int zpos, int xpos) {
    // m is extended beyond the physical square by copying the nearest value
    zpos = zpos < 1 ? 1 : (zpos > n ? n : zpos);
    xpos = xpos < 1 ? 1 : (xpos > n ? n : xpos);
    const double v = model[(long long)(zpos - 1) * n + (xpos - 1)];
    return kind == 0 ? 1.0 / (v * v) : v;
}

__global__ void k_check_model(const double* model, long long count, int* bad) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
         i += (long long)gridDim.x * blockDim.x) {
        const double v = model[i];
        if (!(v > 0.0) || !isfinite(v)) atomicOr(bad, 1);
    }
}

// Symmetric-form 5-point coefficients of every cell grid, stored per grid
// column: diag, the depth coupling between rows j and j+1, and the coupling
// e_k between columns k-1 and k.
__global__ void k_cell_coef(const double* model, int kind, Dims d, const CellDesc* cells,
                            const LayerDesc* layers, double2* diag, double2* cz, double2* e,
                            double2* ax_pool, double2* az_pool) {
    const CellDesc cd = cells[blockIdx.y];
    const LayerDesc ld = layers[cd.layer];
    const int p = d.p;
    const double ih2 = 1.0 / (d.h * d.h);
    const double w2 = d.omega * d.omega;
    const long long total = (long long)cd.Wc * cd.HL;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int k = (int)(q / cd.HL), j = (int)(q % cd.HL);
        const double xp = k - p + 1, zp = j - p + 1;           // local positions
        const double2 ax = pml_alpha(xp, cd.nc, p, d.beta);
        const double2 axm = pml_alpha(xp - 0.5, cd.nc, p, d.beta);
        const double2 axp = pml_alpha(xp + 0.5, cd.nc, p, d.beta);
        const double2 az = pml_alpha(zp, ld.nl, p, d.beta);
        const double2 azm = pml_alpha(zp - 0.5, ld.nl, p, d.beta);
        const double2 azp = pml_alpha(zp + 0.5, ld.nl, p, d.beta);
        const double2 iax = cinv(ax), iaz = cinv(az);
        const double m = model_m(model, kind, d.n, ld.first - p + j, cd.first - p + k);
        double2 t1 = cmul(cadd(axm, axp), iaz);
        double2 t2 = cmul(cadd(azm, azp), iax);
        double2 t3 = cmul(iax, iaz);
        double2 dg;
        dg.x = (t1.x + t2.x) * ih2 - w2 * m * t3.x;
        dg.y = (t1.y + t2.y) * ih2 - w2 * m * t3.y;
        const long long o = cd.off_coef + q;
        diag[o] = dg;
        double2 c = cmul(azp, iax);
        c.x *= -ih2; c.y *= -ih2;
        cz[o] = c;
        double2 ev = cmul(axm, iaz);
        ev.x *= -ih2; ev.y *= -ih2;
        e[o] = ev;
        if (j == 0) ax_pool[(long long)cd.gidx * d.Wcmax + k] = ax;
        if (k == 0 && cd.cell == 0) az_pool[(long long)cd.layer * d.HLmax + j] = az;
    }
}

// Global operator (residual of the refinement, Sec. 5 footnote) and the
// gradient weight w = 1/(alpha_x alpha_z).
__global__ void k_global_coef(const double* model, int kind, Dims d, double2* gdiag,
                              double2* gcx, double2* gcz, double2* wext) {
    const int W = d.W, p = d.p;
    const double ih2 = 1.0 / (d.h * d.h);
    const double w2 = d.omega * d.omega;
    const long long total = (long long)W * W;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int Z = (int)(q / W), X = (int)(q % W);
        const double xp = X - p + 1, zp = Z - p + 1;
        const double2 ax = pml_alpha(xp, d.n, p, d.beta);
        const double2 axm = pml_alpha(xp - 0.5, d.n, p, d.beta);
        const double2 axp = pml_alpha(xp + 0.5, d.n, p, d.beta);
        const double2 az = pml_alpha(zp, d.n, p, d.beta);
        const double2 azm = pml_alpha(zp - 0.5, d.n, p, d.beta);
        const double2 azp = pml_alpha(zp + 0.5, d.n, p, d.beta);
        const double2 iax = cinv(ax), iaz = cinv(az);
        const double m = model_m(model, kind, d.n, (int)zp, (int)xp);
        double2 t1 = cmul(cadd(axm, axp), iaz);
        double2 t2 = cmul(cadd(azm, azp), iax);
        double2 t3 = cmul(iax, iaz);
        double2 dg;
        dg.x = (t1.x + t2.x) * ih2 - w2 * m * t3.x;
        dg.y = (t1.y + t2.y) * ih2 - w2 * m * t3.y;
        gdiag[q] = dg;
        double2 cx = cmul(axp, iaz); cx.x *= -ih2; cx.y *= -ih2;
        double2 c2 = cmul(azp, iax); c2.x *= -ih2; c2.y *= -ih2;
        gcx[q] = cx;
        gcz[q] = c2;
        wext[q] = t3;
    }
}

void launch_check_model(const double* model, long long count, int* bad_flag, hipStream_t st) {
    hipLaunchKernelGGL(k_check_model, dim3(256), dim3(256), 0, st, model, count, bad_flag);
}

void launch_build_coef(const double* model, int model_kind, const Dims& d,
                       const CellDesc* cells_dev, const LayerDesc* layers_dev, int ncells,
                       const CellDesc* cells_host, double2* diag, double2* cz, double2* e,
                       double2* ax_pool, double2* az_pool, double2* gdiag, double2* gcx,
                       double2* gcz, double2* wext, int* bad_flag, hipStream_t st) {
    (void)cells_host;
    hipLaunchKernelGGL(k_check_model, dim3(256), dim3(256), 0, st, model, (long long)d.n * d.n,
                       bad_flag);
    hipLaunchKernelGGL(k_cell_coef, dim3(64, ncells), dim3(256), 0, st, model, model_kind, d,
                       cells_dev, layers_dev, diag, cz, e, ax_pool, az_pool);
    hipLaunchKernelGGL(k_global_coef, dim3(1024), dim3(256), 0, st, model, model_kind, d, gdiag,
                       gcx, gcz, wext);
}

// ---------------------------------------------------------------------------
// elementwise helpers

template <typename T>
__global__ void k_axpby(C2<T>* y, const C2<T>* x, double2 a, double2 b, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        C2<T> xv = x ? x[i] : mk<T>((T)0, (T)0);
        C2<T> yv = y[i];
        C2<T> ta = mk<T>((T)a.x, (T)a.y), tb = mk<T>((T)b.x, (T)b.y);
        y[i] = cadd(cmul(ta, xv), cmul(tb, yv));
    }
}

template <typename T>
void launch_axpby(C2<T>* y, const C2<T>* x, double2 a, double2 b, long long n, hipStream_t st) {
    if (n <= 0) return;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_axpby<T>), dim3(blocks), dim3(256), 0, st, y, x, a, b, n);
}
template void launch_axpby<double>(double2*, const double2*, double2, double2, long long, hipStream_t);
template void launch_axpby<float>(float2*, const float2*, double2, double2, long long, hipStream_t);

__global__ void k_cast_d2f(float2* y, const double2* x, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double2 v = x[i];
        y[i] = make_float2((float)v.x, (float)v.y);
    }
}
// y = x widened to FP64; also into y2 where given (one read of x for two
// destinations)
__global__ void k_cast_f2d(double2* y, double2* y2, const float2* x, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        float2 v = x[i];
        const double2 d = make_double2((double)v.x, (double)v.y);
        y[i] = d;
        if (y2) y2[i] = d;
    }
}
void launch_cast_d2f(float2* y, const double2* x, long long n, hipStream_t st) {
    if (n <= 0) return;
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_cast_d2f, dim3(blocks), dim3(256), 0, st, y, x, n);
}
void launch_cast_f2d(double2* y, const float2* x, long long n, hipStream_t st, double2* y2) {
    if (n <= 0) return;
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_cast_f2d, dim3(blocks), dim3(256), 0, st, y, y2, x, n);
}

__global__ void k_conj_copy(double2* y, const double2* x, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double2 v = x[i];
        y[i] = make_double2(v.x, -v.y);
    }
}
void launch_conj_copy(double2* y, const double2* x, long long n, hipStream_t st) {
    if (n <= 0) return;
    int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_conj_copy, dim3(blocks), dim3(256), 0, st, y, x, n);
}

// ---------------------------------------------------------------------------
// GMRES reductions on batch-fastest vectors: element (i, b) at i * B + b.

constexpr int RD_THREADS = 256;

// partial[(chunk * nv + v) * B + b] = sum_{i in chunk} conj(V_v[i,b]) w[i,b]
// Up to DV basis vectors per workgroup, so w is read once per DV of them.
constexpr int DV = 8;

// Threads per batch column of the reduction kernels: the largest power of
// two with per * B <= RD_THREADS (at least 1).
__device__ inline int rd_per(int B) {
    int per = 1;
    while (2 * per * B <= RD_THREADS) per *= 2;
    return per;
}

// Column sums of NV quantities per thread: thread tid = sub * bcols + col
// (sub < per, a power of two) holds acc[v] of column col; the sums over sub
// are formed by halving, all quantities at once, and left in acc of the
// threads with sub = 0.  red: NV * RD_THREADS entries of LDS.
template <int NV>
__device__ inline void reduce_columns(double2 (&acc)[NV], int nout, int per, int bcols,
                                      double2* red) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int v = 0; v < NV; ++v)
        if (v < nout) red[v * RD_THREADS + tid] = acc[v];
    __syncthreads();
    const int sub = tid / bcols;
    for (int h = per / 2; h > 0; h >>= 1) {
        if (sub < h) {
#pragma unroll
            for (int v = 0; v < NV; ++v)
                if (v < nout) {
                    const double2 o = red[v * RD_THREADS + tid + h * bcols];
                    red[v * RD_THREADS + tid].x += o.x;
                    red[v * RD_THREADS + tid].y += o.y;
                }
        }
        __syncthreads();
    }
    if (tid < bcols) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (v < nout) acc[v] = red[v * RD_THREADS + tid];
    }
    __syncthreads();
}

// Partial sums of conj(V_v) w (or |w|^2 when V is null) for the up to NVT
// vectors v0 .. v0 + NVT - 1 of this workgroup row (blockIdx.y); NVT is the
// vector count itself for passes over at most DV vectors, so registers scale
// with it, and for up to four vectors two rows per thread are in flight.
template <int NVT>
__global__ void __launch_bounds__(RD_THREADS)
k_dots(const double2* V, long long vstride, int nv, const double2* w, long long n, int B,
       double2* partial, int nchunks) {
    __shared__ double2 red[NVT * RD_THREADS];
    const int v0 = blockIdx.y * NVT;
    const int nvb = nv - v0 < NVT ? nv - v0 : NVT;
    const int tid = threadIdx.x;
    const int per = rd_per(B);                                    // threads per column
    const int bcols = B < RD_THREADS ? B : RD_THREADS;
    const long long chunk = (n + nchunks - 1) / nchunks;
    const long long i0 = blockIdx.x * chunk;
    const long long i1 = (i0 + chunk < n) ? i0 + chunk : n;
    for (int bb = 0; bb < B; bb += bcols) {
        double2 acc[NVT];
#pragma unroll
        for (int v = 0; v < NVT; ++v) acc[v] = make_double2(0.0, 0.0);
        const int b = bb + tid % bcols;
        const int sub = tid / bcols;
        if (sub < per && b < B) {
            auto row = [&](double2 c, const double2 (&a)[NVT]) {
#pragma unroll
                for (int v = 0; v < NVT; ++v) {
                    if (v < nvb) {
                        acc[v].x += a[v].x * c.x + a[v].y * c.y;
                        acc[v].y += a[v].x * c.y - a[v].y * c.x;
                    }
                }
            };
            auto load = [&](long long q, double2 (&a)[NVT]) {
                const double2 c = w[q];
#pragma unroll
                for (int v = 0; v < NVT; ++v)
                    a[v] = (V && v < nvb) ? gload<double>(V + (v0 + v) * vstride + q) : c;
                return c;
            };
            long long i = i0 + sub;
            constexpr bool TWO = NVT <= 4;
            for (; TWO && i + per < i1; i += 2 * per) {
                double2 a0[NVT], a1[NVT];
                const double2 c0 = load(i * B + b, a0);
                const double2 c1 = load((i + per) * B + b, a1);
                row(c0, a0);
                row(c1, a1);
            }
            for (; i < i1; i += per) {
                double2 a0[NVT];
                const double2 c0 = load(i * B + b, a0);
                row(c0, a0);
            }
        }
        reduce_columns<NVT>(acc, nvb, per, bcols, red);
        if (tid < bcols && bb + tid < B)
            for (int v = 0; v < nvb; ++v)
                partial[((long long)blockIdx.x * nv + v0 + v) * B + bb + tid] = acc[v];
    }
}

void launch_dots(const double2* V, long long vstride, int nv, const double2* w, long long n,
                 int B, double2* partial, int nchunks, hipStream_t st) {
#define HZ_DOTS(NVC)                                                                           \
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_dots<NVC>), dim3(nchunks, (nv + NVC - 1) / NVC),      \
                       dim3(RD_THREADS), 0, st, V, vstride, nv, w, n, B, partial, nchunks)
    switch (nv) {
    case 1: HZ_DOTS(1); break;
    case 2: HZ_DOTS(2); break;
    case 3: HZ_DOTS(3); break;
    case 4: HZ_DOTS(4); break;
    case 5: HZ_DOTS(5); break;
    case 6: HZ_DOTS(6); break;
    case 7: HZ_DOTS(7); break;
    default: HZ_DOTS(DV); break;
    }
#undef HZ_DOTS
}

// One Gram-Schmidt pass fused with the reductions of the next step:
//   w <- w + sgn * sum_{v < nv} coef[v][b] V_v      (stored back to w)
// then, for the updated w, partial sums of conj(V_v) w for v < nv (norm = 0,
// nv outputs) or of |w|^2 (norm = 1, one output), laid out as k_dots'.  The
// basis values of an element stay in registers between the two halves, so
// V and w are read once for both (nv <= UD_MAX = 8).
constexpr int UD_MAX = 8;

// NV (the number of basis vectors) is a template parameter, so that the
// registers of a pass scale with it (all eight at once took 143 registers,
// three waves per SIMD, and the 1024-workgroup launch ran in two rounds), and
// for up to four vectors two rows per thread are in flight per loop step.
template <int NV>
__global__ void __launch_bounds__(RD_THREADS)
k_update_dots(double2* __restrict__ w, const double2* __restrict__ V, long long vstride,
              const double2* __restrict__ coef, double sgn, long long n, int B, int norm,
              double2* __restrict__ partial, int nchunks) {
    __shared__ double2 red[NV * RD_THREADS];
    const int tid = threadIdx.x;
    const int per = rd_per(B);
    const int bcols = B < RD_THREADS ? B : RD_THREADS;
    const long long chunk = (n + nchunks - 1) / nchunks;
    const long long i0 = blockIdx.x * chunk;
    const long long i1 = (i0 + chunk < n) ? i0 + chunk : n;
    const int nout = norm ? 1 : NV;
    for (int bb = 0; bb < B; bb += bcols) {
        double2 acc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[v] = make_double2(0.0, 0.0);
        const int b = bb + tid % bcols;
        const int sub = tid / bcols;
        if (sub < per && b < B) {
            double2 h[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) h[v] = coef[(long long)v * B + b];
            // one row: w <- w + sgn V h, then the products with the new w
            auto row = [&](double2 x, const double2 (&vv)[NV], long long q) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    x.x += sgn * (h[v].x * vv[v].x - h[v].y * vv[v].y);
                    x.y += sgn * (h[v].x * vv[v].y + h[v].y * vv[v].x);
                }
                w[q] = x;
                if (norm) {
                    acc[0].x += x.x * x.x + x.y * x.y;
                } else {
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        acc[v].x += vv[v].x * x.x + vv[v].y * x.y;
                        acc[v].y += vv[v].x * x.y - vv[v].y * x.x;
                    }
                }
            };
            long long i = i0 + sub;
            // two rows per step only where the registers allow four waves
            // per SIMD (the passes over many vectors have loads enough)
            constexpr bool TWO = NV <= 4;
            for (; TWO && i + per < i1; i += 2 * per) {
                const long long q0 = i * B + b, q1 = (i + per) * B + b;
                const double2 x0 = w[q0], x1 = w[q1];
                double2 v0[NV], v1[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    v0[v] = gload<double>(V + v * vstride + q0);
                    v1[v] = gload<double>(V + v * vstride + q1);
                }
                row(x0, v0, q0);
                row(x1, v1, q1);
            }
            for (; i < i1; i += per) {
                const long long q0 = i * B + b;
                double2 v0[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) v0[v] = gload<double>(V + v * vstride + q0);
                row(w[q0], v0, q0);
            }
        }
        reduce_columns<NV>(acc, nout, per, bcols, red);
        if (tid < bcols && bb + tid < B)
            for (int v = 0; v < nout; ++v)
                partial[((long long)blockIdx.x * nout + v) * B + bb + tid] = acc[v];
    }
}

bool launch_update_dots(double2* w, const double2* V, long long vstride, int nv,
                        const double2* coef, double sgn, long long n, int B, int norm,
                        double2* partial, int nchunks, hipStream_t st) {
    if (nv < 1 || nv > UD_MAX) return false;
#define HZ_UD(NVC)                                                                          \
    case NVC:                                                                               \
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_update_dots<NVC>), dim3(nchunks), dim3(RD_THREADS), \
                           0, st, w, V, vstride, coef, sgn, n, B, norm, partial, nchunks); \
        break;
    switch (nv) {
        HZ_UD(1) HZ_UD(2) HZ_UD(3) HZ_UD(4) HZ_UD(5) HZ_UD(6) HZ_UD(7) HZ_UD(8)
    }
#undef HZ_UD
    return true;
}

void launch_norms(const double2* w, long long n, int B, double2* partial, int nchunks,
                  hipStream_t st) {
    launch_dots(nullptr, 0LL, 1, w, n, B, partial, nchunks, st);
}

// out[q] = sum_c partial[c * count + q]: one workgroup per output entry, a
// strided pass over the chunks and a tree in LDS (fixed order: deterministic)
__global__ void __launch_bounds__(RD_THREADS)
k_reduce_partials(const double2* partial, int nchunks, int count, double2* out) {
    __shared__ double2 red[RD_THREADS];
    const int q = blockIdx.x;
    double2 s = make_double2(0.0, 0.0);
    for (int c = threadIdx.x; c < nchunks; c += RD_THREADS) {
        const double2 v = partial[(long long)c * count + q];
        s.x += v.x; s.y += v.y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = RD_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[threadIdx.x].x += red[threadIdx.x + h].x;
            red[threadIdx.x].y += red[threadIdx.x + h].y;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[q] = red[0];
}
void launch_reduce_partials(const double2* partial, int nchunks, int count, double2* out,
                            hipStream_t st) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_reduce_partials, dim3(count), dim3(RD_THREADS), 0, st, partial, nchunks,
                       count, out);
}

// out[i,b] = c0[b] x0[i,b] + c1[b] x1[i,b] (+ c2[b] x2[i,b]), coef = [3][B]
// (per-column complex coefficients; out may alias an input)
__global__ void k_lincomb3(double2* out, const double2* x0, const double2* x1, const double2* x2,
                           const double2* coef, long long n, int B) {
    const long long total = n * B;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int b = (int)(q % B);
        const double2 c0 = coef[b], c1 = coef[B + b];
        const double2 a0 = x0[q], a1 = x1[q];
        double2 r = make_double2(c0.x * a0.x - c0.y * a0.y + c1.x * a1.x - c1.y * a1.y,
                                 c0.x * a0.y + c0.y * a0.x + c1.x * a1.y + c1.y * a1.x);
        if (x2) {
            const double2 c2 = coef[2 * B + b], a2 = x2[q];
            r.x += c2.x * a2.x - c2.y * a2.y;
            r.y += c2.x * a2.y + c2.y * a2.x;
        }
        out[q] = r;
    }
}
void launch_lincomb3(double2* out, const double2* x0, const double2* x1, const double2* x2,
                     const double2* coef, long long n, int B, hipStream_t st) {
    const long long total = n * B;
    const int blocks = (int)std::min<long long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_lincomb3, dim3(blocks), dim3(256), 0, st, out, x0, x1, x2, coef, n, B);
}

__global__ void k_fill_zero(double2* y, long long n) {
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x)
        y[q] = make_double2(0.0, 0.0);
}
void launch_fill_zero(double2* y, long long n, hipStream_t st) {
    const int blocks = (int)std::min<long long>((n + 255) / 256, 16384);
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, st, y, n);
}

// w[i,b] += sgn * sum_v coef[v,b] V_v[i,b]
__global__ void k_update_basis(double2* w, const double2* V, long long vstride, int nv,
                               const double2* coef, long long n, int B, double sgn) {
    const long long total = n * B;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int b = (int)(q % B);
        double2 acc = make_double2(0.0, 0.0);
        for (int v = 0; v < nv; ++v) {
            const double2 c = coef[(long long)v * B + b];
            const double2 x = V[v * vstride + q];
            acc.x += c.x * x.x - c.y * x.y;
            acc.y += c.x * x.y + c.y * x.x;
        }
        const double2 w0 = w[q];
        w[q] = make_double2(w0.x + sgn * acc.x, w0.y + sgn * acc.y);
    }
}
void launch_update_basis(double2* w, const double2* V, long long vstride, int nv,
                         const double2* coef, long long n, int B, hipStream_t st, double sgn) {
    const long long total = n * B;
    int blocks = (int)std::min<long long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_update_basis, dim3(blocks), dim3(256), 0, st, w, V, vstride, nv, coef,
                       n, B, sgn);
}

// y[i,b] = s[b] x[i,b], also into y2 when given (a second copy of the new
// Krylov vector for the operator plans' fixed input buffer)
__global__ void k_scale_cols(double2* y, double2* y2, const double2* x, const double2* s,
                             long long n, int B) {
    const long long total = n * B;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const double2 c = s[q % B];
        const double2 v = x[q];
        const double2 r = make_double2(c.x * v.x - c.y * v.y, c.x * v.y + c.y * v.x);
        y[q] = r;
        if (y2) y2[q] = r;
    }
}
void launch_scale_cols(double2* y, const double2* x, const double2* s, long long n, int B,
                       hipStream_t st, double2* y2) {
    const long long total = n * B;
    int blocks = (int)std::min<long long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_scale_cols, dim3(blocks), dim3(256), 0, st, y, y2, x, s, n, B);
}

// The same scaled by 1 / |x_b| from the squared norms n2[b].x (0 for a zero
// norm), without a separate kernel for the scales
__global__ void k_scale_cols_inv_norm(double2* y, double2* y2, const double2* x,
                                      const double2* n2, long long n, int B) {
    const long long total = n * B;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const double m = n2[q % B].x;
        const double c = m > 0.0 ? 1.0 / sqrt(m) : 0.0;
        const double2 v = x[q];
        const double2 r = make_double2(c * v.x, c * v.y);
        y[q] = r;
        if (y2) y2[q] = r;
    }
}
void launch_scale_cols_inv_norm(double2* y, double2* y2, const double2* x, const double2* n2,
                                long long n, int B, hipStream_t st) {
    const long long total = n * B;
    int blocks = (int)std::min<long long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_scale_cols_inv_norm, dim3(blocks), dim3(256), 0, st, y, y2, x, n2, n, B);
}

// ---------------------------------------------------------------------------
// layout conversions

// Both conversions go through LDS: a workgroup moves a TT x TT block of
// (batch column, grid column) pairs of one grid row, reading along the grid
// row and writing along the batch (or the reverse), both coalesced in 1 KB
// runs (one wave per 64-element row).  The tile (66.5 KB) is dynamic LDS.
constexpr int TT = 64;
constexpr int TT_LDS = TT * (TT + 1) * (int)sizeof(double2);

// rhs[b][z][x] (physical) -> f_ext[Z][X][b] (extended, batch fastest), zero in
// the PML, and flag the layer whose owned rows hold extended row Z when the
// block carries a nonzero source.  Grid: (column tiles x batch tiles, row
// groups of TZ rows); the loads of the next row are in flight while the
// current tile is written out.
constexpr int TZ = 4;

__global__ void __launch_bounds__(256)
k_rhs_to_ext(const double2* __restrict__ rhs, int B, int n, int p, int W,
             double2* __restrict__ f_ext, const LayerDesc* layers, int L, int* active) {
    extern __shared__ double2 cv_tile[];
    __shared__ int any;
    auto tile = [&](int r, int c) -> double2& { return cv_tile[r * (TT + 1) + c]; };
    const int xt = (W + TT - 1) / TT;
    const int X0 = (blockIdx.x % xt) * TT, b0 = (blockIdx.x / xt) * TT;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;      // 4 rows of 64 lanes
    constexpr int RS = 256 / TT;                                  // rows per pass
    constexpr int RPT = TT / RS;                                  // tile rows per thread
    double2 v[RPT];
    auto load = [&](int Z) {
        const int z = Z - p;
        const bool row_in = z >= 0 && z < n;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {                            // r: batch column
            const int r = ty + q * RS;
            const int b = b0 + r, x = X0 + tx - p;
            v[q] = make_double2(0.0, 0.0);
            if (row_in && b < B && x >= 0 && x < n) v[q] = rhs[((long long)b * n + z) * n + x];
        }
    };
    const int Zb = blockIdx.y * TZ;
    if (Zb < W) load(Zb);
    for (int Z = Zb; Z < min(W, Zb + TZ); ++Z) {
        if (threadIdx.x == 0) any = 0;
        __syncthreads();
        bool nz = false;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            nz = nz || v[q].x != 0.0 || v[q].y != 0.0;
            tile(ty + q * RS, tx) = v[q];
        }
        if (nz) any = 1;
        __syncthreads();
        if (Z + 1 < min(W, Zb + TZ)) load(Z + 1);
        for (int r = ty; r < TT; r += RS) {                       // r: grid column
            const int X = X0 + r, b = b0 + tx;
            if (X < W && b < B) f_ext[((long long)Z * W + X) * B + b] = tile(tx, r);
        }
        if (active && threadIdx.x == 0 && any) {
            for (int l = 0; l < L; ++l) {
                const int lo = layers[l].row0 + layers[l].own_r0;
                const int hi = layers[l].row0 + layers[l].own_r1;
                if (Z >= lo && Z <= hi) { atomicOr(&active[l], 1); break; }
            }
        }
        __syncthreads();
    }
}

// the conversions' dynamic LDS above the default limit, set once per device
static void cv_lds_attr(const void* fn, int* done) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        dev = 0;
    }
    if (!done[dev]) {
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, TT_LDS) !=
            hipSuccess)
            (void)hipGetLastError();
        done[dev] = 1;
    }
}

void launch_rhs_to_ext(const double2* rhs, int B, int n, int p, int W, double2* f_ext,
                       const LayerDesc* layers_dev, int L, int* layer_active, hipStream_t st) {
    static int done[64] = {0};
    cv_lds_attr(reinterpret_cast<const void*>(&k_rhs_to_ext), done);
    const int xt = (W + TT - 1) / TT, bt = (B + TT - 1) / TT;
    hipLaunchKernelGGL(k_rhs_to_ext, dim3(xt * bt, (W + TZ - 1) / TZ), dim3(256), TT_LDS, st, rhs,
                       B, n, p, W, f_ext, layers_dev, L, layer_active);
}

// u[Z][X][b] (extended, batch fastest) -> out[b][z][x] on the physical grid
// (physical = 1) or out[b][Z][X] on the extended grid, conjugated if asked.
// Grid: (column tiles x batch tiles, row groups of TZ rows).
__global__ void __launch_bounds__(256)
k_ext_to_out(const double2* __restrict__ u, int B, int n, int p, int W, double2* __restrict__ out,
             int physical, int conj) {
    extern __shared__ double2 cv_tile[];
    auto tile = [&](int r, int c) -> double2& { return cv_tile[r * (TT + 1) + c]; };
    const int side = physical ? n : W;
    const int off = physical ? p : 0;
    const int xt = (side + TT - 1) / TT;
    const int x0 = (blockIdx.x % xt) * TT, b0 = (blockIdx.x / xt) * TT;
    const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
    constexpr int RS = 256 / TT;
    constexpr int RPT = TT / RS;
    double2 v[RPT];
    auto load = [&](int z) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) {                            // r: grid column
            const int r = ty + q * RS;
            const int x = x0 + r, b = b0 + tx;
            v[q] = make_double2(0.0, 0.0);
            if (x < side && b < B) v[q] = u[((long long)(z + off) * W + x + off) * B + b];
            if (conj) v[q].y = -v[q].y;
        }
    };
    const int zb = blockIdx.y * TZ;
    if (zb < side) load(zb);
    for (int z = zb; z < min(side, zb + TZ); ++z) {
#pragma unroll
        for (int q = 0; q < RPT; ++q) tile(ty + q * RS, tx) = v[q];
        __syncthreads();
        if (z + 1 < min(side, zb + TZ)) load(z + 1);
        for (int r = ty; r < TT; r += RS) {                       // r: batch column
            const int b = b0 + r, x = x0 + tx;
            if (b < B && x < side) out[((long long)b * side + z) * side + x] = tile(tx, r);
        }
        __syncthreads();
    }
}
void launch_ext_to_out(const double2* u_ext, int B, int n, int p, int W, double2* out,
                       int physical, int conj, hipStream_t st) {
    static int done[64] = {0};
    cv_lds_attr(reinterpret_cast<const void*>(&k_ext_to_out), done);
    const int side = physical ? n : W;
    const int xt = (side + TT - 1) / TT, bt = (B + TT - 1) / TT;
    hipLaunchKernelGGL(k_ext_to_out, dim3(xt * bt, (side + TZ - 1) / TZ), dim3(256), TT_LDS, st,
                       u_ext, B, n, p, W, out, physical, conj);
}

__global__ void k_transpose_bfast(const double2* src, double2* dst, int B, long long n, int to_bfast) {
    const long long total = n * B;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        // q indexes the destination
        if (to_bfast) {
            const long long i = q / B; const int b = (int)(q % B);
            dst[q] = src[(long long)b * n + i];
        } else {
            const int b = (int)(q / n); const long long i = q % n;
            dst[q] = src[i * B + b];
        }
    }
}
void launch_transpose_bfast(const double2* src, double2* dst, int B, long long n, int to_bfast,
                            hipStream_t st) {
    const long long total = n * B;
    int blocks = (int)std::min<long long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_transpose_bfast, dim3(blocks), dim3(256), 0, st, src, dst, B, n, to_bfast);
}

// ---------------------------------------------------------------------------
// Per right-hand side, over the extended grid (batch fastest), without
// storing the residual: partial[blk * B + b] = (sum |f - H u|^2, sum |f|^2)
// over the workgroup's node range.  Sums are collected in LDS (dynamic,
// 2 B doubles); when B divides the workgroup size every thread keeps one
// column and adds once at the end.
__global__ void __launch_bounds__(256)
k_residual_norms(const double2* __restrict__ u, const double2* __restrict__ f,
                 const double2* __restrict__ gd, const double2* __restrict__ gcx,
                 const double2* __restrict__ gcz, int W, int B, long long nodes_per_block,
                 double2* __restrict__ partial) {
    extern __shared__ double rn_sh[];
    for (int i = threadIdx.x; i < 2 * B; i += blockDim.x) rn_sh[i] = 0.0;
    __syncthreads();
    const long long nodes = (long long)W * W;
    const long long n0 = blockIdx.x * nodes_per_block;
    const long long n1 = n0 + nodes_per_block < nodes ? n0 + nodes_per_block : nodes;
    const bool fixed = (blockDim.x % B) == 0;
    double sr = 0.0, sf = 0.0;
    for (long long q = n0 * B + threadIdx.x; q < n1 * B; q += blockDim.x) {
        const int b = (int)(q % B);
        const long long g = q / B;
        const int Z = (int)(g / W), X = (int)(g % W);
        double2 acc = cmul(gd[g], u[q]);
        if (X + 1 < W) acc = cfma(gcx[g], u[q + B], acc);
        if (X > 0) acc = cfma(gcx[g - 1], u[q - B], acc);
        if (Z + 1 < W) acc = cfma(gcz[g], u[q + (long long)W * B], acc);
        if (Z > 0) acc = cfma(gcz[g - W], u[q - (long long)W * B], acc);
        const double2 fv = f[q];
        const double rx = fv.x - acc.x, ry = fv.y - acc.y;
        const double r2 = rx * rx + ry * ry, f2 = fv.x * fv.x + fv.y * fv.y;
        if (fixed) {
            sr += r2;
            sf += f2;
        } else {
            atomicAdd(&rn_sh[2 * b], r2);
            atomicAdd(&rn_sh[2 * b + 1], f2);
        }
    }
    if (fixed) {                                  // this thread's column throughout
        const int b = (int)((n0 * B + threadIdx.x) % B);
        atomicAdd(&rn_sh[2 * b], sr);
        atomicAdd(&rn_sh[2 * b + 1], sf);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x)
        partial[(long long)blockIdx.x * B + b] = make_double2(rn_sh[2 * b], rn_sh[2 * b + 1]);
}
// Same norms for B <= 256 by marching down the grid: a workgroup holds XW =
// 256 / B groups of B threads, group g owns RX adjacent grid columns and a
// band of zb rows, and a thread owns one RHS of its group: it carries u at
// rows z - 1, z, z + 1 over its RX columns and one halo column on each side
// in registers, so u is read (RX + 2) / RX times and f once (a thread per
// column would fetch each u entry three times, as the x neighbour of two
// other workgroups).  Workgroups are numbered so that each XCD (slot L runs
// on XCD L mod 8) takes one contiguous run of (band, column group): the
// halo columns then come from the same L2.  RX = 4 (u read 1.5 times) keeps
// a thread within 128 registers, four waves per SIMD; RX = 8 took 212
// registers, two waves per SIMD, and ran at half the HBM rate.
constexpr int RN_RX = 4;

__global__ void __launch_bounds__(256, 4)
k_residual_norms_march(const double2* __restrict__ u, const double2* __restrict__ f,
                       const double2* __restrict__ gd, const double2* __restrict__ gcx,
                       const double2* __restrict__ gcz, int W, int B, int XW, int nxg, int zb,
                       double2* __restrict__ partial) {
    extern __shared__ double rn_sh[];
    for (int i = threadIdx.x; i < 2 * B; i += blockDim.x) rn_sh[i] = 0.0;
    const int total = (int)gridDim.x, Lb = (int)blockIdx.x;
    const int xcd = Lb & 7, loc = Lb >> 3, q8 = total >> 3, r8 = total & 7;
    const int tile = (xcd < r8 ? xcd * (q8 + 1) : r8 * (q8 + 1) + (xcd - r8) * q8) + loc;
    const int xg = tile % nxg, zc = tile / nxg;
    const int xo = threadIdx.x / B, b = threadIdx.x % B;
    const int xs = (xg * XW + xo) * RN_RX;           // first owned column
    const int z0 = zc * zb, z1 = min(W, z0 + zb);
    __syncthreads();
    double sr = 0.0, sf = 0.0;
    if (xo < XW && xs < W && z0 < z1) {
        const double2 zero = make_double2(0.0, 0.0);
        auto at = [&](int z, int xx) { return ((long long)z * W + xx) * B + b; };
        // window columns xs - 1 .. xs + RN_RX (zero outside the grid)
        auto load_row = [&](int z, double2* r) {
#pragma unroll
            for (int c = 0; c < RN_RX + 2; ++c) {
                const int xx = xs - 1 + c;
                r[c] = zero;
                if (z >= 0 && z < W && xx >= 0 && xx < W) r[c] = gload<double>(u + at(z, xx));
            }
        };
        double2 um[RN_RX + 2], uc[RN_RX + 2], un[RN_RX + 2];
        load_row(z0 - 1, um);
        load_row(z0, uc);
        for (int z = z0; z < z1; ++z) {
            load_row(z + 1, un);
            double2 fv[RN_RX];
#pragma unroll
            for (int c = 0; c < RN_RX; ++c) {
                fv[c] = zero;
                if (xs + c < W) fv[c] = gload<double>(f + at(z, xs + c));
            }
#pragma unroll
            for (int c = 0; c < RN_RX; ++c) {
                const int x = xs + c;
                if (x < W) {
                    const long long g = (long long)z * W + x;
                    double2 acc = cmul(gd[g], uc[c + 1]);
                    if (x + 1 < W) acc = cfma(gcx[g], uc[c + 2], acc);
                    if (x > 0) acc = cfma(gcx[g - 1], uc[c], acc);
                    if (z + 1 < W) acc = cfma(gcz[g], un[c + 1], acc);
                    if (z > 0) acc = cfma(gcz[g - W], um[c + 1], acc);
                    const double rx = fv[c].x - acc.x, ry = fv[c].y - acc.y;
                    sr += rx * rx + ry * ry;
                    sf += fv[c].x * fv[c].x + fv[c].y * fv[c].y;
                }
            }
#pragma unroll
            for (int c = 0; c < RN_RX + 2; ++c) {
                um[c] = uc[c];
                uc[c] = un[c];
            }
        }
    }
    if (xo < XW) {
        atomicAdd(&rn_sh[2 * b], sr);
        atomicAdd(&rn_sh[2 * b + 1], sf);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < B; c += blockDim.x)
        partial[(long long)blockIdx.x * B + c] = make_double2(rn_sh[2 * c], rn_sh[2 * c + 1]);
}

// Workgroups (= partial rows) of launch_residual_norms for a partial buffer
// of cap rows: up to 16 row bands per column group when marching, else the
// node-ordered kernel with at most 2048 workgroups.
int residual_norms_blocks(int W, int B, int cap) {
    const long long nodes = (long long)W * W;
    const int flat = (int)std::max<long long>(1, std::min<long long>(std::min(cap, 2048), nodes / 64));
    if (B > 256) return flat;
    const int XW = 256 / B, nxg = (W + XW * RN_RX - 1) / (XW * RN_RX);
    if (nxg > cap) return flat;
    return nxg * std::max(1, std::min(16, cap / nxg));
}

void launch_residual_norms(const double2* u, const double2* f, const double2* gdiag,
                           const double2* gcx, const double2* gcz, int W, int B, double2* partial,
                           int nblocks, hipStream_t st) {
    const int XW = B <= 256 ? 256 / B : 1, nxg = (W + XW * RN_RX - 1) / (XW * RN_RX);
    if (B <= 256 && nblocks >= nxg && nblocks % nxg == 0 && nblocks / nxg <= 16) {
        // marching layout (residual_norms_blocks gives a multiple of nxg
        // here; nz bands of zb rows cover all W rows)
        const int nz = nblocks / nxg;
        const int zb = (W + nz - 1) / nz;
        hipLaunchKernelGGL(k_residual_norms_march, dim3(nblocks), dim3(256),
                           sizeof(double) * 2 * B, st, u, f, gdiag, gcx, gcz, W, B, XW, nxg, zb,
                           partial);
        return;
    }
    const long long nodes = (long long)W * W;
    const long long per = (nodes + nblocks - 1) / nblocks;
    hipLaunchKernelGGL(k_residual_norms, dim3(nblocks), dim3(256), sizeof(double) * 2 * B, st, u,
                       f, gdiag, gcx, gcz, W, B, per, partial);
}

// ---------------------------------------------------------------------------
// r = f - H u on the extended grid (FP64)
__global__ void k_residual(const double2* u, const double2* f, double2* r, const double2* gd,
                           const double2* gcx, const double2* gcz, int W, int B, int bfast) {
    const long long total = (long long)W * W * B;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        int b, Z, X;
        if (bfast) { b = (int)(q % B); long long node = q / B; Z = (int)(node / W); X = (int)(node % W); }
        else { b = (int)(q / ((long long)W * W)); long long node = q % ((long long)W * W); Z = (int)(node / W); X = (int)(node % W); }
        auto idx = [&](int z, int x) -> long long {
            return bfast ? (((long long)z * W + x) * B + b) : ((long long)b * W * W + (long long)z * W + x);
        };
        const long long g = (long long)Z * W + X;
        double2 acc = cmul(gd[g], u[q]);
        if (X + 1 < W) acc = cfma(gcx[g], u[idx(Z, X + 1)], acc);
        if (X > 0) acc = cfma(gcx[g - 1], u[idx(Z, X - 1)], acc);
        if (Z + 1 < W) acc = cfma(gcz[g], u[idx(Z + 1, X)], acc);
        if (Z > 0) acc = cfma(gcz[g - W], u[idx(Z - 1, X)], acc);
        const double2 fv = f ? f[q] : make_double2(0.0, 0.0);
        r[q] = make_double2(fv.x - acc.x, fv.y - acc.y);
    }
}
void launch_residual(const double2* u, const double2* f, double2* r, const double2* gdiag,
                     const double2* gcx, const double2* gcz, int W, int B, int layout_bfast,
                     hipStream_t st) {
    const long long total = (long long)W * W * B;
    int blocks = (int)std::min<long long>((total + 255) / 256, 16384);
    hipLaunchKernelGGL(k_residual, dim3(blocks), dim3(256), 0, st, u, f, r, gdiag, gcx, gcz, W, B,
                       layout_bfast);
}

// r = P u - d on the receiver row; adjoint source P^T r; partial sums of |r|^2
__global__ void k_misfit(const double2* u, const double2* d, int rec_row, int B, int n, int p,
                         int W, double2* adj, double* Jpart) {
    __shared__ double red[256];
    double acc = 0.0;
    const long long total = (long long)B * n * n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int b = (int)(q / ((long long)n * n));
        const long long rr = q % ((long long)n * n);
        const int z = (int)(rr / n), x = (int)(rr % n);
        double2 v = make_double2(0.0, 0.0);
        if (z == rec_row - 1) {
            const double2 uv = u[(long long)b * W * W + (long long)(z + p) * W + (x + p)];
            const double2 dv = d[(long long)b * n + x];
            v = make_double2(uv.x - dv.x, uv.y - dv.y);
            acc += v.x * v.x + v.y * v.y;
        }
        adj[q] = v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) Jpart[blockIdx.x] = red[0];
}
void launch_misfit(const double2* u_ext, const double2* d_obs, int rec_row, int B, int n, int p,
                   int W, double2* adj, double* Jpart, hipStream_t st) {
    hipLaunchKernelGGL(k_misfit, dim3(MISFIT_PARTS), dim3(256), 0, st, u_ext, d_obs, rec_row, B, n, p, W,
                       adj, Jpart);
}

// g[k] = omega^2 Re sum_b sum_{e -> k} w_e u_b[e] conj(lam_b[e]); u, lam: [b][Z][X]
__global__ void k_misfit_grad(const double2* u, const double2* lam, int B, int W, int n, int p,
                              const double2* wext, double omega, double* g) {
    const long long total = (long long)n * n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(q / n), x = (int)(q % n);     // physical, 0-based
        const int Z0 = (z == 0) ? 0 : z + p, Z1 = (z == n - 1) ? W - 1 : z + p;
        const int X0 = (x == 0) ? 0 : x + p, X1 = (x == n - 1) ? W - 1 : x + p;
        double acc = 0.0;
        for (int Z = Z0; Z <= Z1; ++Z)
            for (int X = X0; X <= X1; ++X) {
                const long long e = (long long)Z * W + X;
                const double2 w = wext[e];
                for (int b = 0; b < B; ++b) {
                    const double2 a = u[(long long)b * W * W + e];
                    const double2 l = lam[(long long)b * W * W + e];
                    // u * conj(lam)
                    const double2 t = make_double2(a.x * l.x + a.y * l.y, a.y * l.x - a.x * l.y);
                    acc += w.x * t.x - w.y * t.y;
                }
            }
        g[q] = omega * omega * acc;
    }
}
void launch_misfit_grad(const double2* u, const double2* lam, int B, int W, int n, int p,
                        const double2* wext, double omega, double* g, hipStream_t st) {
    const long long total = (long long)n * n;
    int blocks = (int)std::min<long long>((total + 255) / 256, 8192);
    hipLaunchKernelGGL(k_misfit_grad, dim3(blocks), dim3(256), 0, st, u, lam, B, W, n, p, wext,
                       omega, g);
}

}  // namespace hz
