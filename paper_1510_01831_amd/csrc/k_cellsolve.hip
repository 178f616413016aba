// Batched cell solves with the stored Schur factors (online local solves of
// Alg. 7 and the offline Green's-function probes, Sec. 4.3).
//
// With X_k = S_k^{-1} and the column couplings e_k, H^{l,c} x = b is solved by
//   forward:   y_0 = b_0,  y_k = b_k - e_k o (X_{k-1} y_{k-1})
//   backward:  x_{W-1} = X_{W-1} y_{W-1},  x_k = X_k (y_k - e_{k+1} o x_{k+1})
// where o is the elementwise product over the rows of a column.
//
// One workgroup handles one cell and NB right-hand sides; the current column
// vector lives in LDS, the factor blocks stream through LDS tiles, the
// forward iterates are kept in a global scratch for the backward sweep.
// Sources are assembled on the fly (volume source, App. C equivalent sources
// on the layer interface rows, column equivalent sources of the inner traces,
// or unit probes) and the results are sampled as they are produced.
#include "hz_common.h"

namespace hz {

constexpr int CS_THREADS = 256;
constexpr int CS_HLMAX = 224;
constexpr int CS_KC = 16;

template <typename T>
__device__ inline C2<T> to_t(double2 v) { return mk<T>((T)v.x, (T)v.y); }

template <typename T, int NB>
__device__ inline C2<T> cell_source(const CellSolveArgs<T>& a, const CellDesc& cd,
                                    const LayerDesc& ld, int k, int j, int b) {
    const int p = a.p;
    const double ih2 = 1.0 / (a.h * a.h);
    C2<T> z = mk<T>((T)0, (T)0);
    const int B = a.B;
    if (a.mode == SOLVE_GRID) {
        return a.g_grid[((long long)j * cd.Wc + k) * B + b];
    }
    const bool own_col = (k >= cd.own_c0 && k <= cd.own_c1);
    if (a.mode == SOLVE_PROBE) {
        const int probe = a.probe0 + b;
        if (probe < cd.ncol) {
            int q = probe;
            int right = 0;
            if (!cd.has_left) right = 1;
            else if (q >= 2 * cd.HL) { right = 1; q -= 2 * cd.HL; }
            const int ab = q / cd.HL, jj = q - ab * cd.HL;
            if (j != jj) return z;
            int kk; double sg;
            if (!right) { kk = ab == 0 ? p : p - 1; sg = ab == 0 ? 1.0 : -1.0; }
            else { kk = ab == 0 ? p + cd.nc : p + cd.nc - 1; sg = ab == 0 ? -1.0 : 1.0; }
            if (k != kk) return z;
            double2 iz = cinv(a.alpha_z[(long long)cd.layer * a.HLmax + j]);
            return mk<T>((T)(sg * iz.x * ih2), (T)(sg * iz.y * ih2));
        } else {
            const int t = probe - cd.ncol;
            const int si = t / cd.s, ci = t - si * cd.s;
            if (k != cd.own_c0 + ci) return z;
            const int lid = ld.slot_id[si];
            int rr; double sg;
            if (lid == 0) { rr = p; sg = 1.0; }
            else if (lid == 1) { rr = p - 1; sg = -1.0; }
            else if (lid == 2) { rr = p + ld.nl; sg = -1.0; }
            else { rr = p + ld.nl - 1; sg = 1.0; }
            if (j != rr) return z;
            double2 ix = cinv(a.alpha_x[(long long)cd.gidx * a.Wcmax + k]);
            return mk<T>((T)(sg * ix.x * ih2), (T)(sg * ix.y * ih2));
        }
    }
    // SOLVE_SAMPLE / SOLVE_VOLUME
    C2<T> v = z;
    const long long W = a.W;
    const bool own_row = (j >= ld.own_r0 && j <= ld.own_r1);
    if (a.f_ext && own_col && own_row && (!a.layer_active || a.layer_active[cd.layer])) {
        v = a.f_ext[(((long long)(ld.row0 + j)) * W + cd.col0 + k) * B + b];
    }
    if (a.mode == SOLVE_VOLUME) {
        if (own_col) {
            const C2<T>* top = a.top_pair ? a.top_pair[cd.layer] : nullptr;
            const C2<T>* bot = a.bot_pair ? a.bot_pair[cd.layer] : nullptr;
            const long long col = cd.col0 + k;
            if (top && (j == p || j == p - 1)) {
                double2 ix = cinv(a.alpha_x[(long long)cd.gidx * a.Wcmax + k]);
                C2<T> s = to_t<T>(mk<double>(ix.x * ih2, ix.y * ih2));
                if (j == p) v = cfma(s, top[(0 * W + col) * B + b], v);
                else v = csub(v, cmul(s, top[(1 * W + col) * B + b]));
            }
            if (bot && (j == p + ld.nl - 1 || j == p + ld.nl)) {
                double2 ix = cinv(a.alpha_x[(long long)cd.gidx * a.Wcmax + k]);
                C2<T> s = to_t<T>(mk<double>(ix.x * ih2, ix.y * ih2));
                if (j == p + ld.nl - 1) v = cfma(s, bot[(1 * W + col) * B + b], v);
                else v = csub(v, cmul(s, bot[(0 * W + col) * B + b]));
            }
        }
        if (a.inner_v && ld.J > 0) {
            const C2<T>* iv = a.inner_v + ld.off_inner * B;
            const int HL = cd.HL;
            const bool kl = cd.has_left && (k == p || k == p - 1);
            const bool kr = cd.has_right && (k == p + cd.nc || k == p + cd.nc - 1);
            if (kl || kr) {
                double2 iz = cinv(a.alpha_z[(long long)cd.layer * a.HLmax + j]);
                C2<T> s = to_t<T>(mk<double>(iz.x * ih2, iz.y * ih2));
                if (kl) {
                    const int jf = cd.cell - 1;
                    if (k == p) v = cfma(s, iv[(((long long)jf * 2 + 0) * HL + j) * B + b], v);
                    else v = csub(v, cmul(s, iv[(((long long)jf * 2 + 1) * HL + j) * B + b]));
                }
                if (kr) {
                    const int jf = cd.cell;
                    if (k == p + cd.nc) v = csub(v, cmul(s, iv[(((long long)jf * 2 + 0) * HL + j) * B + b]));
                    else v = cfma(s, iv[(((long long)jf * 2 + 1) * HL + j) * B + b], v);
                }
            }
        }
    }
    return v;
}

template <typename T, int NB>
__device__ inline void cell_emit(const CellSolveArgs<T>& a, const CellDesc& cd,
                                 const LayerDesc& ld, int k, int j, int b, C2<T> x) {
    const int p = a.p;
    const int B = a.B;
    const long long W = a.W;
    const bool own_col = (k >= cd.own_c0 && k <= cd.own_c1);
    switch (a.mode) {
    case SOLVE_GRID:
        a.x_grid[((long long)j * cd.Wc + k) * B + b] = x;
        break;
    case SOLVE_PROBE: {
        const long long probe = a.probe0 + b;
        C2<T>* CS = a.CSpool + cd.off_CS;
        C2<T>* Q = a.Qpool + cd.off_Q;
        if (cd.has_left && k == p) CS[(long long)j * cd.R + probe] = x;
        if (cd.has_right && k == p + cd.nc - 1)
            CS[((long long)(cd.has_left ? cd.HL : 0) + j) * cd.R + probe] = x;
        if (own_col) {
            for (int si = 0; si < ld.nslot; ++si)
                if (ld.slot_row[si] == j)
                    Q[((long long)si * cd.s + (k - cd.own_c0)) * cd.R + probe] = x;
        }
    } break;
    case SOLVE_SAMPLE: {
        C2<T>* ir = a.inner_rhs + ld.off_inner * B;
        const int HL = cd.HL;
        if (cd.has_left && k == p)
            ir[(((long long)(cd.cell - 1) * 2 + 1) * HL + j) * B + b] = x;
        if (cd.has_right && k == p + cd.nc - 1)
            ir[(((long long)cd.cell * 2 + 0) * HL + j) * B + b] = x;
        if (own_col) {
            for (int si = 0; si < ld.nslot; ++si)
                if (ld.slot_row[si] == j)
                    a.rows_out[(((long long)cd.layer * MAXSLOT + si) * W + cd.col0 + k) * B + b] = x;
        }
    } break;
    case SOLVE_VOLUME:
        if (own_col && j >= ld.own_r0 && j <= ld.own_r1)
            a.u_ext[(((long long)(ld.row0 + j)) * W + cd.col0 + k) * B + b] = x;
        break;
    default:
        break;
    }
}

// t = X * v for an HL x HL block X (row-major, global) and v [HL][NB] in LDS;
// thread owns column c = tid % NB and rows j = tid / NB + m * (CS_THREADS/NB).
template <typename T, int NB, int MR>
__device__ inline void block_matvec(const C2<T>* __restrict__ X, int HL, const C2<T>* vs,
                                    C2<T> (*Xs)[CS_KC + 1], C2<T> acc[MR]) {
    const int tid = threadIdx.x;
    constexpr int RG = CS_THREADS / NB;
    const int c = tid % NB;
    const int j0 = tid / NB;
#pragma unroll
    for (int m = 0; m < MR; ++m) acc[m] = mk<T>((T)0, (T)0);
    for (int i0 = 0; i0 < HL; i0 += CS_KC) {
        const int kc = min(CS_KC, HL - i0);
        __syncthreads();
        for (int idx = tid; idx < HL * CS_KC; idx += CS_THREADS) {
            const int r = idx / CS_KC, ii = idx - r * CS_KC;
            Xs[r][ii] = (ii < kc) ? X[(long long)r * HL + i0 + ii] : mk<T>((T)0, (T)0);
        }
        __syncthreads();
        for (int ii = 0; ii < kc; ++ii) {
            const C2<T> vv = vs[(i0 + ii) * NB + c];
#pragma unroll
            for (int m = 0; m < MR; ++m) {
                const int j = j0 + m * RG;
                if (j < HL) acc[m] = cfma(Xs[j][ii], vv, acc[m]);
            }
        }
    }
}

template <typename T, int NB>
__global__ void __launch_bounds__(CS_THREADS) k_cell_solve(CellSolveArgs<T> a) {
    constexpr int RG = CS_THREADS / NB;
    constexpr int MR = (CS_HLMAX + RG - 1) / RG;
    __shared__ C2<T> vs[CS_HLMAX * NB];
    __shared__ C2<T> Xs[CS_HLMAX][CS_KC + 1];

    const int gc = a.cell_list[blockIdx.x];
    const CellDesc cd = a.cells[gc];
    const LayerDesc ld = a.layers[cd.layer];
    const int HL = cd.HL, Wc = cd.Wc;
    const int b0 = blockIdx.y * NB;
    if (a.mode == SOLVE_PROBE && a.probe0 + b0 >= cd.R) return;   // uniform per workgroup
    const int tid = threadIdx.x;
    const int c = tid % NB;
    const int j0 = tid / NB;
    const int b = b0 + c;
    const bool bvalid = b < a.B && (a.mode != SOLVE_PROBE || a.probe0 + b < cd.R);
    const long long nn = (long long)HL * HL;
    const C2<T>* Xf = a.X + cd.off_X;
    const C2<T>* ee = a.coef_e + cd.off_coef;
    C2<T>* Y = a.Y + ((long long)blockIdx.x * gridDim.y + blockIdx.y) * a.y_stride;
    C2<T> acc[MR];

    // ---- forward sweep
    for (int k = 0; k < Wc; ++k) {
        if (k > 0) block_matvec<T, NB, MR>(Xf + (long long)(k - 1) * nn, HL, vs, Xs, acc);
        C2<T> yv[MR];
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int j = j0 + m * RG;
            if (j < HL) {
                C2<T> s = bvalid ? cell_source<T, NB>(a, cd, ld, k, j, b) : mk<T>((T)0, (T)0);
                if (k > 0) s = csub(s, cmul(ee[(long long)k * HL + j], acc[m]));
                yv[m] = s;
                Y[((long long)k * HL + j) * NB + c] = s;
            }
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int j = j0 + m * RG;
            if (j < HL) vs[j * NB + c] = yv[m];
        }
        __syncthreads();
    }
    // ---- backward sweep
    for (int k = Wc - 1; k >= 0; --k) {
        if (k < Wc - 1) {
            // v <- y_k - e_{k+1} o x_{k+1}   (elementwise, own entries)
#pragma unroll
            for (int m = 0; m < MR; ++m) {
                const int j = j0 + m * RG;
                if (j < HL) {
                    C2<T> xv = vs[j * NB + c];
                    vs[j * NB + c] = csub(Y[((long long)k * HL + j) * NB + c],
                                          cmul(ee[(long long)(k + 1) * HL + j], xv));
                }
            }
        }
        block_matvec<T, NB, MR>(Xf + (long long)k * nn, HL, vs, Xs, acc);
        __syncthreads();
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int j = j0 + m * RG;
            if (j < HL) {
                vs[j * NB + c] = acc[m];
                if (bvalid) cell_emit<T, NB>(a, cd, ld, k, j, b, acc[m]);
            }
        }
        __syncthreads();
    }
}

template <typename T>
void launch_cell_solve(const CellSolveArgs<T>& a, int ncells_launch, int nb_chunks,
                       hipStream_t st) {
    (void)nb_chunks;
    if (a.B <= 1) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cell_solve<T, 1>), dim3(ncells_launch, 1), dim3(CS_THREADS), 0, st, a);
    } else if (a.B <= 4) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cell_solve<T, 4>), dim3(ncells_launch, 1), dim3(CS_THREADS), 0, st, a);
    } else {
        const int chunks = (a.B + 15) / 16;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cell_solve<T, 16>), dim3(ncells_launch, chunks), dim3(CS_THREADS), 0, st, a);
    }
}

template void launch_cell_solve<double>(const CellSolveArgs<double>&, int, int, hipStream_t);
template void launch_cell_solve<float>(const CellSolveArgs<float>&, int, int, hipStream_t);

}  // namespace hz
