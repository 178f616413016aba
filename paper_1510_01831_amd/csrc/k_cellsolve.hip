// Batched cell solves with the stored Schur factors (online local solves of
// Alg. 7 and the offline Green's-function probes, Sec. 4.3).
//
// With X_k = S_k^{-1} and the column couplings e_k, H^{l,c} x = b is solved by
//   forward:   y_0 = b_0,  y_k = b_k - e_k o (X_{k-1} y_{k-1})
//   backward:  x_{W-1} = X_{W-1} y_{W-1},  x_k = X_k (y_k - e_{k+1} o x_{k+1})
// where o is the elementwise product over the rows of a column.
//
// One workgroup handles one cell and NB right-hand sides.  The current
// column block lives in LDS; the X_k blocks stream from HBM/L2 in their 16x4
// MFMA tile order (each wave load is 1 KB contiguous); the forward iterates go
// to a global scratch for the backward sweep.  NB >= 16 runs the block
// products on the matrix cores (four real MFMAs per complex tile product);
// NB <= 4 is a matrix-vector product reduced across the four lanes that share
// a row.  Sources are assembled on the fly (volume source, App. C equivalent
// sources on the layer interface rows, column equivalent sources of the inner
// traces, or unit probes) and results are sampled as they are produced.
// The solve mode is a template parameter so each mode is its own kernel.
#include "hz_common.h"
#include "hz_mfma.h"

namespace hz {

constexpr int CS_THREADS = 256;
constexpr int CS_HLPMAX = 224;

template <typename T>
__device__ inline C2<T> to_t(double2 v) { return mk<T>((T)v.x, (T)v.y); }

template <typename T, int MODE>
__device__ inline C2<T> cell_source(const CellSolveArgs<T>& a, const CellDesc& cd,
                                    const LayerDesc& ld, int k, int j, int b) {
    const int p = a.p;
    const double ih2 = 1.0 / (a.h * a.h);
    C2<T> z = mk<T>((T)0, (T)0);
    const int B = a.B;
    if (j >= cd.HL) return z;
    if constexpr (MODE == SOLVE_GRID) {
        return a.g_grid[((long long)j * cd.Wc + k) * B + b];
    }
    const bool own_col = (k >= cd.own_c0 && k <= cd.own_c1);
    if constexpr (MODE == SOLVE_PROBE) {
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
    if constexpr (MODE == SOLVE_VOLUME) {
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

template <typename T, int MODE>
__device__ inline void cell_emit(const CellSolveArgs<T>& a, const CellDesc& cd,
                                 const LayerDesc& ld, int k, int j, int b, C2<T> x) {
    const int p = a.p;
    const int B = a.B;
    const long long W = a.W;
    if (j >= cd.HL) return;
    const bool own_col = (k >= cd.own_c0 && k <= cd.own_c1);
    if constexpr (MODE == SOLVE_GRID) {
        a.x_grid[((long long)j * cd.Wc + k) * B + b] = x;
    } else if constexpr (MODE == SOLVE_PROBE) {
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
    } else if constexpr (MODE == SOLVE_SAMPLE) {
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
    } else {
        if (own_col && j >= ld.own_r0 && j <= ld.own_r1)
            a.u_ext[(((long long)(ld.row0 + j)) * W + cd.col0 + k) * B + b] = x;
    }
}

template <typename T>
__device__ inline C2<T> e_coef(const C2<T>* ee, int k, int j, int HL) {
    return j < HL ? ee[(long long)k * HL + j] : mk<T>((T)0, (T)0);
}

// ===========================================================================
// NB <= 4: lanes run along the tile's 4 columns, each lane owning one row of
// a 16-row tile; the 4 partial sums of a row are combined with two shuffles.
template <typename T, int NB, int MODE>
__global__ void __launch_bounds__(CS_THREADS) k_cs_gemv(CellSolveArgs<T> a) {
    constexpr int MRT = (CS_HLPMAX / 16 + 3) / 4;   // row tiles per wave (4 for 224 rows)
    __shared__ C2<T> vs[CS_HLPMAX * NB];

    const int gc = a.cell_list[blockIdx.x];
    const CellDesc cd = a.cells[gc];
    const LayerDesc ld = a.layers[cd.layer];
    const int HL = cd.HL, HLp = cd.HLp, Wc = cd.Wc;
    const int RT = HLp >> 4, KS = HLp >> 2;
    const int b0 = blockIdx.y * NB;
    if (MODE == SOLVE_PROBE && a.probe0 + b0 >= cd.R) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const long long np2 = (long long)HLp * HLp;
    const C2<T>* Xf = a.X + cd.off_X;
    const C2<T>* ee = a.coef_e + cd.off_coef;
    C2<T>* Y = a.Y + ((long long)blockIdx.x * gridDim.y + blockIdx.y) * a.y_stride;
    auto bval = [&](int c) {
        const int b = b0 + c;
        return b < a.B && (MODE != SOLVE_PROBE || a.probe0 + b < cd.R);
    };
    for (int q = tid; q < HLp * NB; q += CS_THREADS) vs[q] = mk<T>((T)0, (T)0);
    __syncthreads();

    C2<T> acc[MRT][NB];
    auto matvec = [&](const C2<T>* Xk) {
#pragma unroll
        for (int m = 0; m < MRT; ++m)
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[m][c] = mk<T>((T)0, (T)0);
#pragma unroll
        for (int m = 0; m < MRT; ++m) {
            const int R = w + 4 * m;
            if (R < RT) {
                const C2<T>* base = Xk + ((long long)R * KS << 6) + lane;
#pragma unroll 8
                for (int s = 0; s < KS; ++s) {
                    const C2<T> x = base[(long long)s << 6];
                    const int cc = 4 * s + (lane >> 4);
#pragma unroll
                    for (int c = 0; c < NB; ++c) acc[m][c] = cfma(x, vs[cc * NB + c], acc[m][c]);
                }
            }
        }
#pragma unroll
        for (int m = 0; m < MRT; ++m)
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                C2<T> v = acc[m][c];
                v.x += __shfl_xor(v.x, 16, 64); v.y += __shfl_xor(v.y, 16, 64);
                v.x += __shfl_xor(v.x, 32, 64); v.y += __shfl_xor(v.y, 32, 64);
                acc[m][c] = v;
            }
    };

    // ---- forward sweep
    for (int k = 0; k < Wc; ++k) {
        if (k > 0) matvec(Xf + (long long)(k - 1) * np2);
        __syncthreads();
        if (lane < 16) {
#pragma unroll
            for (int m = 0; m < MRT; ++m) {
                const int R = w + 4 * m;
                if (R < RT) {
                    const int j = R * 16 + lane;
#pragma unroll
                    for (int c = 0; c < NB; ++c) {
                        C2<T> s = bval(c) ? cell_source<T, MODE>(a, cd, ld, k, j, b0 + c)
                                          : mk<T>((T)0, (T)0);
                        if (k > 0) s = csub(s, cmul(e_coef<T>(ee, k, j, HL), acc[m][c]));
                        vs[j * NB + c] = s;
                        Y[((long long)k * HLp + j) * NB + c] = s;
                    }
                }
            }
        }
        __syncthreads();
    }
    // ---- backward sweep
    for (int k = Wc - 1; k >= 0; --k) {
        if (k < Wc - 1) {
            for (int q = tid; q < HLp * NB; q += CS_THREADS) {
                const int j = q / NB;
                vs[q] = csub(Y[(long long)k * HLp * NB + q], cmul(e_coef<T>(ee, k + 1, j, HL), vs[q]));
            }
            __syncthreads();
        }
        matvec(Xf + (long long)k * np2);
        __syncthreads();
        if (lane < 16) {
#pragma unroll
            for (int m = 0; m < MRT; ++m) {
                const int R = w + 4 * m;
                if (R < RT) {
                    const int j = R * 16 + lane;
#pragma unroll
                    for (int c = 0; c < NB; ++c) {
                        vs[j * NB + c] = acc[m][c];
                        if (bval(c)) cell_emit<T, MODE>(a, cd, ld, k, j, b0 + c, acc[m][c]);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ===========================================================================
// NB in {16, 32}: block products on the matrix cores.  Wave w owns row tiles
// w, w+4, ...; the B operand (column block) is read from LDS, the A operand
// (factor tile) straight from global memory in MFMA order.
template <typename T, int NB, int MODE>
__global__ void __launch_bounds__(CS_THREADS) k_cs_mfma(CellSolveArgs<T> a) {
    constexpr int MRT = (CS_HLPMAX / 16 + 3) / 4;
    constexpr int NCT = NB / 16;
    using acc_t = typename Mf<T>::acc;
    __shared__ C2<T> vs[CS_HLPMAX * NB];

    const int gc = a.cell_list[blockIdx.x];
    const CellDesc cd = a.cells[gc];
    const LayerDesc ld = a.layers[cd.layer];
    const int HL = cd.HL, HLp = cd.HLp, Wc = cd.Wc;
    const int RT = HLp >> 4, KS = HLp >> 2;
    const int b0 = blockIdx.y * NB;
    if (MODE == SOLVE_PROBE && a.probe0 + b0 >= cd.R) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lc = lane & 15, lk = lane >> 4;
    const long long np2 = (long long)HLp * HLp;
    const C2<T>* Xf = a.X + cd.off_X;
    const C2<T>* ee = a.coef_e + cd.off_coef;
    C2<T>* Y = a.Y + ((long long)blockIdx.x * gridDim.y + blockIdx.y) * a.y_stride;
    auto bval = [&](int c) {
        const int b = b0 + c;
        return b < a.B && (MODE != SOLVE_PROBE || a.probe0 + b < cd.R);
    };
    for (int q = tid; q < HLp * NB; q += CS_THREADS) vs[q] = mk<T>((T)0, (T)0);
    __syncthreads();

    acc_t cr[MRT][NCT], ci[MRT][NCT];
    auto matmul = [&](const C2<T>* Xk) {
#pragma unroll
        for (int m = 0; m < MRT; ++m)
#pragma unroll
            for (int t = 0; t < NCT; ++t) { cr[m][t] = mf_zero<T>(); ci[m][t] = mf_zero<T>(); }
#pragma unroll 2
        for (int s = 0; s < KS; ++s) {
            C2<T> bv[NCT];
#pragma unroll
            for (int t = 0; t < NCT; ++t) bv[t] = vs[(4 * s + lk) * NB + t * 16 + lc];
#pragma unroll
            for (int m = 0; m < MRT; ++m) {
                const int R = w + 4 * m;
                if (R < RT) {
                    const C2<T> x = Xk[(((long long)R * KS + s) << 6) + lane];
#pragma unroll
                    for (int t = 0; t < NCT; ++t) cmma<T>(x.x, x.y, bv[t].x, bv[t].y, cr[m][t], ci[m][t]);
                }
            }
        }
    };

    // accumulators -> LDS (each lane its own entries)
    auto store_acc = [&]() {
#pragma unroll
        for (int m = 0; m < MRT; ++m) {
            const int R = w + 4 * m;
            if (R < RT) {
#pragma unroll
                for (int t = 0; t < NCT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int j = R * 16 + Mf<T>::row(lane, v);
                        vs[j * NB + t * 16 + lc] = mk<T>(cr[m][t][v], ci[m][t][v]);
                    }
            }
        }
    };
    const int nq = HLp * NB;

    // ---- forward sweep
    for (int k = 0; k < Wc; ++k) {
        if (k > 0) {
            matmul(Xf + (long long)(k - 1) * np2);
            __syncthreads();
            store_acc();
            __syncthreads();
        }
        // y_k = b_k - e_k o t, thread-strided over (row, column) with the
        // batch column fastest (coalesced sources and scratch)
        for (int q = tid; q < nq; q += CS_THREADS) {
            const int j = q / NB, c = q - j * NB;
            C2<T> yv = bval(c) ? cell_source<T, MODE>(a, cd, ld, k, j, b0 + c) : mk<T>((T)0, (T)0);
            if (k > 0) yv = csub(yv, cmul(e_coef<T>(ee, k, j, HL), vs[q]));
            vs[q] = yv;
            Y[(long long)k * nq + q] = yv;
        }
        __syncthreads();
    }
    // ---- backward sweep
    for (int k = Wc - 1; k >= 0; --k) {
        if (k < Wc - 1) {
            for (int q = tid; q < nq; q += CS_THREADS) {
                const int j = q / NB;
                vs[q] = csub(Y[(long long)k * nq + q], cmul(e_coef<T>(ee, k + 1, j, HL), vs[q]));
            }
            __syncthreads();
        }
        matmul(Xf + (long long)k * np2);
        __syncthreads();
        store_acc();
        __syncthreads();
        for (int q = tid; q < nq; q += CS_THREADS) {
            const int j = q / NB, c = q - j * NB;
            if (bval(c)) cell_emit<T, MODE>(a, cd, ld, k, j, b0 + c, vs[q]);
        }
    }
}

template <typename T, int MODE>
void launch_mode(const CellSolveArgs<T>& a, int ncells, hipStream_t st) {
    const int nb = a.nb > 0 ? a.nb : cs_nb(a.B);
    const int chunks = (a.B + nb - 1) / nb;
    dim3 grid(ncells, chunks), blk(CS_THREADS);
    switch (nb) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cs_gemv<T, 1, MODE>), grid, blk, 0, st, a); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cs_gemv<T, 2, MODE>), grid, blk, 0, st, a); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cs_gemv<T, 4, MODE>), grid, blk, 0, st, a); break;
    case 16: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cs_mfma<T, 16, MODE>), grid, blk, 0, st, a); break;
    default: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cs_mfma<T, 32, MODE>), grid, blk, 0, st, a); break;
    }
}

template <typename T>
void launch_cell_solve(const CellSolveArgs<T>& a, int ncells_launch, int nb_chunks,
                       hipStream_t st) {
    (void)nb_chunks;
    switch (a.mode) {
    case SOLVE_GRID: launch_mode<T, SOLVE_GRID>(a, ncells_launch, st); break;
    case SOLVE_PROBE: launch_mode<T, SOLVE_PROBE>(a, ncells_launch, st); break;
    case SOLVE_SAMPLE: launch_mode<T, SOLVE_SAMPLE>(a, ncells_launch, st); break;
    default: launch_mode<T, SOLVE_VOLUME>(a, ncells_launch, st); break;
    }
}

template void launch_cell_solve<double>(const CellSolveArgs<double>&, int, int, hipStream_t);
template void launch_cell_solve<float>(const CellSolveArgs<float>&, int, int, hipStream_t);

}  // namespace hz
