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

constexpr int CS_THREADS = 1024;    // single-RHS cell solve (16 waves)
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
                if (j == p) v = cfma(s, gload<T>(top + (0 * W + col) * B + b), v);
                else v = csub(v, cmul(s, gload<T>(top + (1 * W + col) * B + b)));
            }
            if (bot && (j == p + ld.nl - 1 || j == p + ld.nl)) {
                double2 ix = cinv(a.alpha_x[(long long)cd.gidx * a.Wcmax + k]);
                C2<T> s = to_t<T>(mk<double>(ix.x * ih2, ix.y * ih2));
                if (j == p + ld.nl - 1) v = cfma(s, gload<T>(bot + (1 * W + col) * B + b), v);
                else v = csub(v, cmul(s, gload<T>(bot + (0 * W + col) * B + b)));
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
                    if (k == p) v = cfma(s, gload<T>(iv + (((long long)jf * 2 + 0) * HL + j) * B + b), v);
                    else v = csub(v, cmul(s, gload<T>(iv + (((long long)jf * 2 + 1) * HL + j) * B + b)));
                }
                if (kr) {
                    const int jf = cd.cell;
                    if (k == p + cd.nc) v = csub(v, cmul(s, gload<T>(iv + (((long long)jf * 2 + 0) * HL + j) * B + b)));
                    else v = cfma(s, gload<T>(iv + (((long long)jf * 2 + 1) * HL + j) * B + b), v);
                }
            }
        }
    }
    return v;
}

// Per-workgroup constants of the source assembly, fetched once: whether the
// volume source is read in this layer, the interface pair and inner-trace
// pointers, and (in LDS) the scaled PML factors 1/(alpha_z h^2) per row and
// 1/(alpha_x h^2) per column of the cell.
template <typename T>
struct SrcCtx {
    bool act;
    const C2<T>* top;
    const C2<T>* bot;
    const C2<T>* iv;
    const double2* izs;     // [HLp] (LDS)
    const double2* ixs;     // [Wc]  (LDS)
};

template <typename T, int MODE>
__device__ inline C2<T> cell_source_ctx(const CellSolveArgs<T>& a, const CellDesc& cd,
                                        const LayerDesc& ld, const SrcCtx<T>& sc, int k, int j,
                                        int b) {
    const int p = a.p;
    const C2<T> z = mk<T>((T)0, (T)0);
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
            const double2 iz = sc.izs[j];
            return mk<T>((T)(sg * iz.x), (T)(sg * iz.y));
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
            const double2 ix = sc.ixs[k];
            return mk<T>((T)(sg * ix.x), (T)(sg * ix.y));
        }
    }
    // SOLVE_SAMPLE / SOLVE_VOLUME
    C2<T> v = z;
    const long long W = a.W;
    const bool own_row = (j >= ld.own_r0 && j <= ld.own_r1);
    if (sc.act && own_col && own_row)
        v = a.f_ext[(((long long)(ld.row0 + j)) * W + cd.col0 + k) * B + b];
    if constexpr (MODE == SOLVE_VOLUME) {
        if (own_col) {
            const long long col = cd.col0 + k;
            if (sc.top && (j == p || j == p - 1)) {
                const C2<T> s = to_t<T>(sc.ixs[k]);
                if (j == p) v = cfma(s, gload<T>(sc.top + (0 * W + col) * B + b), v);
                else v = csub(v, cmul(s, gload<T>(sc.top + (1 * W + col) * B + b)));
            }
            if (sc.bot && (j == p + ld.nl - 1 || j == p + ld.nl)) {
                const C2<T> s = to_t<T>(sc.ixs[k]);
                if (j == p + ld.nl - 1) v = cfma(s, gload<T>(sc.bot + (1 * W + col) * B + b), v);
                else v = csub(v, cmul(s, gload<T>(sc.bot + (0 * W + col) * B + b)));
            }
        }
        if (sc.iv) {
            const int HL = cd.HL;
            const bool kl = cd.has_left && (k == p || k == p - 1);
            const bool kr = cd.has_right && (k == p + cd.nc || k == p + cd.nc - 1);
            if (kl || kr) {
                const C2<T> s = to_t<T>(sc.izs[j]);
                if (kl) {
                    const int jf = cd.cell - 1;
                    if (k == p) v = cfma(s, gload<T>(sc.iv + (((long long)jf * 2 + 0) * HL + j) * B + b), v);
                    else v = csub(v, cmul(s, gload<T>(sc.iv + (((long long)jf * 2 + 1) * HL + j) * B + b)));
                }
                if (kr) {
                    const int jf = cd.cell;
                    if (k == p + cd.nc) v = csub(v, cmul(s, gload<T>(sc.iv + (((long long)jf * 2 + 0) * HL + j) * B + b)));
                    else v = cfma(s, gload<T>(sc.iv + (((long long)jf * 2 + 1) * HL + j) * B + b), v);
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
        if (a.CPpool) {
            C2<T>* CP = a.CPpool + cd.off_CP;
            const int HL = cd.HL;
            if (cd.has_left && (k == p - 1 || k == p))
                CP[((long long)(k - p + 1) * HL + j) * cd.R + probe] = x;
            if (cd.has_right && (k == p + cd.nc - 1 || k == p + cd.nc))
                CP[((long long)((cd.has_left ? 2 : 0) + k - (p + cd.nc - 1)) * HL + j) * cd.R +
                   probe] = x;
        }
        if (own_col) {
            for (int si = 0; si < ld.nslot; ++si)
                if (ld.slot_row[si] == j)
                    Q[((long long)si * cd.s + (k - cd.own_c0)) * cd.R + probe] = x;
        }
    } else if constexpr (MODE == SOLVE_SAMPLE) {
        const int HL = cd.HL;
        if (a.inner_pol) {
            // left pair (positions 0, 1) -> q of interface cell-1, right pair
            // (n_c, n_c + 1) -> d of interface cell
            C2<T>* ir = a.inner_rhs + 2 * ld.off_inner * B;
            const int J = ld.J;
            if (cd.has_left && (k == p - 1 || k == p))
                ir[((((long long)J + cd.cell - 1) * 2 + (k - p + 1)) * HL + j) * B + b] = x;
            if (cd.has_right && (k == p + cd.nc - 1 || k == p + cd.nc))
                ir[((((long long)cd.cell) * 2 + (k - (p + cd.nc - 1))) * HL + j) * B + b] = x;
        } else {
            C2<T>* ir = a.inner_rhs + ld.off_inner * B;
            if (cd.has_left && k == p)
                ir[(((long long)(cd.cell - 1) * 2 + 1) * HL + j) * B + b] = x;
            if (cd.has_right && k == p + cd.nc - 1)
                ir[(((long long)cd.cell * 2 + 0) * HL + j) * B + b] = x;
        }
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

// First column of a cell that holds a source or an output: the left pair of
// the inner interface (p - 1, p) or the first own column.  The columns left
// of it (the overlap into the left neighbour's PML) carry neither, so the
// forward sweep starts there (its iterates are zero before) and the backward
// sweep stops there (nothing left of it is read).  Grid solves use them all.
template <int MODE>
__device__ inline int first_live_col(const CellDesc& cd, int p) {
    if (MODE == SOLVE_GRID) return 0;
    int k = cd.own_c0;
    if (cd.has_left && p - 1 < k) k = p - 1;
    return k < 0 ? 0 : k;
}

// ===========================================================================
// NB <= 4: lanes run along the tile's 4 columns, each lane owning one row of
// a 16-row tile; the 4 partial sums of a row are combined with two shuffles.
#ifndef CS_GV_UL4
#define CS_GV_UL4 4
#endif
#ifndef CS_GV_UL1
#define CS_GV_UL1 10
#endif
template <typename T, int NB, int MODE>
__global__ void __launch_bounds__(CS_THREADS) k_cs_gemv(CellSolveArgs<T> a) {
    // A step's matrix-vector product reads a whole HLp x HLp factor block
    // and one workgroup serves a cell, so the step time is the time to have
    // the block in flight: 16 waves, each taking one row tile over 1/NS of
    // the column quads (NS = 2 for HLp > 64), with all of its loads issued
    // before the products.  Partial row sums meet in LDS.
    constexpr int NSMAX = 4;
    constexpr int WAVES = CS_THREADS / 64;
    __shared__ C2<T> vs[CS_HLPMAX * NB];
    __shared__ C2<T> part[2 * CS_HLPMAX * NB];     // NS * HLp <= 2 * CS_HLPMAX

    const int gc = a.cell_list[blockIdx.x];
    const CellDesc cd = a.cells[gc];
    const LayerDesc& ld = a.layers[cd.layer];
    const int HL = cd.HL, HLp = cd.HLp, Wc = cd.Wc;
    const int RT = HLp >> 4, KS = HLp >> 2;
    const int NS = RT >= WAVES / 2 ? 2 : (RT >= WAVES / 4 ? 4 : NSMAX);
    const int KSP = (KS + NS - 1) / NS;             // column quads per item
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

    // part[h][row][c] = sum over quad range h of X_k[row][.] vs[.][c]
    auto matvec = [&](const C2<T>* Xk) {
        for (int item = w; item < RT * NS; item += WAVES) {
            const int R = item % RT, h = item / RT;
            const int s0 = h * KSP, s1 = min(KS, s0 + KSP);
            C2<T> acc[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) acc[c] = mk<T>((T)0, (T)0);
            const C2<T>* base = Xk + ((long long)R * KS << 6) + lane;
            // loads in flight per lane; a last partial group re-reads its
            // final quad for the missing ones (same cache line) and zeroes
            // them, so it is issued as one group too (no branch between the
            // loads and their products)
            constexpr int UL = NB >= 4 ? CS_GV_UL4 : CS_GV_UL1;
            for (int s = s0; s < s1; s += UL) {
                C2<T> x[UL];
#pragma unroll
                for (int u = 0; u < UL; ++u)
                    x[u] = gload<T>(base + ((long long)min(s + u, s1 - 1) << 6));
#pragma unroll
                for (int u = 0; u < UL; ++u) {
                    const bool live = s + u < s1;
                    const int cc = 4 * min(s + u, s1 - 1) + (lane >> 4);
                    const C2<T> xv = mk<T>(live ? x[u].x : (T)0, live ? x[u].y : (T)0);
#pragma unroll
                    for (int c = 0; c < NB; ++c) acc[c] = cfma(xv, vs[cc * NB + c], acc[c]);
                }
            }
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                C2<T> v = acc[c];
                v.x += __shfl_xor(v.x, 16, 64); v.y += __shfl_xor(v.y, 16, 64);
                v.x += __shfl_xor(v.x, 32, 64); v.y += __shfl_xor(v.y, 32, 64);
                if (lane < 16) part[(h * HLp + R * 16 + lane) * NB + c] = v;
            }
        }
    };
    auto rowsum = [&](int j, int c) {
        C2<T> v = part[j * NB + c];
        for (int h = 1; h < NS; ++h) v = cadd(v, part[(h * HLp + j) * NB + c]);
        return v;
    };

    // thread tid owns entry q = tid of the column block (HLp NB <= 896 <
    // 1024 entries); the loads of a step that do not depend on its product
    // (the sources and e_k in the forward sweep, the stored iterate and
    // e_{k+1} in the backward sweep) are issued before the product and are
    // in flight during it
    static_assert(CS_HLPMAX * 4 <= CS_THREADS, "one column-block entry per thread");
    const int q = tid, qj = q / NB, qc = q % NB;
    const bool mine = q < HLp * NB;
    const C2<T> zero = mk<T>((T)0, (T)0);
    const int k0 = first_live_col<MODE>(cd, a.p);
    // SOLVE_SAMPLE with one or two columns (the volume source of a layer,
    // point sources): the iterates are zero before the first column that
    // holds a source of this workgroup's columns, so the forward sweep
    // starts there (Wc: none); the backward sweep still runs down to k0.
    // (Wider batches are set by their chunk whose first source lies near
    // the first column; for them the scan would only cost time.)
    int kf = k0;
    if constexpr (MODE == SOLVE_SAMPLE && NB <= 2) {
        __shared__ int kfirst;
        if (tid == 0) kfirst = Wc;
        __syncthreads();
        const int ncols = Wc - k0;
        int km = Wc;
        for (long long e = tid; e < (long long)HL * ncols * NB; e += CS_THREADS) {
            const int c = (int)(e % NB);
            const long long r = e / NB;
            const int k = k0 + (int)(r % ncols), j = (int)(r / ncols);
            if (k < km && bval(c)) {
                const C2<T> v = cell_source<T, MODE>(a, cd, ld, k, j, b0 + c);
                if (v.x != (T)0 || v.y != (T)0) km = k;
            }
        }
        atomicMin(&kfirst, km);
        __syncthreads();
        kf = kfirst;
    }
    // ---- forward sweep
    for (int k = kf; k < Wc; ++k) {
        C2<T> src = zero, ek = zero;
        if (mine) {
            if (bval(qc)) src = cell_source<T, MODE>(a, cd, ld, k, qj, b0 + qc);
            if (k > kf) ek = e_coef<T>(ee, k, qj, HL);
        }
        if (k > kf) matvec(Xf + (long long)(k - 1) * np2);
        __syncthreads();
        if (mine) {
            C2<T> s = src;
            if (k > kf) s = csub(s, cmul(ek, rowsum(qj, qc)));
            vs[q] = s;
            Y[(long long)k * HLp * NB + q] = s;
        }
        __syncthreads();
    }
    // ---- backward sweep
    C2<T> ynext = zero, enext = zero;      // Y_k and e_{k+1} of the next step down
    for (int k = Wc - 1; k >= k0; --k) {
        if (k < Wc - 1) {
            if (mine) vs[q] = csub(ynext, cmul(enext, vs[q]));
            __syncthreads();
        }
        if (mine && k > k0) {
            ynext = k - 1 >= kf ? Y[(long long)(k - 1) * HLp * NB + q] : zero;
            enext = e_coef<T>(ee, k, qj, HL);
        }
        matvec(Xf + (long long)k * np2);
        __syncthreads();
        if (mine) {
            const C2<T> x = rowsum(qj, qc);
            vs[q] = x;
            if (bval(qc)) cell_emit<T, MODE>(a, cd, ld, k, qj, b0 + qc, x);
        }
        __syncthreads();
    }
}

// ===========================================================================
// NB in {16, 32}: block products on the matrix cores, NW waves per workgroup
// (8; 12 for cells of 129-160 rows, see below).  Wave w owns the 16-row
// tiles w and w + NW (MC of them, a
// per-wave constant chosen once by a wave-uniform switch).  The A operand (factor tile) streams
// from global memory in MFMA order with a two-group register double buffer;
// the B operand (current column block) is read from LDS.  The elementwise
// updates y = b - e o t run on the accumulators in registers: each lane keeps
// its own entries, so the forward iterates go to a lane-private, coalesced
// scratch and the sources and scratch reads of the next step are issued
// before the block product that they wait for.
constexpr int CS_MF_WAVES = 8;        // waves of the default instance
#ifndef CS_U1
#define CS_U1 4
#endif
#ifndef CS_U10
#define CS_U10 4
#endif
#ifndef CS_U2
#define CS_U2 2
#endif

// Grid column of the point source of probe `probe` (the columns used by the
// SOLVE_PROBE branch of cell_source).
__device__ inline int probe_col(const CellDesc& cd, int p, int probe) {
    if (probe < cd.ncol) {
        int q = probe, right = 0;
        if (!cd.has_left) right = 1;
        else if (q >= 2 * cd.HL) { right = 1; q -= 2 * cd.HL; }
        const int ab = q / cd.HL;
        return right ? (ab == 0 ? p + cd.nc : p + cd.nc - 1) : (ab == 0 ? p : p - 1);
    }
    return cd.own_c0 + (probe - cd.ncol) % cd.s;
}

// Add (re, im) to entry v of a complex accumulator (Gauss's three-product
// form: re = P1 - P2 and im = P3 - P1 - P2, so P1 += re and P3 += re + im).
template <typename T>
__device__ inline void acc_add(CAcc<T, true>& a, int v, T re, T im) {
    a.p1[v] += re;
    a.p3[v] += re + im;
}
template <typename T>
__device__ inline void acc_add(CAcc<T, false>& a, int v, T re, T im) {
    a.r[v] += re;
    a.i[v] += im;
}

// NW = 12 (cells of 129-160 rows, up to ten row tiles): waves 0-7 own row
// tiles 0-7; waves 8 + 2i and 9 + 2i share row tile 8 + i, each taking one
// part of the k steps of its block products.  The second leaves its partial
// sums in LDS (pbuf), the first adds them after the step's barrier and does
// the tile's updates.  Three waves per SIMD then carry equal matrix-core
// work; with ten waves two SIMDs held three of them and two held two.
template <typename T, int NB, int MODE, int MC, int NW>
__device__ __forceinline__ void cs_mfma_body(const CellSolveArgs<T>& a, const CellDesc& cd,
                                             const LayerDesc& ld, C2<T>* vs, double2* izs,
                                             double2* ixs, C2<T>* pbuf, int b0, long long slot) {
    constexpr int NCT = NB / 16;
    constexpr int MCA = MC > 0 ? MC : 1;
    constexpr bool SPLIT = NW == 12;
    // k steps per register group.  Ten waves run at three waves per SIMD,
    // 170 registers per lane: four k steps (4 KB of factor in flight per
    // wave) fit except for the FP64 volume solve and the 32-column FP32
    // probes, which keep two (with four they spill)
    constexpr bool U10_SMALL = (sizeof(T) == 8 && MODE == SOLVE_VOLUME) ||
                               (sizeof(T) == 4 && NB == 32 && MODE == SOLVE_PROBE);
    constexpr int U = NW > CS_MF_WAVES ? (U10_SMALL ? 2 : CS_U10)
                                       : (MC > 1 ? CS_U2 : CS_U1);
    const int HL = cd.HL, HLp = cd.HLp, Wc = cd.Wc;
    const int KS = HLp >> 2;                  // multiple of 4
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int lc = lane & 15, lk = lane >> 4;
    // first row tile of the wave, and its part of a shared tile (-1: whole)
    const int tw = SPLIT && w >= 8 ? 8 + ((w - 8) >> 1) : w;
    const int part = SPLIT && w >= 8 ? ((w - 8) & 1) : -1;
    const bool owner = part <= 0;             // does the tile's updates
    const int kmid = ((KS / 2) / U) * U;      // split point of a shared tile's k steps
    const int ks0 = part == 1 ? kmid : 0, ks1 = part == 0 ? kmid : KS;
    const long long np2 = (long long)HLp * HLp;
    const long long nq = (long long)HLp * NB;
    const C2<T>* __restrict__ Xf = a.X + cd.off_X;
    const C2<T>* __restrict__ ee = a.coef_e + cd.off_coef;
    C2<T>* __restrict__ Y = a.Y + slot * a.y_stride;
    const C2<T> z = mk<T>((T)0, (T)0);

    auto row_of = [&](int m, int v) { return (tw + NW * m) * 16 + Mf<T>::row(lane, v); };
    auto yidx = [&](int m, int t, int v) {
        return ((long long)((tw + NW * m) * NCT + t) * 4 + v) * 64 + lane;
    };
    auto bval = [&](int c) {
        const int b = b0 + c;
        return b < a.B && (MODE != SOLVE_PROBE || a.probe0 + b < cd.R);
    };

    CAcc<T, HZ_GAUSS3 != 0> ac[MCA][NCT];
    auto matmul = [&](const C2<T>* __restrict__ Xk) {
#pragma unroll
        for (int m = 0; m < MCA; ++m)
#pragma unroll
            for (int t = 0; t < NCT; ++t) ac[m][t].zero();
        if constexpr (MC > 0) {
            const C2<T>* xp[MC];
#pragma unroll
            for (int m = 0; m < MC; ++m)
                xp[m] = Xk + (((long long)(tw + NW * m) * KS) << 6) + lane;
            C2<T> xa[U][MC], xb[U][MC];
            auto load = [&](C2<T> (&dst)[U][MC], int s0) {
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int m = 0; m < MC; ++m) dst[u][m] = xp[m][(long long)(s0 + u) << 6];
            };
            auto mult = [&](const C2<T> (&src)[U][MC], int s0) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    C2<T> bv[NCT];
#pragma unroll
                    for (int t = 0; t < NCT; ++t) bv[t] = vs[(4 * (s0 + u) + lk) * NB + t * 16 + lc];
#pragma unroll
                    for (int m = 0; m < MC; ++m)
#pragma unroll
                        for (int t = 0; t < NCT; ++t)
                            ac[m][t].add(src[u][m].x, src[u][m].y, bv[t].x, bv[t].y);
                }
            };
            load(xa, ks0);
            for (int s = ks0; s < ks1; s += 2 * U) {
                if (s + U < ks1) load(xb, s + U);
                mult(xa, s);
                if (s + U >= ks1) break;
                if (s + 2 * U < ks1) load(xa, s + 2 * U);
                mult(xb, s + U);
            }
        }
    };
    // a shared tile's partial sums: the second part stores them, the first
    // adds them to its accumulators (after a barrier)
    auto tval = [&](int m, int t, int v) { return mk<T>(ac[m][t].re(v), ac[m][t].im(v)); };
    auto pidx = [&](int t, int v) { return (((tw - 8) * NCT + t) * 4 + v) * 64 + lane; };
    auto put_part = [&]() {
        if constexpr (SPLIT && MC > 0) {
#pragma unroll
            for (int t = 0; t < NCT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) pbuf[pidx(t, v)] = tval(0, t, v);
        }
    };
    auto add_part = [&]() {
        if constexpr (SPLIT && MC > 0) {
#pragma unroll
            for (int t = 0; t < NCT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const C2<T> q = pbuf[pidx(t, v)];
                    acc_add(ac[0][t], v, q.x, q.y);
                }
        }
    };

    // per-workgroup source constants
    {
        const double ih2 = 1.0 / (a.h * a.h);
        for (int j = threadIdx.x; j < HLp; j += NW * 64) {
            double2 v = make_double2(0.0, 0.0);
            if (j < HL) {
                const double2 iz = cinv(a.alpha_z[(long long)cd.layer * a.HLmax + j]);
                v = make_double2(iz.x * ih2, iz.y * ih2);
            }
            izs[j] = v;
        }
        for (int k = threadIdx.x; k < Wc; k += NW * 64) {
            const double2 ix = cinv(a.alpha_x[(long long)cd.gidx * a.Wcmax + k]);
            ixs[k] = make_double2(ix.x * ih2, ix.y * ih2);
        }
    }
    SrcCtx<T> sc;
    sc.act = a.f_ext && (!a.layer_active || a.layer_active[cd.layer]);
    sc.top = (MODE == SOLVE_VOLUME && a.top_pair) ? a.top_pair[cd.layer] : nullptr;
    sc.bot = (MODE == SOLVE_VOLUME && a.bot_pair) ? a.bot_pair[cd.layer] : nullptr;
    sc.iv = (MODE == SOLVE_VOLUME && a.inner_v && ld.J > 0) ? a.inner_v + ld.off_inner * a.B
                                                             : nullptr;
    sc.izs = izs;
    sc.ixs = ixs;
    __syncthreads();

    C2<T> pv[MCA][NCT][4];   // prefetched sources (forward) / iterates (backward)
    C2<T> pe[MCA][4];        // prefetched coupling coefficients

    // The forward sweep starts at the first live column (above); a probe
    // batch's sources are point sources, so for it y_k = 0 before the first
    // column kmin that holds one, and the sweep starts there.
    const int kstop = first_live_col<MODE>(cd, a.p);
    int kmin = kstop;
    if constexpr (MODE == SOLVE_PROBE) {
        int c = Wc;
        if (lane < NB && bval(lane)) c = probe_col(cd, a.p, a.probe0 + b0 + lane);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) c = min(c, __shfl_xor(c, off));
        kmin = __builtin_amdgcn_readfirstlane(c);
    }

    // ---- forward sweep: y_0 = b_0, y_k = b_k - e_k o (X_{k-1} y_{k-1})
    auto fwd_update = [&](int k) {
#pragma unroll
        for (int m = 0; m < MC; ++m)
#pragma unroll
            for (int t = 0; t < NCT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    C2<T> y = pv[m][t][v];
                    if (k > kmin) y = csub(y, cmul(pe[m][v], tval(m, t, v)));
                    pv[m][t][v] = y;
                    Y[(long long)k * nq + yidx(m, t, v)] = y;
                }
    };
    for (int k = kmin; k < Wc; ++k) {
        if (owner) {
#pragma unroll
            for (int m = 0; m < MC; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = row_of(m, v);
                    pe[m][v] = k > kmin ? e_coef<T>(ee, k, j, HL) : z;
#pragma unroll
                    for (int t = 0; t < NCT; ++t) {
                        const int c = t * 16 + lc;
                        pv[m][t][v] = bval(c) ? cell_source_ctx<T, MODE>(a, cd, ld, sc, k, j, b0 + c) : z;
                    }
                }
        }
        if (k > kmin) {
            matmul(Xf + (long long)(k - 1) * np2);
            if (part == 1) put_part();
        }
        if (part < 0) fwd_update(k);
        __syncthreads();                      // all block products of this step done
        if (part == 0) {
            if (k > kmin) add_part();
            fwd_update(k);
        }
        if (owner) {
#pragma unroll
            for (int m = 0; m < MC; ++m)
#pragma unroll
                for (int t = 0; t < NCT; ++t)
#pragma unroll
                    for (int v = 0; v < 4; ++v) vs[row_of(m, v) * NB + t * 16 + lc] = pv[m][t][v];
        }
        __syncthreads();
    }
    // ---- backward sweep: x_{W-1} = X_{W-1} y_{W-1}, x_k = X_k (y_k - e_{k+1} o x_{k+1}),
    // down to the first live column
    auto bwd_update = [&](int k) {
#pragma unroll
        for (int m = 0; m < MC; ++m)
#pragma unroll
            for (int t = 0; t < NCT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int c = t * 16 + lc;
                    const C2<T> x = tval(m, t, v);
                    if (bval(c)) cell_emit<T, MODE>(a, cd, ld, k, row_of(m, v), b0 + c, x);
                    pv[m][t][v] = csub(pv[m][t][v], cmul(pe[m][v], x));
                }
    };
    for (int k = Wc - 1; k >= kstop; --k) {
        if (k > kstop && owner) {
#pragma unroll
            for (int m = 0; m < MC; ++m)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    pe[m][v] = e_coef<T>(ee, k, row_of(m, v), HL);
#pragma unroll
                    for (int t = 0; t < NCT; ++t)
                        pv[m][t][v] = k - 1 >= kmin ? Y[(long long)(k - 1) * nq + yidx(m, t, v)] : z;
                }
        }
        matmul(Xf + (long long)k * np2);
        if (part == 1) put_part();
        if (part < 0) bwd_update(k);
        // the shared tiles' partial sums cross between waves at every step
        if (SPLIT || k > kstop) __syncthreads();
        if (part == 0) {
            add_part();
            bwd_update(k);
        }
        if (k > kstop) {
            if (owner) {
#pragma unroll
                for (int m = 0; m < MC; ++m)
#pragma unroll
                    for (int t = 0; t < NCT; ++t)
#pragma unroll
                        for (int v = 0; v < 4; ++v) vs[row_of(m, v) * NB + t * 16 + lc] = pv[m][t][v];
            }
            __syncthreads();
        }
    }
}

// MCMAX = 1 serves cells of up to NW row tiles with fewer registers;
// MCMAX = 2 serves up to 2 NW.
template <typename T, int NB, int MODE, int MCMAX, int NW>
__global__ void __launch_bounds__(NW * 64) k_cs_mfma(CellSolveArgs<T> a) {
    extern __shared__ __align__(16) unsigned char cs_lds[];
    C2<T>* vs = reinterpret_cast<C2<T>*>(cs_lds);
    const int hlp_max = (a.HLmax + 15) / 16 * 16;
    double2* izs = reinterpret_cast<double2*>(cs_lds + (size_t)hlp_max * NB * sizeof(C2<T>));
    double2* ixs = izs + hlp_max;
    C2<T>* pbuf = reinterpret_cast<C2<T>*>(ixs + a.Wcmax);     // NW = 12: shared-tile partials
    // 1-D grid over (cell, batch chunk), chunks fastest, in XCD-contiguous
    // order: the chunks of a cell stream the same factor blocks through one
    // XCD's L2 at about the same time
    const int chunks = (a.B + NB - 1) / NB;
    const int item = xcd_tile(blockIdx.x, (int)gridDim.x);
    const int ci = item / chunks, ch = item - ci * chunks;
    const int gc = a.cell_list[ci];
    const CellDesc cd = a.cells[gc];
    const LayerDesc& ld = a.layers[cd.layer];
    const int b0 = ch * NB;
    if (MODE == SOLVE_PROBE && a.probe0 + b0 >= cd.R) return;   // whole workgroup
    const long long slot = (long long)ci * chunks + ch;
    const int RT = cd.HLp >> 4;
    const int w = threadIdx.x >> 6;
    // tiles w and w + NW (HLp <= 224 gives at most 14 tiles); NW = 12: the
    // wave's tile of at most ten
    const int tw = NW == 12 && w >= 8 ? 8 + ((w - 8) >> 1) : w;
    const int mc = NW == 12 ? (tw < RT ? 1 : 0) : (RT > w ? (RT - w + NW - 1) / NW : 0);
    // every branch passes the same sequence of barriers
    if (mc == 0) cs_mfma_body<T, NB, MODE, 0, NW>(a, cd, ld, vs, izs, ixs, pbuf, b0, slot);
    else if (MCMAX == 1 || mc == 1) cs_mfma_body<T, NB, MODE, 1, NW>(a, cd, ld, vs, izs, ixs, pbuf, b0, slot);
    else cs_mfma_body<T, NB, MODE, MCMAX, NW>(a, cd, ld, vs, izs, ixs, pbuf, b0, slot);
}

template <typename T, int NB, int MODE, int MCMAX, int NW>
void launch_cs_mfma_mc(const CellSolveArgs<T>& a, dim3 grid, size_t lds, hipStream_t st) {
    static bool attr = false;
    if (!attr) {
        // if the device refuses, a launch needing more LDS fails and is reported
        if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cs_mfma<T, NB, MODE, MCMAX, NW>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
            (void)hipGetLastError();
        attr = true;
    }
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cs_mfma<T, NB, MODE, MCMAX, NW>), grid, dim3(NW * 64),
                       lds, st, a);
}

template <typename T, int NB, int MODE>
void launch_cs_mfma(const CellSolveArgs<T>& a, dim3 grid, hipStream_t st) {
    const int hlp = (a.HLmax + 15) / 16 * 16;     // largest HLp of any cell
    // column block, then the row and column PML scalings
    const size_t lds = (size_t)hlp * NB * sizeof(C2<T>) + (size_t)(hlp + a.Wcmax) * sizeof(double2);
    if (hlp <= 16 * CS_MF_WAVES) launch_cs_mfma_mc<T, NB, MODE, 1, CS_MF_WAVES>(a, grid, lds, st);
    else if (hlp <= 160)        // plus the partial sums of the two shared tiles
        launch_cs_mfma_mc<T, NB, MODE, 1, 12>(a, grid, lds + 2 * (NB / 16) * 4 * 64 * sizeof(C2<T>), st);
    else launch_cs_mfma_mc<T, NB, MODE, 2, CS_MF_WAVES>(a, grid, lds, st);
}

template <typename T, int MODE>
void launch_mode(const CellSolveArgs<T>& a, int ncells, hipStream_t st) {
    const int nb = a.nb > 0 ? a.nb : cs_nb_cap(a.B);
    const int chunks = (a.B + nb - 1) / nb;
    dim3 grid(ncells, chunks), blk(CS_THREADS);
    const dim3 grid1((unsigned)(ncells * chunks));      // matrix-core kernels: 1-D
    switch (nb) {
    case 1: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cs_gemv<T, 1, MODE>), grid, blk, 0, st, a); break;
    case 2: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cs_gemv<T, 2, MODE>), grid, blk, 0, st, a); break;
    case 4: hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cs_gemv<T, 4, MODE>), grid, blk, 0, st, a); break;
    case 16: launch_cs_mfma<T, 16, MODE>(a, grid1, st); break;
    default: launch_cs_mfma<T, 32, MODE>(a, grid1, st); break;
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
