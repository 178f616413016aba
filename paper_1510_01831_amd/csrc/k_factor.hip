// Offline factorisations (Sec. 4.3.1, Table 2: "LU factorizations").
//
// * Every cell operator H^{l,c} is block tridiagonal along x with one block
//   per grid column (HL x HL, itself tridiagonal in depth) and diagonal
//   couplings between neighbouring columns.  Eliminating the columns left to
//   right gives the Schur complements
//       S_0 = A_0,   S_k = A_k - diag(e_k) S_{k-1}^{-1} diag(e_k),
//   whose inverses X_k = S_k^{-1} are stored (the cell's block LDU factors).
// * The inner SIE of each layer is block tridiagonal with blocks of 2 HL; its
//   block LU without pivoting (Sec. 4.2.2) needs the inverses of its diagonal
//   blocks.
// Both use the same in-place Gauss-Jordan inversion with partial pivoting by
// rows that are never physically swapped: at step k the pivot row r_k is the
// unused row with the largest |S[r][k]|; at the end the array holds
// X[k][r_j] at position [r_k][j].
#include "hz_common.h"

namespace hz {

constexpr int GJ_THREADS = 512;
constexpr int GJ_NMAX = 448;    // largest matrix order handled (2 HL <= 448)

#ifndef HZ_GJ_REG
#define HZ_GJ_REG 1             // register-resident cell recursion for HL <= 128
#endif

template <typename T>
__device__ inline T cabs2(C2<T> a) { return a.x * a.x + a.y * a.y; }

// Maximum over the 64 lanes of a wave, returned to every lane: DPP steps
// within each row of 16 lanes, row broadcasts across rows, then lane 63.
template <int CTRL, int ROWMASK>
__device__ inline double dpp_max_step(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWMASK, 0xF, false);
    const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWMASK, 0xF, false);
    return fmax(v, __hiloint2double(hi2, lo2));
}
template <int CTRL, int ROWMASK>
__device__ inline float dpp_max_step(float v) {
    const int b = __float_as_int(v);
    return fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(b, b, CTRL, ROWMASK, 0xF, false)));
}
template <typename T>
__device__ inline T wave_max(T v) {
    v = dpp_max_step<0xB1, 0xF>(v);     // quad_perm [1,0,3,2]
    v = dpp_max_step<0x4E, 0xF>(v);     // quad_perm [2,3,0,1]
    v = dpp_max_step<0x124, 0xF>(v);    // row_ror:4
    v = dpp_max_step<0x128, 0xF>(v);    // row_ror:8
    v = dpp_max_step<0x142, 0xA>(v);    // row_bcast:15 into rows 1 and 3
    v = dpp_max_step<0x143, 0xC>(v);    // row_bcast:31 into rows 2 and 3
    if constexpr (sizeof(T) == 8) {
        const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
        const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
        return __hiloint2double(hi, lo);
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
    }
}

// Pivot statistics of one block inversion (wave-uniform values): exact zero
// pivots are flagged at once; at the end, the ratio of the smallest to the
// largest pivot magnitude is compared with PIVOT_RATIO_MIN and folded into
// the launch's minimum.
template <typename T>
struct PivotStats {
    T pmax2 = (T)0, pmin2 = (T)-1;
    __device__ void add(T best2) {
        pmax2 = fmax(pmax2, best2);
        pmin2 = pmin2 < (T)0 ? best2 : fmin(pmin2, best2);
    }
    __device__ void finish(FactorFlags* ff) const {
        if (threadIdx.x != 0) return;
        double ratio = 0.0;
        if (pmax2 > (T)0 && pmin2 > (T)0) ratio = sqrt((double)pmin2 / (double)pmax2);
        if (!(ratio > PIVOT_RATIO_MIN)) atomicOr(&ff->singular, 1);
        atomicMin(&ff->min_ratio_bits, (unsigned long long)__double_as_longlong(ratio));
    }
};


// Invert the n x n matrix in `work` (row-major, row stride n; thread-owned
// entries: entry e = r*n + j is only ever touched by thread e % blockDim.x)
// and write the inverse to `out` (row stride ldo).  `work` is destroyed.
// LDS: colbuf[2][GJ_NMAX], prow[GJ_NMAX], pivrow/pivstep.  Every wave runs
// the pivot search itself (DPP wave max, then a ballot for the smallest row
// attaining it) and keeps its own used-row flags, so a step costs two
// barriers; a thread walks its entries with 32-bit row/column counters.
// out_tiled > 0: write the inverse in the 16x4 MFMA tile layout of order
// out_tiled (padded entries untouched); otherwise row-major with stride ldo.
template <typename T>
__device__ void gj_invert(C2<T>* work, C2<T>* out, int n, long long ldo, FactorFlags* ff,
                          int out_tiled = 0) {
    constexpr int SR = (GJ_NMAX + 63) / 64;
    __shared__ C2<T> colbuf[2][GJ_NMAX];
    __shared__ C2<T> prow[GJ_NMAX];
    __shared__ int pivrow[GJ_NMAX];
    __shared__ int pivstep[GJ_NMAX];

    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const int lane = tid & 63;
    const int nn = n * n;
    // entry e = tid + q nt sits at (r0 + q dr + carries, c0 + q dc mod n)
    const int dr = nt / n, dc = nt % n, r0 = tid / n, c0 = tid % n;
    bool used[SR];
#pragma unroll
    for (int s = 0; s < SR; ++s) used[s] = false;
    for (int r = tid; r < n; r += nt) { pivrow[r] = r; pivstep[r] = r; }
    {   // publish column 0
        int r = r0, j = c0;
        for (int e = tid; e < nn; e += nt) {
            if (j == 0) colbuf[0][r] = work[e];
            r += dr; j += dc;
            if (j >= n) { j -= n; ++r; }
        }
    }
    __syncthreads();
    int cur = 0;
    PivotStats<T> pst;
    for (int k = 0; k < n; ++k) {
        // ---- pivot search over unused rows (ties -> smallest row)
        T v[SR];
#pragma unroll
        for (int s = 0; s < SR; ++s) {
            const int r = lane + 64 * s;
            v[s] = (T)-1;
            if (r < n && !used[s]) v[s] = cabs2<T>(colbuf[cur][r]);
        }
        T best = v[0];
#pragma unroll
        for (int s = 1; s < SR; ++s) best = fmax(best, v[s]);
        best = wave_max(best);
        int pr = -1;
#pragma unroll
        for (int s = SR - 1; s >= 0; --s) {
            const unsigned long long m = __ballot(v[s] >= (T)0 && v[s] == best);
            if (m) pr = 64 * s + __ffsll((long long)m) - 1;
        }
        // pr < 0 only if no candidate compared (NaN input): flag it and keep
        // every index in range
        if (pr < 0) { pr = 0; best = (T)0; }
        pr = __builtin_amdgcn_readfirstlane(pr);
        pst.add(best);
#pragma unroll
        for (int s = 0; s < SR; ++s)
            if (pr == lane + 64 * s) used[s] = true;
        const C2<T> pv = colbuf[cur][pr];
        C2<T> inv = mk<T>((T)0, (T)0);
        if (best <= (T)0) {
            if (tid == 0) atomicOr(&ff->singular, 1);
        } else {
            const T den = (T)1 / (pv.x * pv.x + pv.y * pv.y);
            inv = mk<T>(pv.x * den, -pv.y * den);
        }
        if (tid == 0) { pivrow[k] = pr; pivstep[pr] = k; }
        // ---- publish the pivot row (pre-update values); entry pr*n + j is
        // owned by thread (pr*n + j) % nt
        {
            const int rb = pr * n;
            for (int j = ((tid - rb) % nt + nt) % nt; j < n; j += nt) prow[j] = work[rb + j];
        }
        __syncthreads();
        // ---- update, publishing column k+1 for the next search; a thread's
        // entries go in groups of four so that four loads are in flight
        const int nxt = cur ^ 1;
        auto upd = [&](int r, int j, C2<T> a) {
            C2<T> w;
            if (r == pr) {
                w = (j == k) ? inv : cmul(prow[j], inv);
            } else {
                const C2<T> f = cmul(colbuf[cur][r], inv);
                if (j == k) {
                    w = mk<T>(-f.x, -f.y);
                } else {
                    const C2<T> pj = prow[j];
                    w = mk<T>(a.x - (f.x * pj.x - f.y * pj.y), a.y - (f.x * pj.y + f.y * pj.x));
                }
            }
            if (j == k + 1) colbuf[nxt][r] = w;
            return w;
        };
        int r = r0, j = c0;
        int e = tid;
        for (; e + 3 * nt < nn; e += 4 * nt) {
            int rr[4], jj[4];
            C2<T> a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                rr[u] = r; jj[u] = j;
                a[u] = work[e + u * nt];
                r += dr; j += dc;
                if (j >= n) { j -= n; ++r; }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) work[e + u * nt] = upd(rr[u], jj[u], a[u]);
        }
        for (; e < nn; e += nt) {
            work[e] = upd(r, j, work[e]);
            r += dr; j += dc;
            if (j >= n) { j -= n; ++r; }
        }
        cur = nxt;
        __syncthreads();
    }
    pst.finish(ff);
    // ---- unscramble: X[pivstep[r]][pivrow[j]] = work[r][j]
    {
        int r = r0, j = c0;
        for (int e = tid; e < nn; e += nt) {
            const int oi = pivstep[r], oj = pivrow[j];
            if (out_tiled) out[xt_index(oi, oj, out_tiled)] = work[e];
            else out[(long long)oi * ldo + oj] = work[e];
            r += dr; j += dc;
            if (j >= n) { j -= n; ++r; }
        }
    }
    __syncthreads();
}

// One workgroup per cell: the Schur recursion over the Wc grid columns.
template <typename T>
__global__ void __launch_bounds__(GJ_THREADS)
k_cell_factor(const CellDesc* __restrict__ cells, const double2* __restrict__ diag,
              const double2* __restrict__ cz, const double2* __restrict__ e,
              C2<T>* __restrict__ Xpool, C2<T>* __restrict__ workpool, long long work_stride,
              FactorFlags* ff) {
    const CellDesc cd = cells[blockIdx.x];
    const int HL = cd.HL, Wc = cd.Wc, HLp = cd.HLp;
    const long long nn = (long long)HL * HL;
    const long long np2 = (long long)HLp * HLp;
    C2<T>* work = workpool + (long long)blockIdx.x * work_stride;
    C2<T>* X = Xpool + cd.off_X;
    const double2* dg = diag + cd.off_coef;
    const double2* zz = cz + cd.off_coef;
    const double2* ee = e + cd.off_coef;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int k = 0; k < Wc; ++k) {
        // S_k = A_k - diag(e_k) X_{k-1} diag(e_k), written with the ownership
        // pattern of gj_invert (entry e owned by thread e % nt).
        const C2<T>* Xp = X + (long long)(k - 1) * np2;
        for (long long q = tid; q < nn; q += nt) {
            int r = (int)(q / HL), j = (int)(q % HL);
            double2 a; a.x = 0.0; a.y = 0.0;
            if (r == j) a = dg[(long long)k * HL + r];
            else if (j == r + 1) a = zz[(long long)k * HL + r];
            else if (r == j + 1) a = zz[(long long)k * HL + j];
            C2<T> v = mk<T>((T)a.x, (T)a.y);
            if (k > 0) {
                double2 er = ee[(long long)k * HL + r];
                double2 ej = ee[(long long)k * HL + j];
                C2<T> x = Xp[xt_index(r, j, HLp)];
                C2<T> t = cmul(cmul(mk<T>((T)er.x, (T)er.y), x), mk<T>((T)ej.x, (T)ej.y));
                v = csub(v, t);
            }
            work[q] = v;
        }
        if (HLp != HL) {       // zero the padding of the tiled block
            C2<T>* Xk = X + (long long)k * np2;
            for (long long q = tid; q < np2; q += nt) {
                const int tile = (int)(q >> 6), ln = (int)(q & 63);
                const int i = (tile / (HLp >> 2)) * 16 + (ln & 15);
                const int j = (tile % (HLp >> 2)) * 4 + (ln >> 4);
                if (i >= HL || j >= HL) Xk[q] = mk<T>((T)0, (T)0);
            }
        }
        __syncthreads();
        gj_invert<T>(work, X + (long long)k * np2, HL, HL, ff, HLp);
    }
}

// Register-resident variant of the cell recursion for HL <= NM (NM = 64 or
// 128): the Schur complement of the current grid column stays in registers
// for the whole Gauss-Jordan elimination, so an elimination step reads no
// global memory.  Thread t owns rows rg + 32 i (i < NM/32) and columns
// cg + 16 jj (jj < NM/16), rg = t / 16, cg = t % 16 (so one row's owners
// are 16 lanes of one wave); entries outside the
// HL x HL block are zero and stay zero.  Step k with pivot row p is the
// rank-1 update
//     a[r][j] <- a[r][j] - c_r P_j   (r != p),      a[p][j] <- P_j,
// where c is column k before the step, P_j = a[p][j] / a[p][k] (j != k),
// P_k = 1 / a[p][k], and column k is cleared first so that it ends as
// -c_r / a[p][k].  Only the pivot column (published by its owners at the end
// of the previous step) and the scaled pivot row pass through LDS; every wave
// runs the pivot search itself (a DPP max over its lanes, then a ballot for
// the smallest row attaining it), so a step costs two barriers.  The pivoting
// rule and the unscrambled output are those of gj_invert.
//
// Register layout: a[jj] is a vector over the owned rows, element 2i the
// real and 2i+1 the imaginary part of row rg + 32 i.  The pivot row's slot
// i = p / 32 is wave-uniform but known only at run time; indexing the vector
// with it compiles to register-relative moves (no scratch).  The column slot
// k / 16 is made a compile-time constant by unrolling the step loop over it.
template <typename T, int N>
using vecT = T __attribute__((ext_vector_type(N)));

template <typename T, int NM, int CR, int CL>
__global__ void __launch_bounds__(GJ_THREADS)
k_cell_factor_reg(const CellDesc* __restrict__ cells, const double2* __restrict__ diag,
                  const double2* __restrict__ cz, const double2* __restrict__ e,
                  C2<T>* __restrict__ Xpool, FactorFlags* ff) {
    constexpr int R = NM / 32, C = CR + CL, SR = (NM + 63) / 64, LW = 16 * CL;
    static_assert(NM % 32 == 0 && 16 * C >= NM, "layout must cover the block");
    using V = vecT<T, 2 * R>;
    __shared__ C2<T> colbuf[2][NM];
    __shared__ C2<T> prow[16 * C];
    __shared__ int pivrow[NM];
    __shared__ int pivstep[NM];
    // columns 16 CR .. 16 C - 1 live in LDS, row-major with row length LW
    extern __shared__ __align__(16) unsigned char fac_dyn[];
    C2<T>* lm = reinterpret_cast<C2<T>*>(fac_dyn);
    const CellDesc cd = cells[blockIdx.x];
    const int n = cd.HL, Wc = cd.Wc, HLp = cd.HLp;
    const long long np2 = (long long)HLp * HLp;
    C2<T>* X = Xpool + cd.off_X;
    const double2* dg = diag + cd.off_coef;
    const double2* zz = cz + cd.off_coef;
    const double2* ee = e + cd.off_coef;
    const int tid = threadIdx.x, lane = tid & 63;
    const int rg = tid >> 4, cg = tid & 15;
    const C2<T> zero = mk<T>((T)0, (T)0);
    V a[CR];
    for (int col = 0; col < Wc; ++col) {
        // S_col = A_col - diag(e_col) X_{col-1} diag(e_col); every load uses
        // an in-range index and out-of-block entries are selected away
        const C2<T>* Xp = X + (long long)(col - 1) * np2;
        const long long cb = (long long)col * n;
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int r = rg + 32 * i;
            const int rc = r < n ? r : 0;
            const double2 dr = dg[cb + rc], zr = zz[cb + rc], zm = zz[cb + (rc > 0 ? rc - 1 : 0)];
            const double2 ev = ee[cb + rc];
            const C2<T> er = mk<T>((T)ev.x, (T)ev.y);
#pragma unroll
            for (int jj = 0; jj < C; ++jj) {
                const int j = cg + 16 * jj;
                const bool in = r < n && j < n;
                const double2 av = (j == r) ? dr : (j == r + 1) ? zr : (j == r - 1) ? zm
                                 : make_double2(0.0, 0.0);
                C2<T> v = mk<T>((T)av.x, (T)av.y);
                if (col > 0) {
                    const double2 evj = ee[cb + (in ? j : 0)];
                    const C2<T> x = Xp[xt_index(in ? r : 0, in ? j : 0, HLp)];
                    v = csub(v, cmul(cmul(er, x), mk<T>((T)evj.x, (T)evj.y)));
                }
                v = in ? v : zero;
                if (jj < CR) {
                    a[jj < CR ? jj : 0][2 * i] = v.x;
                    a[jj < CR ? jj : 0][2 * i + 1] = v.y;
                } else {
                    lm[r * LW + cg + 16 * (jj - CR)] = v;
                }
            }
        }
        if (cg == 0) {
#pragma unroll
            for (int i = 0; i < R; ++i) colbuf[0][rg + 32 * i] = mk<T>(a[0][2 * i], a[0][2 * i + 1]);
        }
        bool used[SR];
#pragma unroll
        for (int s = 0; s < SR; ++s) used[s] = false;
        for (int r = tid; r < NM; r += GJ_THREADS) { pivrow[r] = r; pivstep[r] = r; }
        __syncthreads();
        int cur = 0;
        PivotStats<T> pst;
#pragma unroll
        for (int kj = 0; kj < C; ++kj) {
            for (int kc = 0; kc < 16; ++kc) {
                const int k = kj * 16 + kc;
                if (k >= n) break;
                // pivot search (every wave): largest |c_r|^2 over unused rows,
                // ties to the smallest row; -1 marks a row out of the race
                T v[SR];
#pragma unroll
                for (int s = 0; s < SR; ++s) {
                    const int r = lane + 64 * s;
                    v[s] = (T)-1;
                    if (r < n && !used[s]) v[s] = cabs2<T>(colbuf[cur][r]);
                }
                T best = v[0];
#pragma unroll
                for (int s = 1; s < SR; ++s) best = fmax(best, v[s]);
                best = wave_max(best);
                int pr = -1;
#pragma unroll
                for (int s = SR - 1; s >= 0; --s) {
                    const unsigned long long m = __ballot(v[s] >= (T)0 && v[s] == best);
                    if (m) pr = 64 * s + __ffsll((long long)m) - 1;
                }
                // pr < 0 only if no candidate compared (NaN input): flag it
                // and keep every index in range
                if (pr < 0) { pr = 0; best = (T)0; }
                pr = __builtin_amdgcn_readfirstlane(pr);
                pst.add(best);
                const C2<T> pv = colbuf[cur][pr];
                C2<T> inv = zero;
                if (best <= (T)0) {
                    if (tid == 0) atomicOr(&ff->singular, 1);
                } else {
                    const T den = (T)1 / (pv.x * pv.x + pv.y * pv.y);
                    inv = mk<T>(pv.x * den, -pv.y * den);
                }
#pragma unroll
                for (int s = 0; s < SR; ++s)
                    if (pr == lane + 64 * s) used[s] = true;
                const int pi = pr >> 5, prg = pr & 31;
                // scaled pivot row, from its owners (16 lanes of one wave)
                if (rg == prg) {
#pragma unroll
                    for (int jj = 0; jj < C; ++jj) {
                        C2<T> v;
                        if (jj < CR) v = mk<T>(a[jj < CR ? jj : 0][2 * pi], a[jj < CR ? jj : 0][2 * pi + 1]);
                        else v = lm[pr * LW + cg + 16 * (jj - CR)];
                        prow[cg + 16 * jj] = (jj == kj && cg == kc) ? inv : cmul(v, inv);
                    }
                }
                if (tid == 0) { pivrow[k] = pr; pivstep[pr] = k; }
                __syncthreads();
                C2<T> cc[R];
#pragma unroll
                for (int i = 0; i < R; ++i) cc[i] = colbuf[cur][rg + 32 * i];
                if (kj < CR) {
                    if (cg == kc) a[kj < CR ? kj : 0] = (V)(T)0;
                }
#pragma unroll
                for (int jj = 0; jj < C; ++jj) {
                    const C2<T> P = prow[cg + 16 * jj];
#pragma unroll
                    for (int i = 0; i < R; ++i) {
                        T re, im;
                        if (jj < CR) {
                            re = a[jj < CR ? jj : 0][2 * i];
                            im = a[jj < CR ? jj : 0][2 * i + 1];
                        } else {
                            const C2<T> w = lm[(rg + 32 * i) * LW + cg + 16 * (jj - CR)];
                            const bool clr = jj == kj && cg == kc;
                            re = clr ? (T)0 : w.x;
                            im = clr ? (T)0 : w.y;
                        }
                        re = re - cc[i].x * P.x;
                        im = im - cc[i].x * P.y;
                        re = re + cc[i].y * P.y;
                        im = im - cc[i].y * P.x;
                        if (jj < CR) {
                            a[jj < CR ? jj : 0][2 * i] = re;
                            a[jj < CR ? jj : 0][2 * i + 1] = im;
                        } else {
                            lm[(rg + 32 * i) * LW + cg + 16 * (jj - CR)] = mk<T>(re, im);
                        }
                    }
                }
                if (rg == prg) {
#pragma unroll
                    for (int jj = 0; jj < C; ++jj) {
                        const C2<T> P = prow[cg + 16 * jj];
                        if (jj < CR) {
                            a[jj < CR ? jj : 0][2 * pi] = P.x;
                            a[jj < CR ? jj : 0][2 * pi + 1] = P.y;
                        } else {
                            lm[pr * LW + cg + 16 * (jj - CR)] = P;
                        }
                    }
                }
                // publish column k + 1 for the next search
                const int k1 = k + 1;
                if (k1 < n) {
                    const int kj1 = kc < 15 ? kj : kj + 1, kc1 = kc < 15 ? kc + 1 : 0;
#pragma unroll
                    for (int jq = kj; jq <= kj + 1 && jq < C; ++jq) {
                        if (jq == kj1 && cg == kc1) {
#pragma unroll
                            for (int i = 0; i < R; ++i) {
                                C2<T> w;
                                if (jq < CR) w = mk<T>(a[jq < CR ? jq : 0][2 * i], a[jq < CR ? jq : 0][2 * i + 1]);
                                else w = lm[(rg + 32 * i) * LW + cg + 16 * (jq - CR)];
                                colbuf[cur ^ 1][rg + 32 * i] = w;
                            }
                        }
                    }
                }
                cur ^= 1;
                __syncthreads();
            }
        }
        pst.finish(ff);
        // unscramble: X_col[pivstep[r]][pivrow[j]] = a[r][j]; padding zero
        C2<T>* Xk = X + (long long)col * np2;
        int ps[R];
#pragma unroll
        for (int i = 0; i < R; ++i) ps[i] = pivstep[rg + 32 * i];
#pragma unroll
        for (int jj = 0; jj < C; ++jj) {
            const int j = cg + 16 * jj;
            const int pcj = pivrow[j < NM ? j : 0];
#pragma unroll
            for (int i = 0; i < R; ++i) {
                const int r = rg + 32 * i;
                const bool in = r < n && j < n;
                C2<T> w;
                if (jj < CR) w = mk<T>(a[jj < CR ? jj : 0][2 * i], a[jj < CR ? jj : 0][2 * i + 1]);
                else w = lm[r * LW + cg + 16 * (jj - CR)];
                if (r < HLp && j < HLp)
                    Xk[xt_index(in ? ps[i] : r, in ? pcj : j, HLp)] = in ? w : zero;
            }
        }
        __syncthreads();
    }
}

// LDS bytes of the LDS-resident columns of k_cell_factor_reg.
template <typename T, int NM, int CL>
constexpr size_t fac_lds_bytes() { return (size_t)NM * 16 * CL * sizeof(C2<T>); }

template <typename T>
__global__ void __launch_bounds__(GJ_THREADS)
k_invert_batch(C2<T>* const* mats, C2<T>* const* outs, const int* ns, C2<T>* workpool,
               long long work_stride, FactorFlags* ff) {
    const int n = ns[blockIdx.x];
    C2<T>* work = workpool + (long long)blockIdx.x * work_stride;
    const C2<T>* src = mats[blockIdx.x];
    const long long nn = (long long)n * n;
    for (long long q = threadIdx.x; q < nn; q += blockDim.x) work[q] = src[q];
    __syncthreads();
    gj_invert<T>(work, outs[blockIdx.x], n, n, ff);
}

template <typename T>
void launch_cell_factor(const CellDesc* cells_dev, int ncells, const Dims& d,
                        const double2* diag, const double2* cz, const double2* e,
                        C2<T>* Xpool, C2<T>* work, long long work_stride, FactorFlags* ff,
                        hipStream_t st) {
#if HZ_GJ_REG
    if (d.HLmax <= 64) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cell_factor_reg<T, 64, 4, 0>), dim3(ncells),
                           dim3(GJ_THREADS), 0, st, cells_dev, diag, cz, e, Xpool, ff);
        return;
    }
    if (d.HLmax <= 128) {
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cell_factor_reg<T, 128, 8, 0>), dim3(ncells),
                           dim3(GJ_THREADS), 0, st, cells_dev, diag, cz, e, Xpool, ff);
        return;
    }
    if (d.HLmax <= 160) {
        // 7 column slots in registers, 3 (48 columns) in LDS
        constexpr size_t lds = fac_lds_bytes<T, 160, 3>();
        static bool attr = false;
        if (!attr) {
            // if the device refuses, the launch fails and is reported
            if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_cell_factor_reg<T, 160, 7, 3>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
                (void)hipGetLastError();
            attr = true;
        }
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cell_factor_reg<T, 160, 7, 3>), dim3(ncells),
                           dim3(GJ_THREADS), lds, st, cells_dev, diag, cz, e, Xpool, ff);
        return;
    }
#endif
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cell_factor<T>), dim3(ncells), dim3(GJ_THREADS), 0, st,
                       cells_dev, diag, cz, e, Xpool, work, work_stride, ff);
}

template <typename T>
void launch_invert_batch(C2<T>* const* mats, C2<T>* const* outs, const int* ns, int count,
                         C2<T>* work, long long work_stride, FactorFlags* ff, hipStream_t st) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_invert_batch<T>), dim3(count), dim3(GJ_THREADS), 0, st,
                       mats, outs, ns, work, work_stride, ff);
}

template void launch_cell_factor<double>(const CellDesc*, int, const Dims&, const double2*,
                                         const double2*, const double2*, double2*, double2*,
                                         long long, FactorFlags*, hipStream_t);
template void launch_cell_factor<float>(const CellDesc*, int, const Dims&, const double2*,
                                        const double2*, const double2*, float2*, float2*,
                                        long long, FactorFlags*, hipStream_t);
template void launch_invert_batch<double>(double2* const*, double2* const*, const int*, int,
                                          double2*, long long, FactorFlags*, hipStream_t);
template void launch_invert_batch<float>(float2* const*, float2* const*, const int*, int,
                                         float2*, long long, FactorFlags*, hipStream_t);

}  // namespace hz
