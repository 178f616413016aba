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

template <typename T>
__device__ inline T cabs2(C2<T> a) { return a.x * a.x + a.y * a.y; }

// Invert the n x n matrix in `work` (row-major, row stride n; thread-owned
// entries: entry e = r*n + j is only ever touched by thread e % blockDim.x)
// and write the inverse to `out` (row stride ldo).  `work` is destroyed.
// LDS: colbuf[2][GJ_NMAX], prow[GJ_NMAX], pivrow/pivstep/used, reduction.
// out_tiled > 0: write the inverse in the 16x4 MFMA tile layout of order
// out_tiled (padded entries untouched); otherwise row-major with stride ldo.
template <typename T>
__device__ void gj_invert(C2<T>* work, C2<T>* out, int n, long long ldo, int* sing_flag,
                          int out_tiled = 0) {
    __shared__ C2<T> colbuf[2][GJ_NMAX];
    __shared__ C2<T> prow[GJ_NMAX];
    __shared__ int pivrow[GJ_NMAX];
    __shared__ int pivstep[GJ_NMAX];
    __shared__ int used[GJ_NMAX];
    __shared__ T redv[GJ_THREADS];
    __shared__ int redi[GJ_THREADS];
    __shared__ int s_pr;
    __shared__ C2<T> s_inv;

    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const long long nn = (long long)n * n;
    for (int r = tid; r < n; r += nt) used[r] = 0;
    // publish column 0
    for (long long e = tid; e < nn; e += nt) {
        int j = (int)(e % n);
        if (j == 0) colbuf[0][e / n] = work[e];
    }
    __syncthreads();
    int cur = 0;
    for (int k = 0; k < n; ++k) {
        // ---- pivot search over unused rows (ties -> smallest row)
        T best = (T)-1;
        int bi = n;
        for (int r = tid; r < n; r += nt) {
            if (!used[r]) {
                T v = cabs2<T>(colbuf[cur][r]);
                if (v > best) { best = v; bi = r; }
            }
        }
        redv[tid] = best;
        redi[tid] = bi;
        __syncthreads();
        for (int s = nt >> 1; s > 0; s >>= 1) {
            if (tid < s) {
                T v2 = redv[tid + s];
                int i2 = redi[tid + s];
                if (v2 > redv[tid] || (v2 == redv[tid] && i2 < redi[tid])) {
                    redv[tid] = v2; redi[tid] = i2;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            int pr = redi[0];
            C2<T> pv = colbuf[cur][pr];
            if (redv[0] <= (T)0) {
                atomicOr(sing_flag, 1);
                s_inv = mk<T>((T)0, (T)0);
            } else {
                T den = (T)1 / (pv.x * pv.x + pv.y * pv.y);
                s_inv = mk<T>(pv.x * den, -pv.y * den);
            }
            s_pr = pr;
            used[pr] = 1;
            pivrow[k] = pr;
            pivstep[pr] = k;
        }
        __syncthreads();
        const int pr = s_pr;
        const C2<T> inv = s_inv;
        // ---- publish the pivot row (pre-update values); each thread reads
        // only the entries of row pr it owns (e = tid mod nt)
        {
            const long long r0 = (long long)pr * n;
            long long e0 = r0 + ((tid - (int)(r0 % nt)) % nt + nt) % nt;
            for (long long e = e0; e < r0 + n; e += nt) prow[e - r0] = work[e];
        }
        __syncthreads();
        // ---- update, publishing column k+1 for the next search
        const int nxt = cur ^ 1;
        for (long long e = tid; e < nn; e += nt) {
            int r = (int)(e / n);
            int j = (int)(e % n);
            C2<T> v;
            if (r == pr) {
                v = (j == k) ? inv : cmul(prow[j], inv);
            } else {
                C2<T> f = cmul(colbuf[cur][r], inv);
                if (j == k) {
                    v = mk<T>(-f.x, -f.y);
                } else {
                    C2<T> w = work[e];
                    C2<T> pj = prow[j];
                    v = mk<T>(w.x - (f.x * pj.x - f.y * pj.y), w.y - (f.x * pj.y + f.y * pj.x));
                }
            }
            work[e] = v;
            if (j == k + 1) colbuf[nxt][r] = v;
        }
        cur = nxt;
        __syncthreads();
    }
    // ---- unscramble: X[pivstep[r]][pivrow[j]] = work[r][j]
    for (long long e = tid; e < nn; e += nt) {
        int r = (int)(e / n);
        int j = (int)(e % n);
        const int oi = pivstep[r], oj = pivrow[j];
        if (out_tiled) out[xt_index(oi, oj, out_tiled)] = work[e];
        else out[(long long)oi * ldo + oj] = work[e];
    }
    __syncthreads();
}

// One workgroup per cell: the Schur recursion over the Wc grid columns.
template <typename T>
__global__ void __launch_bounds__(GJ_THREADS)
k_cell_factor(const CellDesc* __restrict__ cells, const double2* __restrict__ diag,
              const double2* __restrict__ cz, const double2* __restrict__ e,
              C2<T>* __restrict__ Xpool, C2<T>* __restrict__ workpool, long long work_stride,
              int* sing_flag) {
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
        gj_invert<T>(work, X + (long long)k * np2, HL, HL, sing_flag, HLp);
    }
}

template <typename T>
__global__ void __launch_bounds__(GJ_THREADS)
k_invert_batch(C2<T>* const* mats, C2<T>* const* outs, const int* ns, C2<T>* workpool,
               long long work_stride, int* sing_flag) {
    const int n = ns[blockIdx.x];
    C2<T>* work = workpool + (long long)blockIdx.x * work_stride;
    const C2<T>* src = mats[blockIdx.x];
    const long long nn = (long long)n * n;
    for (long long q = threadIdx.x; q < nn; q += blockDim.x) work[q] = src[q];
    __syncthreads();
    gj_invert<T>(work, outs[blockIdx.x], n, n, sing_flag);
}

template <typename T>
void launch_cell_factor(const CellDesc* cells_dev, int ncells, const Dims& d,
                        const double2* diag, const double2* cz, const double2* e,
                        C2<T>* Xpool, C2<T>* work, long long work_stride, int* sing_flag,
                        hipStream_t st) {
    (void)d;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cell_factor<T>), dim3(ncells), dim3(GJ_THREADS), 0, st,
                       cells_dev, diag, cz, e, Xpool, work, work_stride, sing_flag);
}

template <typename T>
void launch_invert_batch(C2<T>* const* mats, C2<T>* const* outs, const int* ns, int count,
                         C2<T>* work, long long work_stride, int* sing_flag, hipStream_t st) {
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_invert_batch<T>), dim3(count), dim3(GJ_THREADS), 0, st,
                       mats, outs, ns, work, work_stride, sing_flag);
}

template void launch_cell_factor<double>(const CellDesc*, int, const Dims&, const double2*,
                                         const double2*, const double2*, double2*, double2*,
                                         long long, int*, hipStream_t);
template void launch_cell_factor<float>(const CellDesc*, int, const Dims&, const double2*,
                                        const double2*, const double2*, float2*, float2*,
                                        long long, int*, hipStream_t);
template void launch_invert_batch<double>(double2* const*, double2* const*, const int*, int,
                                          double2*, long long, int*, hipStream_t);
template void launch_invert_batch<float>(float2* const*, float2* const*, const int*, int,
                                         float2*, long long, int*, hipStream_t);

}  // namespace hz
