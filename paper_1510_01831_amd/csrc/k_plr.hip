// Partitioned low-rank form of the interface operators (eq. factorization
// and its PLR footnote, Sec. 4.3; accuracy eps of the caption of Fig. 9).
//
// A dense operator block A (row-major, row stride lda) is cut into square
// tiles of PLR_TILE; a tile whose rank-revealing QR reaches the tile's
// Frobenius budget delta = eps ||A||_F / sqrt(T) (T tiles in the block) at a
// rank r with r (t_r + t_c) < t_r t_c is stored as U (t_r x r) and
// W (r x t_c), A_tile ~ U W; otherwise it stays dense.  Householder QR with
// column pivoting: after r steps A P = Q [R11 R12; 0 R22] and the discarded
// part has Frobenius norm ||R22||_F, which is checked at every step, so the
// whole block satisfies ||A - A_plr||_F <= eps ||A||_F.  U = Q[:, :r]
// (column-major: lane i reads row i of a column), W = [R11 R12] P^T
// (row-major: lane j reads column j of a row), dense tiles column-major, so
// that every wave load is consecutive lanes on consecutive entries.
//
// Application (single right-hand side, the HBM-bound form): one wave per
// tile writes the tile's partial product to a scratch (dense: D x; low rank:
// U (W x)); a second kernel adds the partials of each tile row in tile order
// (deterministic) and applies the task's epilogue.
#include "hz_common.h"

namespace hz {

constexpr int PLR_THREADS = 256;

// Frobenius norm squared of every tile (one workgroup per tile).
template <typename T>
__global__ void __launch_bounds__(PLR_THREADS)
k_plr_tile_norms(const PlrBlock<T>* __restrict__ blocks, const PlrTile* __restrict__ tiles,
                 double* __restrict__ norm2) {
    const PlrTile tl = tiles[blockIdx.x];
    const PlrBlock<T> bk = blocks[tl.block];
    __shared__ double red[PLR_THREADS];
    double acc = 0.0;
    for (int e = threadIdx.x; e < tl.tr * tl.tc; e += PLR_THREADS) {
        const int i = e / tl.tc, j = e - i * tl.tc;
        const C2<T> a = gload<T>(bk.A + (long long)(tl.i0 + i) * bk.lda + tl.j0 + j);
        acc += (double)a.x * a.x + (double)a.y * a.y;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = PLR_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) norm2[blockIdx.x] = red[0];
}

// Rank-revealing QR of every tile.  write = 0: only the rank (tl.rank is
// written to ranks[]); write = 1: the factors (or the dense tile) go to the
// pool at the tile's offset.  delta2[t]: the tile's Frobenius budget squared.
template <typename T>
__global__ void __launch_bounds__(PLR_THREADS)
k_plr_compress(const PlrBlock<T>* __restrict__ blocks, const PlrTile* __restrict__ tiles,
               const double* __restrict__ delta2, int* __restrict__ ranks,
               C2<T>* __restrict__ pool, int write) {
    constexpr int TS = PLR_TILE;
    __shared__ C2<T> A[TS * TS];                  // column-major, leading dimension TS
    __shared__ C2<T> V[TS * PLR_RMAX];            // Householder vectors (column k from row k)
    __shared__ T beta[PLR_RMAX];
    __shared__ double nrm[TS];
    __shared__ int perm[TS];
    __shared__ double red[PLR_THREADS];
    __shared__ int ired[PLR_THREADS];
    __shared__ C2<T> wv[TS];
    const PlrTile tl = tiles[blockIdx.x];
    const PlrBlock<T> bk = blocks[tl.block];
    const int tr = tl.tr, tc = tl.tc, tid = threadIdx.x;
    const double d2 = delta2[blockIdx.x];
    for (int e = tid; e < tr * tc; e += PLR_THREADS) {
        const int i = e / tc, j = e - i * tc;
        A[i + j * TS] = gload<T>(bk.A + (long long)(tl.i0 + i) * bk.lda + tl.j0 + j);
    }
    for (int j = tid; j < tc; j += PLR_THREADS) perm[j] = j;
    __syncthreads();
    // largest rank that stores fewer entries than the tile
    int rlim = (tr * tc - 1) / (tr + tc);
    if (rlim > PLR_RMAX) rlim = PLR_RMAX;
    const int kmax = min(tr, tc);
    int rank = -1;
    for (int k = 0; k <= kmax; ++k) {
        // squared norms of the remaining columns (rows k..tr-1)
        for (int j = tid; j < tc; j += PLR_THREADS) {
            double s = 0.0;
            if (j >= k)
                for (int i = k; i < tr; ++i) {
                    const C2<T> a = A[i + j * TS];
                    s += (double)a.x * a.x + (double)a.y * a.y;
                }
            nrm[j] = s;
        }
        __syncthreads();
        // remaining Frobenius norm squared and the pivot column
        double s = 0.0, best = -1.0;
        int bj = min(k, tc - 1);
        for (int j = k + tid; j < tc; j += PLR_THREADS) {
            s += nrm[j];
            if (nrm[j] > best) { best = nrm[j]; bj = j; }
        }
        red[tid] = s;
        ired[tid] = bj;
        __syncthreads();
        for (int h = PLR_THREADS / 2; h > 0; h >>= 1) {
            if (tid < h) {
                red[tid] += red[tid + h];
                const int a = ired[tid], b = ired[tid + h];
                // larger norm wins, ties to the smaller column
                if (nrm[b] > nrm[a] || (nrm[b] == nrm[a] && b < a)) ired[tid] = b;
            }
            __syncthreads();
        }
        const double rem2 = red[0];
        const int p = ired[0];
        __syncthreads();
        if (rem2 <= d2) { rank = k; break; }
        if (k >= rlim || k == kmax) break;           // no saving: dense
        // swap columns k and p
        if (p != k) {
            for (int i = tid; i < tr; i += PLR_THREADS) {
                const C2<T> t0 = A[i + k * TS];
                A[i + k * TS] = A[i + p * TS];
                A[i + p * TS] = t0;
            }
            if (tid == 0) { const int t0 = perm[k]; perm[k] = perm[p]; perm[p] = t0; }
        }
        __syncthreads();
        // Householder vector of column k (rows k..tr-1): v = x - alpha e_0,
        // alpha = -exp(i arg x_0) ||x||, H = I - beta v v^H, beta = 2 / ||v||^2
        if (tid == 0) {
            double xn = 0.0;
            for (int i = k; i < tr; ++i) {
                const C2<T> a = A[i + k * TS];
                xn += (double)a.x * a.x + (double)a.y * a.y;
            }
            xn = sqrt(xn);
            const C2<T> x0 = A[k + k * TS];
            const double a0 = sqrt((double)x0.x * x0.x + (double)x0.y * x0.y);
            double ph_re = 1.0, ph_im = 0.0;
            if (a0 > 0.0) { ph_re = x0.x / a0; ph_im = x0.y / a0; }
            const double al_re = -ph_re * xn, al_im = -ph_im * xn;
            const double v0_re = x0.x - al_re, v0_im = x0.y - al_im;
            double vn = v0_re * v0_re + v0_im * v0_im;
            for (int i = k + 1; i < tr; ++i) {
                const C2<T> a = A[i + k * TS];
                vn += (double)a.x * a.x + (double)a.y * a.y;
            }
            beta[k] = vn > 0.0 ? (T)(2.0 / vn) : (T)0;
            V[k + k * TS] = mk<T>((T)v0_re, (T)v0_im);
            wv[0] = mk<T>((T)al_re, (T)al_im);
        }
        __syncthreads();
        for (int i = k + 1 + tid; i < tr; i += PLR_THREADS) V[i + k * TS] = A[i + k * TS];
        if (tid == 0) A[k + k * TS] = wv[0];
        for (int i = k + 1 + tid; i < tr; i += PLR_THREADS) A[i + k * TS] = mk<T>((T)0, (T)0);
        __syncthreads();
        // apply H to the columns k+1..tc-1: w_j = v^H a_j, a_j -= beta v w_j
        const T bt = beta[k];
        for (int j = k + 1 + tid; j < tc; j += PLR_THREADS) {
            C2<T> w = mk<T>((T)0, (T)0);
            for (int i = k; i < tr; ++i) w = cfma(cconj(V[i + k * TS]), A[i + j * TS], w);
            w = cscale(w, bt);
            for (int i = k; i < tr; ++i) A[i + j * TS] = csub(A[i + j * TS], cmul(V[i + k * TS], w));
        }
        __syncthreads();
    }
    if (!write) {
        if (tid == 0) ranks[blockIdx.x] = rank;
        return;
    }
    C2<T>* out = pool + tl.off;
    if (tl.rank < 0) {                                // dense tile, column-major
        for (int e = tid; e < tr * tc; e += PLR_THREADS) {
            const int i = e / tc, j = e - i * tc;
            out[i + (long long)j * tr] = gload<T>(bk.A + (long long)(tl.i0 + i) * bk.lda + tl.j0 + j);
        }
        return;
    }
    const int r = tl.rank;
    if (r == 0) return;
    // W = [R11 R12] P^T (r x tc, row-major): W[q, perm[j]] = R[q, j]
    C2<T>* W = out + (long long)tr * r;
    for (int e = tid; e < r * tc; e += PLR_THREADS) {
        const int q = e / tc, j = e - q * tc;
        W[(long long)q * tc + perm[j]] = j >= q ? A[q + j * TS] : mk<T>((T)0, (T)0);
    }
    __syncthreads();                                  // R read; A's storage becomes U
    // U = H_0 ... H_{r-1} [I_r; 0], one column per thread, in LDS
    for (int e = tid; e < tr * r; e += PLR_THREADS) {
        const int i = e % tr, q = e / tr;
        A[i + q * TS] = mk<T>((T)(i == q ? 1 : 0), (T)0);
    }
    __syncthreads();
    for (int k = r - 1; k >= 0; --k) {
        for (int q = tid; q < r; q += PLR_THREADS) {
            C2<T> w = mk<T>((T)0, (T)0);
            for (int i = k; i < tr; ++i) w = cfma(cconj(V[i + k * TS]), A[i + q * TS], w);
            w = cscale(w, beta[k]);
            for (int i = k; i < tr; ++i) A[i + q * TS] = csub(A[i + q * TS], cmul(V[i + k * TS], w));
        }
        __syncthreads();
    }
    for (int e = tid; e < tr * r; e += PLR_THREADS) {
        const int i = e % tr, q = e / tr;
        out[i + (long long)q * tr] = A[i + q * TS];
    }
}

// Gather x[k] of a task (its k-th input row, column b) through the segments.
template <typename T>
__device__ inline C2<T> task_x(const GemmTask<T>& t, int k, int b) {
    for (int s = 0; s < t.nseg; ++s) {
        const int rel = k - t.seg_k0[s];
        if (rel >= 0 && rel < t.seg_len[s])
            return t.seg_ptr[s] ? gload<T>(t.seg_ptr[s] + (long long)rel * t.ldx + b)
                                : mk<T>((T)0, (T)0);
    }
    return mk<T>((T)0, (T)0);
}

// Whether column range [j0, j0 + tc) of a task meets a non-null segment.
template <typename T>
__device__ inline bool task_cols_live(const GemmTask<T>& t, int j0, int tc) {
    for (int s = 0; s < t.nseg; ++s)
        if (t.seg_ptr[s] && t.seg_k0[s] < j0 + tc && j0 < t.seg_k0[s] + t.seg_len[s]) return true;
    return false;
}

// Sum of a complex value over the 64 lanes of a wave, in every lane.
template <typename T>
__device__ inline C2<T> wave_sum(C2<T> v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    return v;
}

// Pass 1: one wave per tile of each task (tasks on blockIdx.y); partial
// products of the tile to part[(t.plr_part + tile) * PLR_TILE + row].
// Tiles whose columns meet only absent input segments write zeros.  Loads
// are issued in groups of PLR_G independent ones per lane (a single-RHS
// product is bound by memory latency otherwise).
constexpr int PLR_G = 8;
template <typename T>
__global__ void __launch_bounds__(PLR_THREADS)
k_plr_apply_tiles(const GemmTask<T>* __restrict__ tasks, C2<T>* __restrict__ part) {
    constexpr int TS = PLR_TILE;
    __shared__ C2<T> xs[PLR_THREADS / 64][TS];
    const GemmTask<T>& t = tasks[blockIdx.y];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int tile = blockIdx.x * (PLR_THREADS / 64) + wv;
    const int ntile = t.plr_ntr * t.plr_ntc;
    if (tile >= ntile) return;                        // whole wave
    const PlrTile tl = t.plr[tile];
    const C2<T>* src = t.plr_pool + tl.off;
    const int tr = tl.tr, tc = tl.tc;
    const C2<T> z = mk<T>((T)0, (T)0);
    C2<T> y = z;
    if (tl.rank == 0 || !task_cols_live(t, tl.j0, tc)) {
        gstore<T>(part + (t.plr_part + tile) * TS + lane, y);
        return;
    }
    const C2<T> xl = lane < tc ? task_x<T>(t, tl.j0 + lane, 0) : z;
    xs[wv][lane] = xl;
    __builtin_amdgcn_wave_barrier();
    const int il = lane < tr ? lane : 0;
    if (tl.rank < 0) {                                // dense, column-major
        for (int j0 = 0; j0 < tc; j0 += PLR_G) {
            C2<T> a[PLR_G];
#pragma unroll
            for (int u = 0; u < PLR_G; ++u)
                a[u] = j0 + u < tc ? gload<T>(src + il + (long long)(j0 + u) * tr) : z;
#pragma unroll
            for (int u = 0; u < PLR_G; ++u) y = cfma(a[u], xs[wv][(j0 + u) & (TS - 1)], y);
        }
    } else {
        const int r = tl.rank;
        const C2<T>* W = src + (long long)tr * r;     // r x tc, row-major
        const int jl = lane < tc ? lane : 0;
        for (int q0 = 0; q0 < r; q0 += PLR_G) {
            C2<T> w[PLR_G], u[PLR_G];
#pragma unroll
            for (int g = 0; g < PLR_G; ++g) {
                w[g] = q0 + g < r ? gload<T>(W + (long long)(q0 + g) * tc + jl) : z;
                u[g] = q0 + g < r ? gload<T>(src + il + (long long)(q0 + g) * tr) : z;
            }
#pragma unroll
            for (int g = 0; g < PLR_G; ++g) {
                // t_q = sum_j W[q, j] x_j (every lane), then y_i += U[i, q] t_q
                const C2<T> tq = wave_sum<T>(lane < tc ? cmul(w[g], xl) : z);
                y = cfma(u[g], tq, y);
            }
        }
    }
    gstore<T>(part + (t.plr_part + tile) * TS + lane, lane < tr ? y : z);
}

// Pass 2: one wave per tile row of each task: the partials of the row's
// tiles added in tile order, then the epilogue.
template <typename T>
__global__ void __launch_bounds__(PLR_THREADS)
k_plr_apply_rows(const GemmTask<T>* __restrict__ tasks, const C2<T>* __restrict__ part) {
    constexpr int TS = PLR_TILE;
    const GemmTask<T>& t = tasks[blockIdx.y];
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (PLR_THREADS / 64) + (threadIdx.x >> 6);
    if (row >= t.plr_ntr) return;
    const int i = row * TS + lane;
    if (i >= t.m) return;
    C2<T> acc = mk<T>((T)0, (T)0);
    const C2<T>* p = part + (t.plr_part + (long long)row * t.plr_ntc) * TS + lane;
    const int n = t.plr_ntc;
    for (int q0 = 0; q0 < n; q0 += PLR_G) {
        C2<T> v[PLR_G];
#pragma unroll
        for (int g = 0; g < PLR_G; ++g)
            v[g] = q0 + g < n ? gload<T>(p + (long long)(q0 + g) * TS) : mk<T>((T)0, (T)0);
#pragma unroll
        for (int g = 0; g < PLR_G; ++g) acc = cadd(acc, v[g]);
    }
    // epilogue: out = add0 + c1 add1 + alpha acc on the task's output segments
    for (int s = 0; s < t.noseg; ++s) {
        const int rel = i - t.oseg_i0[s];
        if (rel >= 0 && rel < t.oseg_len[s]) {
            const long long off = (long long)rel * t.ldo;
            C2<T> v = cscale(acc, t.alpha);
            if (t.oseg_add0[s]) v = cadd(v, gload<T>(t.oseg_add0[s] + off));
            if (t.oseg_add1[s]) v = cadd(v, cscale(gload<T>(t.oseg_add1[s] + off), t.c1[s]));
            gstore<T>(t.oseg_ptr[s] + off, v);
            return;
        }
    }
}

template <typename T>
void launch_plr_tile_norms(const PlrBlock<T>* blocks, const PlrTile* tiles, int ntiles,
                           double* norm2, hipStream_t st) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_plr_tile_norms<T>), dim3(ntiles), dim3(PLR_THREADS), 0,
                       st, blocks, tiles, norm2);
}

template <typename T>
void launch_plr_compress(const PlrBlock<T>* blocks, const PlrTile* tiles, int ntiles,
                         const double* delta2, int* ranks, C2<T>* pool, int write,
                         hipStream_t st) {
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_plr_compress<T>), dim3(ntiles), dim3(PLR_THREADS), 0, st,
                       blocks, tiles, delta2, ranks, pool, write);
}

template <typename T>
void launch_plr_apply(const GemmTask<T>* tasks_dev, int ntasks, int max_tiles, int max_rows,
                      C2<T>* part, hipStream_t st) {
    if (ntasks <= 0) return;
    constexpr int WPB = PLR_THREADS / 64;
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_plr_apply_tiles<T>),
                       dim3((max_tiles + WPB - 1) / WPB, ntasks), dim3(PLR_THREADS), 0, st,
                       tasks_dev, part);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_plr_apply_rows<T>),
                       dim3((max_rows + WPB - 1) / WPB, ntasks), dim3(PLR_THREADS), 0, st,
                       tasks_dev, (const C2<T>*)part);
}

template void launch_plr_tile_norms<double>(const PlrBlock<double>*, const PlrTile*, int, double*,
                                            hipStream_t);
template void launch_plr_tile_norms<float>(const PlrBlock<float>*, const PlrTile*, int, double*,
                                           hipStream_t);
template void launch_plr_compress<double>(const PlrBlock<double>*, const PlrTile*, int,
                                          const double*, int*, double2*, int, hipStream_t);
template void launch_plr_compress<float>(const PlrBlock<float>*, const PlrTile*, int,
                                         const double*, int*, float2*, int, hipStream_t);
template void launch_plr_apply<double>(const GemmTask<double>*, int, int, int, double2*,
                                       hipStream_t);
template void launch_plr_apply<float>(const GemmTask<float>*, int, int, int, float2*, hipStream_t);

}  // namespace hz
