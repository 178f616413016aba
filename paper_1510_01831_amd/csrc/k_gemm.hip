// Segmented batched complex GEMM:  out = add0 + c1 * add1 + alpha * A x
// over a list of tasks.  Used for every dense operator application of the
// interface factorisation (M_f, the inner block LU substitutions, and the
// combined [M_u | D_loc] output operator), online and offline.
//
// x rows are gathered from up to NSEG contiguous segments (trace pairs, inner
// traces), the output rows are scattered to up to NOSEG contiguous segments,
// and every vector row holds B batch values contiguously (batch fastest).
#include <algorithm>

#include "hz_common.h"
#include "hz_mfma.h"

namespace hz {

constexpr int GV_THREADS = 256;
constexpr int GV_ROWS = 4;           // rows per workgroup (one per wave)

template <typename T>
__device__ inline C2<T> shfl_down_c(C2<T> v, int d) {
    C2<T> r;
    r.x = __shfl_down(v.x, d, 64);
    r.y = __shfl_down(v.y, d, 64);
    return r;
}

template <typename T>
__device__ inline void epilogue(const GemmTask<T>& t, int i, int b, C2<T> acc) {
    for (int s = 0; s < t.noseg; ++s) {
        const int rel = i - t.oseg_i0[s];
        if (rel >= 0 && rel < t.oseg_len[s]) {
            const long long off = (long long)rel * t.ldo + b;
            C2<T> v = cscale(acc, t.alpha);
            const C2<T>* a0 = t.oseg_add0[s];
            const C2<T>* a1 = t.oseg_add1[s];
            if (a0) v = cadd(v, gload<T>(a0 + off));
            if (a1) v = cadd(v, cscale(gload<T>(a1 + off), t.c1[s]));
            gstore<T>(t.oseg_ptr[s] + off, v);
            return;
        }
    }
}

// A load of an operator entry that is streamed once per launch, marked
// nontemporal (it should not displace the cached input vector).
template <typename T>
__device__ __forceinline__ C2<T> gload_stream(const C2<T>* p) {
    using V = T __attribute__((ext_vector_type(2)));
    const V v = __builtin_nontemporal_load((const __attribute__((address_space(1))) V*)p);
    return mk<T>(v.x, v.y);
}

// B == 1: each wave reduces one row at a time, lanes run along k.
template <typename T>
__global__ void __launch_bounds__(GV_THREADS) k_gemv(const GemmTask<T>* __restrict__ tasks) {
    const GemmTask<T>& t = tasks[blockIdx.z];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int rr = wave; rr < GV_ROWS; rr += GV_THREADS / 64) {
        const int i = blockIdx.x * GV_ROWS + rr;
        if (i >= t.m) break;
        const C2<T>* Ar = t.A + (long long)i * t.lda;
        // GV_U loads of A and x in flight per lane, guarded at the end of a
        // segment instead of a one-load remainder loop (a single-RHS product
        // is bound by memory latency: every round trip of a row's stream
        // counts); three accumulators leave the registers to the loads
        constexpr int GV_U = 6, GV_ACC = 3;
        C2<T> au[GV_ACC];
#pragma unroll
        for (int u = 0; u < GV_ACC; ++u) au[u] = mk<T>((T)0, (T)0);
        for (int s = 0; s < t.nseg; ++s) {
            const C2<T>* xp = t.seg_ptr[s];
            if (!xp) continue;
            const int k0 = t.seg_k0[s], len = t.seg_len[s];
            const long long ldx = t.ldx;
            for (int kk = lane; kk < len; kk += 64 * GV_U) {
                C2<T> av[GV_U], xv[GV_U];
#pragma unroll
                for (int u = 0; u < GV_U; ++u) {
                    const bool in = kk + 64 * u < len;
                    av[u] = in ? gload_stream<T>(Ar + k0 + kk + 64 * u) : mk<T>((T)0, (T)0);
                    xv[u] = in ? gload<T>(xp + (long long)(kk + 64 * u) * ldx) : mk<T>((T)0, (T)0);
                }
#pragma unroll
                for (int u = 0; u < GV_U; ++u) au[u % GV_ACC] = cfma(av[u], xv[u], au[u % GV_ACC]);
            }
        }
        C2<T> acc = cadd(cadd(au[0], au[1]), au[2]);
        for (int d = 32; d > 0; d >>= 1) {
            C2<T> o = shfl_down_c<T>(acc, d);
            acc.x += o.x; acc.y += o.y;
        }
        if (lane == 0) epilogue<T>(t, i, 0, acc);
    }
}

constexpr int TM = 32, TB = 32, TK = 16;

// B > 1: 32 x 32 output tile, 16-deep k chunks staged in LDS, 2 x 2 per thread.
template <typename T>
__global__ void __launch_bounds__(GV_THREADS)
k_gemm_tiled(const GemmTask<T>* __restrict__ tasks, int B) {
    const GemmTask<T>& t = tasks[blockIdx.z];
    const int i0 = blockIdx.x * TM;
    if (i0 >= t.m) return;
    const int b0 = blockIdx.y * TB;
    if (t.ncol > 0) B = t.ncol;
    if (b0 >= B) return;
    __shared__ C2<T> As[TM][TK + 1];
    __shared__ C2<T> Xs[TK][TB + 1];
    const int tid = threadIdx.x;
    const int tr = (tid / 16) * 2;      // 16 row pairs
    const int tc = (tid % 16) * 2;      // 16 column pairs
    C2<T> acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) acc[a][c] = mk<T>((T)0, (T)0);
    for (int s = 0; s < t.nseg; ++s) {
        const C2<T>* xp = t.seg_ptr[s];
        if (!xp) continue;
        const int k0 = t.seg_k0[s], len = t.seg_len[s];
        for (int kc = 0; kc < len; kc += TK) {
            __syncthreads();
            for (int idx = tid; idx < TM * TK; idx += GV_THREADS) {
                const int r = idx / TK, q = idx % TK;
                const int i = i0 + r;
                As[r][q] = (i < t.m && kc + q < len) ? gload<T>(t.A + (long long)i * t.lda + k0 + kc + q)
                                                     : mk<T>((T)0, (T)0);
            }
            for (int idx = tid; idx < TK * TB; idx += GV_THREADS) {
                const int q = idx / TB, c = idx % TB;
                const int b = b0 + c;
                Xs[q][c] = (kc + q < len && b < B) ? gload<T>(xp + (long long)(kc + q) * t.ldx + b)
                                                   : mk<T>((T)0, (T)0);
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < TK; ++q) {
                const C2<T> a0 = As[tr][q], a1 = As[tr + 1][q];
                const C2<T> x0 = Xs[q][tc], x1 = Xs[q][tc + 1];
                acc[0][0] = cfma(a0, x0, acc[0][0]);
                acc[0][1] = cfma(a0, x1, acc[0][1]);
                acc[1][0] = cfma(a1, x0, acc[1][0]);
                acc[1][1] = cfma(a1, x1, acc[1][1]);
            }
        }
    }
    for (int a = 0; a < 2; ++a) {
        const int i = i0 + tr + a;
        if (i >= t.m) continue;
        for (int c = 0; c < 2; ++c) {
            const int b = b0 + tc + c;
            if (b < B) epilogue<T>(t, i, b, acc[a][c]);
        }
    }
}

// Batched: MT x TBM output tile per workgroup on the matrix cores.  The k
// range (all segments) is walked in KC-deep chunks; chunk c+1 is fetched into
// registers while chunk c is multiplied out of one of two LDS buffers, so one
// barrier per chunk separates the loads from the products.  The 4 waves form
// a 2 x 2 grid, each computing (MT/2) x (TBM/2) as 16x16 complex tiles (four
// real MFMAs per 4-deep k step).
// Operand cursor for the current input segment, set once per segment.  The
// block size (256) is a multiple of KC and of TBM, so entry e of a thread's
// share of a chunk sits at a fixed row or k offset from entry 0: one base
// pointer per operand plus uniform strides (few registers per lane, so more
// workgroups and chunks in flight fit on a CU).
//   A entry e: row  tid / KC + e (256 / KC),   k offset tid % KC
//   x entry e: k offset tid / TBM + e (256 / TBM), column tid % TBM
template <typename T, int MT, int TBM, int KC>
struct GemmCursor {
    static constexpr int NA = MT * KC / GV_THREADS;    // A entries per thread
    static constexpr int NX = KC * TBM / GV_THREADS;   // x entries per thread
    static constexpr int RA = GV_THREADS / KC;         // A rows between entries
    static constexpr int QX = GV_THREADS / TBM;        // x rows between entries
    static_assert(GV_THREADS % KC == 0 && GV_THREADS % TBM == 0, "cursor layout");
    const C2<T>* a0;        // A entry 0 (row clamped into range)
    const C2<T>* x0;        // x entry 0 (column clamped into range)
    long long astep;        // RA * lda
    long long ldx;
    int qa, qx;             // k offset of A entries / of x entry 0 inside a chunk
    unsigned amask;         // bit e: A entry e's row is inside the task
    bool xok;               // the thread's x column is inside the batch
    int sg, len;

    __device__ __forceinline__ void set(const GemmTask<T>& t, int s, int i0, int b0, int B,
                                        int tid) {
        sg = s;
        len = t.seg_len[s];
        ldx = t.ldx;
        const long long lda = t.lda;
        const int k0 = t.seg_k0[s], m = t.m;
        const int r0 = i0 + tid / KC;
        qa = tid % KC;
        amask = 0;
#pragma unroll
        for (int e = 0; e < NA; ++e)
            if (r0 + e * RA < m) amask |= 1u << e;
        astep = (long long)RA * lda;
        a0 = t.A + (long long)(r0 < m ? r0 : 0) * lda + k0 + qa;
        const int c = tid % TBM;
        qx = tid / TBM;
        xok = b0 + c < B;
        x0 = t.seg_ptr[s] + (long long)qx * ldx + (xok ? b0 + c : 0);
    }
};

template <typename T, int MT, int TBM, int KC>
struct GemmStage {
    using Cur = GemmCursor<T, MT, TBM, KC>;
    static constexpr int NA = Cur::NA;
    static constexpr int NX = Cur::NX;
    C2<T> a[NA], x[NX];

    // chunk starting at k offset kc of the cursor's segment
    __device__ __forceinline__ void load(const Cur& cu, int kc) {
        const bool ka = kc + cu.qa < cu.len;
#pragma unroll
        for (int e = 0; e < NA; ++e)
            a[e] = (ka && ((cu.amask >> e) & 1u)) ? gload<T>(cu.a0 + e * cu.astep + kc)
                                                  : mk<T>((T)0, (T)0);
        const long long xo = (long long)kc * cu.ldx;
#pragma unroll
        for (int e = 0; e < NX; ++e)
            x[e] = (cu.xok && kc + cu.qx + e * Cur::QX < cu.len)
                       ? gload<T>(cu.x0 + (long long)e * Cur::QX * cu.ldx + xo)
                       : mk<T>((T)0, (T)0);
    }
    __device__ __forceinline__ void stash(C2<T> (*As)[KC + 1], C2<T> (*Xs)[TBM + 1], int tid) const {
#pragma unroll
        for (int e = 0; e < NA; ++e) {
            const int idx = tid + e * GV_THREADS;
            As[idx / KC][idx % KC] = a[e];
        }
#pragma unroll
        for (int e = 0; e < NX; ++e) {
            const int idx = tid + e * GV_THREADS;
            Xs[idx / TBM][idx % TBM] = x[e];
        }
    }
};

// next non-empty chunk after (sg, kc); sg == nseg when none is left
template <typename T, int KC>
__device__ __forceinline__ void next_chunk(const GemmTask<T>& t, int& sg, int& kc) {
    kc += KC;
    while (sg < t.nseg && (!t.seg_ptr[sg] || kc >= t.seg_len[sg])) { ++sg; kc = 0; }
}

// OFFLINE selects a separate instantiation (same code) for the factorisation
// stage, so per-kernel profiles of the solve phase hold only solve launches.
// Tile order (xcd_tile): each XCD is given one contiguous run of the (task,
// row tile, column tile) sequence, column tiles fastest: the workgroups that
// share a row block of A and a task's x run together and read them once into
// that XCD's L2.

// DEEP: two register stages, so the loads of chunk c+2 are issued while chunk
// c is multiplied and chunk c+1 waits in registers (two chunk periods to hide
// the load latency instead of one).
//
// NBUF: LDS buffers per operand.  Two let the next chunk be stashed while the
// current one is multiplied (one barrier per chunk); one halves the LDS of a
// workgroup at the price of a second barrier.  The 32 x 32 tiles with 32-deep
// chunks use one: at two (33.8 KB for complex64) only four workgroups fit on
// a CU, so a launch of 1216 split-k workgroups ran in two rounds; at one
// (16.9 KB) registers allow five per CU (complex128: two -> four).
//
// splits > 1 (split k): the splits workgroups of an output
// tile (adjacent slots, hence one XCD) each take a contiguous share of the
// tile's k chunks and store their raw accumulators to ws; a second kernel
// (k_gemm_split_reduce) adds the shares in index order and applies the
// epilogue.  The kernel boundary orders the two passes, so no workgroup
// waits on another and no fence is needed.
template <typename T, int MT, int TBM, int KC, bool OFFLINE, bool DEEP = false, int NBUF = 2>
__global__ void __launch_bounds__(GV_THREADS, 2)
k_gemm_mfma(const GemmTask<T>* __restrict__ tasks, int B, int row_tiles, int col_tiles,
            int splits, C2<T>* __restrict__ ws) {
    constexpr int RTW = MT / 32;                 // row tiles per wave
    constexpr int CTW = TBM / 32;                // column tiles per wave
    const int per_task = row_tiles * col_tiles * splits;
    const int tile = xcd_tile(blockIdx.x, (int)gridDim.x);
    const int task = tile / per_task, rem = tile - task * per_task;
    const int sp = rem % splits, rc = rem / splits;
    const int rt = rc / col_tiles, ct = rc - rt * col_tiles;
    const GemmTask<T>& t = tasks[task];
    const int i0 = rt * MT;
    if (i0 >= t.m) return;
    if (t.ncol > 0) B = t.ncol;
    const int b0 = ct * TBM;
    if (b0 >= B) return;
    __shared__ C2<T> As[NBUF][MT][KC + 1];
    __shared__ C2<T> Xs[NBUF][KC][TBM + 1];
    // the LDS buffer a chunk is stashed into: with one buffer the stash waits
    // behind a barrier until every wave has finished multiplying the last one
    auto nbuf = [](int b) { return NBUF == 2 ? b : 0; };
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lc = lane & 15, lk = lane >> 4;
    const int wr = (w >> 1) * (MT / 2), wc = (w & 1) * (TBM / 2);
    // (two workgroups per CU are requested: the FP64 64 x 64 tile with three
    // accumulator sets then fits in 256 registers per lane without spilling)
    CAcc<T, HZ_GAUSS3 != 0> acc[RTW][CTW];
#pragma unroll
    for (int a = 0; a < RTW; ++a)
#pragma unroll
        for (int c = 0; c < CTW; ++c) acc[a][c].zero();
    auto multiply = [&](int buf) {
        buf = nbuf(buf);
#pragma unroll
        for (int s4 = 0; s4 < KC / 4; ++s4) {
            C2<T> av[RTW], bv[CTW];
#pragma unroll
            for (int a = 0; a < RTW; ++a) av[a] = As[buf][wr + a * 16 + lc][s4 * 4 + lk];
#pragma unroll
            for (int c = 0; c < CTW; ++c) bv[c] = Xs[buf][s4 * 4 + lk][wc + c * 16 + lc];
#pragma unroll
            for (int a = 0; a < RTW; ++a)
#pragma unroll
                for (int c = 0; c < CTW; ++c)
                    acc[a][c].add(av[a].x, av[a].y, bv[c].x, bv[c].y);
        }
    };
    int sg = 0, kc = -KC;
    next_chunk<T, KC>(t, sg, kc);
    int left = 1 << 30;                          // chunks this workgroup takes
    if (splits > 1) {
        int nch = 0;
        for (int q = 0; q < t.nseg; ++q)
            if (t.seg_ptr[q] && t.seg_len[q] > 0) nch += (t.seg_len[q] + KC - 1) / KC;
        const int cb = (int)((long long)sp * nch / splits);
        left = (int)((long long)(sp + 1) * nch / splits) - cb;
        for (int q = 0; q < cb && sg < t.nseg; ++q) next_chunk<T, KC>(t, sg, kc);
        if (left <= 0) sg = t.nseg;
    }
    GemmCursor<T, MT, TBM, KC> cu;
    // load chunk (s, k), moving the cursor to segment s first if needed
    auto load = [&](GemmStage<T, MT, TBM, KC>& st, int s, int k) {
        if (s != cu.sg) cu.set(t, s, i0, b0, B, tid);
        st.load(cu, k);
    };
    cu.sg = -1;
    if (sg < t.nseg && !DEEP) {
        GemmStage<T, MT, TBM, KC> stage;
        load(stage, sg, kc);
        stage.stash(As[0], Xs[0], tid);
        __syncthreads();
        int buf = 0;
        while (true) {
            int ns = sg, nk = kc;
            next_chunk<T, KC>(t, ns, nk);
            const bool more = ns < t.nseg && left > 1;
            if (more) load(stage, ns, nk);
            multiply(buf);
            if (!more) break;
            if (NBUF == 1) __syncthreads();
            stage.stash(As[nbuf(buf ^ 1)], Xs[nbuf(buf ^ 1)], tid);
            __syncthreads();
            buf ^= 1;
            sg = ns;
            kc = nk;
            --left;
        }
    } else if (sg < t.nseg) {
        // chunk positions: (s0,k0) in LDS, (s1,k1) in registers p, (s2,k2)
        // being loaded into registers q; the two register stages swap roles
        // every chunk (loop unrolled by two so that they keep fixed names)
        GemmStage<T, MT, TBM, KC> p, q;
        // chunk positions are produced in order; after `left` of them the
        // workgroup's share of a split tile is done
        int remaining = left - 1;
        auto nxt = [&](int& s, int& k) {
            if (remaining <= 0) { s = t.nseg; return; }
            --remaining;
            next_chunk<T, KC>(t, s, k);
        };
        load(p, sg, kc);
        p.stash(As[0], Xs[0], tid);
        int s1 = sg, k1 = kc;
        nxt(s1, k1);
        if (s1 < t.nseg) load(p, s1, k1);
        __syncthreads();
        int buf = 0;
        while (true) {
            int s2 = s1, k2 = k1;
            if (s1 < t.nseg) nxt(s2, k2);
            if (s2 < t.nseg) load(q, s2, k2);
            multiply(buf);
            if (s1 >= t.nseg) break;
            if (NBUF == 1) __syncthreads();
            p.stash(As[nbuf(buf ^ 1)], Xs[nbuf(buf ^ 1)], tid);
            __syncthreads();
            buf ^= 1;
            int s3 = s2, k3 = k2;
            if (s2 < t.nseg) nxt(s3, k3);
            if (s3 < t.nseg) load(p, s3, k3);
            multiply(buf);
            if (s2 >= t.nseg) break;
            if (NBUF == 1) __syncthreads();
            q.stash(As[nbuf(buf ^ 1)], Xs[nbuf(buf ^ 1)], tid);
            __syncthreads();
            buf ^= 1;
            s1 = s3;
            k1 = k3;
        }
    }
    if (splits > 1) {
        constexpr int NV = RTW * CTW * 4;
        const long long tile_id = ((long long)task * row_tiles + rt) * col_tiles + ct;
        C2<T>* mine = ws + ((tile_id * splits + sp) * GV_THREADS + tid) * NV;
#pragma unroll
        for (int a = 0; a < RTW; ++a)
#pragma unroll
            for (int c = 0; c < CTW; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    gstore<T>(mine + (a * CTW + c) * 4 + v, mk<T>(acc[a][c].re(v), acc[a][c].im(v)));
        return;
    }
    if constexpr (RTW * CTW == 1) {
        // 32 x 32 tiles (short launches of the sweeps): the epilogue reads
        // of the thread's four entries are issued together before the stores
        C2<T>* dst[4];
        C2<T> ad0[4], ad1[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = i0 + wr + Mf<T>::row(lane, v);
            const int b = b0 + wc + lc;
            dst[v] = nullptr;
            ad0[v] = mk<T>((T)0, (T)0);
            ad1[v] = mk<T>((T)0, (T)0);
            if (i >= t.m || b >= B) continue;
            for (int sg = 0; sg < t.noseg; ++sg) {
                const int rel = i - t.oseg_i0[sg];
                if (rel < 0 || rel >= t.oseg_len[sg]) continue;
                const long long off = (long long)rel * t.ldo + b;
                dst[v] = t.oseg_ptr[sg] + off;
                if (t.oseg_add0[sg]) ad0[v] = gload<T>(t.oseg_add0[sg] + off);
                if (t.oseg_add1[sg]) ad1[v] = cscale(gload<T>(t.oseg_add1[sg] + off), t.c1[sg]);
                break;
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (dst[v])
                gstore<T>(dst[v], cadd(cadd(cscale(mk<T>(acc[0][0].re(v), acc[0][0].im(v)), t.alpha),
                                            ad0[v]), ad1[v]));
        return;
    }
#pragma unroll
    for (int a = 0; a < RTW; ++a)
#pragma unroll
        for (int c = 0; c < CTW; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wr + a * 16 + Mf<T>::row(lane, v);
                const int b = b0 + wc + c * 16 + lc;
                if (i < t.m && b < B) epilogue<T>(t, i, b, mk<T>(acc[a][c].re(v), acc[a][c].im(v)));
            }
}

// Second pass of split k: one workgroup per output tile; thread tid adds, in
// split order, the partial accumulators that thread tid of each split
// workgroup stored (same register-to-element map as k_gemm_mfma) and applies
// the task's epilogue (same arithmetic order as the unsplit kernels).  All
// partial loads of a thread are issued before the sums and all epilogue reads
// before the stores, instead of two dependent round trips per entry.
template <typename T, int MT, int TBM>
__global__ void __launch_bounds__(GV_THREADS)
k_gemm_split_reduce(const GemmTask<T>* __restrict__ tasks, int B, int row_tiles, int col_tiles,
                    int splits, const C2<T>* __restrict__ ws) {
    constexpr int RTW = MT / 32, CTW = TBM / 32, NV = RTW * CTW * 4;
    constexpr int SMAX = 8;                      // largest split of the split kinds
    const int per_task = row_tiles * col_tiles;
    const int tile = blockIdx.x;
    const int task = tile / per_task, rc = tile - task * per_task;
    const int rt = rc / col_tiles, ct = rc - rt * col_tiles;
    const GemmTask<T>& t = tasks[task];
    const int i0 = rt * MT;
    if (i0 >= t.m) return;
    if (t.ncol > 0) B = t.ncol;
    const int b0 = ct * TBM;
    if (b0 >= B) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int lc = lane & 15;
    const int wr = (w >> 1) * (MT / 2), wc = (w & 1) * (TBM / 2);
    const C2<T>* base = ws + (long long)tile * splits * GV_THREADS * NV + (long long)tid * NV;
    const long long sstride = (long long)GV_THREADS * NV;
    C2<T> sum[NV];
#pragma unroll
    for (int e = 0; e < NV; ++e) sum[e] = gload<T>(base + e);
#pragma unroll
    for (int q = 1; q < SMAX; ++q) {
        if (q >= splits) break;
        C2<T> part[NV];
#pragma unroll
        for (int e = 0; e < NV; ++e) part[e] = gload<T>(base + q * sstride + e);
#pragma unroll
        for (int e = 0; e < NV; ++e) sum[e] = cadd(sum[e], part[e]);
    }
    // epilogue: output segment and offset of every entry, then the adds
    C2<T>* dst[NV];
    C2<T> ad0[NV], ad1[NV];        // add0 and c1 * add1 of each entry (zero when absent)
#pragma unroll
    for (int a = 0; a < RTW; ++a)
#pragma unroll
        for (int c = 0; c < CTW; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int e = (a * CTW + c) * 4 + v;
                const int i = i0 + wr + a * 16 + Mf<T>::row(lane, v);
                const int b = b0 + wc + c * 16 + lc;
                dst[e] = nullptr;
                ad0[e] = mk<T>((T)0, (T)0);
                ad1[e] = mk<T>((T)0, (T)0);
                if (i >= t.m || b >= B) continue;
                for (int sg = 0; sg < t.noseg; ++sg) {
                    const int rel = i - t.oseg_i0[sg];
                    if (rel < 0 || rel >= t.oseg_len[sg]) continue;
                    const long long off = (long long)rel * t.ldo + b;
                    dst[e] = t.oseg_ptr[sg] + off;
                    if (t.oseg_add0[sg]) ad0[e] = gload<T>(t.oseg_add0[sg] + off);
                    if (t.oseg_add1[sg]) ad1[e] = cscale(gload<T>(t.oseg_add1[sg] + off), t.c1[sg]);
                    break;
                }
            }
#pragma unroll
    for (int e = 0; e < NV; ++e)
        if (dst[e]) gstore<T>(dst[e], cadd(cadd(cscale(sum[e], t.alpha), ad0[e]), ad1[e]));
}

template <typename T>
__global__ void k_copy(C2<T>* __restrict__ y, const C2<T>* __restrict__ x, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        y[i] = x[i];
}

template <typename T>
void launch_copy(C2<T>* y, const C2<T>* x, long long n, hipStream_t st) {
    if (n <= 0) return;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_copy<T>), dim3(blocks), dim3(256), 0, st, y, x, n);
}
template void launch_copy<double>(double2*, const double2*, long long, hipStream_t);
template void launch_copy<float>(float2*, const float2*, long long, hipStream_t);

// which kernel launch_gemm runs for a launch of this shape
GemmKernel gemm_kernel(int ntasks, int max_m, int B) {
    if (B == 1) return GEMM_GEMV;
    if (B < 16) return GEMM_TILED;
    const long long big = (long long)ntasks * ((max_m + 63) / 64) * ((B + 63) / 64);
    return (B >= 64 && big >= 512) ? GEMM_MFMA64 : GEMM_MFMA32;
}

const char* gemm_kernel_name(GemmKernel k) {
    switch (k) {
    case GEMM_GEMV: return "gemv";
    case GEMM_TILED: return "gemm_tiled";
    case GEMM_MFMA64: return "gemm_mfma64";
    case GEMM_MFMA32K16: return "gemm_mfma32k16";
    case GEMM_MFMA32D: return "gemm_mfma32d";
    case GEMM_MFMA64D: return "gemm_mfma64d";
    case GEMM_MFMA32X64: return "gemm_mfma32x64";
    case GEMM_MFMA64X32: return "gemm_mfma64x32";
    case GEMM_MFMA64S2: return "gemm_mfma64s2";
    case GEMM_MFMA64S4: return "gemm_mfma64s4";
    case GEMM_MFMA32S2: return "gemm_mfma32s2";
    case GEMM_MFMA32S4: return "gemm_mfma32s4";
    case GEMM_MFMA32S8: return "gemm_mfma32s8";
    case GEMM_MFMA64S8: return "gemm_mfma64s8";
    case GEMM_MFMA32X64S4: return "gemm_mfma32x64s4";
    case GEMM_MFMA32X64S8: return "gemm_mfma32x64s8";
    case GEMM_MFMA32DS4: return "gemm_mfma32ds4";
    case GEMM_MFMA32DS8: return "gemm_mfma32ds8";
    default: return "gemm_mfma32";
    }
}

template <typename T, bool OFFLINE>
void launch_gemm_mfma(GemmKernel kind, const GemmTask<T>* tasks_dev, int ntasks, int max_m, int B,
                      hipStream_t st, const GemmSplitWs* sw) {
    // split k: pass 1 stores each workgroup's partial tile, pass 2 adds them
    int splits = 0, mt = 0, tbm = 0;
    switch (kind) {
    case GEMM_MFMA64S2: splits = 2; mt = 64; tbm = 64; break;
    case GEMM_MFMA64S4: splits = 4; mt = 64; tbm = 64; break;
    case GEMM_MFMA64S8: splits = 8; mt = 64; tbm = 64; break;
    case GEMM_MFMA32S2: splits = 2; mt = 32; tbm = 32; break;
    case GEMM_MFMA32S4: splits = 4; mt = 32; tbm = 32; break;
    case GEMM_MFMA32S8: splits = 8; mt = 32; tbm = 32; break;
    case GEMM_MFMA32X64S4: splits = 4; mt = 32; tbm = 64; break;
    case GEMM_MFMA32X64S8: splits = 8; mt = 32; tbm = 64; break;
    case GEMM_MFMA32DS4: splits = 4; mt = 32; tbm = 32; break;
    case GEMM_MFMA32DS8: splits = 8; mt = 32; tbm = 32; break;
    default: break;
    }
    const bool deep = kind == GEMM_MFMA32DS4 || kind == GEMM_MFMA32DS8;
    if (splits > 0) {
        const int rt = (max_m + mt - 1) / mt, ct = (B + tbm - 1) / tbm;
        const long long tiles = (long long)rt * ct * ntasks;
        const long long need = tiles * splits * (long long)mt * tbm * (long long)sizeof(C2<T>);
        if (sw && sw->ws && need <= sw->ws_bytes) {
            C2<T>* ws = (C2<T>*)sw->ws;
            const dim3 g1((unsigned)(tiles * splits)), g2((unsigned)tiles), blk(GV_THREADS);
            if (mt == 64) {
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 64, 64, 16, OFFLINE>), g1, blk, 0,
                                   st, tasks_dev, B, rt, ct, splits, ws);
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_split_reduce<T, 64, 64>), g2, blk, 0, st,
                                   tasks_dev, B, rt, ct, splits, (const C2<T>*)ws);
            } else if (tbm == 64) {
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 32, 64, 32, OFFLINE>), g1, blk, 0,
                                   st, tasks_dev, B, rt, ct, splits, ws);
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_split_reduce<T, 32, 64>), g2, blk, 0, st,
                                   tasks_dev, B, rt, ct, splits, (const C2<T>*)ws);
            } else {
                if (deep)
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 32, 32, 32, OFFLINE, true, 1>), g1,
                                       blk, 0, st, tasks_dev, B, rt, ct, splits, ws);
                else
                    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 32, 32, 32, OFFLINE, false, 1>), g1,
                                       blk, 0, st, tasks_dev, B, rt, ct, splits, ws);
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_split_reduce<T, 32, 32>), g2, blk, 0, st,
                                   tasks_dev, B, rt, ct, splits, (const C2<T>*)ws);
            }
            return;
        }
        // no room for the partial tiles: the unsplit kernel of the same tile
        kind = mt == 64 ? GEMM_MFMA64 : tbm == 64 ? GEMM_MFMA32X64 : deep ? GEMM_MFMA32D : GEMM_MFMA32;
    }
    // big launches: 64 x 64 tiles; otherwise 32 x 32 tiles with deeper
    // chunks, which keep more workgroups busy and fewer chunks in flight
    if (kind == GEMM_MFMA64) {
        const int rt = (max_m + 63) / 64, ct = (B + 63) / 64;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 64, 64, 16, OFFLINE>),
                           dim3(rt * ct * ntasks), dim3(GV_THREADS), 0, st, tasks_dev, B, rt, ct, 1,
                           (C2<T>*)nullptr);
    } else if (kind == GEMM_MFMA32K16) {
        const int rt = (max_m + 31) / 32, ct = (B + 31) / 32;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 32, 32, 16, OFFLINE>),
                           dim3(rt * ct * ntasks), dim3(GV_THREADS), 0, st, tasks_dev, B, rt, ct, 1,
                           (C2<T>*)nullptr);
    } else if (kind == GEMM_MFMA32X64) {
        const int rt = (max_m + 31) / 32, ct = (B + 63) / 64;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 32, 64, 32, OFFLINE>),
                           dim3(rt * ct * ntasks), dim3(GV_THREADS), 0, st, tasks_dev, B, rt, ct, 1,
                           (C2<T>*)nullptr);
    } else if (kind == GEMM_MFMA64X32) {
        const int rt = (max_m + 63) / 64, ct = (B + 31) / 32;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 64, 32, 32, OFFLINE>),
                           dim3(rt * ct * ntasks), dim3(GV_THREADS), 0, st, tasks_dev, B, rt, ct, 1,
                           (C2<T>*)nullptr);
    } else if (kind == GEMM_MFMA32D) {
        const int rt = (max_m + 31) / 32, ct = (B + 31) / 32;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 32, 32, 32, OFFLINE, true, 1>),
                           dim3(rt * ct * ntasks), dim3(GV_THREADS), 0, st, tasks_dev, B, rt, ct, 1,
                           (C2<T>*)nullptr);
    } else if (kind == GEMM_MFMA64D) {
        const int rt = (max_m + 63) / 64, ct = (B + 63) / 64;
        constexpr int KCD = sizeof(T) == 4 ? 32 : 16;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 64, 64, KCD, OFFLINE, true>),
                           dim3(rt * ct * ntasks), dim3(GV_THREADS), 0, st, tasks_dev, B, rt, ct, 1,
                           (C2<T>*)nullptr);
    } else {
        const int rt = (max_m + 31) / 32, ct = (B + 31) / 32;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_mfma<T, 32, 32, 32, OFFLINE, false, 1>),
                           dim3(rt * ct * ntasks), dim3(GV_THREADS), 0, st, tasks_dev, B, rt, ct, 1,
                           (C2<T>*)nullptr);
    }
}

template <typename T>
void launch_gemm(const GemmTask<T>* tasks_dev, int ntasks, int max_m, int B, hipStream_t st,
                 bool offline, int kind_choice, const GemmSplitWs* sw) {
    if (ntasks <= 0 || max_m <= 0) return;
    GemmKernel kind = gemm_kernel(ntasks, max_m, B);
    if (kind_choice >= GEMM_MFMA32 && kind >= GEMM_MFMA32) kind = (GemmKernel)kind_choice;
    if (kind == GEMM_GEMV) {
        dim3 grid((max_m + GV_ROWS - 1) / GV_ROWS, 1, ntasks);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemv<T>), grid, dim3(GV_THREADS), 0, st, tasks_dev);
    } else if (kind == GEMM_TILED) {
        dim3 grid((max_m + TM - 1) / TM, (B + TB - 1) / TB, ntasks);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_gemm_tiled<T>), grid, dim3(GV_THREADS), 0, st,
                           tasks_dev, B);
    } else if (offline) {
        launch_gemm_mfma<T, true>(kind, tasks_dev, ntasks, max_m, B, st, sw);
    } else {
        launch_gemm_mfma<T, false>(kind, tasks_dev, ntasks, max_m, B, st, sw);
    }
}

template void launch_gemm<double>(const GemmTask<double>*, int, int, int, hipStream_t, bool, int,
                                  const GemmSplitWs*);
template void launch_gemm<float>(const GemmTask<float>*, int, int, int, hipStream_t, bool, int,
                                 const GemmSplitWs*);

}  // namespace hz
