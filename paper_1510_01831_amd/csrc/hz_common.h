// Internal declarations shared by the HIP kernels and the host orchestration.
//
// Storage conventions (all device arrays):
//  * complex numbers are interleaved (double2 / float2);
//  * every online vector is stored "batch fastest": element (i, b) of a batch
//    of B vectors lives at [i * B + b];
//  * a cell grid is stored column by column (x slowest): node (row j, col k)
//    at [k * HL + j], because the cell factorisation eliminates whole columns;
//  * dense operators are row-major.
#pragma once
#include <algorithm>
#include <cstdlib>

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace hz {

template <typename T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <typename T> using C2 = typename cplx_t<T>::type;

template <typename T> __host__ __device__ inline C2<T> mk(T x, T y) { C2<T> r; r.x = x; r.y = y; return r; }
template <typename C> __host__ __device__ inline C cadd(C a, C b) { C r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename C> __host__ __device__ inline C csub(C a, C b) { C r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename C> __host__ __device__ inline C cmul(C a, C b) {
    C r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// c + a * b
template <typename C> __host__ __device__ inline C cfma(C a, C b, C c) {
    C r; r.x = c.x + a.x * b.x - a.y * b.y; r.y = c.y + a.x * b.y + a.y * b.x; return r;
}
template <typename C> __host__ __device__ inline C cconj(C a) { C r; r.x = a.x; r.y = -a.y; return r; }
template <typename C, typename S> __host__ __device__ inline C cscale(C a, S s) { C r; r.x = a.x * s; r.y = a.y * s; return r; }

// alpha = 1/(1 + i beta (d/delta)^2) at a (possibly half-integer) position of
// an axis whose own nodes are 1..n_own (quadratic PML of App. A with
// C = beta omega delta; sigma = 0 on the closed physical interval).
__host__ __device__ inline double2 pml_alpha(double pos, int n_own, int p, double beta) {
    double2 r; r.x = 1.0; r.y = 0.0;
    if (p == 0) return r;
    double d = pos < 0.0 ? -pos : 0.0;
    double dr = pos - (n_own + 1);
    if (dr > d) d = dr;
    d /= p;
    double s = beta * d * d;
    double den = 1.0 / (1.0 + s * s);
    r.x = den; r.y = -s * den;
    return r;
}

__host__ __device__ inline double2 cinv(double2 a) {
    double den = 1.0 / (a.x * a.x + a.y * a.y);
    double2 r; r.x = a.x * den; r.y = -a.y * den; return r;
}

// ---------------------------------------------------------------------------
// descriptors (plain structs, copied to the device)

constexpr int MAXSLOT = 4;
constexpr int MISFIT_PARTS = 256;
// Workgroup slot L of a 1-D launch runs on XCD L mod 8 (round-robin
// dispatch).  xcd_tile maps slots to work items so that each XCD gets one
// contiguous run of the item sequence: items next to each other in that
// sequence (the tiles that share operands, the batch chunks of one cell)
// run on one XCD at about the same time and share its L2.
__device__ __forceinline__ int xcd_tile(int L, int total) {
    const int xcd = L & 7, local = L >> 3;
    const int q = total >> 3, r = total & 7;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + local;
}

// Status of the block inversions of a factorisation.  A block is reported
// singular when a pivot is exactly zero or when its smallest pivot magnitude
// is at most PIVOT_RATIO_MIN times its largest (partial pivoting: the pivots
// bound the block's condition from below, and a ratio below 2^-26 leaves
// fewer than half of the FP64 digits); min_ratio_bits holds the smallest
// ratio seen, as the bits of a non-negative double (atomicMin order).
struct FactorFlags {
    int singular;
    int pad;
    unsigned long long min_ratio_bits;
};
constexpr double PIVOT_RATIO_MIN = 1.4901161193847656e-08;   // 2^-26   // workgroups (and partial sums) of k_misfit

struct LayerDesc {
    int index;           // 0-based layer index
    int first, last;     // owned physical rows (1-based, global)
    int nl, HL;          // owned physical rows, grid rows (nl + 2 p)
    int row0;            // extended-grid array row of local array row 0 (= first - 1)
    int own_r0, own_r1;  // owned local array rows (inclusive)
    int has_top, has_bot;
    int nslot;           // interface rows of this layer (0, 2 or 4)
    int slot_row[MAXSLOT];   // stored slot -> local array row
    int slot_id[MAXSLOT];    // stored slot -> logical slot (0 top-a, 1 top-b, 2 bot-a, 3 bot-b)
    int slot_of[MAXSLOT];    // logical slot -> stored slot or -1
    int cell_begin;      // global index of the layer's first cell
    int J;               // inner interfaces (cells - 1)
    long long off_Sinv;  // inner LU: Sinv_j [2HL][2HL], j < J
    long long off_Lfac;  // L_j^a [HL][2HL], j = 1..J-1 (slot j-1)
    long long off_inner; // offset (complex elements, per batch column) of the layer's inner vector
};

struct CellDesc {
    int layer, cell, gidx;   // layer index, cell index in the layer, global cell index
    int HL, Wc, nc;          // grid rows, grid columns, owned physical columns
    int HLp;                 // HL rounded up to a multiple of 16 (padded factor blocks)
    int first;               // first owned physical column (1-based, global)
    int col0;                // extended-grid array column of cell-local array column 0
    int own_c0, own_c1, s;   // owned cell-local array columns (inclusive), count
    int has_left, has_right, adj;
    int nslot;               // = layer nslot
    int ncol;                // column probes = adj * 2 HL
    int R;                   // probes = ncol + nslot * s
    long long off_coef;      // diag/cz/e: [Wc][HL] each
    long long off_X;         // X_k = S_k^{-1}: [Wc][HLp x HLp in 16x4 MFMA tiles, see xt_index]
    long long off_Q;         // Q = [M_u | D_loc]: [nslot * s][R]
    long long off_CS;        // column samples: [adj * HL][R] (left side first)
    long long off_CP;        // pair-column samples (nested polarized traces): [adj * 2 HL][R],
                             // left pair (positions 0, 1) first, then the right pair (n_c, n_c + 1)
};

struct Dims {
    int n, p, W, L, Lc, K;   // K = L - 1 interfaces
    double h, omega, beta;
    int HLmax, Wcmax, HLpmax;
};

// A device pointer seen as a global-memory pointer, so that accesses compile
// to global_load / global_store.  Pointers read from a task table are
// otherwise generic, and a generic (flat) access also counts against the LDS
// wait counter: every LDS wait would then wait for the prefetch loads too.
template <typename T>
__device__ __forceinline__ C2<T> gload(const C2<T>* p) {
    using V = T __attribute__((ext_vector_type(2)));
    const V v = *(const __attribute__((address_space(1))) V*)p;
    return mk<T>(v.x, v.y);
}
template <typename T>
__device__ __forceinline__ void gstore(C2<T>* p, C2<T> v) {
    using V = T __attribute__((ext_vector_type(2)));
    V w;
    w.x = v.x;
    w.y = v.y;
    *(__attribute__((address_space(1))) V*)p = w;
}

// Position of entry (i, j) of an HLp x HLp Schur inverse stored as 16x4 tiles
// in MFMA operand order: tile (i/16, j/4), lane (i%16) + 16 (j%4).  A wave
// reads one tile as 1 KB of contiguous complex values.
__host__ __device__ inline long long xt_index(int i, int j, int HLp) {
    return (((long long)(i >> 4) * (HLp >> 2) + (j >> 2)) << 6) + (i & 15) + ((j & 3) << 4);
}

// ---------------------------------------------------------------------------
// generic segmented GEMM:  out[i] = add0[i] + c1 * add1[i] + alpha * sum_k A[i][k] x[k]
// for one right-hand-side batch; x rows come from up to NSEG contiguous
// segments, output rows go to up to NOSEG contiguous segments.

constexpr int NSEG = 6;
constexpr int NOSEG = 4;

// Partitioned low-rank form of an operator block (k_plr.hip): square tiles
// of PLR_TILE, each dense (column-major, rank -1), zero (rank 0) or the
// factors U (tr x r) then W (r x tc), both column-major, at `off` complex
// elements into the pool.  Ranks above PLR_RMAX are stored dense.
constexpr int PLR_TILE = 64;
constexpr int PLR_RMAX = 32;
struct PlrTile {
    int block;           // index of the block (offline compression only)
    int i0, j0, tr, tc;  // tile origin and size in the block
    int rank;
    long long off;
};
template <typename T>
struct PlrBlock {        // a dense block to compress: row-major, row stride lda
    const C2<T>* A;
    long long lda;
};

template <typename T>
struct GemmTask {
    const C2<T>* A;      // row-major, row stride lda
    long long lda;
    int m, k;            // rows, columns (k counts the gathered x rows)
    int nseg;
    int seg_k0[NSEG];
    int seg_len[NSEG];
    const C2<T>* seg_ptr[NSEG];   // x row r of the segment at seg_ptr + r * ldx (NULL = zeros)
    int noseg;
    int oseg_i0[NOSEG];
    int oseg_len[NOSEG];
    C2<T>* oseg_ptr[NOSEG];
    const C2<T>* oseg_add0[NOSEG];
    const C2<T>* oseg_add1[NOSEG];
    T c1[NOSEG];
    T alpha;
    long long ldx;       // row stride of every x segment (complex elements)
    long long ldo;       // row stride of the output / add0 / add1 segments
    int ncol;            // batch columns of this task (0 = the launch's B)
    // PLR form of A (single-RHS launches of the preconditioner), or NULL:
    // plr_ntr x plr_ntc tiles, row-major, factors in plr_pool
    const PlrTile* plr;
    const C2<T>* plr_pool;
    int plr_ntr, plr_ntc;
    long long plr_part;  // first tile of this task in the launch's partial-product scratch
};

// Workspace of the split-k variants: partial tiles (bytes).
struct GemmSplitWs {
    void* ws = nullptr;              // partial tiles of the split-k variants
    long long ws_bytes = 0;
};

// ---------------------------------------------------------------------------
// cell solve (Schur recursion) arguments

enum SolveMode { SOLVE_GRID = 0, SOLVE_PROBE = 1, SOLVE_SAMPLE = 2, SOLVE_VOLUME = 3 };

template <typename T>
struct CellSolveArgs {
    int mode;
    int B;               // batch columns handled in total (per cell)
    int nb;              // batch columns per workgroup (cs_nb)
    const CellDesc* cells;
    const LayerDesc* layers;
    const int* cell_list;        // cells handled by this launch (grid.x index -> global cell)
    const C2<T>* X;              // factor pool
    const C2<T>* coef_e;         // e pool (same layout as coef, complex)
    const double2* alpha_x;      // per cell: alpha_x at own nodes [Wcmax] (cell profile), FP64
    const double2* alpha_z;      // per layer: alpha_z at nodes [HLmax], FP64
    C2<T>* Y;                    // scratch for the forward sweep: per workgroup [Wc][HLp][NB]
    long long y_stride;          // complex elements per launch-cell in Y
    // SOLVE_GRID: g/x on the cell grid [HL][Wc][B] (row-major grid) for one cell
    const C2<T>* g_grid; C2<T>* x_grid;
    // SOLVE_PROBE: outputs Q (row samples) and CS (column samples) into the pools,
    // and the pair-column samples into CPpool when it is set
    C2<T>* Qpool; C2<T>* CSpool; C2<T>* CPpool;
    int probe0;                  // first probe handled (chunking over R)
    // SOLVE_SAMPLE / SOLVE_VOLUME: volume source on the extended grid [W][W][B] (or NULL)
    const C2<T>* f_ext;
    const int* layer_active;     // per layer: source present (may be NULL = all)
    // interface-row sources (reconstruction): polarized-style pairs per layer,
    // top pair / bottom pair pointers given per layer through a table
    const C2<T>* const* top_pair;   // [L] -> [2][W][B] or NULL
    const C2<T>* const* bot_pair;   // [L] -> [2][W][B] or NULL
    const C2<T>* inner_v;        // inner traces (column sources), base of per-layer vectors
    long long inner_ld;          // per-layer stride in complex elements (J*2*HLmax*B)
    // outputs
    C2<T>* inner_rhs;            // SOLVE_SAMPLE: column samples -> inner rhs (per layer)
    int inner_pol;               // SOLVE_SAMPLE: inner rhs of the polarized inner system
                                 // ([d|q][J][2][HL][B] per layer, stride 2 J 2 HLmax B)
    C2<T>* rows_out;             // SOLVE_SAMPLE: row samples [L][nslot=4][W][B]
    C2<T>* u_ext;                // SOLVE_VOLUME: [W][W][B]
    double h;
    int n, p, W, HLmax, Wcmax;
};

// ---------------------------------------------------------------------------
// launchers (defined in the .hip files)

void launch_check_model(const double* model, long long count, int* bad_flag, hipStream_t st);

void launch_build_coef(const double* model, int model_kind, const Dims& d,
                       const CellDesc* cells_dev, const LayerDesc* layers_dev, int ncells,
                       const CellDesc* cells_host, double2* diag, double2* cz, double2* e,
                       double2* ax_pool, double2* az_pool, double2* gdiag, double2* gcx,
                       double2* gcz, double2* wext, int* bad_flag, hipStream_t st);

template <typename T>
void launch_cell_factor(const CellDesc* cells_dev, int ncells, const Dims& d,
                        const double2* diag, const double2* cz, const double2* e,
                        C2<T>* Xpool, C2<T>* work, long long work_stride, FactorFlags* ff,
                        hipStream_t st);

template <typename T>
void launch_invert_batch(C2<T>* const* mats, C2<T>* const* outs, const int* ns, int count,
                         C2<T>* work, long long work_stride, FactorFlags* ff, hipStream_t st);

template <typename T>
void launch_cell_solve(const CellSolveArgs<T>& a, int ncells_launch, int nb_chunks,
                       hipStream_t st);

// PLR compression and application (k_plr.hip)
template <typename T>
void launch_plr_tile_norms(const PlrBlock<T>* blocks, const PlrTile* tiles, int ntiles,
                           double* norm2, hipStream_t st);
template <typename T>
void launch_plr_compress(const PlrBlock<T>* blocks, const PlrTile* tiles, int ntiles,
                         const double* delta2, int* ranks, C2<T>* pool, int write,
                         hipStream_t st);
// part: PLR_TILE partial entries per tile, a task's tiles from its plr_part
template <typename T>
void launch_plr_apply(const GemmTask<T>* tasks_dev, int ntasks, int max_tiles, int max_rows,
                      C2<T>* part, hipStream_t st);

// B = number of batch columns; ldx/ldo come from the tasks.
// offline = launch from the factorisation stage (separate kernel instance);
// kind_choice = a matrix-core variant picked by the autotuner (-1: default)
template <typename T>
void launch_gemm(const GemmTask<T>* tasks_dev, int ntasks, int max_m, int B, hipStream_t st,
                 bool offline = false, int kind_choice = -1, const GemmSplitWs* sw = nullptr);

// the GEMM kernel launch_gemm selects for a shape (for per-kernel profiles);
// the matrix-core variants are 64x64 tiles / 16-deep chunks, 32x32 / 32-deep
// and 32x32 / 16-deep
// GEMM_MFMA32D / GEMM_MFMA64D: the 32x32 and 64x64 tiles with two chunks of
// loads in flight (64x64 with 32-deep chunks in complex64).
// GEMM_MFMA32X64 / GEMM_MFMA64X32: 32 x 64 and 64 x 32 output tiles (rows x
// batch columns), 32-deep chunks.
// GEMM_MFMA64S2 / GEMM_MFMA64S4: 64x64 tiles with the k chunks of a tile split
// over 2 / 4 workgroups that store partial tiles, then a reduction kernel
// (needs a GemmSplitWs large enough; otherwise GEMM_MFMA64).
// GEMM_MFMA32S2 / S4 / S8: the same split over 32x32 tiles, 32-deep chunks
// (short launches with long k: more workgroups per output tile);
// GEMM_MFMA64S8, GEMM_MFMA32X64S4 / S8: 64x64 and 32 x 64 tiles split 8 / 4 / 8
// ways; GEMM_MFMA32DS4 / DS8: 32x32 tiles with two chunks in flight, split
// 4 / 8 ways.
enum GemmKernel { GEMM_GEMV = 0, GEMM_TILED = 1, GEMM_MFMA32 = 2, GEMM_MFMA64 = 3,
                  GEMM_MFMA32K16 = 4, GEMM_MFMA32D = 5, GEMM_MFMA64D = 6,
                  GEMM_MFMA32X64 = 7, GEMM_MFMA64X32 = 8, GEMM_MFMA64S2 = 9,
                  GEMM_MFMA64S4 = 10, GEMM_MFMA32S2 = 11, GEMM_MFMA32S4 = 12,
                  GEMM_MFMA32S8 = 13, GEMM_MFMA64S8 = 14, GEMM_MFMA32X64S4 = 15,
                  GEMM_MFMA32X64S8 = 16, GEMM_MFMA32DS4 = 17, GEMM_MFMA32DS8 = 18 };

GemmKernel gemm_kernel(int ntasks, int max_m, int B);
const char* gemm_kernel_name(GemmKernel k);

template <typename T>
void launch_copy(C2<T>* y, const C2<T>* x, long long n, hipStream_t st);

// number of right-hand sides one cell-solve workgroup handles for a batch B:
// the largest value, used to size the per-workgroup scratch
inline int cs_nb_cap(int B) {
    if (B <= 1) return 1;
    if (B <= 2) return 2;
    if (B <= 4) return 4;
    return B <= 16 ? 16 : 32;
}

// and the value used for a launch of `ncells` cells whose largest padded
// height is `hlp` (elements of `elem` bytes).  With few cells, 16 columns
// instead of 32 doubles the workgroups and halves each one's sequential work;
// cells taller than 160 rows keep 16 columns (two row tiles per wave leave no
// registers for 32), and so do FP64 cells taller than 128 rows (the ten-wave
// kernel has 170 registers per lane).
// HZ_CELL_NB overrides the choice (1, 2, 4, 16 or 32; clamped to the cap).
inline int cs_nb_max(int hlp, int elem) {
    return (hlp > 160 || (elem > 8 && hlp > 128)) ? 16 : 32;
}
inline int cs_nb(int B, int ncells, int hlp, int elem) {
    int nb = cs_nb_cap(B);
    if (nb == 32 && ((long long)ncells * ((B + 31) / 32) < 512 || cs_nb_max(hlp, elem) < 32))
        nb = 16;
    if (const char* e = std::getenv("HZ_CELL_NB")) {
        const int o = std::atoi(e);
        if (o == 1 || o == 2 || o == 4 || o == 16 || o == 32)
            nb = std::min(std::min(o, cs_nb_cap(B)), cs_nb_max(hlp, elem));
    }
    return nb;
}

// vector / reduction kernels (FP64 unless templated)
template <typename T>
void launch_axpby(C2<T>* y, const C2<T>* x, double2 a, double2 b, long long n, hipStream_t st);
void launch_cast_d2f(float2* y, const double2* x, long long n, hipStream_t st);
void launch_cast_f2d(double2* y, const float2* x, long long n, hipStream_t st,
                     double2* y2 = nullptr);
void launch_dots(const double2* V, long long vstride, int nv, const double2* w, long long n,
                 int B, double2* partial, int nchunks, hipStream_t st);
void launch_reduce_partials(const double2* partial, int nchunks, int count, double2* out,
                            hipStream_t st);
void launch_lincomb3(double2* out, const double2* x0, const double2* x1, const double2* x2,
                     const double2* coef, long long n, int B, hipStream_t st);
void launch_fill_zero(double2* y, long long n, hipStream_t st);
void launch_update_basis(double2* w, const double2* V, long long vstride, int nv,
                         const double2* coef, long long n, int B, hipStream_t st,
                         double sgn = 1.0);
void launch_scale_cols(double2* y, const double2* x, const double2* s, long long n, int B,
                       hipStream_t st, double2* y2 = nullptr);
void launch_scale_cols_inv_norm(double2* y, double2* y2, const double2* x, const double2* n2,
                                long long n, int B, hipStream_t st);
void launch_norms(const double2* w, long long n, int B, double2* partial, int nchunks,
                  hipStream_t st);
// w += sgn * V coef, then partial sums of V^H w (norm = 0) or |w|^2 (norm = 1);
// false (nothing launched) when nv is outside 1..8
bool launch_update_dots(double2* w, const double2* V, long long vstride, int nv,
                        const double2* coef, double sgn, long long n, int B, int norm,
                        double2* partial, int nchunks, hipStream_t st);
void launch_rhs_to_ext(const double2* rhs, int B, int n, int p, int W, double2* f_ext,
                       const LayerDesc* layers_dev, int L, int* layer_active, hipStream_t st);
void launch_ext_to_out(const double2* u_ext, int B, int n, int p, int W, double2* out,
                       int physical, int conj, hipStream_t st);
// (sum |f - H u|^2, sum |f|^2) per column over node ranges -> partial[nblocks][B]
// (needs 16 B bytes of LDS)
int residual_norms_blocks(int W, int B, int cap);
void launch_residual_norms(const double2* u, const double2* f, const double2* gdiag,
                           const double2* gcx, const double2* gcz, int W, int B, double2* partial,
                           int nblocks, hipStream_t st);
void launch_residual(const double2* u, const double2* f, double2* r, const double2* gdiag,
                     const double2* gcx, const double2* gcz, int W, int B, int layout_bfast,
                     hipStream_t st);
void launch_misfit_grad(const double2* u, const double2* lam, int B, int W, int n, int p,
                        const double2* wext, double omega, double* g, hipStream_t st);
void launch_misfit(const double2* u_ext, const double2* d_obs, int rec_row, int B, int n, int p,
                   int W, double2* adj, double* Jpart, hipStream_t st);
void launch_conj_copy(double2* y, const double2* x, long long n, hipStream_t st);
void launch_transpose_bfast(const double2* src, double2* dst, int B, long long n, int to_bfast,
                            hipStream_t st);

}  // namespace hz
