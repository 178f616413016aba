// Host orchestration of the nested polarized-traces solver behind the C-ABI
// of include/hz.h.
//
//  hz_setup   -- partitions (layers, cells, Sec. 4 / Fig. 5), coefficients (App. A)
//  hz_factor  -- cell Schur factors, cell Green's-function probes giving the
//                interface operators of eq. factorization, inner block LU
//                (Sec. 4.2.2)
//  hz_solve   -- Alg. 6: RHS formation (Alg. 7 volume mode in the layers that
//                hold sources), GMRES on P^GS M (Sec. 3.1), reconstruction
//                (Alg. 7 volume mode in every layer).  HZ_MIXED applies the
//                preconditioner with complex64 operators inside flexible
//                GMRES; HZ_MIXED_REFINE runs the whole solve in complex64
//                inside an FP64 iterative refinement on the volume.
//
// Every dense operator application is a list of GemmTask records executed by
// the segmented GEMM kernels; the lists of the GMRES operators (M and P^GS)
// are built once per batch size ("plans") and replayed.
#include "hz.h"
#include "hz_common.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

using namespace hz;

namespace {

thread_local std::string g_err;

struct HzError {
    hz_status s;
    std::string msg;
};

[[noreturn]] void raise(hz_status s, const std::string& m) { throw HzError{s, m}; }

#define HIPCHK(x)                                                                        \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess)                                                            \
            raise(HZ_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_) + " (line " + \
                                  std::to_string(__LINE__) + ")");                       \
    } while (0)

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// device allocations owned by a context
struct Arena {
    std::unordered_map<void*, size_t> sizes;
    long long bytes = 0;
    void* alloc(size_t n) {
        if (n == 0) n = 16;
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, n);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            raise(HZ_ENOMEM, "hipMalloc of " + std::to_string(n) + " bytes failed");
        }
        sizes[p] = n;
        bytes += (long long)n;
        return p;
    }
    void release(void* p, size_t /*n: recorded at allocation*/) {
        if (!p) return;
        auto it = sizes.find(p);
        if (it != sizes.end()) {
            bytes -= (long long)it->second;
            sizes.erase(it);
            (void)hipFree(p);
        }
    }
    void free_all() {
        for (auto& kv : sizes) (void)hipFree(kv.first);
        sizes.clear();
        bytes = 0;
    }
};

template <typename T>
struct Ops {                       // factors and interface operators in precision T
    C2<T>* X = nullptr;
    C2<T>* e = nullptr;
    C2<T>* Q = nullptr;
    C2<T>* CS = nullptr;
    C2<T>* Sinv = nullptr;
    C2<T>* Lfac = nullptr;
    C2<T>* Qc = nullptr;           // composed output operators [Q_x S^{-1} | Q_u] per side and cell
    C2<T>* CP = nullptr;           // pair-column samples (nested polarized traces)
};

enum LaunchKind { L_GEMM = 0, L_AXPBY = 1, L_COPY = 2, L_INNER = 3 };

template <typename T>
struct LaunchRec {
    int kind;
    long long off;        // first task
    int ntasks, max_m;
    C2<T>* y; const C2<T>* x; double2 a, b; long long n;   // vector ops
    double bytes, flops;  // algorithmic traffic / work of a GEMM launch
    int choice = -1;      // GEMM kernel picked by the autotuner (-1: default)
    bool plr = false;     // every task applies its operator in PLR form (B = 1)
    int plr_tiles = 0, plr_rows = 0;   // largest tile count / tile-row count of a task
    double bytes_dense = 0;            // algorithmic bytes of the dense form of a PLR launch
};

// Partitioned low-rank operators of the preconditioner (precision T): the
// factors of all compressed blocks in one pool, the tiles in one table, and
// per block (keyed by its first entry, as plan tasks point to it) the first
// tile and the tile grid.
template <typename T>
struct PlrStore {
    C2<T>* pool = nullptr;
    PlrTile* tiles = nullptr;
    std::vector<PlrTile> host;
    struct Ref { long long first; int ntr, ntc; };
    std::map<const void*, Ref> blocks;
    long long stored = 0, dense = 0;   // complex elements
    C2<T>* part = nullptr;             // partial products of one launch's tiles
    long long part_tiles = 0;
};

template <typename T> struct Plan;

// Nested polarized traces: one inner solve of a set of independent layer
// jobs (Sec. 4.2.1).  Job i's polarized inner right-hand side rhs_i
// ([d|q][J][2][HL_i][B]) is packed into column block i of the workspace
// vectors, rows [dq * 2 J HLmax, + 2 J HL_i) (the rest stays zero), so that
// the whole set is one batch of NJ * B columns for GMRES; the traces
// s = d + q go to out_i ([J][2][HL_i][B]).
template <typename T>
struct InnerRec {
    struct Job { int layer; const C2<T>* rhs; C2<T>* out; };
    std::vector<Job> jobs;
    bool loose = false;          // inside the preconditioner: the loose inner tolerance
    long long n = 0;             // rows of a workspace vector (4 J HLmax)
    int ncols = 0;               // NJ * B
    Arena* ar = nullptr;
    C2<T>* wA = nullptr;         // inner M: wA -> wB, inner P^GS: wB -> wC
    C2<T>* wB = nullptr;
    C2<T>* wC = nullptr;
    C2<T>* S = nullptr;          // s = d + q of wA (the d rows only)
    void* jobtab = nullptr;      // device table of the jobs (pack / unpack)
    std::unique_ptr<Plan<T>> M, P;
    ~InnerRec() {
        if (!ar) return;
        for (void* q : {(void*)wA, (void*)wB, (void*)wC, (void*)S, jobtab}) ar->release(q, 0);
    }
};

template <typename T>
struct Plan {
    GemmTask<T>* dev = nullptr;
    size_t dev_bytes = 0;
    std::vector<GemmTask<T>> tasks;
    std::vector<LaunchRec<T>> launches;
    std::vector<std::unique_ptr<InnerRec<T>>> inner;   // L_INNER records (off = index)
    bool inner_loose = false;            // its inner solves are inside the preconditioner
    hipGraph_t graph = nullptr;          // the launches captured once, replayed after
    hipGraphExec_t exec = nullptr;
    std::string name;                    // profiling family of the whole replay
    ~Plan() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

template <typename T>
struct LayerJob {
    int layer = 0;
    const C2<T>* top = nullptr;
    const C2<T>* bot = nullptr;
    const C2<T>* inner_add = nullptr;
    C2<T>* iy = nullptr;
    C2<T>* ix = nullptr;
    int side = 1;
    C2<T>* out = nullptr;
    const C2<T>* add0 = nullptr;
    const C2<T>* add1 = nullptr;
    int add1_row = 0;
    T c1 = 0;
    T alpha = 1;
    bool use_x = true;
    bool phase3 = true;
};

template <typename T>
struct Work {
    int Bcap = 0;
    C2<T>* f_ext = nullptr;    // [W][W][B]
    C2<T>* u_ext = nullptr;    // [W][W][B]
    C2<T>* rows_out = nullptr; // [L][4][W][B]
    C2<T>* gf = nullptr;       // [L][J][2][HLmax][B]
    C2<T>* iy[2] = {nullptr, nullptr};
    C2<T>* ix[2] = {nullptr, nullptr};
    C2<T>* pA = nullptr;       // polarized vectors [4KW][B]
    C2<T>* pB = nullptr;
    C2<T>* pC = nullptr;
    C2<T>* sv = nullptr;       // s = d + q, [K][2W][B]
    C2<T>* Y = nullptr;        // forward-sweep scratch of the cell solves
    long long y_stride = 0;
    int y_wgs = 0;
    const C2<T>** pair_tab = nullptr;   // device [2L]: top pairs then bottom pairs
    std::map<int, std::unique_ptr<Plan<T>>> sie, pre;
    std::map<std::string, std::unique_ptr<Plan<T>>> jobs;   // RHS formation / reconstruction
};

struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t next = 0;
    struct Pending { std::string fam; size_t e0, e1; double bytes, flops; };
    std::vector<Pending> pend;
    std::map<std::string, hz_kstat> acc;
};

}  // namespace

struct hz_ctx {
    hz_params prm{};
    Dims d{};
    int state = 0;                 // 1 set up, 2 factored
    hipStream_t st = nullptr;
    hipStream_t own_st = nullptr;  // stream created by the context (blocking, default priority)
    bool use_graphs = true;
    int compose = 1;               // output operators composed with the inner SIE inverse:
                                   // 0 never, 1 where it pays (compose_jobs), 2 always
    bool offline = false;          // inside the factorisation stage
    bool tune = true;              // autotune GEMM kernels and cell-solve widths (HZ_TUNE=0: off)
    bool inner_pt = false;         // nested polarized traces: the inner SIE iterated (Sec. 4.2.1)
    double inner_tol_loose = 1e-6; // inner GMRES tolerance inside the preconditioner
    double inner_tol_tight = 1e-12;// inner GMRES tolerance elsewhere (building blocks)
    double inner_tol_solve = 0.0;  // the same inside hz_solve / hz_adjoint (0 outside)
    int inner_iters_max = 0;       // largest inner GMRES iteration count since the last reset
    long long CP_elems = 0;
    int force_kind = -1;           // HZ_GEMM_KIND: one matrix-core GEMM kernel for every launch
    GemmSplitWs gsw;               // workspace of the split-k GEMM variants (allocated once)
    std::map<std::string, int> cs_tuned;   // (mode, B, cells) -> cell-solve batch width
    Arena arena;
    std::vector<LayerDesc> layers;
    std::vector<CellDesc> cells;
    LayerDesc* d_layers = nullptr;
    CellDesc* d_cells = nullptr;
    int* d_all_cells = nullptr;    // 0 .. ncells-1 (contiguous cell lists point into it)
    int* d_cell_list = nullptr;    // [ncells] other cell lists
    double* model = nullptr;
    double2 *diag = nullptr, *cz = nullptr, *e = nullptr;
    double2 *ax_pool = nullptr, *az_pool = nullptr;
    double2 *gdiag = nullptr, *gcx = nullptr, *gcz = nullptr, *wext = nullptr;
    int* flags = nullptr;          // [0] bad model
    FactorFlags* fflags = nullptr; // pivot status of the factorisation's block inversions
    double min_pivot_ratio = 0.0;  // smallest pivot ratio of the last factorisation
    int* layer_active = nullptr;   // [L]
    long long coef_elems = 0, X_elems = 0, Q_elems = 0, CS_elems = 0, Sinv_elems = 0, Lfac_elems = 0;
    long long inner_per_layer = 0; // J * 2 * HLmax
    long long Qc_elems = 0;
    std::vector<long long> qc_off; // [(layer * 2 + side) * Lc + cell] -> offset in Qc, -1 if none
    std::vector<int> qc_ld;        // row length of that block (J 2 HL + nslot s)
    Ops<double> o64;
    Ops<float> o32;
    Work<double> w64;
    Work<float> w32;
    PlrStore<double> plr64;
    PlrStore<float> plr32;
    // FP64 GMRES / refinement workspace
    int g_cap_B = 0, g_cap_m = 0;
    double2 *Z = nullptr;          // flexible GMRES: preconditioned basis
    double2 *V = nullptr, *gw = nullptr, *gb = nullptr, *gx = nullptr, *gpart = nullptr,
            *gsmall = nullptr, *gcoef = nullptr;
    int gpart_chunks = 0;
    double2* gh = nullptr;         // GMRES projections of both passes and |w|^2, on the device
    // inner GMRES (nested polarized traces): Krylov basis and reductions
    long long i_cap = 0; int i_cap_m = 0, i_cap_cols = 0, i_chunks = 0;
    double2 *iV = nullptr, *ipart = nullptr, *ismall = nullptr, *icoef = nullptr, *ih = nullptr;
    // its Givens state on the device (rotated Hessenberg columns packed by
    // column, rotations, rotated residual, per-column status) and the
    // per-iteration convergence flags with their pinned host copies
    double2 *iR = nullptr, *isn = nullptr, *ig = nullptr;
    double *ics = nullptr, *ibeta = nullptr;
    int *idone = nullptr, *ikfin = nullptr, *iflag = nullptr;
    int* h_iflag = nullptr;
    hipEvent_t iev = nullptr;
    double2 *u64 = nullptr, *f64 = nullptr, *r64 = nullptr;   // refinement [W][W][B]
    std::vector<std::vector<std::complex<double>>> g_hess;     // host Hessenberg storage of GMRES
    double2* h_pin = nullptr;      // pinned host buffer for the small per-iteration reads
    int device = 0;                // device current at hz_setup
    double* misfit_scratch = nullptr; // this device's copy of the file-scope scratch array
    size_t h_pin_elems = 0;
    hz_timing timing{};
    Prof prof;
};

namespace {

// ---------------------------------------------------------------------------
// small helpers

template <typename T> Ops<T>& ops(hz_ctx* c);
template <> Ops<double>& ops<double>(hz_ctx* c) { return c->o64; }
template <> Ops<float>& ops<float>(hz_ctx* c) { return c->o32; }
template <typename T> Work<T>& work(hz_ctx* c);
template <> Work<double>& work<double>(hz_ctx* c) { return c->w64; }
template <> Work<float>& work<float>(hz_ctx* c) { return c->w32; }
template <typename T> PlrStore<T>& plr_store(hz_ctx* c);
template <> PlrStore<double>& plr_store<double>(hz_ctx* c) { return c->plr64; }
template <> PlrStore<float>& plr_store<float>(hz_ctx* c) { return c->plr32; }

template <typename T>
C2<T>* alloc_c(hz_ctx* c, long long n) {
    return (C2<T>*)c->arena.alloc((size_t)n * sizeof(C2<T>));
}

std::vector<std::pair<int, int>> partition(int n, int parts) {
    std::vector<std::pair<int, int>> out;
    int base = n / parts, extra = n % parts, start = 1;
    for (int k = 0; k < parts; ++k) {
        int size = base + (k < extra ? 1 : 0);
        out.push_back({start, start + size - 1});
        start += size;
    }
    return out;
}

// ---------------------------------------------------------------------------
// partitions and descriptors

void build_descriptors(hz_ctx* c) {
    const Dims& d = c->d;
    const int p = d.p;
    auto lparts = partition(d.n, d.L);
    auto cparts = partition(d.n, d.Lc);
    c->layers.clear();
    c->cells.clear();
    int HLmax = 0, Wcmax = 0;
    for (auto& lp : lparts) HLmax = std::max(HLmax, lp.second - lp.first + 1 + 2 * p);
    for (auto& cp : cparts) Wcmax = std::max(Wcmax, cp.second - cp.first + 1 + 2 * p);
    c->d.HLmax = HLmax;
    c->d.Wcmax = Wcmax;
    c->d.HLpmax = (HLmax + 15) / 16 * 16;
    const int J = d.Lc - 1;
    c->inner_per_layer = (long long)J * 2 * HLmax;
    long long off_coef = 0, off_X = 0, off_Q = 0, off_CS = 0, off_Sinv = 0, off_Lfac = 0, off_CP = 0;
    for (int l = 0; l < d.L; ++l) {
        LayerDesc ld{};
        ld.index = l;
        ld.first = lparts[l].first;
        ld.last = lparts[l].second;
        ld.nl = ld.last - ld.first + 1;
        ld.HL = ld.nl + 2 * p;
        ld.row0 = ld.first - 1;
        ld.own_r0 = (l == 0) ? 0 : p;
        ld.own_r1 = (l == d.L - 1) ? ld.HL - 1 : p + ld.nl - 1;
        ld.has_top = l > 0;
        ld.has_bot = l < d.L - 1;
        ld.nslot = 0;
        for (int s = 0; s < MAXSLOT; ++s) { ld.slot_of[s] = -1; ld.slot_row[s] = -1; ld.slot_id[s] = -1; }
        auto add_slot = [&](int lid, int row) {
            ld.slot_of[lid] = ld.nslot;
            ld.slot_row[ld.nslot] = row;
            ld.slot_id[ld.nslot] = lid;
            ld.nslot++;
        };
        if (ld.has_top) { add_slot(0, p - 1); add_slot(1, p); }
        if (ld.has_bot) { add_slot(2, p + ld.nl - 1); add_slot(3, p + ld.nl); }
        ld.cell_begin = l * d.Lc;
        ld.J = J;
        ld.off_Sinv = off_Sinv;
        off_Sinv += (long long)J * (2LL * ld.HL) * (2LL * ld.HL);
        ld.off_Lfac = off_Lfac;
        off_Lfac += (long long)std::max(J - 1, 0) * ld.HL * (2LL * ld.HL);
        ld.off_inner = (long long)l * c->inner_per_layer;
        c->layers.push_back(ld);
        for (int k = 0; k < d.Lc; ++k) {
            CellDesc cd{};
            cd.layer = l;
            cd.cell = k;
            cd.gidx = l * d.Lc + k;
            cd.HL = ld.HL;
            cd.HLp = (ld.HL + 15) / 16 * 16;
            cd.first = cparts[k].first;
            cd.nc = cparts[k].second - cparts[k].first + 1;
            cd.Wc = cd.nc + 2 * p;
            cd.col0 = cd.first - 1;
            cd.own_c0 = (k == 0) ? 0 : p;
            cd.own_c1 = (k == d.Lc - 1) ? cd.Wc - 1 : p + cd.nc - 1;
            cd.s = cd.own_c1 - cd.own_c0 + 1;
            cd.has_left = k > 0;
            cd.has_right = k < d.Lc - 1;
            cd.adj = cd.has_left + cd.has_right;
            cd.nslot = ld.nslot;
            cd.ncol = cd.adj * 2 * cd.HL;
            cd.R = cd.ncol + cd.nslot * cd.s;
            cd.off_coef = off_coef;
            off_coef += (long long)cd.Wc * cd.HL;
            cd.off_X = off_X;
            off_X += (long long)cd.Wc * cd.HLp * cd.HLp;
            cd.off_Q = off_Q;
            off_Q += (long long)cd.nslot * cd.s * cd.R;
            cd.off_CS = off_CS;
            off_CS += (long long)cd.adj * cd.HL * cd.R;
            cd.off_CP = off_CP;
            off_CP += (long long)cd.adj * 2 * cd.HL * cd.R;
            c->cells.push_back(cd);
        }
    }
    c->coef_elems = off_coef;
    c->X_elems = off_X;
    c->Q_elems = off_Q;
    c->CS_elems = off_CS;
    c->Sinv_elems = off_Sinv;
    c->Lfac_elems = off_Lfac;
    c->CP_elems = off_CP;
    if (c->inner_pt) {                 // no inner factorisation
        c->Sinv_elems = 0;
        c->Lfac_elems = 0;
    } else {
        c->CP_elems = 0;
    }
}

void sync(hz_ctx* c) { HIPCHK(hipStreamSynchronize(c->st)); }

// Pinned host staging of at least `elems` complex values (reads of Krylov
// projections: a pageable destination would be copied through a bounce
// buffer on every iteration).  Valid until the next call.
double2* pinned(hz_ctx* c, size_t elems) {
    if (c->h_pin_elems < elems) {
        if (c->h_pin) (void)hipHostFree(c->h_pin);
        c->h_pin = nullptr;
        c->h_pin_elems = 0;
        const size_t want = std::max<size_t>(elems, 4096);
        if (hipHostMalloc((void**)&c->h_pin, sizeof(double2) * want, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            c->h_pin = nullptr;
            raise(HZ_ENOMEM, "hipHostMalloc of the staging buffer failed");
        }
        c->h_pin_elems = want;
    }
    return c->h_pin;
}

void upload(hz_ctx* c, void* dst, const void* src, size_t bytes) {
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->st));
    sync(c);
}

// ---------------------------------------------------------------------------
// profiling (events on the context stream around each dense launch)

size_t prof_event(hz_ctx* c) {
    Prof& P = c->prof;
    if (P.next == P.pool.size()) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        P.pool.push_back(e);
    }
    const size_t i = P.next++;
    HIPCHK(hipEventRecord(P.pool[i], c->st));
    return i;
}

void prof_flush(hz_ctx* c) {
    Prof& P = c->prof;
    if (P.pend.empty()) { P.next = 0; return; }
    sync(c);
    for (const auto& q : P.pend) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, P.pool[q.e0], P.pool[q.e1]));
        // one record per kernel family and launch shape (launches of one
        // shape have the same algorithmic flops), so per-launch averages
        // describe one kind of launch
        const std::string key = q.fam + "#" + std::to_string(std::llround(q.flops)) + "#" +
                                std::to_string(std::llround(q.bytes));
        hz_kstat& k = P.acc[key];
        std::snprintf(k.name, sizeof(k.name), "%s", q.fam.c_str());
        k.launches += 1;
        k.ms += ms;
        k.bytes += q.bytes;
        k.flops += q.flops;
    }
    P.pend.clear();
    P.next = 0;
}

template <typename T>
std::string fam_name(const char* base) {
    return std::string(base) + (sizeof(T) == sizeof(double) ? "_c128" : "_c64");
}

// ---------------------------------------------------------------------------
// GEMM plans for layer jobs (design: phases M_f -> inner LU -> [M_u | D_loc])

template <typename T>
GemmTask<T> blank_task() {
    GemmTask<T> t;
    std::memset(&t, 0, sizeof(t));
    t.alpha = (T)1;
    return t;
}

template <typename T>
const C2<T>* pair_row(const C2<T>* pair, int row, int col, int W, int B) {
    return pair ? pair + ((long long)row * W + col) * B : nullptr;
}

template <typename T>
void add_launch(Plan<T>& pl, long long first, int maxm, int B) {
    LaunchRec<T> r{};
    r.kind = L_GEMM;
    r.off = first;
    r.ntasks = (int)(pl.tasks.size() - first);
    r.max_m = maxm;
    // algorithmic traffic: every operator entry that meets a nonzero input
    // segment, every input and output vector element, every addend
    double bytes = 0, flops = 0;
    const double cs = sizeof(C2<T>);
    for (size_t q = first; q < pl.tasks.size(); ++q) {
        const GemmTask<T>& t = pl.tasks[q];
        long long kk = 0;
        for (int s = 0; s < t.nseg; ++s)
            if (t.seg_ptr[s]) kk += t.seg_len[s];
        int adds = 0;
        for (int s = 0; s < t.noseg; ++s) adds += (t.oseg_add0[s] != nullptr) + (t.oseg_add1[s] != nullptr);
        const int nb = t.ncol > 0 ? t.ncol : B;
        bytes += cs * ((double)t.m * kk + (double)kk * nb + (double)t.m * nb * (1.0 + (t.noseg ? (double)adds / t.noseg : 0.0)));
        flops += 8.0 * t.m * kk * nb;
    }
    r.bytes = bytes;
    r.flops = flops;
    if (r.ntasks > 0) pl.launches.push_back(r);
}

template <typename T>
void add_vec(Plan<T>& pl, int kind, C2<T>* y, const C2<T>* x, double2 a, double2 b, long long n) {
    LaunchRec<T> r{};
    r.kind = kind;
    r.y = y; r.x = x; r.a = a; r.b = b; r.n = n;
    pl.launches.push_back(r);
}

// Whether a set of jobs takes its samples through the composed operators
// Qc = [Q_x S^{-1} | Q_u] or through the inner block-LU substitutions and
// Q = [Q_x | Q_u].  Qc has J 2 HL columns for the inner right-hand side where
// Q has the cell's adj 2 HL inner-trace columns, so composing costs
// 2 s (J 2 HL - adj 2 HL) more operator entries per cell and job; the
// substitutions cost (8J - 4) HL^2 entries per job and 3J - 2 dependent
// launches, shared by all jobs of the set.  A sequential sweep step (one
// job) is worth composing; a batch of many parallel jobs (the SIE product,
// the reflections) is not once J is large (n = 2047, L_c = 8: Qc doubles the
// SIE product's flops).  The estimate takes the saved entries at the
// matrix-core rate (B >= 16) or at the HBM rate (streamed once, small B),
// against 25 us per added dependent launch.  mode 2 (HZ_COMPOSE=2) composes
// every set, 0 none.
template <typename T>
bool compose_jobs(hz_ctx* c, const std::vector<LayerJob<T>>& jobs, int B) {
    const Dims& d = c->d;
    const int J = d.Lc - 1;
    if (c->inner_pt || J <= 0 || c->compose == 0 || ops<T>(c).Qc == nullptr) return false;
    if (c->compose == 2) return true;
    double saved = 0.0;                       // operator entries per right-hand side
    for (const auto& jb : jobs) {
        if (!jb.phase3) continue;
        const LayerDesc& ld = c->layers[jb.layer];
        const double HL = ld.HL, NI = 2.0 * J * HL;
        for (int k = 0; k < d.Lc; ++k) {
            const CellDesc& cd = c->cells[ld.cell_begin + k];
            saved += 2.0 * cd.s * (NI - cd.ncol);
        }
        saved -= (8.0 * J - 4.0) * HL * HL;
    }
    const double rate = sizeof(T) == sizeof(double) ? 60e12 : 120e12;
    const double t_saved = std::max(saved * B * 8.0 / rate, saved * sizeof(C2<T>) / 5e12);
    return t_saved <= (3.0 * J - 2.0) * 25e-6;
}

// Append the three phases of a set of independent layer jobs to a plan.
// keep_composed: take the composed operators whenever they exist (the PLR
// form compresses Qc, not Q).
template <typename T>
void plan_jobs(hz_ctx* c, Plan<T>& pl, const std::vector<LayerJob<T>>& jobs, int B,
               bool keep_composed = false) {
    const Dims& d = c->d;
    const int W = d.W;
    const int J = d.Lc - 1;
    Ops<T>& o = ops<T>(c);
    // with the composed output operators, only jobs that need the inner
    // traces themselves (no phase 3) run the block LU substitutions
    const bool pt = c->inner_pt && J > 0;
    const bool comp = !pt && J > 0 && o.Qc != nullptr && c->compose != 0 &&
                      (keep_composed || compose_jobs<T>(c, jobs, B));
    std::vector<LayerJob<T>> p2;
    for (const auto& jb : jobs)
        if (!(comp && jb.phase3)) p2.push_back(jb);
    // ---- phase 1: inner right-hand sides from the interface-row sources
    if (J > 0) {
        long long first = pl.tasks.size();
        int maxm = 0;
        for (const auto& jb : jobs) {
            const LayerDesc& ld = c->layers[jb.layer];
            for (int k = 0; k < d.Lc; ++k) {
                const CellDesc& cd = c->cells[ld.cell_begin + k];
                GemmTask<T> t = blank_task<T>();
                t.A = o.CS + cd.off_CS + cd.ncol;
                t.lda = cd.R;
                t.m = cd.adj * cd.HL;
                t.k = cd.nslot * cd.s;
                if (pt) {                     // both columns of each pair
                    t.A = o.CP + cd.off_CP + cd.ncol;
                    t.m = cd.adj * 2 * cd.HL;
                }
                t.ldx = B;
                t.ldo = B;
                t.nseg = 0;
                for (int si = 0; si < ld.nslot; ++si) {
                    const int lid = ld.slot_id[si];
                    const C2<T>* pr = lid < 2 ? jb.top : jb.bot;
                    t.seg_k0[t.nseg] = si * cd.s;
                    t.seg_len[t.nseg] = cd.s;
                    t.seg_ptr[t.nseg] = pair_row<T>(pr, lid % 2, cd.col0 + cd.own_c0, W, B);
                    t.nseg++;
                }
                t.noseg = 0;
                const long long HLB = (long long)cd.HL * B;
                if (pt) {
                    // left pair -> q of interface k-1, right pair -> d of interface k
                    if (cd.has_left) {
                        const long long off = ((long long)J + k - 1) * 2 * HLB;
                        t.oseg_i0[t.noseg] = 0;
                        t.oseg_len[t.noseg] = 2 * cd.HL;
                        t.oseg_ptr[t.noseg] = jb.iy + off;
                        t.oseg_add0[t.noseg] = jb.inner_add ? jb.inner_add + off : nullptr;
                        t.noseg++;
                    }
                    if (cd.has_right) {
                        const long long off = (long long)k * 2 * HLB;
                        t.oseg_i0[t.noseg] = cd.has_left ? 2 * cd.HL : 0;
                        t.oseg_len[t.noseg] = 2 * cd.HL;
                        t.oseg_ptr[t.noseg] = jb.iy + off;
                        t.oseg_add0[t.noseg] = jb.inner_add ? jb.inner_add + off : nullptr;
                        t.noseg++;
                    }
                    maxm = std::max(maxm, t.m);
                    pl.tasks.push_back(t);
                    continue;
                }
                if (cd.has_left) {
                    const long long off = ((long long)(k - 1) * 2 + 1) * HLB;
                    t.oseg_i0[t.noseg] = 0;
                    t.oseg_len[t.noseg] = cd.HL;
                    t.oseg_ptr[t.noseg] = jb.iy + off;
                    t.oseg_add0[t.noseg] = jb.inner_add ? jb.inner_add + off : nullptr;
                    t.noseg++;
                }
                if (cd.has_right) {
                    const long long off = ((long long)k * 2 + 0) * HLB;
                    t.oseg_i0[t.noseg] = cd.has_left ? cd.HL : 0;
                    t.oseg_len[t.noseg] = cd.HL;
                    t.oseg_ptr[t.noseg] = jb.iy + off;
                    t.oseg_add0[t.noseg] = jb.inner_add ? jb.inner_add + off : nullptr;
                    t.noseg++;
                }
                maxm = std::max(maxm, t.m);
                pl.tasks.push_back(t);
            }
        }
        add_launch(pl, first, maxm, B);
        // ---- phase 2 (nested polarized traces): the inner polarized systems
        // of all jobs, iterated together
        if (pt && !p2.empty()) {
            auto ir = std::make_unique<InnerRec<T>>();
            for (const auto& jb : p2) ir->jobs.push_back({jb.layer, jb.iy, jb.ix});
            ir->loose = pl.inner_loose;
            LaunchRec<T> r{};
            r.kind = L_INNER;
            r.off = (long long)pl.inner.size();
            pl.inner.push_back(std::move(ir));
            pl.launches.push_back(r);
        }
        // ---- phase 2: block LU substitutions across the cells (inner sweeps)
        if (!pt && !p2.empty()) {
            for (int j = 1; j < J; ++j) {                       // forward
                long long f2 = pl.tasks.size();
                int mm = 0;
                for (const auto& jb : p2) {
                    const LayerDesc& ld = c->layers[jb.layer];
                    const int HL = ld.HL;
                    const long long blk = 2LL * HL * B;
                    GemmTask<T> t = blank_task<T>();
                    t.A = o.Lfac + ld.off_Lfac + (long long)(j - 1) * HL * 2 * HL;
                    t.lda = 2 * HL;
                    t.m = HL;
                    t.k = 2 * HL;
                    t.ldx = B; t.ldo = B;
                    t.nseg = 1;
                    t.seg_k0[0] = 0; t.seg_len[0] = 2 * HL; t.seg_ptr[0] = jb.iy + (j - 1) * blk;
                    t.noseg = 1;
                    t.oseg_i0[0] = 0; t.oseg_len[0] = HL; t.oseg_ptr[0] = jb.iy + j * blk;
                    t.oseg_add0[0] = jb.iy + j * blk;
                    t.alpha = (T)-1;
                    mm = std::max(mm, t.m);
                    pl.tasks.push_back(t);
                }
                add_launch(pl, f2, mm, B);
            }
            for (int j = J - 1; j >= 0; --j) {                  // backward
                if (j < J - 1) {
                    long long f2 = pl.tasks.size();
                    int mm = 0;
                    for (const auto& jb : p2) {
                        const LayerDesc& ld = c->layers[jb.layer];
                        const int HL = ld.HL;
                        const long long blk = 2LL * HL * B;
                        const CellDesc& cn = c->cells[ld.cell_begin + j + 1];   // cell right of iface j
                        GemmTask<T> t = blank_task<T>();
                        // y_j.b - C_j x_{j+1},  C_j = -(left-column samples of cell j+1, right probes)
                        t.A = o.CS + cn.off_CS + 2LL * HL;      // left rows, right probes
                        t.lda = cn.R;
                        t.m = HL;
                        t.k = 2 * HL;
                        t.ldx = B; t.ldo = B;
                        t.nseg = 1;
                        t.seg_k0[0] = 0; t.seg_len[0] = 2 * HL; t.seg_ptr[0] = jb.ix + (j + 1) * blk;
                        t.noseg = 1;
                        t.oseg_i0[0] = 0; t.oseg_len[0] = HL;
                        t.oseg_ptr[0] = jb.iy + j * blk + (long long)HL * B;
                        t.oseg_add0[0] = jb.iy + j * blk + (long long)HL * B;
                        t.alpha = (T)1;
                        mm = std::max(mm, t.m);
                        pl.tasks.push_back(t);
                    }
                    add_launch(pl, f2, mm, B);
                }
                long long f2 = pl.tasks.size();
                int mm = 0;
                for (const auto& jb : p2) {
                    const LayerDesc& ld = c->layers[jb.layer];
                    const int HL = ld.HL;
                    const long long blk = 2LL * HL * B;
                    GemmTask<T> t = blank_task<T>();
                    t.A = o.Sinv + ld.off_Sinv + (long long)j * 4 * HL * HL;
                    t.lda = 2 * HL;
                    t.m = 2 * HL;
                    t.k = 2 * HL;
                    t.ldx = B; t.ldo = B;
                    t.nseg = 1;
                    t.seg_k0[0] = 0; t.seg_len[0] = 2 * HL; t.seg_ptr[0] = jb.iy + j * blk;
                    t.noseg = 1;
                    t.oseg_i0[0] = 0; t.oseg_len[0] = 2 * HL; t.oseg_ptr[0] = jb.ix + j * blk;
                    mm = std::max(mm, t.m);
                    pl.tasks.push_back(t);
                }
                add_launch(pl, f2, mm, B);
            }
        }
    }
    // ---- phase 3: samples on the requested interface rows
    long long first = pl.tasks.size();
    int maxm = 0;
    for (const auto& jb : jobs) {
        if (!jb.phase3) continue;
        const LayerDesc& ld = c->layers[jb.layer];
        const int so_a = ld.slot_of[jb.side == 0 ? 0 : 2];
        if (so_a < 0) raise(HZ_EINVAL, "layer has no interface on the requested side");
        for (int k = 0; k < d.Lc; ++k) {
            const CellDesc& cd = c->cells[ld.cell_begin + k];
            GemmTask<T> t = blank_task<T>();
            t.A = o.Q + cd.off_Q + (long long)so_a * cd.s * cd.R;
            t.lda = cd.R;
            t.m = 2 * cd.s;
            t.k = cd.R;
            t.ldx = B; t.ldo = B;
            t.nseg = 0;
            const long long HLB = (long long)cd.HL * B;
            int x0 = cd.ncol;                    // first column of the interface-row sources
            if (comp) {                          // [Q_x S^{-1} | Q_u] applied to [iy; pair]
                const long long q = ((long long)jb.layer * 2 + jb.side) * d.Lc + k;
                t.A = o.Qc + c->qc_off[q];
                t.lda = c->qc_ld[q];
                t.k = c->qc_ld[q];
                t.seg_k0[0] = 0;
                t.seg_len[0] = J * 2 * cd.HL;
                t.seg_ptr[0] = jb.iy;
                t.nseg = 1;
                x0 = J * 2 * cd.HL;
            } else {
                if (cd.has_left) {
                    t.seg_k0[t.nseg] = 0;
                    t.seg_len[t.nseg] = 2 * cd.HL;
                    t.seg_ptr[t.nseg] = jb.ix + (long long)(k - 1) * 2 * HLB;
                    t.nseg++;
                }
                if (cd.has_right) {
                    t.seg_k0[t.nseg] = cd.has_left ? 2 * cd.HL : 0;
                    t.seg_len[t.nseg] = 2 * cd.HL;
                    t.seg_ptr[t.nseg] = jb.ix + (long long)k * 2 * HLB;
                    t.nseg++;
                }
            }
            if (jb.use_x) {
                for (int si = 0; si < ld.nslot; ++si) {
                    const int lid = ld.slot_id[si];
                    const C2<T>* pr = lid < 2 ? jb.top : jb.bot;
                    t.seg_k0[t.nseg] = x0 + si * cd.s;
                    t.seg_len[t.nseg] = cd.s;
                    t.seg_ptr[t.nseg] = pair_row<T>(pr, lid % 2, cd.col0 + cd.own_c0, W, B);
                    t.nseg++;
                }
            }
            t.noseg = 2;
            for (int r = 0; r < 2; ++r) {
                const long long off = ((long long)r * W + cd.col0 + cd.own_c0) * B;
                t.oseg_i0[r] = r * cd.s;
                t.oseg_len[r] = cd.s;
                t.oseg_ptr[r] = jb.out + off;
                t.oseg_add0[r] = jb.add0 ? jb.add0 + off : nullptr;
                t.oseg_add1[r] = (jb.add1 && jb.add1_row == r) ? jb.add1 + off : nullptr;
                t.c1[r] = jb.c1;
            }
            t.alpha = jb.alpha;
            maxm = std::max(maxm, t.m);
            pl.tasks.push_back(t);
        }
    }
    add_launch(pl, first, maxm, B);
}

template <typename T>
void plan_upload(hz_ctx* c, Plan<T>& pl) {
    const size_t bytes = pl.tasks.size() * sizeof(GemmTask<T>);
    if (bytes == 0) return;
    if (pl.dev_bytes < bytes) {
        if (pl.dev) c->arena.release(pl.dev, pl.dev_bytes);
        pl.dev = (GemmTask<T>*)c->arena.alloc(bytes);
        pl.dev_bytes = bytes;
    }
    upload(c, pl.dev, pl.tasks.data(), bytes);
}

template <typename T>
void plan_launches(hz_ctx* c, Plan<T>& pl, int B);

// Autotuner for the matrix-core GEMM launches of a solve plan.  Each launch is
// timed with every candidate kernel on its own operator blocks, with the
// input segments and outputs redirected to scratch buffers (plans that update
// vectors in place are not disturbed), and the fastest kernel is kept in the
// launch record.  Runs once, when the plan is built for a batch size.
// 64 MB of partial tiles for the split-k GEMM variants (a launch whose
// partials do not fit runs the unsplit kernel)
void ensure_split_ws(hz_ctx* c) {
    if (c->gsw.ws) return;
    c->gsw.ws_bytes = 64LL << 20;
    c->gsw.ws = c->arena.alloc((size_t)c->gsw.ws_bytes);
}

template <typename T>
void tune_plan(hz_ctx* c, Plan<T>& pl, int B) {
    ensure_split_ws(c);
    if (c->force_kind >= GEMM_MFMA32) {
        for (auto& r : pl.launches)
            if (r.kind == L_GEMM) r.choice = c->force_kind;
        return;
    }
    if (!c->tune || B < 16 || pl.launches.empty()) return;
    // Trials read the launch's own inputs (reading disturbs nothing) and write
    // every output segment to its own place in a scratch buffer, so that they
    // see the launch's real memory traffic: with one shared input buffer the
    // inputs stayed in L2 and tiles that re-read them looked cheaper than they
    // are.  add0 / add1 are dropped (they only add a read per output entry).
    long long out_elems = 1;
    int max_tasks = 1;
    for (const auto& r : pl.launches) {
        max_tasks = std::max(max_tasks, r.ntasks);
        long long tot = 0;
        for (int q2 = 0; q2 < r.ntasks; ++q2) {
            const GemmTask<T>& t = pl.tasks[r.off + q2];
            for (int q = 0; q < t.noseg; ++q) tot += (long long)t.oseg_len[q] * t.ldo;
        }
        out_elems = std::max(out_elems, tot);
    }
    C2<T>* sout = alloc_c<T>(c, out_elems);
    GemmTask<T>* dt = (GemmTask<T>*)c->arena.alloc(sizeof(GemmTask<T>) * max_tasks);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (auto& r : pl.launches) {
        if (r.kind != L_GEMM) continue;
        if (gemm_kernel(r.ntasks, r.max_m, B) < GEMM_MFMA32) continue;
        std::vector<GemmTask<T>> tt(pl.tasks.begin() + r.off, pl.tasks.begin() + r.off + r.ntasks);
        long long at = 0;
        for (auto& t : tt) {
            for (int q = 0; q < t.noseg; ++q) {
                t.oseg_ptr[q] = sout + at;
                at += (long long)t.oseg_len[q] * t.ldo;
                t.oseg_add0[q] = nullptr;
                t.oseg_add1[q] = nullptr;
            }
        }
        upload(c, dt, tt.data(), sizeof(GemmTask<T>) * tt.size());
        // the heuristic's kernel first; another replaces it only when more
        // than 3% faster, so near-ties give the same choice from run to run
        const int dflt = (int)gemm_kernel(r.ntasks, r.max_m, B);
        float best = 1e30f;
        for (int cand : {dflt, (int)GEMM_MFMA64, (int)GEMM_MFMA32, (int)GEMM_MFMA32K16,
                         (int)GEMM_MFMA32D, (int)GEMM_MFMA64D, (int)GEMM_MFMA32X64,
                         (int)GEMM_MFMA64X32, (int)GEMM_MFMA64S2, (int)GEMM_MFMA64S4,
                         (int)GEMM_MFMA32S2, (int)GEMM_MFMA32S4, (int)GEMM_MFMA32S8,
                         (int)GEMM_MFMA64S8, (int)GEMM_MFMA32X64S4, (int)GEMM_MFMA32X64S8,
                         (int)GEMM_MFMA32DS4, (int)GEMM_MFMA32DS8}) {
            if (cand == dflt && best < 1e30f) continue;
            // launches big enough for 64 x 64 tiles keep 64-row tiles: there
            // the back-to-back trial launches find their inputs in cache and
            // favour 32-row tiles that re-read them, which lose in the solve
            if (dflt == GEMM_MFMA64 &&
                !(cand == GEMM_MFMA64 || cand == GEMM_MFMA64D || cand == GEMM_MFMA64X32 ||
                  cand == GEMM_MFMA64S2 || cand == GEMM_MFMA64S4 || cand == GEMM_MFMA64S8))
                continue;
            if ((cand == GEMM_MFMA64 || cand == GEMM_MFMA64D || cand == GEMM_MFMA32X64 ||
                 cand == GEMM_MFMA64S2 || cand == GEMM_MFMA64S4 || cand == GEMM_MFMA64S8 ||
                 cand == GEMM_MFMA32X64S4 || cand == GEMM_MFMA32X64S8) && B < 64)
                continue;
            launch_gemm<T>(dt, r.ntasks, r.max_m, B, c->st, false, cand, &c->gsw);   // warm-up
            HIPCHK(hipEventRecord(e0, c->st));
            for (int rep = 0; rep < 3; ++rep)
                launch_gemm<T>(dt, r.ntasks, r.max_m, B, c->st, false, cand, &c->gsw);
            HIPCHK(hipEventRecord(e1, c->st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            if (best == 1e30f || ms < 0.97f * best) { best = ms; r.choice = cand; }
        }
    }
    HIPCHK(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->arena.release(sout, 0);
    c->arena.release(dt, 0);
}

template <typename T>
void inner_solve(hz_ctx* c, InnerRec<T>& r, int B);

// Replay a plan: through its captured HIP graph when graphs are enabled and
// profiling is off, launch by launch (one event pair per kernel) otherwise.
template <typename T>
void plan_run(hz_ctx* c, Plan<T>& pl, int B) {
    // plans with inner iterations read the inner residuals on the host
    if (c->use_graphs && c->st && !pl.name.empty() && !c->prof.on && pl.inner.empty()) {
        if (!pl.exec) {
            HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
            plan_launches<T>(c, pl, B);
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamEndCapture(c->st, &g));
            pl.graph = g;
            HIPCHK(hipGraphInstantiate(&pl.exec, g, nullptr, nullptr, 0));
        }
        HIPCHK(hipGraphLaunch(pl.exec, c->st));
        return;
    }
    plan_launches<T>(c, pl, B);
}

template <typename T>
void plan_launches(hz_ctx* c, Plan<T>& pl, int B) {
    const bool prof = c->prof.on;
    for (const auto& r : pl.launches) {
        if (r.kind == L_GEMM && r.plr) {
            size_t e0 = prof ? prof_event(c) : 0;
            launch_plr_apply<T>(pl.dev + r.off, r.ntasks, r.plr_tiles, r.plr_rows,
                                plr_store<T>(c).part, c->st);
            if (prof) {
                size_t e1 = prof_event(c);
                c->prof.pend.push_back({fam_name<T>("plr_gemv"), e0, e1, r.bytes, r.flops});
            }
        } else if (r.kind == L_GEMM) {
            size_t e0 = prof ? prof_event(c) : 0;
            launch_gemm<T>(pl.dev + r.off, r.ntasks, r.max_m, B, c->st, c->offline, r.choice,
                           &c->gsw);
            if (prof) {
                size_t e1 = prof_event(c);
                const GemmKernel kk = gemm_kernel(r.ntasks, r.max_m, B);
                const char* k = gemm_kernel_name(r.choice >= 0 && kk >= GEMM_MFMA32
                                                     ? (GemmKernel)r.choice : kk);
                c->prof.pend.push_back({fam_name<T>(k), e0, e1, r.bytes, r.flops});
            }
        } else if (r.kind == L_AXPBY) {
            launch_axpby<T>(r.y, r.x, r.a, r.b, r.n, c->st);
        } else if (r.kind == L_COPY) {
            launch_copy<T>(r.y, r.x, r.n, c->st);
        } else if (r.kind == L_INNER) {
            inner_solve(c, *pl.inner[r.off], B);
        }
    }
    HIPCHK(hipGetLastError());
}

// polarized vector helpers: d_k / q_k pairs
template <typename T>
C2<T>* dvec(hz_ctx* c, C2<T>* v, int k, int B) { return v + (long long)k * 2 * c->d.W * B; }
template <typename T>
C2<T>* qvec(hz_ctx* c, C2<T>* v, int k, int B) { return v + (long long)(c->d.K + k) * 2 * c->d.W * B; }

template <typename T>
C2<T>* iy_of(hz_ctx* c, int set, int layer, int B) {
    return work<T>(c).iy[set] + (c->inner_pt ? 2 : 1) * c->layers[layer].off_inner * B;
}
// inner right-hand side of the volume source in `layer` (written by SOLVE_SAMPLE)
template <typename T>
C2<T>* gf_of(hz_ctx* c, int layer, int B) {
    return work<T>(c).gf + (c->inner_pt ? 2 : 1) * c->layers[layer].off_inner * B;
}
template <typename T>
C2<T>* ix_of(hz_ctx* c, int set, int layer, int B) {
    return work<T>(c).ix[set] + c->layers[layer].off_inner * B;
}

// M: pA -> pB (eq. M_polarized via the jump conditions)
template <typename T>
void build_sie_plan(hz_ctx* c, Plan<T>& pl, int B) {
    Work<T>& w = work<T>(c);
    const int K = c->d.K;
    const long long pairn = 2LL * c->d.W * B;
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
    // s = d + q
    add_vec<T>(pl, L_COPY, w.sv, w.pA, zero, zero, K * pairn);
    add_vec<T>(pl, L_AXPBY, w.sv, qvec<T>(c, w.pA, 0, B), one, one, K * pairn);
    std::vector<LayerJob<T>> jobs;
    for (int k = 0; k < K; ++k) {
        LayerJob<T> dn;
        dn.layer = k;
        dn.top = k > 0 ? w.sv + (k - 1) * pairn : nullptr;
        dn.bot = qvec<T>(c, w.pA, k, B);
        dn.iy = iy_of<T>(c, 0, k, B);
        dn.ix = ix_of<T>(c, 0, k, B);
        dn.side = 1;
        dn.out = dvec<T>(c, w.pB, k, B);
        dn.add0 = dvec<T>(c, w.pA, k, B);
        dn.add1 = qvec<T>(c, w.pA, k, B);
        dn.add1_row = 0;
        dn.c1 = (T)1;
        dn.alpha = (T)-1;
        jobs.push_back(dn);
        LayerJob<T> up;
        up.layer = k + 1;
        up.top = dvec<T>(c, w.pA, k, B);
        up.bot = k + 1 < K ? w.sv + (k + 1) * pairn : nullptr;
        up.iy = iy_of<T>(c, 1, k + 1, B);
        up.ix = ix_of<T>(c, 1, k + 1, B);
        up.side = 0;
        up.out = qvec<T>(c, w.pB, k, B);
        up.add0 = qvec<T>(c, w.pA, k, B);
        up.add1 = dvec<T>(c, w.pA, k, B);
        up.add1_row = 1;
        up.c1 = (T)1;
        up.alpha = (T)-1;
        jobs.push_back(up);
    }
    plan_jobs<T>(c, pl, jobs, B);
}

// P^GS: pB -> pC (downward sweep, up-going reflections, upward sweep)
template <typename T>
void build_pre_plan(hz_ctx* c, Plan<T>& pl, int B) {
    Work<T>& w = work<T>(c);
    const int K = c->d.K;
    const long long pairn = 2LL * c->d.W * B;
    const double2 zero = make_double2(0.0, 0.0);
    add_vec<T>(pl, L_COPY, dvec<T>(c, w.pC, 0, B), dvec<T>(c, w.pB, 0, B), zero, zero, pairn);
    for (int k = 1; k < K; ++k) {                       // downward sweep (D_down^{-1})
        LayerJob<T> jb;
        jb.layer = k;
        jb.top = dvec<T>(c, w.pC, k - 1, B);
        jb.bot = nullptr;
        jb.iy = iy_of<T>(c, 0, k, B);
        jb.ix = ix_of<T>(c, 0, k, B);
        jb.side = 1;
        jb.out = dvec<T>(c, w.pC, k, B);
        jb.add0 = dvec<T>(c, w.pB, k, B);
        jb.alpha = (T)1;
        plan_jobs<T>(c, pl, {jb}, B);
    }
    if (c->prm.precond == HZ_PRECOND_JACOBI) {          // P^Jac: no reflections, t = v_up
        const double2 zero2 = make_double2(0.0, 0.0);
        add_vec<T>(pl, L_COPY, qvec<T>(c, w.pC, 0, B), qvec<T>(c, w.pB, 0, B), zero2, zero2,
                   K * pairn);
    } else {                                            // t = v_up - L x_down (parallel)
        std::vector<LayerJob<T>> jobs;
        for (int k = 0; k < K; ++k) {
            LayerJob<T> jb;
            jb.layer = k + 1;
            jb.top = dvec<T>(c, w.pC, k, B);
            jb.bot = k + 1 < K ? dvec<T>(c, w.pC, k + 1, B) : nullptr;
            jb.iy = iy_of<T>(c, 0, k + 1, B);
            jb.ix = ix_of<T>(c, 0, k + 1, B);
            jb.side = 0;
            jb.out = qvec<T>(c, w.pC, k, B);
            jb.add0 = qvec<T>(c, w.pB, k, B);
            jb.add1 = dvec<T>(c, w.pC, k, B);
            jb.add1_row = 1;
            jb.c1 = (T)-1;
            jb.alpha = (T)1;
            jobs.push_back(jb);
        }
        // the single-RHS PLR form keeps the composed operators it compressed
        plan_jobs<T>(c, pl, jobs, B, c->prm.plr != 0 && B == 1);
    }
    for (int k = K - 2; k >= 0; --k) {                  // upward sweep (D_up^{-1})
        LayerJob<T> jb;
        jb.layer = k + 1;
        jb.top = nullptr;
        jb.bot = qvec<T>(c, w.pC, k + 1, B);
        jb.iy = iy_of<T>(c, 0, k + 1, B);
        jb.ix = ix_of<T>(c, 0, k + 1, B);
        jb.side = 0;
        jb.out = qvec<T>(c, w.pC, k, B);
        jb.add0 = qvec<T>(c, w.pC, k, B);
        jb.alpha = (T)1;
        plan_jobs<T>(c, pl, {jb}, B);
    }
    (void)pairn;
}

// Switch the GEMM launches of a single-RHS preconditioner plan whose tasks
// all have compressed operators to the PLR kernels (tasks get their tile
// tables and their place in the partial-product scratch).
template <typename T>
void plr_mark(hz_ctx* c, Plan<T>& pl) {
    PlrStore<T>& ps = plr_store<T>(c);
    if (!c->prm.plr || !ps.pool) return;
    const double cs = sizeof(C2<T>);
    long long need = 0;
    for (auto& r : pl.launches) {
        if (r.kind != L_GEMM) continue;
        bool all = true;
        for (int q = 0; q < r.ntasks && all; ++q)
            all = ps.blocks.count((const void*)pl.tasks[r.off + q].A) > 0;
        if (!all) continue;
        long long tot = 0;
        int mt = 0, mr = 0;
        double bytes = 0;
        for (int q = 0; q < r.ntasks; ++q) {
            GemmTask<T>& t = pl.tasks[r.off + q];
            const auto& ref = ps.blocks.at((const void*)t.A);
            t.plr = ps.tiles + ref.first;
            t.plr_pool = ps.pool;
            t.plr_ntr = ref.ntr;
            t.plr_ntc = ref.ntc;
            t.plr_part = tot;
            tot += (long long)ref.ntr * ref.ntc;
            mt = std::max(mt, ref.ntr * ref.ntc);
            mr = std::max(mr, ref.ntr);
            // algorithmic traffic: the stored entries of the tiles that meet a
            // present input segment, the input and output rows
            long long kk = 0;
            for (int s2 = 0; s2 < t.nseg; ++s2)
                if (t.seg_ptr[s2]) kk += t.seg_len[s2];
            for (long long e = ref.first; e < ref.first + (long long)ref.ntr * ref.ntc; ++e) {
                const PlrTile& tl = ps.host[e];
                bool live = false;
                for (int s2 = 0; s2 < t.nseg && !live; ++s2)
                    live = t.seg_ptr[s2] && t.seg_k0[s2] < tl.j0 + tl.tc &&
                           tl.j0 < t.seg_k0[s2] + t.seg_len[s2];
                if (!live) continue;
                bytes += cs * (tl.rank < 0 ? (double)tl.tr * tl.tc : (double)tl.rank * (tl.tr + tl.tc));
            }
            bytes += cs * ((double)kk + 2.0 * t.m);
        }
        r.plr = true;
        r.plr_tiles = mt;
        r.plr_rows = mr;
        r.bytes_dense = r.bytes;
        r.bytes = bytes;
        need = std::max(need, tot);
    }
    if (need > ps.part_tiles) {
        if (ps.part) c->arena.release(ps.part, 0);
        ps.part = alloc_c<T>(c, need * PLR_TILE);
        ps.part_tiles = need;
    }
}

// Single-RHS plans with compressed operators: every PLR launch is timed
// against the dense matrix-vector launch of the same tasks (outputs
// redirected to scratch) and keeps the compressed form only where it is
// faster.  The PLR apply is two dependent kernels, so for short launches of
// small operators its latency outweighs the bytes it saves.
template <typename T>
void tune_plr(hz_ctx* c, Plan<T>& pl) {
    if (!c->tune) return;
    long long out_elems = 1;
    int max_tasks = 0;
    for (const auto& r : pl.launches) {
        if (r.kind != L_GEMM || !r.plr) continue;
        max_tasks = std::max(max_tasks, r.ntasks);
        long long tot = 0;
        for (int q2 = 0; q2 < r.ntasks; ++q2) {
            const GemmTask<T>& t = pl.tasks[r.off + q2];
            for (int q = 0; q < t.noseg; ++q) tot += (long long)t.oseg_len[q] * t.ldo;
        }
        out_elems = std::max(out_elems, tot);
    }
    if (max_tasks == 0) return;
    PlrStore<T>& ps = plr_store<T>(c);
    C2<T>* sout = alloc_c<T>(c, out_elems);
    GemmTask<T>* dt = (GemmTask<T>*)c->arena.alloc(sizeof(GemmTask<T>) * max_tasks);
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (auto& r : pl.launches) {
        if (r.kind != L_GEMM || !r.plr) continue;
        std::vector<GemmTask<T>> tt(pl.tasks.begin() + r.off, pl.tasks.begin() + r.off + r.ntasks);
        long long at = 0;
        for (auto& t : tt)
            for (int q = 0; q < t.noseg; ++q) {
                t.oseg_ptr[q] = sout + at;
                at += (long long)t.oseg_len[q] * t.ldo;
                t.oseg_add0[q] = nullptr;
                t.oseg_add1[q] = nullptr;
            }
        upload(c, dt, tt.data(), sizeof(GemmTask<T>) * tt.size());
        auto timed = [&](bool compressed) {
            auto once = [&] {
                if (compressed)
                    launch_plr_apply<T>(dt, r.ntasks, r.plr_tiles, r.plr_rows, ps.part, c->st);
                else
                    launch_gemm<T>(dt, r.ntasks, r.max_m, 1, c->st, false, -1, &c->gsw);
            };
            once();                                    // warm-up
            HIPCHK(hipEventRecord(e0, c->st));
            for (int rep = 0; rep < 3; ++rep) once();
            HIPCHK(hipEventRecord(e1, c->st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            return ms;
        };
        const float tp = timed(true), td = timed(false);
        if (td < tp) {
            r.plr = false;
            r.bytes = r.bytes_dense;
        }
    }
    HIPCHK(hipGetLastError());
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->arena.release(sout, 0);
    c->arena.release(dt, 0);
}

template <typename T>
Plan<T>& get_plan(hz_ctx* c, bool sie, int B) {
    Work<T>& w = work<T>(c);
    auto& mp = sie ? w.sie : w.pre;
    auto it = mp.find(B);
    if (it != mp.end()) return *it->second;
    auto pl = std::make_unique<Plan<T>>();
    pl->name = fam_name<T>(sie ? "sie_graph" : "precond_graph");
    pl->inner_loose = !sie;
    if (sie) build_sie_plan<T>(c, *pl, B);
    else build_pre_plan<T>(c, *pl, B);
    if (!sie && B == 1) {
        plr_mark<T>(c, *pl);
        tune_plr<T>(c, *pl);
    }
    tune_plan<T>(c, *pl, B);
    plan_upload<T>(c, *pl);
    Plan<T>& ref = *pl;
    mp[B] = std::move(pl);
    return ref;
}

// ---------------------------------------------------------------------------
// nested polarized traces (Sec. 4.2.1): the inner SIE of each layer job as a
// polarized system over the cells (the outer system with layers -> cells),
// iterated by GMRES with the inner Gauss-Seidel sweeps.  The blocks are the
// pair-column samples CP of the cell probes: no inner block is factorised.

constexpr int INNER_MAXIT = 40;

void givens(std::complex<double> a, std::complex<double> b, double& cs, std::complex<double>& sn);

// The inner GMRES keeps its least-squares bookkeeping on the device, one
// thread per right-hand-side column (a single workgroup: the columns are at
// most a few thousand and each does O(j) work per iteration), so that the
// host reads one convergence flag per iteration instead of the Hessenberg
// column.  The arithmetic is that of the host GMRES: complex Givens
// rotations r = (c, s) with c real, zeroing the subdiagonal entry.
constexpr int INNER_STEP_THREADS = 1024;

__device__ inline double cabs_d(double2 a) { return hypot(a.x, a.y); }

// rotation (cs, sn) with  [cs sn; -conj(sn) cs] [a; b] = [r; 0]
__device__ inline void givens_dev(double2 a, double2 b, double& cs, double2& sn) {
    const double ab = cabs_d(b), aa = cabs_d(a);
    if (ab == 0.0) { cs = 1.0; sn = make_double2(0.0, 0.0); return; }
    if (aa == 0.0) { cs = 0.0; sn = make_double2(b.x / ab, -b.y / ab); return; }
    const double t = hypot(aa, ab);
    cs = aa / t;
    const double2 an = make_double2(a.x / aa, a.y / aa);
    sn = cscale(cmul(an, cconj(b)), 1.0 / t);
}

// start: beta = |r0| per column (hb holds |r0|^2), g = beta e_1, columns with
// r0 = 0 done; scale = 1 / beta for the first basis vector
__global__ void __launch_bounds__(INNER_STEP_THREADS)
k_inner_start(const double2* __restrict__ hb, int NB, double* __restrict__ beta,
              double2* __restrict__ g, int* __restrict__ done, int* __restrict__ kfin,
              double2* __restrict__ scale) {
    for (int q = threadIdx.x; q < NB; q += blockDim.x) {
        const double b = sqrt(fmax(0.0, hb[q].x));
        beta[q] = b;
        g[q] = make_double2(b, 0.0);
        done[q] = b == 0.0;
        kfin[q] = 0;
        scale[q] = make_double2(b > 0.0 ? 1.0 / b : 0.0, 0.0);
    }
}

// Arnoldi step j: the new Hessenberg column (projections of both Gram-Schmidt
// passes hA + hB, subdiagonal sqrt(hN)) is rotated by the stored rotations,
// a new rotation zeroes its subdiagonal, the rotated residual g is updated
// and the column is done once |g_{j+1}| <= tol beta.  flag[j] = 1 when every
// column is done.
__global__ void __launch_bounds__(INNER_STEP_THREADS)
k_inner_step(int j, int NB, const double2* __restrict__ hA, const double2* __restrict__ hB,
             const double2* __restrict__ hN, double2* __restrict__ R, double* __restrict__ cs,
             double2* __restrict__ sn, double2* __restrict__ g, const double* __restrict__ beta,
             int* __restrict__ done, int* __restrict__ kfin, double tol, int* __restrict__ flag) {
    int mine = 1;
    double2* Rc = R + (long long)j * (j + 1) / 2 * NB;     // packed column j
    for (int q = threadIdx.x; q < NB; q += blockDim.x) {
        if (done[q]) continue;
        // projections of the two Gram-Schmidt passes (hB null: one pass)
        double2 a = hB ? cadd(hA[q], hB[q]) : hA[q];
        for (int i = 0; i < j; ++i) {
            const long long at = (long long)(i + 1) * NB + q;
            const double2 b = hB ? cadd(hA[at], hB[at]) : hA[at];
            const double ci = cs[(long long)i * NB + q];
            const double2 si = sn[(long long)i * NB + q];
            Rc[(long long)i * NB + q] = cadd(cscale(a, ci), cmul(si, b));
            a = cadd(cscale(cmul(cconj(si), a), -1.0), cscale(b, ci));
        }
        const double nrm = sqrt(fmax(0.0, hN[q].x));
        double cj;
        double2 sj;
        givens_dev(a, make_double2(nrm, 0.0), cj, sj);
        cs[(long long)j * NB + q] = cj;
        sn[(long long)j * NB + q] = sj;
        Rc[(long long)j * NB + q] = cadd(cscale(a, cj), cscale(sj, nrm));
        const double2 gj = g[(long long)j * NB + q];
        const double2 gn = cscale(cmul(cconj(sj), gj), -1.0);
        g[(long long)(j + 1) * NB + q] = gn;
        g[(long long)j * NB + q] = cscale(gj, cj);
        kfin[q] = j + 1;
        if (cabs_d(gn) / beta[q] <= tol || nrm == 0.0) done[q] = 1;
        else mine = 0;
    }
    const int all = __syncthreads_and(mine);
    if (threadIdx.x == 0) flag[j] = all;
}

// y = R^{-1} g over the first kfin[q] rows of each column; coefficients of the
// basis vectors, zero from kfin[q] to kmax
__global__ void k_inner_solve_y(int NB, int kmax, const double2* __restrict__ R,
                                const double2* __restrict__ g, const int* __restrict__ kfin,
                                double2* __restrict__ coef) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= NB) return;
    const int k = kfin[q];
    for (int i = kmax - 1; i >= 0; --i) {
        double2 y = make_double2(0.0, 0.0);
        if (i < k) {
            double2 acc = g[(long long)i * NB + q];
            for (int p2 = i + 1; p2 < k; ++p2)
                acc = csub(acc, cmul(R[((long long)p2 * (p2 + 1) / 2 + i) * NB + q],
                                     coef[(long long)p2 * NB + q]));
            const double2 d = R[((long long)i * (i + 1) / 2 + i) * NB + q];
            const double den = 1.0 / (d.x * d.x + d.y * d.y);
            y = cscale(cmul(acc, cconj(d)), den);
        }
        coef[(long long)i * NB + q] = y;
    }
}
void update_dots_dev(hz_ctx* c, const double2* V, long long vstride, int nv, const double2* coef,
                     double2* w, long long n, int B, int norm, double2* out_dev,
                     double2* part, int max_chunks);

struct InnerJobDev {
    const void* rhs;
    void* out;
    int HL;
    int pad;
};

// rhs_i [d|q][2 J HL_i][B] -> column block i of dst (rows dq 2 J HLmax + r)
template <typename T>
__global__ void k_inner_pack(const InnerJobDev* jobs, C2<T>* dst, int J, int HLmax, int B,
                             long long ld) {
    const InnerJobDev jb = jobs[blockIdx.y];
    const long long rows = 2LL * J * jb.HL;
    const long long total = 2 * rows * B;
    const C2<T>* src = (const C2<T>*)jb.rhs;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const long long rr = q / B;
        const int b = (int)(q - rr * B);
        const int dq = rr >= rows ? 1 : 0;
        const long long r = rr - dq * rows;
        dst[(dq * 2LL * J * HLmax + r) * ld + (long long)blockIdx.y * B + b] = src[q];
    }
}

// traces s = d + q of column block i of x -> out_i [2 J HL_i][B]
template <typename T>
__global__ void k_inner_unpack(const InnerJobDev* jobs, const C2<T>* x, int J, int HLmax, int B,
                               long long ld) {
    const InnerJobDev jb = jobs[blockIdx.y];
    const long long rows = 2LL * J * jb.HL;
    const long long total = rows * B;
    const long long qoff = 2LL * J * HLmax * ld;
    C2<T>* out = (C2<T>*)jb.out;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < total;
         q += (long long)gridDim.x * blockDim.x) {
        const long long r = q / B;
        const int b = (int)(q - r * B);
        const long long at = r * ld + (long long)blockIdx.y * B + b;
        out[q] = cadd(x[at], x[at + qoff]);
    }
}

// pair (rows a then b) of interface j, d (dq = 0) or q (dq = 1), job i
template <typename T>
C2<T>* iw_pair(hz_ctx* c, const InnerRec<T>& r, C2<T>* v, int i, int dq, int j) {
    const int J = c->d.Lc - 1;
    const int HL = c->layers[r.jobs[i].layer].HL;
    const int B = r.ncols / (int)r.jobs.size();
    return v + ((long long)dq * 2 * J * c->d.HLmax + (long long)j * 2 * HL) * r.ncols +
           (long long)i * B;
}

// rows of cell cd's pair-column samples on its left (right = 0) or right pair
template <typename T>
const C2<T>* cp_rows(hz_ctx* c, const CellDesc& cd, int right) {
    return ops<T>(c).CP + cd.off_CP + (right && cd.has_left ? 2LL * cd.HL : 0) * cd.R;
}

// inner M: wA -> wB (s = d + q in S)
template <typename T>
void build_inner_M(hz_ctx* c, InnerRec<T>& r, Plan<T>& pl, int B) {
    const int J = c->d.Lc - 1;
    const long long half = 2LL * J * c->d.HLmax * r.ncols;
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
    add_vec<T>(pl, L_COPY, r.S, r.wA, zero, zero, half);
    add_vec<T>(pl, L_AXPBY, r.S, r.wA + half, one, one, half);
    const long long first = pl.tasks.size();
    int maxm = 0;
    for (int i = 0; i < (int)r.jobs.size(); ++i) {
        const LayerDesc& ld = c->layers[r.jobs[i].layer];
        const int HL = ld.HL;
        const long long hb = (long long)HL * r.ncols;
        for (int j = 0; j < J; ++j) {
            // right rows of cell j: d_j + E_a q_j - R_right[G_T(s_{j-1}) + G_B(q_j)]
            const CellDesc& cj = c->cells[ld.cell_begin + j];
            GemmTask<T> t = blank_task<T>();
            t.A = cp_rows<T>(c, cj, 1);
            t.lda = cj.R;
            t.m = 2 * HL;
            t.ldx = r.ncols; t.ldo = r.ncols;
            t.nseg = 0;
            if (cj.has_left) {
                t.seg_k0[t.nseg] = 0; t.seg_len[t.nseg] = 2 * HL;
                t.seg_ptr[t.nseg] = iw_pair<T>(c, r, r.S, i, 0, j - 1);
                t.nseg++;
            }
            t.seg_k0[t.nseg] = cj.has_left ? 2 * HL : 0; t.seg_len[t.nseg] = 2 * HL;
            t.seg_ptr[t.nseg] = iw_pair<T>(c, r, r.wA, i, 1, j);
            t.nseg++;
            t.k = (cj.has_left ? 2 * HL : 0) + 2 * HL;
            t.noseg = 2;
            t.oseg_i0[0] = 0; t.oseg_len[0] = HL;
            t.oseg_ptr[0] = iw_pair<T>(c, r, r.wB, i, 0, j);
            t.oseg_add0[0] = iw_pair<T>(c, r, r.wA, i, 0, j);
            t.oseg_add1[0] = iw_pair<T>(c, r, r.wA, i, 1, j);
            t.c1[0] = (T)1;
            t.oseg_i0[1] = HL; t.oseg_len[1] = HL;
            t.oseg_ptr[1] = iw_pair<T>(c, r, r.wB, i, 0, j) + hb;
            t.oseg_add0[1] = iw_pair<T>(c, r, r.wA, i, 0, j) + hb;
            t.alpha = (T)-1;
            pl.tasks.push_back(t);
            // left rows of cell j+1: q_j + E_b d_j - R_left[G_T(d_j) + G_B(s_{j+1})]
            const CellDesc& cn = c->cells[ld.cell_begin + j + 1];
            GemmTask<T> u = blank_task<T>();
            u.A = cp_rows<T>(c, cn, 0);
            u.lda = cn.R;
            u.m = 2 * HL;
            u.ldx = r.ncols; u.ldo = r.ncols;
            u.nseg = 1;
            u.seg_k0[0] = 0; u.seg_len[0] = 2 * HL;
            u.seg_ptr[0] = iw_pair<T>(c, r, r.wA, i, 0, j);
            if (cn.has_right) {
                u.seg_k0[1] = 2 * HL; u.seg_len[1] = 2 * HL;
                u.seg_ptr[1] = iw_pair<T>(c, r, r.S, i, 0, j + 1);
                u.nseg = 2;
            }
            u.k = 2 * HL + (cn.has_right ? 2 * HL : 0);
            u.noseg = 2;
            u.oseg_i0[0] = 0; u.oseg_len[0] = HL;
            u.oseg_ptr[0] = iw_pair<T>(c, r, r.wB, i, 1, j);
            u.oseg_add0[0] = iw_pair<T>(c, r, r.wA, i, 1, j);
            u.oseg_i0[1] = HL; u.oseg_len[1] = HL;
            u.oseg_ptr[1] = iw_pair<T>(c, r, r.wB, i, 1, j) + hb;
            u.oseg_add0[1] = iw_pair<T>(c, r, r.wA, i, 1, j) + hb;
            u.oseg_add1[1] = iw_pair<T>(c, r, r.wA, i, 0, j) + hb;
            u.c1[1] = (T)1;
            u.alpha = (T)-1;
            pl.tasks.push_back(u);
            maxm = std::max(maxm, 2 * HL);
        }
    }
    add_launch(pl, first, maxm, B);
}

// inner P^GS: wB -> wC (rightward sweep, reflections, leftward sweep)
template <typename T>
void build_inner_P(hz_ctx* c, InnerRec<T>& r, Plan<T>& pl, int B) {
    const int J = c->d.Lc - 1;
    const int NJ = (int)r.jobs.size();
    const double2 zero = make_double2(0.0, 0.0);
    add_vec<T>(pl, L_COPY, r.wC, r.wB, zero, zero, r.n * r.ncols);
    for (int j = 1; j < J; ++j) {                   // x_j = v_j + R_right^j G_T^j(x_{j-1})
        const long long first = pl.tasks.size();
        int maxm = 0;
        for (int i = 0; i < NJ; ++i) {
            const LayerDesc& ld = c->layers[r.jobs[i].layer];
            const int HL = ld.HL;
            const CellDesc& cj = c->cells[ld.cell_begin + j];
            GemmTask<T> t = blank_task<T>();
            t.A = cp_rows<T>(c, cj, 1);
            t.lda = cj.R;
            t.m = 2 * HL; t.k = 2 * HL;
            t.ldx = r.ncols; t.ldo = r.ncols;
            t.nseg = 1;
            t.seg_k0[0] = 0; t.seg_len[0] = 2 * HL;
            t.seg_ptr[0] = iw_pair<T>(c, r, r.wC, i, 0, j - 1);
            t.noseg = 1;
            t.oseg_i0[0] = 0; t.oseg_len[0] = 2 * HL;
            t.oseg_ptr[0] = iw_pair<T>(c, r, r.wC, i, 0, j);
            t.oseg_add0[0] = iw_pair<T>(c, r, r.wB, i, 0, j);
            t.alpha = (T)1;
            pl.tasks.push_back(t);
            maxm = std::max(maxm, 2 * HL);
        }
        add_launch(pl, first, maxm, B);
    }
    {   // t_j = v^q_j - E_b x_j + R_left^{j+1}[G_T(x_j) + G_B(x_{j+1})]  (all j at once)
        const long long first = pl.tasks.size();
        int maxm = 0;
        for (int i = 0; i < NJ; ++i) {
            const LayerDesc& ld = c->layers[r.jobs[i].layer];
            const int HL = ld.HL;
            const long long hb = (long long)HL * r.ncols;
            for (int j = 0; j < J; ++j) {
                const CellDesc& cn = c->cells[ld.cell_begin + j + 1];
                GemmTask<T> t = blank_task<T>();
                t.A = cp_rows<T>(c, cn, 0);
                t.lda = cn.R;
                t.m = 2 * HL;
                t.ldx = r.ncols; t.ldo = r.ncols;
                t.nseg = 1;
                t.seg_k0[0] = 0; t.seg_len[0] = 2 * HL;
                t.seg_ptr[0] = iw_pair<T>(c, r, r.wC, i, 0, j);
                if (cn.has_right) {
                    t.seg_k0[1] = 2 * HL; t.seg_len[1] = 2 * HL;
                    t.seg_ptr[1] = iw_pair<T>(c, r, r.wC, i, 0, j + 1);
                    t.nseg = 2;
                }
                t.k = 2 * HL + (cn.has_right ? 2 * HL : 0);
                t.noseg = 2;
                t.oseg_i0[0] = 0; t.oseg_len[0] = HL;
                t.oseg_ptr[0] = iw_pair<T>(c, r, r.wC, i, 1, j);
                t.oseg_add0[0] = iw_pair<T>(c, r, r.wB, i, 1, j);
                t.oseg_i0[1] = HL; t.oseg_len[1] = HL;
                t.oseg_ptr[1] = iw_pair<T>(c, r, r.wC, i, 1, j) + hb;
                t.oseg_add0[1] = iw_pair<T>(c, r, r.wB, i, 1, j) + hb;
                t.oseg_add1[1] = iw_pair<T>(c, r, r.wC, i, 0, j) + hb;
                t.c1[1] = (T)-1;
                t.alpha = (T)1;
                pl.tasks.push_back(t);
                maxm = std::max(maxm, 2 * HL);
            }
        }
        add_launch(pl, first, maxm, B);
    }
    for (int j = J - 2; j >= 0; --j) {              // x_j = t_j + R_left^{j+1} G_B^{j+1}(x_{j+1})
        const long long first = pl.tasks.size();
        int maxm = 0;
        for (int i = 0; i < NJ; ++i) {
            const LayerDesc& ld = c->layers[r.jobs[i].layer];
            const int HL = ld.HL;
            const CellDesc& cn = c->cells[ld.cell_begin + j + 1];
            GemmTask<T> t = blank_task<T>();
            t.A = cp_rows<T>(c, cn, 0) + 2 * HL;          // right probes (cell j+1 has a left pair)
            t.lda = cn.R;
            t.m = 2 * HL; t.k = 2 * HL;
            t.ldx = r.ncols; t.ldo = r.ncols;
            t.nseg = 1;
            t.seg_k0[0] = 0; t.seg_len[0] = 2 * HL;
            t.seg_ptr[0] = iw_pair<T>(c, r, r.wC, i, 1, j + 1);
            t.noseg = 1;
            t.oseg_i0[0] = 0; t.oseg_len[0] = 2 * HL;
            t.oseg_ptr[0] = iw_pair<T>(c, r, r.wC, i, 1, j);
            t.oseg_add0[0] = iw_pair<T>(c, r, r.wC, i, 1, j);
            t.alpha = (T)1;
            pl.tasks.push_back(t);
            maxm = std::max(maxm, 2 * HL);
        }
        add_launch(pl, first, maxm, B);
    }
}

void ensure_inner_basis(hz_ctx* c, long long nB, int m, int cols) {
    if (c->i_cap >= nB && c->i_cap_m >= m && c->i_cap_cols >= cols) return;
    for (void* q : {(void*)c->iV, (void*)c->ipart, (void*)c->ismall, (void*)c->icoef, (void*)c->ih,
                    (void*)c->iR, (void*)c->isn, (void*)c->ig, (void*)c->ics, (void*)c->ibeta,
                    (void*)c->idone, (void*)c->ikfin, (void*)c->iflag})
        c->arena.release(q, 0);
    nB = std::max(nB, c->i_cap);
    m = std::max(m, c->i_cap_m);
    cols = std::max(cols, c->i_cap_cols);
    c->i_cap = nB; c->i_cap_m = m; c->i_cap_cols = cols;
    // reduction chunks: enough workgroups for short inner vectors, with the
    // partial sums bounded to 2^25 entries
    c->i_chunks = (int)std::max<long long>(8, std::min<long long>(256, (1LL << 25) / ((m + 2) * (long long)cols)));
    c->iV = (double2*)c->arena.alloc(sizeof(double2) * nB * (m + 1));
    c->ipart = (double2*)c->arena.alloc(sizeof(double2) * c->i_chunks * (m + 2) * (long long)cols);
    c->ismall = (double2*)c->arena.alloc(sizeof(double2) * (m + 2) * (long long)cols);
    c->icoef = (double2*)c->arena.alloc(sizeof(double2) * (m + 2) * (long long)cols);
    c->ih = (double2*)c->arena.alloc(sizeof(double2) * (2 * (m + 1) + 1) * (long long)cols);
    const long long cl = cols;
    c->iR = (double2*)c->arena.alloc(sizeof(double2) * ((long long)m * (m + 1) / 2) * cl);
    c->isn = (double2*)c->arena.alloc(sizeof(double2) * m * cl);
    c->ig = (double2*)c->arena.alloc(sizeof(double2) * (m + 1) * cl);
    c->ics = (double*)c->arena.alloc(sizeof(double) * m * cl);
    c->ibeta = (double*)c->arena.alloc(sizeof(double) * cl);
    c->idone = (int*)c->arena.alloc(sizeof(int) * cl);
    c->ikfin = (int*)c->arena.alloc(sizeof(int) * cl);
    c->iflag = (int*)c->arena.alloc(sizeof(int) * (m + 1));
    if (c->h_iflag) (void)hipHostFree(c->h_iflag);
    c->h_iflag = nullptr;
    if (hipHostMalloc((void**)&c->h_iflag, sizeof(int) * (m + 1), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        c->h_iflag = nullptr;
        raise(HZ_ENOMEM, "hipHostMalloc of the inner convergence flags failed");
    }
    if (!c->iev) HIPCHK(hipEventCreateWithFlags(&c->iev, hipEventDisableTiming));
}

template <typename T>
void inner_setup(hz_ctx* c, InnerRec<T>& r, int B) {
    const Dims& d = c->d;
    const int J = d.Lc - 1;
    const int NJ = (int)r.jobs.size();
    r.n = 4LL * J * d.HLmax;
    r.ncols = NJ * B;
    r.ar = &c->arena;
    const long long nB = r.n * r.ncols;
    r.wA = alloc_c<T>(c, nB);
    r.wB = alloc_c<T>(c, nB);
    r.wC = alloc_c<T>(c, nB);
    r.S = alloc_c<T>(c, nB / 2);
    // padding rows stay zero: the plans write the rows of each job only
    for (C2<T>* q : {r.wA, r.wB, r.wC})
        HIPCHK(hipMemsetAsync(q, 0, sizeof(C2<T>) * nB, c->st));
    HIPCHK(hipMemsetAsync(r.S, 0, sizeof(C2<T>) * (nB / 2), c->st));
    std::vector<InnerJobDev> tab(NJ);
    for (int i = 0; i < NJ; ++i)
        tab[i] = {r.jobs[i].rhs, r.jobs[i].out, c->layers[r.jobs[i].layer].HL, 0};
    r.jobtab = c->arena.alloc(sizeof(InnerJobDev) * NJ);
    upload(c, r.jobtab, tab.data(), sizeof(InnerJobDev) * NJ);
    r.M = std::make_unique<Plan<T>>();
    r.M->name = fam_name<T>("inner_m_graph");
    build_inner_M<T>(c, r, *r.M, B);
    tune_plan<T>(c, *r.M, B);
    r.P = std::make_unique<Plan<T>>();
    r.P->name = fam_name<T>("inner_p_graph");
    build_inner_P<T>(c, r, *r.P, B);
    tune_plan<T>(c, *r.P, B);
    plan_upload<T>(c, *r.M);
    plan_upload<T>(c, *r.P);
}

// Left-preconditioned GMRES on the inner polarized systems of a record, x0 =
// 0, classical Gram-Schmidt with one re-orthogonalisation, per-column
// stopping on the preconditioned residual (the outer driver's scheme, one
// column per job and right-hand side).
template <typename T>
void inner_solve(hz_ctx* c, InnerRec<T>& r, int B) {
    if constexpr (sizeof(T) != sizeof(double)) {
        (void)c; (void)r; (void)B;
        raise(HZ_EINVAL, "nested polarized traces run in complex128 only");
    } else {
        const Dims& d = c->d;
        const int J = d.Lc - 1;
        if (!r.M) inner_setup<T>(c, r, B);
        const long long n = r.n;
        const int NB = r.ncols;
        const int NJ = (int)r.jobs.size();
        const long long nB = n * NB;
        const int m = INNER_MAXIT;
        const double tol = r.loose ? c->inner_tol_loose
                                   : (c->inner_tol_solve > 0 ? c->inner_tol_solve : c->inner_tol_tight);
        ensure_inner_basis(c, nB, m, NB);
        const int chunks = (int)std::min<long long>(c->i_chunks, std::max<long long>(1, n / 8));
        auto idots = [&](const double2* V, int nv, const double2* w, double2* out) {
            launch_dots(V, nB, nv, w, n, NB, c->ipart, chunks, c->st);
            launch_reduce_partials(c->ipart, chunks, nv * NB, out, c->st);
        };
        const dim3 pg(std::max<int>(1, (int)std::min<long long>(4096, (2 * n * B + 255) / 256)), NJ);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inner_pack<T>), pg, dim3(256), 0, c->st,
                           (const InnerJobDev*)r.jobtab, r.wB, J, d.HLmax, B, (long long)NB);
        plan_run<T>(c, *r.P, B);                       // r0 = P b
        double2* V = c->iV;
        HIPCHK(hipMemcpyAsync(V, r.wC, sizeof(double2) * nB, hipMemcpyDeviceToDevice, c->st));
        idots(nullptr, 1, V, c->ismall);
        hipLaunchKernelGGL(k_inner_start, dim3(1), dim3(INNER_STEP_THREADS), 0, c->st, c->ismall, NB,
                           c->ibeta, c->ig, c->idone, c->ikfin, c->icoef);
        launch_scale_cols(V, V, c->icoef, n, NB, c->st, r.wA);   // v_0, also the plans' input
        // The host reads one flag per iteration: every column done.  (Reading
        // it one iteration behind, so that the next one is already queued,
        // was slower: the extra iteration costs more than the wait.)
        int j = 0;
        for (; j < m; ++j) {
            double2* Vn = V + (long long)(j + 1) * nB;
            plan_run<T>(c, *r.M, B);                   // reads v_j from wA
            plan_run<T>(c, *r.P, B);                   // w = P M v_j in wC
            double2* w = r.wC;
            const size_t nh = (size_t)(j + 1) * NB;
            double2* hA = c->ih;
            double2* hB2 = c->ih + nh;
            double2* hN = c->ih + 2 * nh;
            // classical Gram-Schmidt, twice for the tight inner solves and
            // once for the preconditioner's (tolerance 1e-6: the loss of
            // orthogonality of a single pass over a few vectors is far below
            // it); the new vector also goes to wA, the plans' input
            idots(V, j + 1, w, hA);
            const bool cgs2 = !r.loose;
            if (cgs2) {
                update_dots_dev(c, V, nB, j + 1, hA, w, n, NB, 0, hB2, c->ipart, chunks);
                update_dots_dev(c, V, nB, j + 1, hB2, w, n, NB, 1, hN, c->ipart, chunks);
            } else {
                update_dots_dev(c, V, nB, j + 1, hA, w, n, NB, 1, hN, c->ipart, chunks);
            }
            launch_scale_cols_inv_norm(Vn, r.wA, w, hN, n, NB, c->st);
            hipLaunchKernelGGL(k_inner_step, dim3(1), dim3(INNER_STEP_THREADS), 0, c->st, j, NB,
                               (const double2*)hA, cgs2 ? (const double2*)hB2 : nullptr,
                               (const double2*)hN, c->iR,
                               c->ics, c->isn, c->ig, (const double*)c->ibeta, c->idone, c->ikfin,
                               tol, c->iflag);
            HIPCHK(hipMemcpyAsync(c->h_iflag + j, c->iflag + j, sizeof(int), hipMemcpyDeviceToHost,
                                  c->st));
            HIPCHK(hipEventRecord(c->iev, c->st));
            HIPCHK(hipEventSynchronize(c->iev));
            if (c->h_iflag[j]) { ++j; break; }
        }
        c->inner_iters_max = std::max(c->inner_iters_max, j);
        // x = V y into wA (coefficients zero beyond each column's own
        // iteration count), then the traces s = d + q of every job
        const int kmax = j;
        HIPCHK(hipMemsetAsync(r.wA, 0, sizeof(double2) * nB, c->st));
        if (kmax > 0) {
            hipLaunchKernelGGL(k_inner_solve_y, dim3((NB + 255) / 256), dim3(256), 0, c->st, NB, kmax,
                               (const double2*)c->iR, (const double2*)c->ig,
                               (const int*)c->ikfin, c->icoef);
            launch_update_basis(r.wA, V, nB, kmax, c->icoef, n, NB, c->st);
        }
        const dim3 ug(std::max<int>(1, (int)std::min<long long>(4096, (n * B / 2 + 255) / 256)), NJ);
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inner_unpack<T>), ug, dim3(256), 0, c->st,
                           (const InnerJobDev*)r.jobtab, r.wA, J, d.HLmax, B, (long long)NB);
        HIPCHK(hipGetLastError());
    }
}

// ---------------------------------------------------------------------------
// workspaces

// Workspaces for batches up to max_batch.  `volume` adds the volume-solve
// buffers (sources, solutions, cell-solve scratch); the vectors of the
// interface operators are always allocated.
void ensure_refine(hz_ctx* c);

template <typename T>
void ensure_work(hz_ctx* c, int B, bool volume = true) {
    Work<T>& w = work<T>(c);
    const Dims& d = c->d;
    const long long W = d.W;
    if (B > std::max(c->prm.max_batch, 1)) raise(HZ_EINVAL, "batch larger than max_batch");
    B = std::max(B, c->prm.max_batch);
    if (volume && !w.f_ext) {
        if constexpr (sizeof(T) == sizeof(double)) {
            // the FP64 volume buffers are the context's f64 / u64 (same size
            // and layout): solves copy nothing in or out
            ensure_refine(c);
            w.f_ext = c->f64;
            w.u_ext = c->u64;
        } else {
            w.f_ext = alloc_c<T>(c, W * W * B);
            w.u_ext = alloc_c<T>(c, W * W * B);
        }
        w.rows_out = alloc_c<T>(c, (long long)d.L * MAXSLOT * W * B);
        const long long inner = std::max<long long>((long long)d.L * c->inner_per_layer * B, 1);
        w.gf = alloc_c<T>(c, (c->inner_pt ? 2 : 1) * inner);
        // cell-solve scratch: one region per workgroup of a volume solve
        const int nb = cs_nb_cap(B);
        const int chunks = (B + nb - 1) / nb;
        w.y_stride = (long long)d.Wcmax * d.HLpmax * nb;
        w.y_wgs = (int)c->cells.size() * chunks;
        w.Y = alloc_c<T>(c, w.y_stride * w.y_wgs);
    }
    if (w.Bcap >= B) return;
    w.Bcap = B;
    const long long inner = std::max<long long>((long long)d.L * c->inner_per_layer * B, 1);
    for (int s = 0; s < 2; ++s) {
        w.iy[s] = alloc_c<T>(c, (c->inner_pt ? 2 : 1) * inner);   // polarized: [d|q]
        w.ix[s] = alloc_c<T>(c, inner);
    }
    const long long pol = std::max<long long>(4LL * d.K * W * B, 1);
    w.pA = alloc_c<T>(c, pol);
    w.pB = alloc_c<T>(c, pol);
    w.pC = alloc_c<T>(c, pol);
    w.sv = alloc_c<T>(c, std::max<long long>(2LL * d.K * W * B, 1));
    w.pair_tab = (const C2<T>**)c->arena.alloc(sizeof(C2<T>*) * 2 * d.L);
}

// per-layer (top, bottom) trace pairs inside w.sv for the current batch size
template <typename T>
void upload_pair_tab(hz_ctx* c, int B) {
    Work<T>& w = work<T>(c);
    const Dims& d = c->d;
    std::vector<const C2<T>*> tab(2 * d.L, nullptr);
    const long long pairn = 2LL * d.W * B;
    for (int l = 0; l < d.L; ++l) {
        if (l > 0) tab[l] = w.sv + (long long)(l - 1) * pairn;
        if (l < d.L - 1) tab[d.L + l] = w.sv + (long long)l * pairn;
    }
    upload(c, (void*)w.pair_tab, tab.data(), sizeof(C2<T>*) * 2 * d.L);
}

void ensure_gmres(hz_ctx* c, int B, int m) {
    if (c->g_cap_B >= B && c->g_cap_m >= m) return;
    const long long n = 4LL * c->d.K * c->d.W;
    if (c->V) {
        c->arena.release(c->V, 0);
        c->arena.release(c->gw, 0);
        c->arena.release(c->gb, 0);
        c->arena.release(c->gx, 0);
        c->arena.release(c->gpart, 0);
        c->arena.release(c->gsmall, 0);
        c->arena.release(c->gcoef, 0);
        c->arena.release(c->gh, 0);
    }
    B = std::max(B, c->g_cap_B);
    m = std::max(m, c->g_cap_m);
    c->g_cap_B = B;
    c->g_cap_m = m;
    const long long nb = std::max<long long>(n * B, 1);
    c->V = (double2*)c->arena.alloc(sizeof(double2) * nb * (m + 1));
    if (c->prm.precision == HZ_MIXED || c->inner_pt) {
        if (c->Z) c->arena.release(c->Z, 0);
        c->Z = (double2*)c->arena.alloc(sizeof(double2) * nb * m);
    }
    c->gw = (double2*)c->arena.alloc(sizeof(double2) * nb);
    c->gb = (double2*)c->arena.alloc(sizeof(double2) * nb);
    c->gx = (double2*)c->arena.alloc(sizeof(double2) * nb);
    c->gpart_chunks = 1024;
    c->gpart = (double2*)c->arena.alloc(sizeof(double2) * c->gpart_chunks * (m + 2) * B);
    c->gsmall = (double2*)c->arena.alloc(sizeof(double2) * (m + 2) * B);
    c->gcoef = (double2*)c->arena.alloc(sizeof(double2) * (m + 2) * B);
    c->gh = (double2*)c->arena.alloc(sizeof(double2) * (2 * (m + 1) + 1) * B);
}

// ---------------------------------------------------------------------------
// offline stage

template <typename T>
void cell_solve_launch(hz_ctx* c, CellSolveArgs<T> a, const std::vector<int>& list, int Bcols) {
    Work<T>& w = work<T>(c);
    // a contiguous run of cells is a slice of the all-cells table; other
    // lists go to the persistent list buffer (no allocation per solve)
    bool contiguous = true;
    for (size_t i = 1; i < list.size(); ++i) contiguous = contiguous && list[i] == list[0] + (int)i;
    const int* d_list = c->d_all_cells + (list.empty() ? 0 : list[0]);
    if (!contiguous) {
        upload(c, c->d_cell_list, list.data(), sizeof(int) * list.size());
        d_list = c->d_cell_list;
    }
    // all cells of the list with nb batch columns per workgroup, in groups
    // limited by the scratch available
    auto run = [&](int nb, bool prof) {
        const int chunks = (Bcols + nb - 1) / nb;
        const long long wg_elems = (long long)c->d.Wcmax * c->d.HLpmax * nb;
        const int per = (int)std::max<long long>(1, (w.y_stride * w.y_wgs / wg_elems) / chunks);
        a.nb = nb;
        for (size_t g = 0; g < list.size(); g += per) {
            const int cnt = (int)std::min<size_t>(per, list.size() - g);
            a.cell_list = d_list + g;
            a.B = Bcols;
            a.Y = w.Y;
            a.y_stride = wg_elems;
            size_t e0 = prof ? prof_event(c) : 0;
            launch_cell_solve<T>(a, cnt, chunks, c->st);
            HIPCHK(hipGetLastError());
            if (prof) {
                size_t e1 = prof_event(c);
                double bytes = 0, flops = 0;
                for (int q = 0; q < cnt; ++q) {
                    const CellDesc& cd = c->cells[list[g + q]];
                    // the sweeps run over the live columns only (from the left
                    // pair column or the first own column; see the kernels)
                    int k0 = cd.own_c0;
                    if (cd.has_left) k0 = std::min(k0, c->d.p - 1);
                    const double wl = (double)(cd.Wc - std::max(k0, 0));
                    const double blk = wl * cd.HL * cd.HL;
                    // factors read in both sweeps, forward iterates written and
                    // read back, one source and one result per grid node
                    bytes += sizeof(C2<T>) * (2.0 * blk + 4.0 * wl * cd.HL * Bcols);
                    flops += 8.0 * (2.0 * wl - 1.0) * cd.HL * cd.HL * Bcols;
                }
                const char* fam = a.mode == SOLVE_VOLUME ? "cell_solve_volume"
                                  : a.mode == SOLVE_SAMPLE ? "cell_solve_sample" : "cell_solve_other";
                c->prof.pend.push_back({fam_name<T>(fam), e0, e1, bytes, flops});
            }
        }
    };
    int nb = cs_nb(Bcols, (int)list.size(), c->d.HLpmax, (int)sizeof(C2<T>));
    // Autotune the batch width once per (mode, batch, cells): the solve itself
    // is timed with each candidate and the chosen width's output is kept (the
    // matrix-core widths give the same results column by column; the
    // 4-column kernel differs from them by rounding).
    const bool tunable = c->tune && Bcols > 16 && !std::getenv("HZ_CELL_NB") &&
                         (a.mode == SOLVE_SAMPLE || a.mode == SOLVE_VOLUME);
    if (tunable) {
        const std::string key = std::to_string(a.mode) + "|" + std::to_string(Bcols) + "|" +
                                std::to_string(list.size()) + "|" + std::to_string(sizeof(T));
        auto it = c->cs_tuned.find(key);
        if (it != c->cs_tuned.end()) {
            nb = it->second;
        } else {
            hipEvent_t e0, e1;
            HIPCHK(hipEventCreate(&e0));
            HIPCHK(hipEventCreate(&e1));
            float best = 1e30f;
            int best_nb = nb;
            // 4 columns per workgroup (the matrix-vector kernel) only for
            // launches of few workgroups: it reads the factors once per 4
            // columns, but keeps more of them in flight per cell
            const bool narrow = (long long)list.size() * ((Bcols + 15) / 16) < 256;
            int last = 0;
            for (int cand : {32, 16, 4}) {
                if (cand == 32 && cs_nb_max(c->d.HLpmax, (int)sizeof(C2<T>)) < 32) continue;
                if (cand == 4 && !narrow) continue;
                HIPCHK(hipEventRecord(e0, c->st));
                run(cand, false);
                HIPCHK(hipEventRecord(e1, c->st));
                HIPCHK(hipEventSynchronize(e1));
                last = cand;
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                // the earlier candidate is kept unless a later one is more
                // than 3% faster
                if (best == 1e30f || ms < 0.97f * best) { best = ms; best_nb = cand; }
            }
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            c->cs_tuned[key] = best_nb;
            if (best_nb == last) return;         // the last run already wrote the result
            nb = best_nb;
        }
    }
    run(nb, c->prof.on);
}

template <typename T>
CellSolveArgs<T> base_args(hz_ctx* c) {
    CellSolveArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    Ops<T>& o = ops<T>(c);
    a.cells = c->d_cells;
    a.layers = c->d_layers;
    a.X = o.X;
    a.coef_e = o.e;
    a.alpha_x = c->ax_pool;
    a.alpha_z = c->az_pool;
    a.h = c->d.h;
    a.n = c->d.n;
    a.p = c->d.p;
    a.W = c->d.W;
    a.HLmax = c->d.HLmax;
    a.Wcmax = c->d.Wcmax;
    return a;
}

template <typename T>
__global__ void k_inner_diag(const LayerDesc* layers, const int* lays, const CellDesc* cells,
                             const C2<T>* CS, int j, C2<T>* out, long long out_stride) {
    const LayerDesc ld = layers[lays[blockIdx.y]];
    const int HL = ld.HL;
    const int n2 = 2 * HL;
    const CellDesc cl = cells[ld.cell_begin + j];        // left of interface j
    const CellDesc cr = cells[ld.cell_begin + j + 1];    // right of interface j
    C2<T>* o = out + (long long)blockIdx.y * out_stride;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < (long long)n2 * n2;
         q += (long long)gridDim.x * blockDim.x) {
        const int r = (int)(q / n2), col = (int)(q % n2);
        C2<T> v;
        if (r < HL) {       // row a: right-column samples of cell j, its right probes
            const int row = (cl.has_left ? HL : 0) + r;
            const int pc = (cl.has_left ? 2 * HL : 0) + col;
            v = CS[cl.off_CS + (long long)row * cl.R + pc];
        } else {            // row b: left-column samples of cell j+1, its left probes
            v = CS[cr.off_CS + (long long)(r - HL) * cr.R + col];
        }
        v.x = -v.x; v.y = -v.y;
        if (r == col) v.x += (T)1;
        o[q] = v;
    }
}

template <typename T>
__global__ void k_eye(C2<T>* a, int n) {
    const long long nn = (long long)n * n;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nn;
         i += (long long)gridDim.x * blockDim.x)
        a[i] = mk<T>(i / n == i % n ? (T)1 : (T)0, (T)0);
}

// Per cell: whether any of its local-operator coefficients (diagonal,
// vertical coupling, horizontal coupling) differs between two coefficient
// sets (bitwise; the model check excludes NaN).
__global__ void k_coef_changed(const CellDesc* cells, const double2* d0, const double2* z0,
                               const double2* e0, const double2* d1, const double2* z1,
                               const double2* e1, int* changed) {
    const CellDesc cd = cells[blockIdx.x];
    const long long n = (long long)cd.Wc * cd.HL;
    const long long o = cd.off_coef;
    auto ne = [](double2 a, double2 b) {
        return __double_as_longlong(a.x) != __double_as_longlong(b.x) ||
               __double_as_longlong(a.y) != __double_as_longlong(b.y);
    };
    int diff = 0;
    for (long long i = threadIdx.x; i < n; i += blockDim.x)
        diff |= ne(d0[o + i], d1[o + i]) || ne(z0[o + i], z1[o + i]) || ne(e0[o + i], e1[o + i]);
    diff = __syncthreads_or(diff);
    if (threadIdx.x == 0) changed[blockIdx.x] = diff ? 1 : 0;
}

// flag = 1 if the arrays differ anywhere (flag cleared by the caller)
__global__ void k_any_diff(const double2* a, const double2* b, long long n, int* flag) {
    int diff = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        diff |= __double_as_longlong(a[i].x) != __double_as_longlong(b[i].x) ||
                __double_as_longlong(a[i].y) != __double_as_longlong(b[i].y);
    diff = __syncthreads_or(diff);
    if (threadIdx.x == 0 && diff) atomicOr(flag, 1);
}

template <typename T>
void run_jobs(hz_ctx* c, const std::vector<LayerJob<T>>& jobs, int B);

// Composed output operators (offline): for every layer side and cell,
//   Qc = [ Q_x S^{-1} | Q_u ],
// Q_x the row samples of the cell's Green's function driven by the inner
// traces of its two interfaces, S the inner SIE matrix of the layer and Q_u
// the row samples driven by the interface-row sources.  Applying Qc to
// [inner rhs; pair] gives the same samples as solving the inner SIE and then
// applying [Q_x | Q_u]; the inner solve is taken out of the sequential path.
// S^{-1} itself is the inner block LU applied to the identity.
template <typename T>
void build_composed(hz_ctx* c, const std::vector<char>& redo_layer) {
    const Dims& d = c->d;
    const int J = d.Lc - 1;
    Ops<T>& o = ops<T>(c);
    c->qc_off.assign((size_t)d.L * 2 * d.Lc, -1);
    c->qc_ld.assign((size_t)d.L * 2 * d.Lc, 0);
    long long tot = 0;
    for (int l = 0; l < d.L; ++l) {
        const LayerDesc& ld = c->layers[l];
        const int NI = J * 2 * ld.HL;
        for (int side = 0; side < 2; ++side) {
            if (ld.slot_of[side == 0 ? 0 : 2] < 0) continue;
            for (int k = 0; k < d.Lc; ++k) {
                const CellDesc& cd = c->cells[ld.cell_begin + k];
                const size_t q = ((size_t)l * 2 + side) * d.Lc + k;
                c->qc_off[q] = tot;
                c->qc_ld[q] = NI + ld.nslot * cd.s;
                tot += 2LL * cd.s * c->qc_ld[q];
            }
        }
    }
    c->Qc_elems = tot;
    if (!o.Qc) o.Qc = alloc_c<T>(c, std::max<long long>(tot, 1));
    const int NImax = J * 2 * d.HLmax;
    const long long nn = (long long)NImax * NImax;
    C2<T>* E = alloc_c<T>(c, nn);
    C2<T>* IY = alloc_c<T>(c, nn);
    C2<T>* IX = alloc_c<T>(c, nn);
    GemmTask<T>* tdev = (GemmTask<T>*)c->arena.alloc(sizeof(GemmTask<T>) * 2 * d.Lc);
    for (int l = 0; l < d.L; ++l) {
        if (!redo_layer[l]) continue;
        const LayerDesc& ld = c->layers[l];
        const int NI = J * 2 * ld.HL;
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_eye<T>), dim3(1024), dim3(256), 0, c->st, E, NI);
        HIPCHK(hipGetLastError());
        LayerJob<T> jb;
        jb.layer = l;
        jb.inner_add = E;                 // phase 1 without sources: iy = I
        jb.iy = IY;
        jb.ix = IX;                       // -> S^{-1}, [NI][NI]
        jb.phase3 = false;
        run_jobs<T>(c, {jb}, NI);
        std::vector<GemmTask<T>> tasks;
        int maxm = 0;
        for (int side = 0; side < 2; ++side) {
            const int so_a = ld.slot_of[side == 0 ? 0 : 2];
            if (so_a < 0) continue;
            for (int k = 0; k < d.Lc; ++k) {
                const CellDesc& cd = c->cells[ld.cell_begin + k];
                const size_t q = ((size_t)l * 2 + side) * d.Lc + k;
                const int NC = c->qc_ld[q];
                C2<T>* dst = o.Qc + c->qc_off[q];
                const C2<T>* src = o.Q + cd.off_Q + (long long)so_a * cd.s * cd.R;
                GemmTask<T> t = blank_task<T>();
                t.A = src;
                t.lda = cd.R;
                t.m = 2 * cd.s;
                t.k = cd.ncol;
                t.ldx = NI;
                t.ldo = NC;
                t.nseg = 0;
                if (cd.has_left) {
                    t.seg_k0[t.nseg] = 0;
                    t.seg_len[t.nseg] = 2 * ld.HL;
                    t.seg_ptr[t.nseg] = IX + (long long)(k - 1) * 2 * ld.HL * NI;
                    t.nseg++;
                }
                if (cd.has_right) {
                    t.seg_k0[t.nseg] = cd.has_left ? 2 * ld.HL : 0;
                    t.seg_len[t.nseg] = 2 * ld.HL;
                    t.seg_ptr[t.nseg] = IX + (long long)k * 2 * ld.HL * NI;
                    t.nseg++;
                }
                t.noseg = 1;
                t.oseg_i0[0] = 0;
                t.oseg_len[0] = 2 * cd.s;
                t.oseg_ptr[0] = dst;
                t.alpha = 1.0;
                tasks.push_back(t);
                maxm = std::max(maxm, t.m);
                // Q_u: the interface-row-source columns, copied
                HIPCHK(hipMemcpy2DAsync(dst + NI, sizeof(C2<T>) * NC, src + cd.ncol,
                                        sizeof(C2<T>) * cd.R, sizeof(C2<T>) * ld.nslot * cd.s,
                                        2 * cd.s, hipMemcpyDeviceToDevice, c->st));
            }
        }
        if (!tasks.empty()) {
            upload(c, tdev, tasks.data(), sizeof(GemmTask<T>) * tasks.size());
            launch_gemm<T>(tdev, (int)tasks.size(), maxm, NI, c->st, true);
            HIPCHK(hipGetLastError());
        }
        sync(c);
    }
    c->arena.release(E, 0);
    c->arena.release(IY, 0);
    c->arena.release(IX, 0);
    c->arena.release(tdev, 0);
}

template <typename T>
__global__ void k_cast_pool(C2<T>* y, const double2* x, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        y[i] = mk<T>((T)x[i].x, (T)x[i].y);
    }
}

struct OfflineScope {              // marks launches as factorisation-stage launches
    hz_ctx* c;
    explicit OfflineScope(hz_ctx* ctx) : c(ctx) { c->offline = true; }
    ~OfflineScope() { c->offline = false; }
};

// redo: per-cell flags of the cells to (re)factor; nullptr = every cell.
// The inner SIE and the composed operators are rebuilt for the layers that
// hold a redone cell.  T is the precision of the whole offline stage:
// complex128 (HZ_FP64, and HZ_MIXED, which then keeps complex64 copies) or
// complex64 (HZ_MIXED_REFINE: factors, probes, inner LU and composed
// operators computed in FP32, no FP64 operators at all).
template <typename T>
void factor_impl_t(hz_ctx* c, const std::vector<char>* redo) {
    OfflineScope scope(c);
    const Dims& d = c->d;
    const int ncells = (int)c->cells.size();
    std::vector<int> todo;
    for (int i = 0; i < ncells; ++i)
        if (!redo || (*redo)[i]) todo.push_back(i);
    std::vector<char> redo_layer(d.L, 0);
    for (int i : todo) redo_layer[c->cells[i].layer] = 1;
    Ops<T>& o = ops<T>(c);
    if (!o.X) {
        o.X = alloc_c<T>(c, c->X_elems);
        o.Q = alloc_c<T>(c, std::max<long long>(c->Q_elems, 1));
        o.CS = alloc_c<T>(c, std::max<long long>(c->CS_elems, 1));
        o.Sinv = alloc_c<T>(c, std::max<long long>(c->Sinv_elems, 1));
        o.Lfac = alloc_c<T>(c, std::max<long long>(c->Lfac_elems, 1));
        if (c->inner_pt) o.CP = alloc_c<T>(c, std::max<long long>(c->CP_elems, 1));
    }
    if constexpr (sizeof(T) == sizeof(double)) {
        o.e = (C2<T>*)c->e;
    } else {            // the cell solves of the probes read complex64 couplings
        if (!o.e) o.e = alloc_c<T>(c, std::max<long long>(c->coef_elems, 1));
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cast_pool<float>), dim3(4096), dim3(256), 0, c->st,
                           (float2*)o.e, c->e, c->coef_elems);
        HIPCHK(hipGetLastError());
    }
    {
        FactorFlags ff0{0, 0, ~0ULL};
        upload(c, c->fflags, &ff0, sizeof(ff0));
    }
    // temporaries of this call, released on every exit (also on HZ_ESINGULAR)
    struct Temps {
        Arena& a;
        std::vector<void*> v;
        void* keep(void* p) { v.push_back(p); return p; }
        ~Temps() { for (void* p : v) a.release(p, 0); }
    } tmp{c->arena, {}};
    auto check_pivots = [&](const char* what) {
        FactorFlags ff{};
        HIPCHK(hipMemcpy(&ff, c->fflags, sizeof(ff), hipMemcpyDeviceToHost));
        double r = 1.0;
        if (ff.min_ratio_bits != ~0ULL) std::memcpy(&r, &ff.min_ratio_bits, sizeof(r));
        c->min_pivot_ratio = r;
        if (ff.singular) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "%s: pivot ratio %.3g (zero pivot, or below 2^-26 of the "
                          "block's largest pivot)", what, r);
            raise(HZ_ESINGULAR, buf);
        }
    };
    const int nt = (int)todo.size();
    if (nt == 0) return;
    // 1. cell Schur factors (descriptors of the cells to factor, gathered)
    {
        std::vector<CellDesc> sel(nt);
        for (int i = 0; i < nt; ++i) sel[i] = c->cells[todo[i]];
        CellDesc* d_sel = (CellDesc*)tmp.keep(c->arena.alloc(sizeof(CellDesc) * nt));
        upload(c, d_sel, sel.data(), sizeof(CellDesc) * nt);
        const long long ws = (long long)d.HLpmax * d.HLpmax;
        const int batch = std::min(nt, 1024);
        C2<T>* workbuf = (C2<T>*)tmp.keep(alloc_c<T>(c, ws * batch));
        for (int c0 = 0; c0 < nt; c0 += batch) {
            const int cnt = std::min(batch, nt - c0);
            launch_cell_factor<T>(d_sel + c0, cnt, d, c->diag, c->cz, c->e, o.X,
                                       workbuf, ws, c->fflags, c->st);
            HIPCHK(hipGetLastError());
        }
        sync(c);
    }
    check_pivots("cell factorisation");
    // 2. probes: cell Green's functions sampled on the interface rows / columns
    int Rmax = 0;
    for (auto& cd : c->cells) Rmax = std::max(Rmax, cd.R);
    if (Rmax > 0) {
        const int nb = cs_nb(Rmax, ncells, d.HLpmax, (int)sizeof(C2<T>));
        const int chunks = (Rmax + nb - 1) / nb;
        const long long ystride = (long long)d.Wcmax * d.HLpmax * nb;
        // Forward-sweep scratch: a quarter of the free memory, between 4 and
        // 24 GiB, so that a launch holds several waves of workgroups (probe
        // batches differ in length: the forward sweep starts at the batch's
        // first source column) and the dispatcher can balance them.
        size_t mfree = 0, mtot = 0;
        if (hipMemGetInfo(&mfree, &mtot) != hipSuccess) { (void)hipGetLastError(); mfree = 0; }
        const long long budget = std::min<long long>(24LL << 30, std::max<long long>(4LL << 30, (long long)(mfree / 4)));
        long long budget_wgs = std::max<long long>(chunks, budget / (ystride * (long long)sizeof(C2<T>)));
        const int per = (int)std::min<long long>(nt, std::max<long long>(1, budget_wgs / chunks));
        C2<T>* Y = (C2<T>*)tmp.keep(alloc_c<T>(c, ystride * (long long)per * chunks));
        int* d_list = (int*)tmp.keep(c->arena.alloc(sizeof(int) * nt));
        upload(c, d_list, todo.data(), sizeof(int) * nt);
        CellSolveArgs<T> a = base_args<T>(c);
        a.mode = SOLVE_PROBE;
        a.Qpool = o.Q;
        a.CSpool = o.CS;
        a.CPpool = c->inner_pt ? o.CP : nullptr;
        a.probe0 = 0;
        a.B = Rmax;
        a.nb = nb;
        a.Y = Y;
        a.y_stride = ystride;
        for (int g = 0; g < nt; g += per) {
            const int cnt = std::min(per, nt - g);
            a.cell_list = d_list + g;
            launch_cell_solve<T>(a, cnt, chunks, c->st);
            HIPCHK(hipGetLastError());
        }
        sync(c);
    }
    // 3. inner SIE block LU without pivoting (per layer, sequential over
    // interfaces); the nested polarized traces iterate the inner SIE instead
    const int J = c->inner_pt ? 0 : d.Lc - 1;
    std::vector<int> lay;                  // layers to refactor
    for (int l = 0; l < d.L; ++l)
        if (redo_layer[l]) lay.push_back(l);
    if (J > 0) {
        const int L = (int)lay.size();     // compact index i <-> layer lay[i]
        int* d_lay = (int*)tmp.keep(c->arena.alloc(sizeof(int) * L));
        upload(c, d_lay, lay.data(), sizeof(int) * L);
        const long long bs = 4LL * d.HLmax * d.HLmax;       // (2 HLmax)^2
        C2<T>* A = (C2<T>*)tmp.keep(alloc_c<T>(c, bs * L));
        C2<T>* wk = (C2<T>*)tmp.keep(alloc_c<T>(c, bs * L));
        C2<T>** mats = (C2<T>**)tmp.keep(c->arena.alloc(sizeof(void*) * L));
        C2<T>** outs = (C2<T>**)tmp.keep(c->arena.alloc(sizeof(void*) * L));
        int* ns = (int*)tmp.keep(c->arena.alloc(sizeof(int) * L));
        std::vector<int> hn(L);
        std::vector<C2<T>*> hm(L), ho(L);
        for (int i = 0; i < L; ++i) { hn[i] = 2 * c->layers[lay[i]].HL; hm[i] = A + bs * i; }
        upload(c, ns, hn.data(), sizeof(int) * L);
        upload(c, mats, hm.data(), sizeof(void*) * L);
        GemmTask<T>* tdev = (GemmTask<T>*)tmp.keep(c->arena.alloc(sizeof(GemmTask<T>) * 2 * L));
        for (int j = 0; j < J; ++j) {
            hipLaunchKernelGGL(HIP_KERNEL_NAME(k_inner_diag<T>), dim3(64, L), dim3(256), 0, c->st,
                               c->d_layers, d_lay, c->d_cells, o.CS, j, A, bs);
            HIPCHK(hipGetLastError());
            if (j > 0) {
                // L_j^a = B_j^a Sinv_{j-1},  B_j^a = -(right-column samples of cell j, left probes)
                std::vector<GemmTask<T>> t1, t2;
                int mm = 0;
                for (int i = 0; i < L; ++i) {
                    const LayerDesc& ld = c->layers[lay[i]];
                    const int HL = ld.HL;
                    const CellDesc& cj = c->cells[ld.cell_begin + j];
                    GemmTask<T> t = blank_task<T>();
                    t.A = o.CS + cj.off_CS + (long long)HL * cj.R;    // right rows, left probes
                    t.lda = cj.R;
                    t.m = HL; t.k = 2 * HL;
                    t.ldx = 2 * HL; t.ldo = 2 * HL;
                    t.nseg = 1; t.seg_k0[0] = 0; t.seg_len[0] = 2 * HL;
                    t.seg_ptr[0] = o.Sinv + ld.off_Sinv + (long long)(j - 1) * 4 * HL * HL;
                    t.noseg = 1; t.oseg_i0[0] = 0; t.oseg_len[0] = HL;
                    t.oseg_ptr[0] = o.Lfac + ld.off_Lfac + (long long)(j - 1) * HL * 2 * HL;
                    t.alpha = -1.0;
                    t.ncol = 2 * HL;
                    t1.push_back(t);
                    // S_j^a = A_j^a - L_j^a[:, b] C_{j-1}^b,  C_{j-1}^b = -(left-column samples
                    // of cell j, right probes)  ->  A_j^a + L_j^a[:, b] * samples
                    GemmTask<T> u = blank_task<T>();
                    u.A = o.Lfac + ld.off_Lfac + (long long)(j - 1) * HL * 2 * HL + HL;
                    u.lda = 2 * HL;
                    u.m = HL; u.k = HL;
                    u.ldx = cj.R; u.ldo = 2 * HL;
                    u.nseg = 1; u.seg_k0[0] = 0; u.seg_len[0] = HL;
                    u.seg_ptr[0] = o.CS + cj.off_CS + 2LL * HL;      // left rows, right probes
                    u.noseg = 1; u.oseg_i0[0] = 0; u.oseg_len[0] = HL;
                    u.oseg_ptr[0] = A + bs * i;
                    u.oseg_add0[0] = A + bs * i;
                    u.alpha = 1.0;
                    u.ncol = 2 * HL;
                    t2.push_back(u);
                    mm = std::max(mm, 2 * HL);
                }
                upload(c, tdev, t1.data(), sizeof(GemmTask<T>) * L);
                launch_gemm<T>(tdev, L, mm, 2 * d.HLmax, c->st, true);
                HIPCHK(hipGetLastError());
                sync(c);
                upload(c, tdev + L, t2.data(), sizeof(GemmTask<T>) * L);
                launch_gemm<T>(tdev + L, L, mm, 2 * d.HLmax, c->st, true);
                HIPCHK(hipGetLastError());
                sync(c);
            }
            for (int i = 0; i < L; ++i) {
                const LayerDesc& ld = c->layers[lay[i]];
                ho[i] = o.Sinv + ld.off_Sinv + (long long)j * 4 * ld.HL * ld.HL;
            }
            upload(c, outs, ho.data(), sizeof(void*) * L);
            // inverse of an order-2HL block: pack with row stride 2HL (the A buffer is already)
            launch_invert_batch<T>(mats, outs, ns, L, wk, bs, c->fflags, c->st);
            HIPCHK(hipGetLastError());
            sync(c);
        }
        check_pivots("inner block LU");
    }
    // 4. composed output operators
    if (J > 0 && c->compose) build_composed<T>(c, redo_layer);
    // 5. HZ_MIXED: complex64 copies of every operator for the preconditioner
    if constexpr (sizeof(T) == sizeof(double)) {
      if (c->prm.precision == HZ_MIXED) {
        Ops<float>& f = c->o32;
        auto cast = [&](float2*& dst, const double2* src, long long n) {
            if (!dst) dst = alloc_c<float>(c, std::max<long long>(n, 1));
            if (n > 0)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_cast_pool<float>), dim3(4096), dim3(256), 0,
                                   c->st, dst, src, n);
        };
        cast(f.X, o.X, c->X_elems);
        cast(f.e, c->e, c->coef_elems);
        cast(f.Q, o.Q, c->Q_elems);
        cast(f.CS, o.CS, c->CS_elems);
        cast(f.Sinv, o.Sinv, c->Sinv_elems);
        cast(f.Lfac, o.Lfac, c->Lfac_elems);
        if (o.Qc) cast(f.Qc, o.Qc, c->Qc_elems);
        HIPCHK(hipGetLastError());
        sync(c);
      }
    }
}

// Compress the preconditioner's operator blocks in PLR form (offline): the
// composed output operators Qc of every layer side and cell and the
// interface-row columns of the cell samples (M_f).  Tile norms first (the
// per-tile budget eps ||A||_F / sqrt(T) needs the block norm), then the
// ranks (rank-revealing QR without output), then the factors into a pool
// of exactly the stored size.
template <typename T>
void plr_build(hz_ctx* c) {
    PlrStore<T>& ps = plr_store<T>(c);
    if (ps.pool) c->arena.release(ps.pool, 0);
    if (ps.tiles) c->arena.release(ps.tiles, 0);
    ps.pool = nullptr;
    ps.tiles = nullptr;
    ps.host.clear();
    ps.blocks.clear();
    ps.stored = ps.dense = 0;
    const Dims& d = c->d;
    const int J = d.Lc - 1;
    if (!c->prm.plr || J <= 0 || !c->compose) return;
    Ops<T>& o = ops<T>(c);
    if (!o.Qc || !o.CS) return;
    std::vector<PlrBlock<T>> blocks;
    std::vector<long long> bfirst;
    auto add_block = [&](const C2<T>* A, long long lda, int m, int k) {
        if (m <= 0 || k <= 0 || ps.blocks.count((const void*)A)) return;
        const int b = (int)blocks.size();
        blocks.push_back({A, lda});
        const int ntr = (m + PLR_TILE - 1) / PLR_TILE, ntc = (k + PLR_TILE - 1) / PLR_TILE;
        ps.blocks[(const void*)A] = {(long long)ps.host.size(), ntr, ntc};
        bfirst.push_back((long long)ps.host.size());
        for (int i = 0; i < ntr; ++i)
            for (int j = 0; j < ntc; ++j) {
                PlrTile t{};
                t.block = b;
                t.i0 = i * PLR_TILE;
                t.j0 = j * PLR_TILE;
                t.tr = std::min(PLR_TILE, m - t.i0);
                t.tc = std::min(PLR_TILE, k - t.j0);
                t.rank = -1;
                ps.host.push_back(t);
                ps.dense += (long long)t.tr * t.tc;
            }
    };
    for (int l = 0; l < d.L; ++l) {
        const LayerDesc& ld = c->layers[l];
        for (int side = 0; side < 2; ++side)
            for (int k = 0; k < d.Lc; ++k) {
                const size_t q = ((size_t)l * 2 + side) * d.Lc + k;
                if (c->qc_off[q] < 0) continue;
                const CellDesc& cd = c->cells[ld.cell_begin + k];
                add_block(o.Qc + c->qc_off[q], c->qc_ld[q], 2 * cd.s, c->qc_ld[q]);
            }
        if (ld.nslot == 0) continue;
        for (int k = 0; k < d.Lc; ++k) {
            const CellDesc& cd = c->cells[ld.cell_begin + k];
            add_block(o.CS + cd.off_CS + cd.ncol, cd.R, cd.adj * cd.HL, ld.nslot * cd.s);
        }
    }
    const long long nt = (long long)ps.host.size();
    bfirst.push_back(nt);
    if (nt == 0) return;
    if (nt > INT_MAX) raise(HZ_EINVAL, "too many PLR tiles");
    struct Temps {
        Arena& a;
        std::vector<void*> v;
        void* keep(void* p) { v.push_back(p); return p; }
        ~Temps() { for (void* p : v) a.release(p, 0); }
    } tmp{c->arena, {}};
    auto* dblk = (PlrBlock<T>*)tmp.keep(c->arena.alloc(sizeof(PlrBlock<T>) * blocks.size()));
    auto* dtile = (PlrTile*)c->arena.alloc(sizeof(PlrTile) * nt);
    ps.tiles = dtile;
    auto* dnorm = (double*)tmp.keep(c->arena.alloc(sizeof(double) * nt));
    auto* drank = (int*)tmp.keep(c->arena.alloc(sizeof(int) * nt));
    upload(c, dblk, blocks.data(), sizeof(PlrBlock<T>) * blocks.size());
    upload(c, dtile, ps.host.data(), sizeof(PlrTile) * nt);
    launch_plr_tile_norms<T>(dblk, dtile, (int)nt, dnorm, c->st);
    HIPCHK(hipGetLastError());
    std::vector<double> norm2(nt), delta2(nt);
    HIPCHK(hipMemcpyAsync(norm2.data(), dnorm, sizeof(double) * nt, hipMemcpyDeviceToHost, c->st));
    sync(c);
    const double eps = c->prm.plr_eps;
    for (size_t b = 0; b + 1 < bfirst.size(); ++b) {
        double fro2 = 0.0;
        for (long long e = bfirst[b]; e < bfirst[b + 1]; ++e) fro2 += norm2[e];
        const double ntb = (double)(bfirst[b + 1] - bfirst[b]);
        for (long long e = bfirst[b]; e < bfirst[b + 1]; ++e) delta2[e] = eps * eps * fro2 / ntb;
    }
    upload(c, dnorm, delta2.data(), sizeof(double) * nt);
    launch_plr_compress<T>(dblk, dtile, (int)nt, dnorm, drank, nullptr, 0, c->st);
    HIPCHK(hipGetLastError());
    std::vector<int> rank(nt);
    HIPCHK(hipMemcpyAsync(rank.data(), drank, sizeof(int) * nt, hipMemcpyDeviceToHost, c->st));
    sync(c);
    long long off = 0;
    for (long long e = 0; e < nt; ++e) {
        PlrTile& t = ps.host[e];
        t.rank = rank[e];
        t.off = off;
        off += t.rank < 0 ? (long long)t.tr * t.tc : (long long)t.rank * (t.tr + t.tc);
    }
    ps.stored = off;
    ps.pool = alloc_c<T>(c, std::max<long long>(off, 1));
    upload(c, dtile, ps.host.data(), sizeof(PlrTile) * nt);
    launch_plr_compress<T>(dblk, dtile, (int)nt, dnorm, drank, ps.pool, 1, c->st);
    HIPCHK(hipGetLastError());
    sync(c);
}

void factor_impl(hz_ctx* c, const std::vector<char>* redo = nullptr) {
    if (c->prm.precision == HZ_MIXED_REFINE) factor_impl_t<float>(c, redo);
    else factor_impl_t<double>(c, redo);
    // the preconditioner's operators: FP64 in HZ_FP64, complex64 otherwise
    OfflineScope scope(c);
    if (c->prm.precision == HZ_FP64) plr_build<double>(c);
    else plr_build<float>(c);
}

// ---------------------------------------------------------------------------
// online stage, precision T for the local operators

// drop every cached plan (operators, stream or buffers changed)
void clear_plans(hz_ctx* c) {
    c->w64.sie.clear(); c->w64.pre.clear(); c->w64.jobs.clear();
    c->w32.sie.clear(); c->w32.pre.clear(); c->w32.jobs.clear();
}

template <typename T>
void run_jobs(hz_ctx* c, const std::vector<LayerJob<T>>& jobs, int B) {
    Plan<T> pl;
    plan_jobs<T>(c, pl, jobs, B);
    plan_upload<T>(c, pl);
    plan_launches<T>(c, pl, B);
    sync(c);
    if (pl.dev) c->arena.release(pl.dev, pl.dev_bytes);
}

// The same, with the plan kept under `key` (the jobs must be a function of
// the key) and replayed like the operator plans.
template <typename T>
void run_jobs_cached(hz_ctx* c, const std::string& key, const std::vector<LayerJob<T>>& jobs,
                     int B) {
    Work<T>& w = work<T>(c);
    auto it = w.jobs.find(key);
    if (it == w.jobs.end()) {
        auto pl = std::make_unique<Plan<T>>();
        pl->name = fam_name<T>("jobs_graph");
        plan_jobs<T>(c, *pl, jobs, B);
        plan_upload<T>(c, *pl);
        tune_plan<T>(c, *pl, B);
        it = w.jobs.emplace(key, std::move(pl)).first;
    }
    plan_run<T>(c, *it->second, B);
}

std::string jobs_key(const char* kind, int B, const int* active, int L, const void* out) {
    std::string k = std::string(kind) + "|" + std::to_string(B) + "|" +
                    std::to_string((unsigned long long)(uintptr_t)out) + "|";
    for (int l = 0; l < L; ++l) k += active[l] ? '1' : '0';
    return k;
}

// Cell Newton potentials of the volume source in the layers that hold one
// (Alg. 7 lines 3-9): inner right-hand sides -> w.gf, samples on the
// interface rows -> w.rows_out.  Returns false if no layer is active.
template <typename T>
bool sample_sources(hz_ctx* c, int B, const int* active_host) {
    Work<T>& w = work<T>(c);
    const Dims& d = c->d;
    std::vector<int> list;
    for (int l = 0; l < d.L; ++l)
        if (active_host[l])
            for (int k = 0; k < d.Lc; ++k) list.push_back(c->layers[l].cell_begin + k);
    if (list.empty()) return false;
    CellSolveArgs<T> a = base_args<T>(c);
    a.mode = SOLVE_SAMPLE;
    a.f_ext = w.f_ext;
    a.layer_active = nullptr;
    a.inner_rhs = w.gf;
    a.inner_pol = c->inner_pt ? 1 : 0;
    a.rows_out = w.rows_out;
    cell_solve_launch<T>(c, a, list, B);
    return true;
}

// RHS of the polarized system from w.f_ext into polarized vector `out` (T)
template <typename T>
void sie_rhs_impl(hz_ctx* c, int B, C2<T>* out, const int* active_host) {
    Work<T>& w = work<T>(c);
    const Dims& d = c->d;
    const long long pol = 4LL * d.K * d.W * B;
    HIPCHK(hipMemsetAsync(out, 0, sizeof(C2<T>) * pol, c->st));
    if (!sample_sources<T>(c, B, active_host)) return;
    std::vector<LayerJob<T>> jobs;
    for (int l = 0; l < d.L; ++l) {
        if (!active_host[l]) continue;
        const LayerDesc& ld = c->layers[l];
        for (int side = 0; side < 2; ++side) {
            if (side == 0 && !ld.has_top) continue;
            if (side == 1 && !ld.has_bot) continue;
            LayerJob<T> jb;
            jb.layer = l;
            jb.inner_add = gf_of<T>(c, l, B);
            jb.iy = iy_of<T>(c, side, l, B);
            jb.ix = ix_of<T>(c, side, l, B);
            jb.side = side;
            jb.out = side == 1 ? dvec<T>(c, out, l, B) : qvec<T>(c, out, l - 1, B);
            const int so_a = ld.slot_of[side == 0 ? 0 : 2];
            jb.add0 = w.rows_out + ((long long)l * MAXSLOT + so_a) * d.W * B;
            jb.use_x = false;
            jb.alpha = (T)1;
            jobs.push_back(jb);
        }
    }
    run_jobs_cached<T>(c, jobs_key("rhs", B, active_host, d.L, out), jobs, B);
}

// volume reconstruction from traces in w.sv (s = d + q) into w.u_ext
template <typename T>
void reconstruct_impl(hz_ctx* c, int B, const int* active_host) {
    Work<T>& w = work<T>(c);
    const Dims& d = c->d;
    const long long pairn = 2LL * d.W * B;
    const int J = d.Lc - 1;
    if (J > 0) {
        std::vector<LayerJob<T>> jobs;
        for (int l = 0; l < d.L; ++l) {
            LayerJob<T> jb;
            jb.layer = l;
            jb.top = l > 0 ? w.sv + (long long)(l - 1) * pairn : nullptr;
            jb.bot = l < d.L - 1 ? w.sv + (long long)l * pairn : nullptr;
            jb.inner_add = active_host[l] ? gf_of<T>(c, l, B) : nullptr;
            jb.iy = iy_of<T>(c, 0, l, B);
            jb.ix = ix_of<T>(c, 0, l, B);
            jb.phase3 = false;
            jobs.push_back(jb);
        }
        run_jobs_cached<T>(c, jobs_key("rec", B, active_host, d.L, nullptr), jobs, B);
    }
    std::vector<int> list(c->cells.size());
    for (size_t i = 0; i < list.size(); ++i) list[i] = (int)i;
    upload_pair_tab<T>(c, B);
    CellSolveArgs<T> a = base_args<T>(c);
    a.mode = SOLVE_VOLUME;
    a.f_ext = w.f_ext;
    a.layer_active = c->layer_active;
    a.top_pair = w.pair_tab;
    a.bot_pair = w.pair_tab + d.L;
    a.inner_v = J > 0 ? w.ix[0] : nullptr;
    a.u_ext = w.u_ext;
    cell_solve_launch<T>(c, a, list, B);
}

// y = P M x on FP64 vectors (x, y: [n][B]); T selects the operator precision
template <typename T>
void apply_PM(hz_ctx* c, const double2* x, double2* y, int B) {
    Work<T>& w = work<T>(c);
    const long long n = 4LL * c->d.K * c->d.W * B;
    Plan<T>& ps = get_plan<T>(c, true, B);
    Plan<T>& pp = get_plan<T>(c, false, B);
    if constexpr (sizeof(T) == sizeof(double)) {
        HIPCHK(hipMemcpyAsync(w.pA, x, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    } else {
        launch_cast_d2f((float2*)w.pA, x, n, c->st);
    }
    plan_run<T>(c, ps, B);
    plan_run<T>(c, pp, B);
    if constexpr (sizeof(T) == sizeof(double)) {
        HIPCHK(hipMemcpyAsync(y, w.pC, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    } else {
        launch_cast_f2d(y, (const float2*)w.pC, n, c->st);
    }
}

// P on FP64 vectors (used for the preconditioned right-hand side); y2, where
// given, receives the result too
template <typename T>
void apply_P(hz_ctx* c, const double2* x, double2* y, int B, double2* y2 = nullptr) {
    Work<T>& w = work<T>(c);
    const long long n = 4LL * c->d.K * c->d.W * B;
    Plan<T>& pp = get_plan<T>(c, false, B);
    if constexpr (sizeof(T) == sizeof(double)) {
        HIPCHK(hipMemcpyAsync(w.pB, x, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    } else {
        launch_cast_d2f((float2*)w.pB, x, n, c->st);
    }
    plan_run<T>(c, pp, B);
    if constexpr (sizeof(T) == sizeof(double)) {
        HIPCHK(hipMemcpyAsync(y, w.pC, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
        if (y2) HIPCHK(hipMemcpyAsync(y2, w.pC, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    } else {
        launch_cast_f2d(y, (const float2*)w.pC, n, c->st, y2);
    }
}

void givens(std::complex<double> a, std::complex<double> b, double& cs, std::complex<double>& sn) {
    if (std::abs(b) == 0.0) { cs = 1.0; sn = 0.0; return; }
    if (std::abs(a) == 0.0) { cs = 0.0; sn = std::conj(b) / std::abs(b); return; }
    const double t = std::hypot(std::abs(a), std::abs(b));
    cs = std::abs(a) / t;
    sn = (a / std::abs(a)) * std::conj(b) / t;
}

// dots h[v][b] = V_v^H w for v < nv (device -> host)
void dots(hz_ctx* c, const double2* V, long long vstride, int nv, const double2* w, long long n,
          int B, std::vector<std::complex<double>>& out) {
    const int chunks = (int)std::min<long long>(c->gpart_chunks, std::max<long long>(1, n / 32));
    launch_dots(V, vstride, nv, w, n, B, c->gpart, chunks, c->st);
    launch_reduce_partials(c->gpart, chunks, nv * B, c->gsmall, c->st);
    out.resize((size_t)nv * B);
    double2* hp = pinned(c, (size_t)nv * B);
    HIPCHK(hipMemcpyAsync(hp, c->gsmall, sizeof(double2) * nv * B, hipMemcpyDeviceToHost, c->st));
    sync(c);
    for (size_t q = 0; q < out.size(); ++q) out[q] = std::complex<double>(hp[q].x, hp[q].y);
}

// the same reductions left on the device: out_dev[v * B + b]
void dots_dev(hz_ctx* c, const double2* V, long long vstride, int nv, const double2* w,
              long long n, int B, double2* out_dev) {
    const int chunks = (int)std::min<long long>(c->gpart_chunks, std::max<long long>(1, n / 32));
    launch_dots(V, vstride, nv, w, n, B, c->gpart, chunks, c->st);
    launch_reduce_partials(c->gpart, chunks, nv * B, out_dev, c->st);
}

// One Gram-Schmidt pass w -= V coef fused with the next reductions (V^H w,
// or |w|^2 when norm) into out_dev; the separate kernels beyond 8 vectors.
void update_dots_dev(hz_ctx* c, const double2* V, long long vstride, int nv, const double2* coef,
                     double2* w, long long n, int B, int norm, double2* out_dev,
                     double2* part, int max_chunks) {
    // seven or eight vectors take three waves per SIMD: 768 workgroups of
    // four waves then run in one round
    const int cap = nv >= 7 ? std::min(max_chunks, 768) : max_chunks;
    const int chunks = (int)std::min<long long>(cap, std::max<long long>(1, n / 8));
    if (launch_update_dots(w, V, vstride, nv, coef, -1.0, n, B, norm, part, chunks, c->st)) {
        launch_reduce_partials(part, chunks, (norm ? 1 : nv) * B, out_dev, c->st);
        return;
    }
    launch_update_basis(w, V, vstride, nv, coef, n, B, c->st, -1.0);
    launch_dots(norm ? nullptr : V, vstride, norm ? 1 : nv, w, n, B, part, chunks, c->st);
    launch_reduce_partials(part, chunks, (norm ? 1 : nv) * B, out_dev, c->st);
}

void norms(hz_ctx* c, const double2* w, long long n, int B, std::vector<double>& out) {
    std::vector<std::complex<double>> t;
    dots(c, nullptr, 0, 1, w, n, B, t);
    out.resize(B);
    for (int b = 0; b < B; ++b) out[b] = std::sqrt(std::max(0.0, t[b].real()));
}

// M on FP64 vectors with the operators of precision T
template <typename T>
void apply_M(hz_ctx* c, const double2* x, double2* y, int B) {
    Work<T>& w = work<T>(c);
    const long long n = 4LL * c->d.K * c->d.W * B;
    Plan<T>& ps = get_plan<T>(c, true, B);
    if constexpr (sizeof(T) == sizeof(double)) {
        HIPCHK(hipMemcpyAsync(w.pA, x, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    } else {
        launch_cast_d2f((float2*)w.pA, x, n, c->st);
    }
    plan_run<T>(c, ps, B);
    if constexpr (sizeof(T) == sizeof(double)) {
        HIPCHK(hipMemcpyAsync(y, w.pB, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    } else {
        launch_cast_f2d(y, (const float2*)w.pB, n, c->st);
    }
}

// M on FP64 vectors with the FP64 operators
void apply_M64(hz_ctx* c, const double2* x, double2* y, int B) {
    Work<double>& w = c->w64;
    const long long n = 4LL * c->d.K * c->d.W * B;
    Plan<double>& ps = get_plan<double>(c, true, B);
    HIPCHK(hipMemcpyAsync(w.pA, x, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    plan_run<double>(c, ps, B);
    HIPCHK(hipMemcpyAsync(y, w.pB, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
}

// GMRES (Alg. 6) on FP64 vectors, x0 = 0, no restart, classical Gram-Schmidt
// with one re-orthogonalisation, Givens rotations.
//  flex = false: left preconditioning, P M x = P b, both in precision T;
//  flex = true : flexible right preconditioning, M P y = b, x = P y, with M
//                in FP64 and P in complex64 (the preconditioned basis Z is
//                stored, so the inexact P only affects the convergence rate).
template <typename T>
void gmres(hz_ctx* c, const double2* b, double2* x, int B, double tol, int maxit,
           std::vector<int>& iters, std::vector<double>& relres, bool flex = false) {
    const long long n = 4LL * c->d.K * c->d.W;
    const long long nB = n * B;
    ensure_gmres(c, B, maxit);
    double2* V = c->V;
    double2* Z = c->Z;
    const long long vs = nB;
    if (flex) {
        if (!Z) raise(HZ_ESTATE, "flexible GMRES basis missing");
        HIPCHK(hipMemcpyAsync(V, b, sizeof(double2) * nB, hipMemcpyDeviceToDevice, c->st));
    } else {
        apply_P<T>(c, b, V, B);
    }
    std::vector<double> beta;
    norms(c, V, n, B, beta);
    // Hessenberg columns per RHS, kept by the context between solves: every
    // entry read (rows <= column + 1) is written first in the same solve
    auto& Hm = c->g_hess;
    if ((int)Hm.size() < B) Hm.resize(B);
    for (int bb = 0; bb < B; ++bb)
        if (Hm[bb].size() < (size_t)(maxit + 1) * maxit) Hm[bb].resize((size_t)(maxit + 1) * maxit);
    std::vector<std::vector<std::complex<double>>> g(B, std::vector<std::complex<double>>(maxit + 1));
    std::vector<std::vector<double>> cs(B, std::vector<double>(maxit));
    std::vector<std::vector<std::complex<double>>> sn(B, std::vector<std::complex<double>>(maxit));
    std::vector<int> done(B, 0), kfin(B, 0);
    iters.assign(B, 0);
    relres.assign(B, 0.0);
    std::vector<double2> sc(B);
    for (int bb = 0; bb < B; ++bb) {
        g[bb][0] = beta[bb];
        if (beta[bb] == 0.0) { done[bb] = 1; relres[bb] = 0.0; }
        sc[bb] = make_double2(beta[bb] > 0 ? 1.0 / beta[bb] : 0.0, 0.0);
    }
    upload(c, c->gcoef, sc.data(), sizeof(double2) * B);
    launch_scale_cols(V, V, c->gcoef, n, B, c->st);
    std::vector<double> nrm;
    std::vector<double2> coef;
    int j = 0;
    for (; j < maxit; ++j) {
        if (std::all_of(done.begin(), done.end(), [](int v) { return v != 0; })) break;
        double2* Vj = V + (long long)j * vs;
        double2* Vn = V + (long long)(j + 1) * vs;
        // the new vector w: where the last plan of the product runs in FP64,
        // its output buffer itself (overwritten only by the next product)
        double2* wv = c->gw;
        if (flex) {
            // z_j = P v_j is also written into the SIE plan's input
            double2* Zj = Z + (long long)j * vs;
            if (c->inner_pt) apply_P<double>(c, Vj, Zj, B, c->w64.pA);
            else apply_P<float>(c, Vj, Zj, B, c->w64.pA);
            plan_run<double>(c, get_plan<double>(c, true, B), B);
            wv = c->w64.pB;
        } else if constexpr (sizeof(T) == sizeof(double)) {
            HIPCHK(hipMemcpyAsync(c->w64.pA, Vj, sizeof(double2) * nB, hipMemcpyDeviceToDevice, c->st));
            plan_run<double>(c, get_plan<double>(c, true, B), B);
            plan_run<double>(c, get_plan<double>(c, false, B), B);
            wv = c->w64.pC;
        } else {
            apply_PM<T>(c, Vj, c->gw, B);
        }
        // two passes of classical Gram-Schmidt; the projections stay on the
        // device and the host reads both passes and |w|^2 once per iteration
        const size_t nh = (size_t)(j + 1) * B;
        double2* hA = c->gh;
        double2* hB = c->gh + nh;
        double2* hN = c->gh + 2 * nh;
        dots_dev(c, V, vs, j + 1, wv, n, B, hA);
        update_dots_dev(c, V, vs, j + 1, hA, wv, n, B, 0, hB, c->gpart, c->gpart_chunks);
        update_dots_dev(c, V, vs, j + 1, hB, wv, n, B, 1, hN, c->gpart, c->gpart_chunks);
        // next basis vector scaled on the device (columns that have converged
        // keep being normalised; their coefficients beyond convergence are 0)
        launch_scale_cols_inv_norm(Vn, nullptr, wv, hN, n, B, c->st);
        double2* hh = pinned(c, 2 * nh + B);
        HIPCHK(hipMemcpyAsync(hh, c->gh, sizeof(double2) * (2 * nh + B), hipMemcpyDeviceToHost,
                              c->st));
        sync(c);
        std::vector<std::complex<double>> hsum(nh);
        for (size_t q = 0; q < nh; ++q)
            hsum[q] = std::complex<double>(hh[q].x + hh[nh + q].x, hh[q].y + hh[nh + q].y);
        nrm.resize(B);
        for (int bb = 0; bb < B; ++bb) nrm[bb] = std::sqrt(std::max(0.0, hh[2 * nh + bb].x));
        for (int bb = 0; bb < B; ++bb) {
            if (done[bb]) continue;
            auto& H = Hm[bb];
            auto Hat = [&](int r, int col) -> std::complex<double>& { return H[(size_t)r * maxit + col]; };
            for (int i = 0; i <= j; ++i) Hat(i, j) = hsum[(size_t)i * B + bb];
            Hat(j + 1, j) = nrm[bb];
            for (int i = 0; i < j; ++i) {
                std::complex<double> a = Hat(i, j), b2 = Hat(i + 1, j);
                Hat(i, j) = cs[bb][i] * a + sn[bb][i] * b2;
                Hat(i + 1, j) = -std::conj(sn[bb][i]) * a + cs[bb][i] * b2;
            }
            givens(Hat(j, j), Hat(j + 1, j), cs[bb][j], sn[bb][j]);
            std::complex<double> a = Hat(j, j), b2 = Hat(j + 1, j);
            Hat(j, j) = cs[bb][j] * a + sn[bb][j] * b2;
            Hat(j + 1, j) = 0.0;
            g[bb][j + 1] = -std::conj(sn[bb][j]) * g[bb][j];
            g[bb][j] = cs[bb][j] * g[bb][j];
            kfin[bb] = j + 1;
            relres[bb] = std::abs(g[bb][j + 1]) / beta[bb];
            if (relres[bb] <= tol || nrm[bb] == 0.0) done[bb] = 1;
        }
    }
    // x = V y
    const int kmax = *std::max_element(kfin.begin(), kfin.end());
    coef.assign((size_t)std::max(kmax, 1) * B, make_double2(0, 0));
    for (int bb = 0; bb < B; ++bb) {
        const int k = kfin[bb];
        iters[bb] = k;
        std::vector<std::complex<double>> y(k);
        auto& H = Hm[bb];
        for (int i = k - 1; i >= 0; --i) {
            std::complex<double> s = g[bb][i];
            for (int q = i + 1; q < k; ++q) s -= H[(size_t)i * maxit + q] * y[q];
            y[i] = s / H[(size_t)i * maxit + i];
        }
        for (int i = 0; i < k; ++i) coef[(size_t)i * B + bb] = make_double2(y[i].real(), y[i].imag());
    }
    HIPCHK(hipMemsetAsync(x, 0, sizeof(double2) * nB, c->st));
    if (kmax > 0) {
        upload(c, c->gcoef, coef.data(), sizeof(double2) * (size_t)kmax * B);
        launch_update_basis(x, flex ? Z : V, vs, kmax, c->gcoef, n, B, c->st);
    }
    sync(c);
}

// One DD solve of H u = f with f already in work<T>.f_ext; result in work<T>.u_ext.
// Right-preconditioned Bi-CGstab (van der Vorst) on FP64 vectors, x0 = 0,
// shadow residual r0 = b: per iteration two applications of P and of M and
// three host reads of per-column scalars; stops per column on the
// unpreconditioned residual ||b - M x|| <= tol ||b|| (at the half step s or
// the full step r).  Columns that have stopped keep x and r fixed (zero
// coefficients).  P is complex64 when flex (the mixed form) or T = float,
// M is complex128 unless T = float.
template <typename T>
void bicgstab(hz_ctx* c, const double2* b, double2* x, int B, double tol, int maxit,
              std::vector<int>& iters, std::vector<double>& relres, bool flex = false) {
    const long long n = 4LL * c->d.K * c->d.W;
    const long long nB = n * B;
    ensure_gmres(c, B, std::max(maxit, 8));
    // workspace in the Krylov basis buffer: rhat, r (adjacent), p, v, s, t (adjacent), y, z
    double2* rhat = c->V;
    double2* r = c->V + nB;
    double2* p = c->V + 2 * nB;
    double2* v = c->V + 3 * nB;
    double2* sv = c->V + 4 * nB;
    double2* t = c->V + 5 * nB;
    double2* y = c->V + 6 * nB;
    double2* z = c->V + 7 * nB;
    auto P = [&](const double2* in, double2* out) {
        if (flex || sizeof(T) == sizeof(float)) apply_P<float>(c, in, out, B);
        else apply_P<double>(c, in, out, B);
    };
    auto M = [&](const double2* in, double2* out) {
        if (sizeof(T) == sizeof(float)) apply_M<float>(c, in, out, B);
        else apply_M<double>(c, in, out, B);
    };
    std::vector<double2> hv(3 * (size_t)B), cf(3 * (size_t)B);
    auto read = [&](int count) {       // c->gh[0 .. count*B) -> hv
        double2* hp = pinned(c, (size_t)count * B);
        HIPCHK(hipMemcpyAsync(hp, c->gh, sizeof(double2) * count * B,
                              hipMemcpyDeviceToHost, c->st));
        sync(c);
        std::copy(hp, hp + (size_t)count * B, hv.begin());
    };
    auto coefs = [&]() {               // cf -> c->gcoef (3 per column: [j][b])
        HIPCHK(hipMemcpyAsync(c->gcoef, cf.data(), sizeof(double2) * 3 * B,
                              hipMemcpyHostToDevice, c->st));
    };
    using cd = std::complex<double>;
    auto cx = [](double2 a) { return cd(a.x, a.y); };
    auto d2 = [](cd a) { return make_double2(a.real(), a.imag()); };
    // r = rhat = b, x = p = v = 0
    HIPCHK(hipMemcpyAsync(r, b, sizeof(double2) * nB, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(hipMemcpyAsync(rhat, b, sizeof(double2) * nB, hipMemcpyDeviceToDevice, c->st));
    launch_fill_zero(x, nB, c->st);
    launch_fill_zero(p, nB, c->st);
    launch_fill_zero(v, nB, c->st);
    dots_dev(c, nullptr, 0, 1, b, n, B, c->gh);                 // |b|^2
    read(1);
    std::vector<double> nb(B);
    std::vector<cd> rho_prev(B, 1.0), alpha(B, 1.0), omega(B, 1.0);
    std::vector<int> done(B, 0);
    iters.assign(B, 0);
    relres.assign(B, 0.0);
    for (int bb = 0; bb < B; ++bb) {
        nb[bb] = std::sqrt(std::max(0.0, hv[bb].x));
        if (nb[bb] == 0.0) done[bb] = 1;
    }
    for (int it = 1; it <= maxit; ++it) {
        if (std::all_of(done.begin(), done.end(), [](int q) { return q != 0; })) break;
        // rho = (rhat, r)
        dots_dev(c, rhat, nB, 1, r, n, B, c->gh);
        read(1);
        std::vector<cd> rho(B), beta(B, 0.0);
        for (int bb = 0; bb < B; ++bb) {
            rho[bb] = cx(hv[bb]);
            if (done[bb]) continue;
            if (rho[bb] == 0.0) { done[bb] = 1; continue; }          // breakdown
            beta[bb] = (rho[bb] / rho_prev[bb]) * (alpha[bb] / omega[bb]);
        }
        // p = r + beta (p - omega v)
        for (int bb = 0; bb < B; ++bb) {
            const bool a = !done[bb];
            cf[bb] = make_double2(1.0, 0.0);
            cf[B + bb] = d2(a ? beta[bb] : cd(0.0));
            cf[2 * B + bb] = d2(a ? -beta[bb] * omega[bb] : cd(0.0));
        }
        coefs();
        launch_lincomb3(p, r, p, v, c->gcoef, n, B, c->st);
        P(p, y);
        M(y, v);
        // alpha = rho / (rhat, v)
        dots_dev(c, rhat, nB, 1, v, n, B, c->gh);
        read(1);
        for (int bb = 0; bb < B; ++bb) {
            const cd den = cx(hv[bb]);
            if (done[bb] || den == 0.0) { alpha[bb] = 0.0; if (!done[bb]) done[bb] = 1; continue; }
            alpha[bb] = rho[bb] / den;
        }
        // s = r - alpha v
        for (int bb = 0; bb < B; ++bb) {
            cf[bb] = make_double2(1.0, 0.0);
            cf[B + bb] = d2(-alpha[bb]);
            cf[2 * B + bb] = make_double2(0.0, 0.0);
        }
        coefs();
        launch_lincomb3(sv, r, v, nullptr, c->gcoef, n, B, c->st);
        P(sv, z);
        M(z, t);
        // (s, t), (t, t) with w = t and V = [s, t]; |s|^2
        dots_dev(c, sv, nB, 2, t, n, B, c->gh);
        dots_dev(c, nullptr, 0, 1, sv, n, B, c->gh + 2 * B);
        read(3);
        std::vector<int> half(B, 0);
        for (int bb = 0; bb < B; ++bb) {
            if (done[bb]) { omega[bb] = 1.0; continue; }
            const double rs = std::sqrt(std::max(0.0, hv[2 * B + bb].x)) / nb[bb];
            if (rs <= tol) {                                   // converged at the half step
                half[bb] = 1;
                relres[bb] = rs;
                iters[bb] = it;
                omega[bb] = 0.0;
                continue;
            }
            const double tt = hv[B + bb].x;
            if (tt == 0.0) { half[bb] = 1; omega[bb] = 0.0; continue; }     // breakdown
            omega[bb] = std::conj(cx(hv[bb])) / tt;            // (t, s) / (t, t)
        }
        // x = x + alpha y + omega z ; r = s - omega t
        for (int bb = 0; bb < B; ++bb) {
            const bool a = !done[bb];
            cf[bb] = make_double2(1.0, 0.0);
            cf[B + bb] = d2(a ? alpha[bb] : cd(0.0));
            cf[2 * B + bb] = d2(a && !half[bb] ? omega[bb] : cd(0.0));
        }
        coefs();
        launch_lincomb3(x, x, y, z, c->gcoef, n, B, c->st);
        for (int bb = 0; bb < B; ++bb) {
            cf[bb] = make_double2(1.0, 0.0);
            cf[B + bb] = d2(!done[bb] && !half[bb] ? -omega[bb] : cd(0.0));
            cf[2 * B + bb] = make_double2(0.0, 0.0);
        }
        coefs();
        // (for stopped or half-step columns the coefficient is 0 and r = s,
        // which is their residual: s = r there since alpha = 0, or the
        // half-step residual)
        launch_lincomb3(r, sv, t, nullptr, c->gcoef, n, B, c->st);
        dots_dev(c, nullptr, 0, 1, r, n, B, c->gh);
        read(1);
        for (int bb = 0; bb < B; ++bb) {
            if (done[bb]) continue;
            if (half[bb]) { done[bb] = 1; continue; }
            const double rr = std::sqrt(std::max(0.0, hv[bb].x)) / nb[bb];
            relres[bb] = rr;
            iters[bb] = it;
            if (rr <= tol || omega[bb] == 0.0) done[bb] = 1;
            rho_prev[bb] = rho[bb];
        }
    }
    sync(c);
}

template <typename T>
void dd_solve(hz_ctx* c, int B, double tol, int maxit, const std::vector<int>& active,
              std::vector<int>& iters, std::vector<double>& relres, double* t_rhs,
              double* t_gm, double* t_rec, bool flex = false) {
    Work<T>& w = work<T>(c);
    const Dims& d = c->d;
    double t0 = now_s();
    upload(c, c->layer_active, active.data(), sizeof(int) * d.L);
    if (d.K == 0) {
        // single layer: the layer solve is the global solve (Alg. 7 volume mode)
        if (d.Lc > 1) sample_sources<T>(c, B, active.data());
        reconstruct_impl<T>(c, B, active.data());
        iters.assign(B, 0);
        relres.assign(B, 0.0);
        *t_rec += now_s() - t0;
        return;
    }
    const long long n = 4LL * d.K * d.W;
    sie_rhs_impl<T>(c, B, w.pB, active.data());
    // FP64 copy of the polarized RHS
    if constexpr (sizeof(T) == sizeof(double)) {
        HIPCHK(hipMemcpyAsync(c->gb, w.pB, sizeof(double2) * n * B, hipMemcpyDeviceToDevice, c->st));
    } else {
        launch_cast_f2d(c->gb, (const float2*)w.pB, n * B, c->st);
    }
    sync(c);
    double t1 = now_s();
    *t_rhs += t1 - t0;
    if (c->prm.krylov == HZ_KRYLOV_BICGSTAB)
        bicgstab<T>(c, c->gb, c->gx, B, tol, maxit, iters, relres, flex);
    else
        gmres<T>(c, c->gb, c->gx, B, tol, maxit, iters, relres, flex);
    double t2 = now_s();
    *t_gm += t2 - t1;
    // s = d + q  (in T)
    const long long half = 2LL * d.K * d.W * B;
    if constexpr (sizeof(T) == sizeof(double)) {
        HIPCHK(hipMemcpyAsync(w.sv, c->gx, sizeof(double2) * half, hipMemcpyDeviceToDevice, c->st));
        launch_axpby<double>((double2*)w.sv, c->gx + half, make_double2(1, 0), make_double2(1, 0), half, c->st);
    } else {
        launch_axpby<double>(c->gx, c->gx + half, make_double2(1, 0), make_double2(1, 0), half, c->st);
        launch_cast_d2f((float2*)w.sv, c->gx, half, c->st);
    }
    reconstruct_impl<T>(c, B, active.data());
    sync(c);
    *t_rec += now_s() - t2;
}

void check_state(hz_ctx* c, int need) {
    if (!c) raise(HZ_EINVAL, "null context");
    if (c->state < need) raise(HZ_ESTATE, need == 2 ? "call hz_factor first" : "context not set up");
}

// volume residual norms ||f - H u|| / ||f|| per RHS, fields [W][W][B] FP64
void vol_resid(hz_ctx* c, const double2* u, const double2* f, int B, std::vector<double>& out) {
    const long long N = (long long)c->d.W * c->d.W;
    out.resize(B);
    if (B <= 4096) {                        // one pass: norms without storing f - H u
        // gpart holds gpart_chunks * (m + 2) * B entries (m >= 1)
        const long long cap = (long long)c->gpart_chunks * (c->g_cap_m + 2);
        const int nb = residual_norms_blocks(c->d.W, B, (int)std::min<long long>(cap, 1 << 20));
        launch_residual_norms(u, f, c->gdiag, c->gcx, c->gcz, c->d.W, B, c->gpart, nb, c->st);
        launch_reduce_partials(c->gpart, nb, B, c->gsmall, c->st);
        double2* h = pinned(c, B);
        HIPCHK(hipMemcpyAsync(h, c->gsmall, sizeof(double2) * B, hipMemcpyDeviceToHost, c->st));
        sync(c);
        for (int b = 0; b < B; ++b) out[b] = h[b].y > 0 ? std::sqrt(h[b].x / h[b].y) : 0.0;
        return;
    }
    double2* r = c->r64;
    launch_residual(u, f, r, c->gdiag, c->gcx, c->gcz, c->d.W, B, 1, c->st);
    std::vector<double> nr, nf;
    norms(c, r, N, B, nr);
    norms(c, f, N, B, nf);
    for (int b = 0; b < B; ++b) out[b] = nf[b] > 0 ? nr[b] / nf[b] : 0.0;
}

void ensure_refine(hz_ctx* c) {
    if (c->u64) return;
    const long long N = (long long)c->d.W * c->d.W * std::max(c->prm.max_batch, 1);
    c->u64 = (double2*)c->arena.alloc(sizeof(double2) * N);
    c->f64 = (double2*)c->arena.alloc(sizeof(double2) * N);
    c->r64 = (double2*)c->arena.alloc(sizeof(double2) * N);
}

hz_status solve_impl(hz_ctx* c, const void* rhs_dev, int B, void* out_dev, double tol,
                     int max_iter, hz_rhs_stats* stats, hz_timing* timing, int ext_out,
                     int adjoint) {
    check_state(c, 2);
    if (!rhs_dev || !out_dev || B < 1) raise(HZ_EINVAL, "bad solve arguments");
    if (B > std::max(c->prm.max_batch, 1)) raise(HZ_EINVAL, "B exceeds max_batch");
    if (!(tol > 0.0) || max_iter < 1) raise(HZ_EINVAL, "bad tol / max_iter");
    const Dims& d = c->d;
    const long long N = (long long)d.W * d.W;
    double t0 = now_s();
    double t_rhs = 0, t_gm = 0, t_rec = 0;
    ensure_refine(c);
    ensure_gmres(c, B, max_iter);
    const double2* rhs = (const double2*)rhs_dev;
    // f64 = rhs on the extended grid (batch fastest); adjoint: conj(rhs)
    HIPCHK(hipMemsetAsync(c->layer_active, 0, sizeof(int) * d.L, c->st));
    if (adjoint) {
        double2* tmp = c->r64;
        launch_conj_copy(tmp, rhs, (long long)B * d.n * d.n, c->st);
        launch_rhs_to_ext(tmp, B, d.n, d.p, d.W, c->f64, c->d_layers, d.L, c->layer_active, c->st);
    } else {
        launch_rhs_to_ext(rhs, B, d.n, d.p, d.W, c->f64, c->d_layers, d.L, c->layer_active, c->st);
    }
    std::vector<int> active(d.L);
    HIPCHK(hipMemcpyAsync(active.data(), c->layer_active, sizeof(int) * d.L, hipMemcpyDeviceToHost, c->st));
    sync(c);
    std::vector<int> iters(B, 0), it1;
    std::vector<double> relres(B, 0.0), vres;
    int refine_steps = 0;
    bool conv = true;
    std::vector<double> err_est(B, 0.0);
    // nested polarized traces: the inner systems outside the preconditioner
    // are solved well below the outer tolerance (the SIE matrix, the right-
    // hand side and the reconstruction must be exact to it); the
    // preconditioner's loose inner solves make it nonlinear, hence flexible
    // GMRES
    struct InnerTolScope {             // the solve's inner tolerance, reset on every exit
        hz_ctx* c;
        ~InnerTolScope() { c->inner_tol_solve = 0.0; }
    } inner_scope{c};
    c->inner_tol_solve = std::min(1e-10, std::max(1e-13, 0.01 * tol));
    c->inner_iters_max = 0;
    if (c->prm.precision == HZ_FP64 || c->prm.precision == HZ_MIXED) {
        const bool flex = c->prm.precision == HZ_MIXED || c->inner_pt;
        ensure_work<double>(c, B);
        if (c->prm.precision == HZ_MIXED) ensure_work<float>(c, B, false);
        dd_solve<double>(c, B, tol, max_iter, active, iters, relres, &t_rhs, &t_gm, &t_rec, flex);
        for (int b = 0; b < B; ++b) if (!(relres[b] <= tol)) conv = false;
    } else {
        // FP64 iterative refinement around the complex64 nested solver
        ensure_work<float>(c, B);
        Work<float>& w = c->w32;
        HIPCHK(hipMemsetAsync(c->u64, 0, sizeof(double2) * N * B, c->st));
        std::vector<int> all(d.L, 1);
        const double inner_tol = std::max(1e-6, tol);
        const int max_refine = 30;
        std::vector<double> un, dn, dprev(B, 0.0);
        for (int step = 0; step < max_refine; ++step) {
            launch_residual(c->u64, c->f64, c->r64, c->gdiag, c->gcx, c->gcz, d.W, B, 1, c->st);
            launch_cast_d2f(w.f_ext, c->r64, N * B, c->st);
            dd_solve<float>(c, B, inner_tol, max_iter, step == 0 ? active : all, it1, relres,
                            &t_rhs, &t_gm, &t_rec);
            for (int b = 0; b < B; ++b) iters[b] += it1[b];
            launch_cast_f2d(c->r64, w.u_ext, N * B, c->st);          // delta
            launch_axpby<double>(c->u64, c->r64, make_double2(1, 0), make_double2(1, 0), N * B, c->st);
            norms(c, c->r64, N, B, dn);
            norms(c, c->u64, N, B, un);
            refine_steps = step + 1;
            // error of u after this step ~ rho/(1 - rho) ||delta|| with the
            // observed contraction rho = ||delta_k|| / ||delta_{k-1}||
            bool ok = true;
            for (int b = 0; b < B; ++b) {
                const double rel = un[b] > 0 ? dn[b] / un[b] : 0.0;
                double est = 1.0;
                if (step > 0 && dprev[b] > 0) {
                    const double rho = dn[b] / dprev[b];
                    est = rho < 1.0 ? rho / (1.0 - rho) * rel : 1.0;
                }
                if (rel == 0.0) est = 0.0;
                err_est[b] = est;
                dprev[b] = dn[b];
                if (est > tol) ok = false;
            }
            if (ok) break;
            if (step == max_refine - 1) conv = false;
        }
    }
    if (stats) vol_resid(c, c->u64, c->f64, B, vres);
    if (c->prof.on) prof_flush(c);
    launch_ext_to_out(c->u64, B, d.n, d.p, d.W, (double2*)out_dev, ext_out ? 0 : 1, adjoint, c->st);
    HIPCHK(hipGetLastError());
    sync(c);
    const double t_all = now_s() - t0;
    c->timing.t_rhs = t_rhs;
    c->timing.t_gmres = t_gm;
    c->timing.t_recon = t_rec;
    c->timing.t_solve = t_all;
    c->timing.gmres_iters = *std::max_element(iters.begin(), iters.end());
    c->timing.inner_iters = c->inner_iters_max;
    if (timing) *timing = c->timing;
    if (stats) {
        for (int b = 0; b < B; ++b) {
            stats[b].iters = iters[b];
            stats[b].rel_resid = relres[b];
            stats[b].vol_resid = vres.empty() ? -1.0 : vres[b];
            stats[b].refine_steps = refine_steps;
            stats[b].err_est = err_est[b];
        }
    }
    return conv ? HZ_OK : HZ_ENOCONV;
}

hz_status setup_coef(hz_ctx* c, const double* model_dev) {
    const Dims& d = c->d;
    // validate first: a rejected model leaves the context as it was
    HIPCHK(hipMemsetAsync(c->flags, 0, 2 * sizeof(int), c->st));
    launch_check_model(model_dev, (long long)d.n * d.n, c->flags, c->st);
    HIPCHK(hipGetLastError());
    {
        int bad = 0;
        HIPCHK(hipMemcpyAsync(&bad, c->flags, sizeof(int), hipMemcpyDeviceToHost, c->st));
        sync(c);
        if (bad) raise(HZ_EINVAL, "model has NaN, infinite or non-positive entries");
    }
    HIPCHK(hipMemcpyAsync(c->model, model_dev, sizeof(double) * d.n * d.n, hipMemcpyDeviceToDevice, c->st));
    launch_build_coef(c->model, (int)c->prm.model_kind, d, c->d_cells, c->d_layers,
                      (int)c->cells.size(), c->cells.data(), c->diag, c->cz, c->e, c->ax_pool,
                      c->az_pool, c->gdiag, c->gcx, c->gcz, c->wext, c->flags, c->st);
    HIPCHK(hipGetLastError());
    int fl[2];
    HIPCHK(hipMemcpyAsync(fl, c->flags, sizeof(fl), hipMemcpyDeviceToHost, c->st));
    sync(c);
    if (fl[0]) raise(HZ_EINVAL, "model has NaN, infinite or non-positive entries");
    return HZ_OK;
}

#define API_BEGIN try {
#define API_END                                   \
    }                                             \
    catch (const HzError& e) {                    \
        g_err = e.msg;                            \
        return e.s;                               \
    }                                             \
    catch (const std::exception& e) {             \
        g_err = e.what();                         \
        return HZ_EDEVICE;                        \
    }                                             \
    catch (...) {                                 \
        g_err = "unknown error";                  \
        return HZ_EDEVICE;                        \
    }

}  // namespace

// ===========================================================================
// C-ABI

// ---------------------------------------------------------------------------
// Scratch of the allocation-free misfit (hz_misfit_noalloc): the partial sums
// of k_misfit.  One copy per device, held until the process ends.  Host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device (the array's name is a host-side stand-in there).
static __device__ __align__(256) double scratch[hz::MISFIT_PARTS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};

// address of `scratch` on `dev`, which must be the current device
double* misfit_scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) raise(HZ_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            raise(HZ_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        }
        g_scratch_addr[dev] = (double*)p;
    }
    return g_scratch_addr[dev];
}

// J = 1/2 sum of the partials, summed in index order (the order in which
// hz_misfit adds them on the host)
__global__ void k_misfit_total(const double* part, int n, double* J) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *J = 0.5 * s;
}
}  // namespace

extern "C" {

const char* hz_strerror(hz_status s) {
    switch (s) {
    case HZ_OK: return "ok";
    case HZ_EINVAL: return "invalid argument";
    case HZ_ENOMEM: return "out of device memory";
    case HZ_ESTATE: return "call out of order";
    case HZ_ENOCONV: return "GMRES did not converge";
    case HZ_ESINGULAR: return "singular factorisation";
    case HZ_EDEVICE: return "HIP runtime error";
    }
    return "unknown status";
}

const char* hz_last_error(void) { return g_err.c_str(); }

hz_status hz_setup(const double* model_dev, const hz_params* prm, hz_ctx** out) {
    if (out) *out = nullptr;
    hz_ctx* c = nullptr;
    API_BEGIN
    if (!prm || !out || !model_dev) raise(HZ_EINVAL, "null argument");
    const int n = prm->n_x;
    if (n < 2 || prm->n_z != n) raise(HZ_EINVAL, "n_x must equal n_z and be >= 2");
    if (std::fabs(prm->h * (n + 1) - 1.0) > 1e-9) raise(HZ_EINVAL, "h must be 1/(n+1)");
    if (!(prm->omega > 0.0) || !std::isfinite(prm->omega)) raise(HZ_EINVAL, "omega must be > 0");
    if (prm->n_pml < 0) raise(HZ_EINVAL, "n_pml must be >= 0");
    // the equivalent sources of a layer / cell interface sit on the first
    // artificial-PML row / column past the owned ones
    if ((prm->layers > 1 || prm->cells > 1) && prm->n_pml < 1)
        raise(HZ_EINVAL, "a decomposition (layers or cells > 1) needs n_pml >= 1");
    if (prm->layers < 1 || prm->layers > n / 2) raise(HZ_EINVAL, "layers must be in 1..n/2 (>= 2 rows each)");
    if (prm->cells < 1 || prm->cells > n / 2) raise(HZ_EINVAL, "cells must be in 1..n/2 (>= 2 columns each)");
    if (prm->precision != HZ_FP64 && prm->precision != HZ_MIXED &&
        prm->precision != HZ_MIXED_REFINE)
        raise(HZ_EINVAL, "bad precision");
    if (prm->model_kind != HZ_MODEL_VELOCITY && prm->model_kind != HZ_MODEL_SLOWNESS2)
        raise(HZ_EINVAL, "bad model kind");
    if (prm->precond != HZ_PRECOND_GS && prm->precond != HZ_PRECOND_JACOBI)
        raise(HZ_EINVAL, "bad preconditioner");
    if (prm->krylov != HZ_KRYLOV_GMRES && prm->krylov != HZ_KRYLOV_BICGSTAB)
        raise(HZ_EINVAL, "bad Krylov method");
    if (prm->inner != HZ_INNER_LU && prm->inner != HZ_INNER_PT) raise(HZ_EINVAL, "bad inner solver");
    if (prm->inner == HZ_INNER_PT) {
        if (prm->precision != HZ_FP64)
            raise(HZ_EINVAL, "nested polarized traces need precision HZ_FP64");
        if (prm->krylov != HZ_KRYLOV_GMRES)
            raise(HZ_EINVAL, "nested polarized traces need the (flexible) GMRES driver");
        if (!(prm->inner_tol < 1.0)) raise(HZ_EINVAL, "inner_tol must be < 1");
    }
    if (prm->plr != 0 && prm->plr != 1) raise(HZ_EINVAL, "plr must be 0 or 1");
    if (prm->plr && prm->inner != HZ_INNER_LU)
        raise(HZ_EINVAL, "PLR operators need the block-LU inner solver");
    if (prm->plr && !(prm->plr_eps < 1.0)) raise(HZ_EINVAL, "plr_eps must be < 1");
    c = new hz_ctx();
    c->prm = *prm;
    c->inner_pt = prm->inner == HZ_INNER_PT && prm->cells > 1;
    if (c->inner_pt) {
        c->compose = 0;
        c->inner_tol_loose = prm->inner_tol > 0.0 ? prm->inner_tol : 1e-6;
    }
    if (const char* g = std::getenv("HZ_GRAPHS")) c->use_graphs = std::atoi(g) != 0;
    if (const char* g = std::getenv("HZ_COMPOSE"))
        c->compose = c->inner_pt ? 0 : std::min(2, std::max(0, std::atoi(g)));
    if (const char* g = std::getenv("HZ_TUNE")) c->tune = std::atoi(g) != 0;
    if (const char* g = std::getenv("HZ_GEMM_KIND")) {
        const int k = std::atoi(g);
        if (k >= GEMM_MFMA32 && k <= GEMM_MFMA32DS8) c->force_kind = k;
    }
    if (c->prm.pml_beta <= 0.0) c->prm.pml_beta = 2.0;
    if (c->prm.plr_eps <= 0.0) c->prm.plr_eps = 1e-8;
    if (c->prm.max_batch <= 0) c->prm.max_batch = 1;
    Dims& d = c->d;
    d.n = n;
    d.p = prm->n_pml;
    d.W = n + 2 * d.p;
    d.L = prm->layers;
    d.Lc = prm->cells;
    d.K = d.L - 1;
    d.h = 1.0 / (n + 1);
    d.omega = prm->omega;
    d.beta = c->prm.pml_beta;
    build_descriptors(c);
    if (d.HLmax > 224) raise(HZ_EINVAL, "layer grid taller than 224 rows: use more layers");
    if (2 * d.HLmax > 448) raise(HZ_EINVAL, "inner block too large");
    double t0 = now_s();
    // a blocking stream of default priority: ordered after work on the null
    // stream, and capturable into graphs
    HIPCHK(hipStreamCreate(&c->own_st));
    c->st = c->own_st;
    HIPCHK(hipGetDevice(&c->device));
    c->misfit_scratch = misfit_scratch_address(c->device);
    c->d_layers = (LayerDesc*)c->arena.alloc(sizeof(LayerDesc) * d.L);
    c->d_cells = (CellDesc*)c->arena.alloc(sizeof(CellDesc) * c->cells.size());
    upload(c, c->d_layers, c->layers.data(), sizeof(LayerDesc) * d.L);
    upload(c, c->d_cells, c->cells.data(), sizeof(CellDesc) * c->cells.size());
    {
        std::vector<int> all(c->cells.size());
        for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
        c->d_all_cells = (int*)c->arena.alloc(sizeof(int) * all.size());
        c->d_cell_list = (int*)c->arena.alloc(sizeof(int) * all.size());
        upload(c, c->d_all_cells, all.data(), sizeof(int) * all.size());
    }
    c->model = (double*)c->arena.alloc(sizeof(double) * n * n);
    c->diag = alloc_c<double>(c, c->coef_elems);
    c->cz = alloc_c<double>(c, c->coef_elems);
    c->e = alloc_c<double>(c, c->coef_elems);
    c->ax_pool = alloc_c<double>(c, (long long)c->cells.size() * d.Wcmax);
    c->az_pool = alloc_c<double>(c, (long long)d.L * d.HLmax);
    const long long N = (long long)d.W * d.W;
    c->gdiag = alloc_c<double>(c, N);
    c->gcx = alloc_c<double>(c, N);
    c->gcz = alloc_c<double>(c, N);
    c->wext = alloc_c<double>(c, N);
    c->flags = (int*)c->arena.alloc(sizeof(int) * 4);
    c->fflags = (FactorFlags*)c->arena.alloc(sizeof(FactorFlags));
    c->layer_active = (int*)c->arena.alloc(sizeof(int) * d.L);
    setup_coef(c, model_dev);
    c->state = 1;
    c->timing.t_setup = now_s() - t0;
    *out = c;
    return HZ_OK;
    }
    catch (const HzError& e) {
        g_err = e.msg;
        if (c) { c->arena.free_all(); delete c; }
        return e.s;
    }
    catch (...) {
        g_err = "unknown error in hz_setup";
        if (c) { c->arena.free_all(); delete c; }
        return HZ_EDEVICE;
    }
}

hz_status hz_update_model(hz_ctx* c, const double* model_dev) {
    API_BEGIN
    check_state(c, 1);
    if (!model_dev) raise(HZ_EINVAL, "null model");
    setup_coef(c, model_dev);              // a rejected model changes nothing
    c->state = 1;
    return HZ_OK;
    API_END
}

hz_status hz_factor(hz_ctx* c) {
    API_BEGIN
    check_state(c, 1);
    double t0 = now_s();
    c->state = 1;
    factor_impl(c);
    clear_plans(c);
    c->state = 2;
    c->timing.t_factor = now_s() - t0;
    return HZ_OK;
    API_END
}

hz_status hz_update_model_local(hz_ctx* c, const double* model_dev, int* ncells_refactored) {
    API_BEGIN
    check_state(c, 2);
    if (!model_dev) raise(HZ_EINVAL, "null model");
    const Dims& d = c->d;
    const int ncells = (int)c->cells.size();
    double t0 = now_s();
    std::vector<char> redo(ncells, 1);
    {
        const long long ne = c->coef_elems;
        const long long nax = (long long)ncells * d.Wcmax, naz = (long long)d.L * d.HLmax;
        double2* old = alloc_c<double>(c, 3 * ne + nax + naz);
        const size_t cb = sizeof(double2) * ne;
        HIPCHK(hipMemcpyAsync(old, c->diag, cb, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(hipMemcpyAsync(old + ne, c->cz, cb, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(hipMemcpyAsync(old + 2 * ne, c->e, cb, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(hipMemcpyAsync(old + 3 * ne, c->ax_pool, sizeof(double2) * nax, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(hipMemcpyAsync(old + 3 * ne + nax, c->az_pool, sizeof(double2) * naz, hipMemcpyDeviceToDevice, c->st));
        try {
            setup_coef(c, model_dev);      // a rejected model changes nothing
        } catch (...) {
            c->arena.release(old, sizeof(double2) * (3 * ne + nax + naz));
            throw;
        }
        c->state = 1;                      // operators stale until refactored
        int* dchg = (int*)c->arena.alloc(sizeof(int) * (ncells + 1));
        HIPCHK(hipMemsetAsync(dchg + ncells, 0, sizeof(int), c->st));
        hipLaunchKernelGGL(k_coef_changed, dim3(ncells), dim3(256), 0, c->st, c->d_cells, old,
                           old + ne, old + 2 * ne, c->diag, c->cz, c->e, dchg);
        hipLaunchKernelGGL(k_any_diff, dim3(256), dim3(256), 0, c->st, old + 3 * ne, c->ax_pool,
                           nax, dchg + ncells);
        hipLaunchKernelGGL(k_any_diff, dim3(256), dim3(256), 0, c->st, old + 3 * ne + nax,
                           c->az_pool, naz, dchg + ncells);
        HIPCHK(hipGetLastError());
        std::vector<int> chg(ncells + 1);
        HIPCHK(hipMemcpyAsync(chg.data(), dchg, sizeof(int) * (ncells + 1), hipMemcpyDeviceToHost, c->st));
        sync(c);
        c->arena.release(dchg, sizeof(int) * (ncells + 1));
        c->arena.release(old, sizeof(double2) * (3 * ne + nax + naz));
        for (int i = 0; i < ncells; ++i) redo[i] = (chg[ncells] || chg[i]) ? 1 : 0;
    }
    int cnt = 0;
    for (char r : redo) cnt += r;
    factor_impl(c, &redo);
    clear_plans(c);
    c->state = 2;
    c->timing.t_factor = now_s() - t0;
    if (ncells_refactored) *ncells_refactored = cnt;
    return HZ_OK;
    API_END
}

hz_status hz_solve(hz_ctx* c, const void* rhs, int B, void* u, double tol, int max_iter,
                   hz_rhs_stats* stats, hz_timing* timing) {
    API_BEGIN
    return solve_impl(c, rhs, B, u, tol, max_iter, stats, timing, 0, 0);
    API_END
}

hz_status hz_solve_ext(hz_ctx* c, const void* rhs, int B, void* u, double tol, int max_iter,
                       hz_rhs_stats* stats, hz_timing* timing) {
    API_BEGIN
    return solve_impl(c, rhs, B, u, tol, max_iter, stats, timing, 1, 0);
    API_END
}

hz_status hz_adjoint(hz_ctx* c, const void* rhs, int B, void* lam, double tol, int max_iter,
                     hz_rhs_stats* stats) {
    API_BEGIN
    return solve_impl(c, rhs, B, lam, tol, max_iter, stats, nullptr, 0, 1);
    API_END
}

hz_status hz_adjoint_ext(hz_ctx* c, const void* rhs, int B, void* lam, double tol, int max_iter,
                         hz_rhs_stats* stats) {
    API_BEGIN
    return solve_impl(c, rhs, B, lam, tol, max_iter, stats, nullptr, 1, 1);
    API_END
}

hz_status hz_misfit_gradient(hz_ctx* c, const void* u_ext, const void* lam_ext, int B, double* g) {
    API_BEGIN
    check_state(c, 1);
    if (!u_ext || !lam_ext || !g || B < 1) raise(HZ_EINVAL, "bad gradient arguments");
    launch_misfit_grad((const double2*)u_ext, (const double2*)lam_ext, B, c->d.W, c->d.n, c->d.p,
                       c->wext, c->d.omega, g, c->st);
    HIPCHK(hipGetLastError());
    sync(c);
    return HZ_OK;
    API_END
}

hz_status hz_misfit(hz_ctx* c, const void* u_ext, const void* d_obs, int rec_row, int B,
                    void* adj, double* J) {
    API_BEGIN
    check_state(c, 1);
    if (!u_ext || !d_obs || !adj || !J || B < 1 || rec_row < 1 || rec_row > c->d.n)
        raise(HZ_EINVAL, "bad misfit arguments");
    double* part = (double*)c->arena.alloc(sizeof(double) * MISFIT_PARTS);
    launch_misfit((const double2*)u_ext, (const double2*)d_obs, rec_row, B, c->d.n, c->d.p,
                  c->d.W, (double2*)adj, part, c->st);
    HIPCHK(hipGetLastError());
    std::vector<double> hp(MISFIT_PARTS);
    HIPCHK(hipMemcpyAsync(hp.data(), part, sizeof(double) * MISFIT_PARTS, hipMemcpyDeviceToHost, c->st));
    sync(c);
    c->arena.release(part, sizeof(double) * MISFIT_PARTS);
    double s = 0.0;
    for (double v : hp) s += v;
    *J = 0.5 * s;
    return HZ_OK;
    API_END
}

hz_status hz_misfit_noalloc(hz_ctx* c, const void* u_ext, const void* d_obs, int rec_row, int B,
                            void* adj, double* J_dev) {
    API_BEGIN
    check_state(c, 1);
    if (!u_ext || !d_obs || !adj || !J_dev || B < 1 || rec_row < 1 || rec_row > c->d.n)
        raise(HZ_EINVAL, "bad misfit arguments");
    if (!c->misfit_scratch) raise(HZ_ESTATE, "no scratch address for this context's device");
    // the kernel writes every one of its MISFIT_PARTS partial sums, so the
    // array needs no clearing; its size does not depend on B or n
    launch_misfit((const double2*)u_ext, (const double2*)d_obs, rec_row, B, c->d.n, c->d.p,
                  c->d.W, (double2*)adj, c->misfit_scratch, c->st);
    hipLaunchKernelGGL(k_misfit_total, dim3(1), dim3(64), 0, c->st, c->misfit_scratch,
                       MISFIT_PARTS, J_dev);
    HIPCHK(hipGetLastError());
    return HZ_OK;
    API_END
}

hz_status hz_set_stream(hz_ctx* c, void* s) {
    API_BEGIN
    if (!c) raise(HZ_EINVAL, "null context");
    sync(c);
    c->st = s ? (hipStream_t)s : c->own_st;
    // graphs were captured on the previous stream; rebuild lazily
    clear_plans(c);
    return HZ_OK;
    API_END
}

hz_status hz_profile(hz_ctx* c, int on) {
    API_BEGIN
    if (!c) raise(HZ_EINVAL, "null context");
    prof_flush(c);
    c->prof.acc.clear();
    c->prof.on = on != 0;
    return HZ_OK;
    API_END
}

hz_status hz_profile_read(hz_ctx* c, hz_kstat* out, int max, int* count) {
    API_BEGIN
    if (!c || !count) raise(HZ_EINVAL, "null argument");
    prof_flush(c);
    int i = 0;
    for (const auto& kv : c->prof.acc) {
        if (out && i < max) out[i] = kv.second;
        ++i;
    }
    *count = i;
    return HZ_OK;
    API_END
}

hz_status hz_get_info(const hz_ctx* c, hz_info_t* info) {
    if (!c || !info) return HZ_EINVAL;
    info->n = c->d.n;
    info->n_pml = c->d.p;
    info->W = c->d.W;
    info->layers = c->d.L;
    info->cells = c->d.Lc;
    info->trace_len = 4 * c->d.K * c->d.W;
    info->max_batch = c->prm.max_batch;
    info->device_bytes = c->arena.bytes;
    if (c->prm.precision == HZ_FP64) {
        info->plr_bytes = c->plr64.stored * (long long)sizeof(double2);
        info->plr_dense_bytes = c->plr64.dense * (long long)sizeof(double2);
    } else {
        info->plr_bytes = c->plr32.stored * (long long)sizeof(float2);
        info->plr_dense_bytes = c->plr32.dense * (long long)sizeof(float2);
    }
    info->min_pivot_ratio = c->min_pivot_ratio;
    return HZ_OK;
}

hz_status hz_get_timing(const hz_ctx* c, hz_timing* t) {
    if (!c || !t) return HZ_EINVAL;
    *t = c->timing;
    return HZ_OK;
}

void hz_destroy(hz_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    for (hipEvent_t e : c->prof.pool) (void)hipEventDestroy(e);
    clear_plans(c);
    c->arena.free_all();
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    if (c->h_iflag) (void)hipHostFree(c->h_iflag);
    if (c->iev) (void)hipEventDestroy(c->iev);
    if (c->own_st) (void)hipStreamDestroy(c->own_st);
    delete c;
}

// ---- building blocks ---------------------------------------------------------

hz_status hz_apply_layer(hz_ctx* c, int layer, const void* top, const void* bot, int side,
                         void* out, int B) {
    API_BEGIN
    check_state(c, 2);
    if (c->prm.precision == HZ_MIXED_REFINE) raise(HZ_EINVAL, "building blocks need FP64 operators");
    if (layer < 0 || layer >= c->d.L || !out || B < 1 || B > c->prm.max_batch) raise(HZ_EINVAL, "bad arguments");
    const LayerDesc& ld = c->layers[layer];
    if ((side == 0 && !ld.has_top) || (side == 1 && !ld.has_bot) || side < 0 || side > 1)
        raise(HZ_EINVAL, "layer has no interface on that side");
    if ((top && !ld.has_top) || (bot && !ld.has_bot)) raise(HZ_EINVAL, "no such input pair");
    ensure_work<double>(c, B);
    LayerJob<double> jb;
    jb.layer = layer;
    jb.top = (const double2*)top;
    jb.bot = (const double2*)bot;
    jb.iy = iy_of<double>(c, 0, layer, B);
    jb.ix = ix_of<double>(c, 0, layer, B);
    jb.side = side;
    jb.out = (double2*)out;
    jb.alpha = 1.0;
    run_jobs<double>(c, {jb}, B);
    return HZ_OK;
    API_END
}

hz_status hz_apply_sie(hz_ctx* c, const void* x, void* y, int B) {
    API_BEGIN
    check_state(c, 2);
    if (c->prm.precision == HZ_MIXED_REFINE) raise(HZ_EINVAL, "building blocks need FP64 operators");
    if (!x || !y || B < 1 || B > c->prm.max_batch || c->d.K == 0) raise(HZ_EINVAL, "bad arguments");
    ensure_work<double>(c, B);
    Work<double>& w = c->w64;
    const long long n = 4LL * c->d.K * c->d.W * B;
    HIPCHK(hipMemcpyAsync(w.pA, x, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    plan_run<double>(c, get_plan<double>(c, true, B), B);
    HIPCHK(hipMemcpyAsync(y, w.pB, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    sync(c);
    return HZ_OK;
    API_END
}

hz_status hz_apply_precond(hz_ctx* c, const void* x, void* y, int B) {
    API_BEGIN
    check_state(c, 2);
    if (c->prm.precision == HZ_MIXED_REFINE) raise(HZ_EINVAL, "building blocks need FP64 operators");
    if (!x || !y || B < 1 || B > c->prm.max_batch || c->d.K == 0) raise(HZ_EINVAL, "bad arguments");
    ensure_work<double>(c, B);
    Work<double>& w = c->w64;
    const long long n = 4LL * c->d.K * c->d.W * B;
    HIPCHK(hipMemcpyAsync(w.pB, x, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    plan_run<double>(c, get_plan<double>(c, false, B), B);
    HIPCHK(hipMemcpyAsync(y, w.pC, sizeof(double2) * n, hipMemcpyDeviceToDevice, c->st));
    sync(c);
    return HZ_OK;
    API_END
}

hz_status hz_sie_rhs(hz_ctx* c, const void* rhs, void* y, int B) {
    API_BEGIN
    check_state(c, 2);
    if (c->prm.precision == HZ_MIXED_REFINE) raise(HZ_EINVAL, "building blocks need FP64 operators");
    if (!rhs || !y || B < 1 || B > c->prm.max_batch || c->d.K == 0) raise(HZ_EINVAL, "bad arguments");
    ensure_work<double>(c, B);
    ensure_refine(c);
    const Dims& d = c->d;
    HIPCHK(hipMemsetAsync(c->layer_active, 0, sizeof(int) * d.L, c->st));
    launch_rhs_to_ext((const double2*)rhs, B, d.n, d.p, d.W, c->w64.f_ext, c->d_layers, d.L,
                      c->layer_active, c->st);
    std::vector<int> active(d.L);
    HIPCHK(hipMemcpyAsync(active.data(), c->layer_active, sizeof(int) * d.L, hipMemcpyDeviceToHost, c->st));
    sync(c);
    sie_rhs_impl<double>(c, B, (double2*)y, active.data());
    sync(c);
    return HZ_OK;
    API_END
}

hz_status hz_cell_shape(const hz_ctx* c, int layer, int cell, int* HL, int* Wc) {
    if (!c || layer < 0 || layer >= c->d.L || cell < 0 || cell >= c->d.Lc || !HL || !Wc)
        return HZ_EINVAL;
    const CellDesc& cd = c->cells[layer * c->d.Lc + cell];
    *HL = cd.HL;
    *Wc = cd.Wc;
    return HZ_OK;
}

hz_status hz_cell_solve(hz_ctx* c, int layer, int cell, const void* g, void* x, int B) {
    API_BEGIN
    check_state(c, 2);
    if (c->prm.precision == HZ_MIXED_REFINE) raise(HZ_EINVAL, "building blocks need FP64 operators");
    if (layer < 0 || layer >= c->d.L || cell < 0 || cell >= c->d.Lc || !g || !x || B < 1 ||
        B > c->prm.max_batch)
        raise(HZ_EINVAL, "bad arguments");
    ensure_work<double>(c, B);
    CellSolveArgs<double> a = base_args<double>(c);
    a.mode = SOLVE_GRID;
    a.g_grid = (const double2*)g;
    a.x_grid = (double2*)x;
    cell_solve_launch<double>(c, a, {layer * c->d.Lc + cell}, B);
    return HZ_OK;
    API_END
}

hz_status hz_residual(hz_ctx* c, const void* u, const void* f, void* r, int B) {
    API_BEGIN
    check_state(c, 1);
    if (!u || !r || B < 1) raise(HZ_EINVAL, "bad arguments");
    launch_residual((const double2*)u, (const double2*)f, (double2*)r, c->gdiag, c->gcx, c->gcz,
                    c->d.W, B, 0, c->st);
    HIPCHK(hipGetLastError());
    sync(c);
    return HZ_OK;
    API_END
}

}  // extern "C"
