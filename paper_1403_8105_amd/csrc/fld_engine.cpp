// fld_engine.cpp -- host engine and C ABI of libfld (see include/fld.h).
//
// One Engine drives a batch of problems (one problem = one colour channel of
// one volume); a single-volume context is a batch of one.  Every phase of an
// iteration is one launch over a work list that covers all unconverged
// problems.  Memory is laid out z fastest per array; the finest level keeps
// the FP64 state, the multigrid levels keep precision-T copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/fld.h"
#include "fld_internal.h"

using namespace fld;

namespace {

struct DevList {
    Task *d = nullptr;
    int n = 0;
};

struct Level {
    int nx = 0, ny = 0, nz = 0;
    long long n = 0;
    double h = 0.0;
    void *e = nullptr, *b = nullptr, *sa = nullptr, *f = nullptr;
    void *e2 = nullptr;    // finest level, fused sweeps only
    double *band = nullptr;
};

struct Prob {
    int vol = 0, chan = 0;
    int nlev = 0;
    Fine fine{};
    Level lv[kMaxLevels];
    std::vector<double> hist;
    int final_k = 0;     // iteration at which the problem stopped
    int status = FLD_OK;
    int gid0 = 0;        // index of its finest grid in the grid table
    int deep = 0;        // first level of the deep part of the V-cycle (one workgroup)
};

struct Vol {
    int nx, ny, nz;
    long long n;
    double h, sigma_eps;
    double *sig_hat = nullptr;
    bool has_medium = false;
};

int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

constexpr int kRimTaskCells = 256;   // rim voxels per deflation rim task

}  // namespace

struct fld_engine_impl {
    fld_options opt{};
    bool mixed = false, mg = true;
    size_t tsz = 8;
    int nprob = 0;
    std::vector<Vol> vols;
    std::vector<Prob> probs;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // FLD_LOG set (and not "0"): one JSON line per problem and outer
    // iteration on stderr
    const bool log_iters = [] {
        const char *v = std::getenv("FLD_LOG");
        return v && *v && std::strcmp(v, "0") != 0;
    }();
    std::vector<void *> allocs;
    std::string err;

    Fine *d_fines = nullptr;
    Grid *d_grids[2] = {nullptr, nullptr};
    // cluster deflation (built when the media are set)
    bool defl_enabled = false, use_defl = false;
    int ncl_total = 0;
    CTask *d_ctasks = nullptr, *d_rtasks = nullptr;   // cluster-cell and rim tasks
    int n_ctasks = 0, n_rtasks = 0;
    int *d_crange = nullptr, *d_rrange = nullptr, *d_cprob = nullptr;
    double *d_alpha = nullptr, *d_csa = nullptr, *d_cpd = nullptr, *d_cps = nullptr;
    std::vector<void *> defl_allocs;
    int ngrids = 0;
    DevList fine_tasks;
    std::vector<int> fine_range;   // host copy, nprob+1
    int *d_fine_range = nullptr;
    // Anderson dot products: tasks of kAaTaskCells cells, so that each thread
    // sums several quads before the per-task reduction of its 2(m+1) values
    DevList aa_tasks;
    int *d_aa_range = nullptr;
    // fused limiter-residual pass: tiles of every problem, problem by problem
    bool fuse = false;
    // single-pass red-black sweeps of the finest level: tiles of every
    // problem (tile.prob: its level-0 grid)
    bool fuse_rb = false;
    LrTile *d_rbtiles = nullptr;
    int n_rbtiles = 0;
    LrTile *d_lrtiles = nullptr;
    int n_lrtiles = 0;
    int *d_lr_range = nullptr;
    double *d_lrpart = nullptr;
    DevList mid[kMaxLevels], rest[kMaxLevels], gal[kMaxLevels];
    int mid_cells[kMaxLevels] = {};   // cells per smoothing task of each level
    std::vector<Grid> h_grids;        // host copy of the grid table (parity 0)
    DevList coarse_cells[kMaxLevels];   // every cell of level l+1 (deep levels included)
    int *d_coarse_ids = nullptr, *d_deep_roots = nullptr;   // coarsest grids / deep roots
    int n_coarse = 0, n_deep = 0;
    int *d_tail_roots = nullptr;   // problems whose tail runs in one workgroup launch
    int n_tail = 0;
    // The coarsest factorisation runs on a second stream (default priority),
    // forked after the coarse operators are built and joined before the
    // coarsest solve, beside the down-sweep of the finer levels.
    int *d_factor_ids = nullptr;   // coarsest grid of every problem
    int n_factor = 0;
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    long long tail_lds = 0;
    int max_coarse_n = 1, max_coarse_bw = 1;
    // kernel instance choice: kmode 0 FP64 natural, 1 FP32 natural, 2 FP32
    // colour-split, 3 FP32 per problem, 4 FP64 colour-split, 5 FP64 per
    // problem; lsp the layout alone for the level kernels (0 / 1 / 2)
    int kmode = 0, lsp = 0;
    int max_levels = 0;
    double *d_part[4] = {};
    double *d_scal = nullptr;
    // Anderson acceleration: per-problem state and per-task partials
    int *d_aai = nullptr;
    double *d_aad = nullptr, *d_aapart = nullptr;
    int *d_active = nullptr, *d_fail = nullptr;
    std::vector<int> h_active, uploaded_active;
    double *h_scal_pin = nullptr;   // pinned host copies of the scalars and the mask
    int *h_active_pin = nullptr;
    int k_state = 0;               // next outer iteration index (resume)
    bool solved_once = false;

    // HIP-event timing of the hot kernels (options.timing).  Each interval
    // carries its algorithmic bytes per active finest cell; intervals recorded
    // while a graph is captured stay with that graph and are read after every
    // replay.
    struct Timed {
        hipEvent_t a, b;
        int cls;
        double bytes_per_cell;
        double cells;              // active finest cells at launch; < 0: read at harvest
    };
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<Timed> timed, *timed_sink = &timed;
    double acc_ms[4] = {}, acc_launch[4] = {}, acc_bytes[4] = {};
    double fine_cells = 0.0;       // sum of finest-level cells over problems
    bool capturing = false;

    // Events are only ever created outside stream capture: the ones a graph
    // records are made before its capture begins (reserve_graph_events) and
    // handed out from graph_spare while it is captured.
    hipEvent_t next_event()
    {
        if (capturing) {
            if (graph_spare.empty()) {
                note(hipErrorInvalidValue, "graph timing events exhausted");
                return nullptr;
            }
            hipEvent_t e = graph_spare.back();
            graph_spare.pop_back();
            graph_events.push_back(e);
            return e;
        }
        if (ev_used == ev_pool.size()) {
            hipEvent_t e = nullptr;
            note(hipEventCreate(&e), "hipEventCreate");
            ev_pool.push_back(e);
        }
        return ev_pool[ev_used++];
    }
    // Under capture the record becomes an event-record node of the graph,
    // re-recorded on every replay: the node is added after the nodes the
    // stream's capture currently ends with and becomes the dependency of what
    // is captured next.  The dependency list the runtime returns is used only
    // by the very next call, before the capture's dependencies change.
    void record(hipEvent_t e)
    {
        if (!e)
            return;
        if (!capturing) {
            note(hipEventRecord(e, stream), "hipEventRecord");
            return;
        }
        hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
        hipGraph_t g = nullptr;
        const hipGraphNode_t *deps = nullptr;
        size_t nd = 0;
        hipError_t r = hipStreamGetCaptureInfo_v2(stream, &st, nullptr, &g, &deps, &nd);
        if (r != hipSuccess || st != hipStreamCaptureStatusActive || !g) {
            note(r != hipSuccess ? r : hipErrorIllegalState, "hipStreamGetCaptureInfo_v2");
            return;
        }
        hipGraphNode_t node = nullptr;
        r = hipGraphAddEventRecordNode(&node, g, deps, nd, e);
        if (r != hipSuccess) {
            note(r, "hipGraphAddEventRecordNode");
            return;
        }
        note(hipStreamUpdateCaptureDependencies(stream, &node, 1, hipStreamSetCaptureDependencies),
             "hipStreamUpdateCaptureDependencies");
    }
    // Timing events one captured outer iteration records: a pair around every
    // finest-level half-sweep, the limiter, the residual and the direction pass.
    void reserve_graph_events()
    {
        if (!opt.timing)
            return;
        const size_t need = 2 * (size_t)(2 * (opt.nu1 + opt.nu2) + 3);   // finest level only
        while (graph_spare.size() < need) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) {
                note(hipErrorOutOfMemory, "hipEventCreate");
                return;
            }
            graph_spare.push_back(e);
        }
    }
    // First failure of a call whose status is not returned at once.
    hipError_t pending = hipSuccess;
    const char *pending_what = "";
    void note(hipError_t e, const char *what)
    {
        if (e != hipSuccess && pending == hipSuccess) {
            pending = e;
            pending_what = what;
        }
    }
    hipEvent_t tic()
    {
        if (!opt.timing)
            return nullptr;
        hipEvent_t e = next_event();
        record(e);
        return e;
    }
    void toc(hipEvent_t a, int cls, double bytes_per_cell)
    {
        if (!opt.timing)
            return;
        hipEvent_t b = next_event();
        record(b);
        if (!a || !b)
            return;
        // a graph's launches see the problems active when it is replayed
        timed_sink->push_back(
            Timed{a, b, cls, bytes_per_cell, capturing ? -1.0 : active_fine_cells()});
    }
    // Add finished intervals to the accumulators (stream synchronised; for
    // a replayed graph, before the active set changes).
    void harvest(std::vector<Timed> &v, bool clear)
    {
        const double cells = active_fine_cells();
        for (const Timed &t : v) {
            float m = 0.0f;
            note(hipEventElapsedTime(&m, t.a, t.b), "hipEventElapsedTime");
            acc_ms[t.cls] += m;
            acc_launch[t.cls] += 1.0;
            acc_bytes[t.cls] += t.bytes_per_cell * (t.cells < 0.0 ? cells : t.cells);
        }
        if (clear) {
            v.clear();
            ev_used = 0;
        }
    }
    void collect_timing(double ms[4], double launches[4], double bytes[4])
    {
        harvest(timed, true);
        for (int q = 0; q < 4; ++q) {
            ms[q] = acc_ms[q];
            launches[q] = acc_launch[q];
            bytes[q] = acc_bytes[q];
            acc_ms[q] = acc_launch[q] = acc_bytes[q] = 0.0;
        }
    }

    // One graph per ping-pong parity for outer iterations k >= 1: the
    // preconditioner, the conjugate-gradient step and the next limiter and
    // residual passes.
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    std::vector<Timed> graph_timed[2];
    std::vector<hipEvent_t> graph_events, graph_spare;
    bool graphs_ok = true;

    void drop_graphs()
    {
        for (int q = 0; q < 2; ++q) {
            if (graph_exec[q])
                hipGraphExecDestroy(graph_exec[q]);
            graph_exec[q] = nullptr;
            graph_timed[q].clear();
        }
        for (hipEvent_t e : graph_events)
            hipEventDestroy(e);
        graph_events.clear();
        for (hipEvent_t e : graph_spare)
            hipEventDestroy(e);
        graph_spare.clear();
    }

    ~fld_engine_impl()
    {
        if (stream)
            hipStreamSynchronize(stream);
        if (side) {
            hipStreamSynchronize(side);
            hipStreamDestroy(side);
        }
        if (ev_fork)
            hipEventDestroy(ev_fork);
        if (ev_join)
            hipEventDestroy(ev_join);
        for (hipEvent_t e : ev_pool)
            hipEventDestroy(e);
        drop_graphs();
        for (void *p : allocs)
            hipFree(p);
        for (void *p : defl_allocs)
            hipFree(p);
        if (h_scal_pin)
            hipHostFree(h_scal_pin);
        if (h_active_pin)
            hipHostFree(h_active_pin);
        if (own_stream && stream)
            hipStreamDestroy(stream);
    }

    fld_status fail(fld_status s, const char *fmt, ...)
    {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return s;
    }

    fld_status hip_fail(hipError_t e, const char *what)
    {
        if (e == hipErrorOutOfMemory)
            return fail(FLD_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
        return fail(FLD_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
    }

    template <typename P>
    fld_status dalloc(P **p, size_t bytes)
    {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, bytes ? bytes : 8);
        if (e != hipSuccess)
            return hip_fail(e, "hipMalloc");
        allocs.push_back(q);
        *p = (P *)q;
        return FLD_OK;
    }

    fld_status upload_list(const std::vector<Task> &v, DevList &out)
    {
        out.n = (int)v.size();
        if (v.empty())
            return FLD_OK;
        fld_status s = dalloc(&out.d, sizeof(Task) * v.size());
        if (s)
            return s;
        hipError_t e = hipMemcpy(out.d, v.data(), sizeof(Task) * v.size(), hipMemcpyHostToDevice);
        return e == hipSuccess ? FLD_OK : hip_fail(e, "hipMemcpy tasks");
    }

    static void add_tasks(std::vector<Task> &v, int grid, long long n, int cells = kTaskCells)
    {
        for (long long s = 0; s < n; s += cells)
            v.push_back(Task{grid, (int)std::min<long long>(cells, n - s), s});
    }
    // Smoothing sweeps of level l (0 = finest) before (pre) or after the coarse
    // correction: nu_coarse on the levels from coarse_from on when it is set,
    // else nu1 / nu2.  The rule goes by level index, so every problem of a
    // batch sweeps its level l as often as it would alone.
    int sweeps(int l, bool pre) const
    {
        if (l >= 1 && opt.nu_coarse > 0 && l >= opt.coarse_from)
            return opt.nu_coarse;
        return pre ? opt.nu1 : opt.nu2;
    }
    // Largest power-of-two task size in [lo, kTaskCells] that still yields
    // opt.coarse_blocks tasks for n cells.
    int coarse_task(long long n, int lo) const
    {
        int c = kTaskCells;
        while (c > lo && n / c < opt.coarse_blocks)
            c >>= 1;
        return c;
    }

#define CK(x)                                    \
    do {                                         \
        fld_status s_ = (x);                     \
        if (s_ != FLD_OK)                        \
            return s_;                           \
    } while (0)
#define HK(x, what)                              \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess)                    \
            return hip_fail(e_, what);           \
    } while (0)

    // Build every buffer and work list.  dims: per volume (nx,ny,nz); nchan
    // problems per volume.
    fld_status build(const fld_options &o, int nvol, const int *dims, const double *h, int nchan)
    {
        opt = o;
        mixed = opt.precision == FLD_PRECISION_MIXED;
        mg = opt.method == FLD_METHOD_MG;
        tsz = mixed ? 4 : 8;
        HK(hipSetDevice(opt.device), "hipSetDevice");
        if (opt.stream) {
            stream = (hipStream_t)opt.stream;
        } else {
            HK(hipStreamCreate(&stream), "hipStreamCreate");
            own_stream = true;
        }
        vols.resize(nvol);
        for (int v = 0; v < nvol; ++v) {
            Vol &V = vols[v];
            V.nx = dims[3 * v];
            V.ny = dims[3 * v + 1];
            V.nz = dims[3 * v + 2];
            V.n = (long long)V.nx * V.ny * V.nz;
            V.h = h[v];
            const double L = V.h * std::max(V.nx, std::max(V.ny, V.nz));
            V.sigma_eps = opt.sigma_eps > 0.0 ? opt.sigma_eps : 1.0e-3 / L;
            CK(dalloc(&V.sig_hat, sizeof(double) * V.n));
        }
        nprob = nvol * nchan;
        probs.resize(nprob);
        std::vector<Fine> hf(nprob);
        std::vector<Task> ft;
        fine_range.assign(nprob + 1, 0);
        std::vector<Task> at;
        std::vector<int> aa_range(nprob + 1, 0);
        for (int p = 0; p < nprob; ++p) {
            Prob &P = probs[p];
            P.vol = p / nchan;
            P.chan = p % nchan;
            const Vol &V = vols[P.vol];
            Fine &f = P.fine;
            f.nx = V.nx; f.ny = V.ny; f.nz = V.nz; f.prob = p; f.n = V.n;
            f.h = V.h; f.h2 = V.h * V.h; f.eps = opt.eps; f.dghost = opt.eps * V.h;
            f.phi_b = opt.phi_b; f.larsen_n = opt.larsen_n;
            f.mirror = opt.boundary_d == FLD_BOUNDARY_D_MIRROR;
            f.limiter = opt.limiter;
            f.write_sighat = P.chan == 0;
            f.sig_hat = V.sig_hat;
            // colour-split fields of the V-cycle's finest level (e, b, D and
            // sigma_a in the V-cycle's precision): the split smoother needs
            // 8-cell z runs, and the finest level must be smoothed (not the
            // coarsest)
            const bool coarsens = V.nx % 2 == 0 && V.ny % 2 == 0 && V.nz % 2 == 0 &&
                                  V.nx / 2 >= 4 && V.ny / 2 >= 4 && V.nz / 2 >= 4;
            f.split = mg && opt.colour_split && V.nz % 8 == 0 && coarsens;
            const size_t N8 = sizeof(double) * V.n, NT = tsz * V.n;
            // split fields hold whole 64-cell blocks
            const size_t NS = f.split ? tsz * (size_t)((V.n + 63) / 64 * 64) : NT;
            CK(dalloc(&f.sa64, N8));
            CK(dalloc(&f.j, N8));
            CK(dalloc(&f.phi[0], N8));
            CK(dalloc(&f.phi[1], N8));
            CK(dalloc(&f.D64, N8));
            if (!mg)
                CK(dalloc(&f.Dtmp, N8));
            CK(dalloc(&f.b0[0], NS));
            CK(dalloc(&f.b0[1], NS));
            if (mg) {
                CK(dalloc(&f.e0, NS));
                CK(dalloc(&f.p[0], NT));
                CK(dalloc(&f.p[1], NT));
                if (mixed || f.split) {
                    // the smoother's D and sigma_a: FP32, or FP64 colour-split
                    CK(dalloc(&f.D0, NS));
                    CK(dalloc(&f.sa0, NS));
                } else {
                    f.D0 = f.D64;
                    f.sa0 = f.sa64;
                }
                if (opt.aa_m > 0) {
                    CK(dalloc(&f.aa_fprev, NT));
                    HK(hipMemset(f.aa_fprev, 0, NT), "hipMemset");
                    CK(dalloc(&f.aa_dF, NT * (opt.aa_m + 1)));
                    CK(dalloc(&f.aa_dG, NT * (opt.aa_m + 1)));
                }
            } else {
                f.p[0] = f.p[1] = f.b0[1];
                f.e0 = f.b0[1];
            }
            fine_range[p] = (int)ft.size();
            fine_cells += (double)V.n;
            add_tasks(ft, p, V.n);
            fine_range[p + 1] = (int)ft.size();
            aa_range[p] = (int)at.size();
            if (mg && opt.aa_m > 0)
                add_tasks(at, p, V.n, kAaTaskCells);
            aa_range[p + 1] = (int)at.size();
            hf[p] = f;
        }
        {
            int ns = 0;
            for (const Prob &P : probs)
                ns += P.fine.split ? 1 : 0;
            lsp = ns == 0 ? 0 : ns == nprob ? 1 : 2;
            kmode = !mixed ? (lsp == 0 ? 0 : lsp + 3) : lsp + 1;
        }
        CK(upload_list(ft, fine_tasks));
        fuse = mg && opt.fuse_lr != 0;
        for (int p = 0; p < nprob; ++p)
            fuse = fuse && hf[p].nz % 4 == 0;
        if (fuse) {
            std::vector<LrTile> lt;
            std::vector<int> lr_range(nprob + 1, 0);
            for (int p = 0; p < nprob; ++p) {
                const Fine &f = hf[p];
                lr_range[p] = (int)lt.size();
                for (int i0 = 0; i0 < f.nx; i0 += kLrTilePlanes)
                    for (int j0 = 0; j0 < f.ny; j0 += kLrTileRows)
                        for (int k0 = 0; k0 < f.nz; k0 += kLrTileCells)
                            lt.push_back(LrTile{p, i0, std::min(kLrTilePlanes, f.nx - i0), j0, k0});
                lr_range[p + 1] = (int)lt.size();
            }
            n_lrtiles = (int)lt.size();
            CK(dalloc(&d_lrtiles, sizeof(LrTile) * lt.size()));
            HK(hipMemcpy(d_lrtiles, lt.data(), sizeof(LrTile) * lt.size(), hipMemcpyHostToDevice),
               "hipMemcpy");
            CK(dalloc(&d_lr_range, sizeof(int) * (nprob + 1)));
            HK(hipMemcpy(d_lr_range, lr_range.data(), sizeof(int) * (nprob + 1),
                         hipMemcpyHostToDevice), "hipMemcpy");
            CK(dalloc(&d_lrpart, sizeof(double) * lt.size()));
        }
        CK(dalloc(&d_fine_range, sizeof(int) * (nprob + 1)));
        HK(hipMemcpy(d_fine_range, fine_range.data(), sizeof(int) * (nprob + 1),
                     hipMemcpyHostToDevice), "hipMemcpy");
        CK(dalloc(&d_fines, sizeof(Fine) * nprob));
        HK(hipMemcpy(d_fines, hf.data(), sizeof(Fine) * nprob, hipMemcpyHostToDevice), "hipMemcpy");
        size_t maxt = std::max<size_t>(ft.size(), 1);
        for (int q = 0; q < 4; ++q)
            CK(dalloc(&d_part[q], sizeof(double) * maxt));
        CK(dalloc(&d_scal, sizeof(double) * S_COUNT * nprob));
        HK(hipMemset(d_scal, 0, sizeof(double) * S_COUNT * nprob), "hipMemset");
        CK(dalloc(&d_active, sizeof(int) * nprob));
        CK(dalloc(&d_fail, sizeof(int) * nprob));
        HK(hipHostMalloc((void **)&h_scal_pin, sizeof(double) * S_COUNT * nprob, 0),
           "hipHostMalloc");
        HK(hipHostMalloc((void **)&h_active_pin, sizeof(int) * nprob, 0), "hipHostMalloc");
        if (mg && opt.aa_m > 0) {
            CK(dalloc(&d_aai, sizeof(int) * aa_state_ints() * nprob));
            CK(dalloc(&d_aad, sizeof(double) * aa_state_doubles() * nprob));
            HK(hipMemset(d_aad, 0, sizeof(double) * aa_state_doubles() * nprob), "hipMemset");
            CK(upload_list(at, aa_tasks));
            CK(dalloc(&d_aa_range, sizeof(int) * (nprob + 1)));
            HK(hipMemcpy(d_aa_range, aa_range.data(), sizeof(int) * (nprob + 1),
                         hipMemcpyHostToDevice), "hipMemcpy");
            CK(dalloc(&d_aapart, sizeof(double) * 2 * (opt.aa_m + 1) *
                                     std::max<size_t>(at.size(), 1)));
        }
        h_active.assign(nprob, 1);
        if (mg)
            CK(build_hierarchy());
        return FLD_OK;
    }

    fld_status build_hierarchy()
    {
        std::vector<Grid> grids[2];
        fuse_rb = opt.fuse_rb != 0;
        for (int p = 0; p < nprob; ++p)
            fuse_rb = fuse_rb && probs[p].fine.nz % 4 == 0;
        for (int p = 0; p < nprob; ++p) {
            Prob &P = probs[p];
            // levels: 2:1 on all axes while every axis is even and half of it >= 4
            int a = P.fine.nx, b = P.fine.ny, c = P.fine.nz;
            P.nlev = 0;
            for (;;) {
                Level &L = P.lv[P.nlev];
                L.nx = a; L.ny = b; L.nz = c;
                L.n = (long long)a * b * c;
                L.h = P.fine.h * (double)(1LL << P.nlev);
                ++P.nlev;
                if ((a % 2) || (b % 2) || (c % 2) || a / 2 < 4 || b / 2 < 4 || c / 2 < 4 ||
                    P.nlev == kMaxLevels)
                    break;
                a /= 2; b /= 2; c /= 2;
            }
            max_levels = std::max(max_levels, P.nlev);
            for (int l = 0; l < P.nlev; ++l) {
                Level &L = P.lv[l];
                if (l == 0) {
                    L.e = P.fine.e0;
                    L.b = P.fine.b0[0];
                    L.sa = P.fine.sa0;
                    if (fuse_rb)
                        CK(dalloc(&L.e2, tsz * L.n));
                } else {
                    CK(dalloc(&L.e, tsz * L.n));
                    CK(dalloc(&L.b, tsz * L.n));
                    CK(dalloc(&L.sa, tsz * L.n));
                    CK(dalloc(&L.f, tsz * 3 * (size_t)(L.nx + 1) * (L.ny + 1) *
                                        (size_t)face_zstride(L.nz)));
                }
                if (l == P.nlev - 1) {
                    const long long W = (long long)L.ny * L.nz + 1;
                    CK(dalloc(&L.band, sizeof(double) * L.n * W));
                    max_coarse_n = std::max<int>(max_coarse_n, (int)L.n);
                    max_coarse_bw = std::max<int>(max_coarse_bw, L.ny * L.nz);
                }
            }
            P.gid0 = (int)grids[0].size();
            for (int l = 0; l < P.nlev; ++l) {
                const Level &L = P.lv[l];
                Grid g{};
                g.nx = L.nx; g.ny = L.ny; g.nz = L.nz; g.prob = p; g.n = L.n;
                g.h2 = L.h * L.h;
                g.dghost = P.fine.dghost;
                g.fine = l == 0;
                g.split = l == 0 && P.fine.split;
                g.mirror = P.fine.mirror;
                g.finer = l > 0 ? P.gid0 + l - 1 : -1;
                g.coarser = l + 1 < P.nlev ? P.gid0 + l + 1 : -1;
                g.e = L.e; g.b = L.b; g.sa = L.sa; g.D = l == 0 ? P.fine.D0 : nullptr; g.f = L.f;
                g.e2 = L.e2;
                g.band = L.band;
                g.nu_pre = (short)sweeps(l, true);
                g.nu_post = (short)sweeps(l, false);
                grids[0].push_back(g);
                if (l == 0)
                    g.b = P.fine.b0[1];
                grids[1].push_back(g);
            }
        }
        h_grids = grids[0];
        ngrids = (int)grids[0].size();
        if (fuse_rb) {
            std::vector<LrTile> rt;
            for (const Prob &P : probs) {
                const Fine &f = P.fine;
                for (int i0 = 0; i0 < f.nx; i0 += kLrTilePlanes)
                    for (int j0 = 0; j0 < f.ny; j0 += kLrTileRows)
                        for (int k0 = 0; k0 < f.nz; k0 += kLrTileCells)
                            rt.push_back(LrTile{P.gid0, i0, std::min(kLrTilePlanes, f.nx - i0), j0,
                                                k0});
            }
            n_rbtiles = (int)rt.size();
            CK(dalloc(&d_rbtiles, sizeof(LrTile) * rt.size()));
            HK(hipMemcpy(d_rbtiles, rt.data(), sizeof(LrTile) * rt.size(), hipMemcpyHostToDevice),
               "hipMemcpy");
        }
        for (int q = 0; q < 2; ++q) {
            CK(dalloc(&d_grids[q], sizeof(Grid) * ngrids));
            HK(hipMemcpy(d_grids[q], grids[q].data(), sizeof(Grid) * ngrids, hipMemcpyHostToDevice),
               "hipMemcpy grids");
        }
        defl_enabled = opt.deflate_tau > 0.0;
        // deep part: from the first level (below the finest) with at most
        // opt.deep_cells cells; levels above it use the work-list kernels
        // The tail (deep levels and coarsest solve) of a problem runs in one
        // workgroup launch when its levels and LDS footprint fit that kernel,
        // else as the per-phase deep kernels around the coarsest solve.
        std::vector<int> roots, coarsest, tails;
        for (Prob &P : probs) {
            P.deep = P.nlev - 1;
            if (opt.deep_cells > 0)
                for (int l = 1; l < P.nlev; ++l)
                    if (P.lv[l].n <= opt.deep_cells) {
                        P.deep = l;
                        break;
                    }
            const int nd = P.nlev - 1 - P.deep;
            const Level &Lc = P.lv[P.nlev - 1];
            bool fused = nd <= 1 + tail_max_low() &&
                         (nd == 0 || P.lv[P.deep].n <= tail_root_cells());
            long long deep_cells = 0;
            for (int l = P.deep; l < P.nlev - 1; ++l) {
                deep_cells += P.lv[l].n;
                if (l > P.deep && P.lv[l].n > tail_low_cells())
                    fused = false;
            }
            const long long scratch = std::max<long long>(nd ? P.lv[P.deep].n : 0, Lc.n);
            const long long need = tail_lds_need(Lc.n, (long long)Lc.ny * Lc.nz, deep_cells,
                                                 scratch, (int)tsz);
            if (fused && need <= tail_lds_limit()) {
                tails.push_back(P.gid0 + P.deep);
                tail_lds = std::max<long long>(tail_lds, need);
                continue;
            }
            if (P.deep < P.nlev - 1)
                roots.push_back(P.gid0 + P.deep);
            coarsest.push_back(P.gid0 + P.nlev - 1);
        }
        n_tail = (int)tails.size();
        if (n_tail) {
            CK(dalloc(&d_tail_roots, sizeof(int) * n_tail));
            HK(hipMemcpy(d_tail_roots, tails.data(), sizeof(int) * n_tail, hipMemcpyHostToDevice),
               "hipMemcpy");
        }
        n_deep = (int)roots.size();
        if (n_deep) {
            CK(dalloc(&d_deep_roots, sizeof(int) * n_deep));
            HK(hipMemcpy(d_deep_roots, roots.data(), sizeof(int) * n_deep, hipMemcpyHostToDevice),
               "hipMemcpy");
        }
        n_coarse = (int)coarsest.size();
        if (n_coarse) {
            CK(dalloc(&d_coarse_ids, sizeof(int) * n_coarse));
            HK(hipMemcpy(d_coarse_ids, coarsest.data(), sizeof(int) * n_coarse,
                         hipMemcpyHostToDevice), "hipMemcpy");
        }
        {
            std::vector<int> fids;
            for (const Prob &P : probs)
                fids.push_back(P.gid0 + P.nlev - 1);
            n_factor = (int)fids.size();
            CK(dalloc(&d_factor_ids, sizeof(int) * n_factor));
            HK(hipMemcpy(d_factor_ids, fids.data(), sizeof(int) * n_factor,
                         hipMemcpyHostToDevice), "hipMemcpy");
            HK(hipStreamCreateWithFlags(&side, hipStreamNonBlocking), "hipStreamCreateWithFlags");
            HK(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming), "hipEventCreateWithFlags");
            HK(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming), "hipEventCreateWithFlags");
        }
        for (int l = 0; l < max_levels; ++l) {
            std::vector<Task> m, r, g, cc;
            // launch shape: task sizes from the cells all problems hold at this level
            long long nm = 0, nr = 0, ng = 0;
            for (const Prob &P : probs)
                if (l < P.nlev - 1) {
                    const Level &C = P.lv[l + 1];
                    if (l < P.deep) {
                        nm += P.lv[l].n;
                        nr += C.n;
                    }
                    ng += (long long)(C.nx + 1) * (C.ny + 1) * face_zstride(C.nz);
                }
            const int tm = l == 0 ? opt.task_cells0 : coarse_task(nm, 512);
            mid_cells[l] = tm;
            const int tr = coarse_task(nr, 256), tg = coarse_task(ng, 256);
            for (int p = 0; p < nprob; ++p) {
                const Prob &P = probs[p];
                if (l < P.nlev - 1) {
                    if (l < P.deep) {
                        add_tasks(m, P.gid0 + l, P.lv[l].n, tm);
                        add_tasks(r, P.gid0 + l + 1, P.lv[l + 1].n, tr);
                    }
                    const Level &C = P.lv[l + 1];
                    add_tasks(g, P.gid0 + l + 1,
                              (long long)(C.nx + 1) * (C.ny + 1) * face_zstride(C.nz), tg);
                    add_tasks(cc, P.gid0 + l + 1, C.n, 256);
                }
            }
            CK(upload_list(cc, coarse_cells[l]));
            CK(upload_list(m, mid[l]));
            CK(upload_list(r, rest[l]));
            CK(upload_list(g, gal[l]));
        }
        return FLD_OK;
    }

    // ---- medium ---------------------------------------------------------

    fld_status set_problem_medium(int p, const double *d_st, const double *d_al, const double *d_q)
    {
        Prob &P = probs[p];
        const Vol &V = vols[P.vol];
        DevList l;
        // the fine list already holds exactly these tasks
        l.d = fine_tasks.d + fine_range[p];
        l.n = fine_range[p + 1] - fine_range[p];
        launch_setup(stream, P.fine, l.d, l.n, d_st, d_al, d_q, V.sigma_eps, opt.anisotropy_g,
                     d_part[0] + fine_range[p], mixed);
        launch_sum_partials(stream, 1, d_fine_range + p, d_part[0], d_scal + (size_t)p * S_COUNT,
                            S_JN2, nullptr);
        launch_after_setup(stream, 1, d_fines + p, d_scal + (size_t)p * S_COUNT);
        HK(hipGetLastError(), "setup launch");
        return FLD_OK;
    }

    // Clusters of voxels joined by strong faces (classical coefficient
    // ((1/3)/sig_p + (1/3)/sig_s)/2 > tau*L), labelled by union-find and
    // numbered by their first voxel in index order; only clusters of two or
    // more voxels are kept.
    static int label_clusters(const Vol &V, const std::vector<double> &sh, double tau,
                              std::vector<int> &label)
    {
        const long long n = V.n;
        const double thresh = tau * V.h * std::max(V.nx, std::max(V.ny, V.nz));
        std::vector<int> parent(n), size(n, 0), id(n, -1);
        for (long long c = 0; c < n; ++c)
            parent[c] = (int)c;
        auto find = [&](int x) {
            while (parent[x] != x) {
                parent[x] = parent[parent[x]];
                x = parent[x];
            }
            return x;
        };
        auto unite = [&](int a, int b) {
            a = find(a);
            b = find(b);
            if (a != b)
                parent[std::max(a, b)] = std::min(a, b);
        };
        const long long sx = (long long)V.ny * V.nz, sy = V.nz;
        for (int i = 0; i < V.nx; ++i)
            for (int j = 0; j < V.ny; ++j)
                for (int k = 0; k < V.nz; ++k) {
                    const long long c = i * sx + j * sy + k;
                    const double dc = (1.0 / 3.0) / sh[c];
                    if (i + 1 < V.nx && 0.5 * (dc + (1.0 / 3.0) / sh[c + sx]) > thresh)
                        unite((int)c, (int)(c + sx));
                    if (j + 1 < V.ny && 0.5 * (dc + (1.0 / 3.0) / sh[c + sy]) > thresh)
                        unite((int)c, (int)(c + sy));
                    if (k + 1 < V.nz && 0.5 * (dc + (1.0 / 3.0) / sh[c + 1]) > thresh)
                        unite((int)c, (int)(c + 1));
                }
        for (long long c = 0; c < n; ++c)
            size[find((int)c)] += 1;
        int K = 0;
        label.assign(n, -1);
        for (long long c = 0; c < n; ++c) {
            const int r = find((int)c);
            if (size[r] < 2)
                continue;
            if (id[r] < 0)
                id[r] = K++;
            label[c] = id[r];
        }
        return K;
    }

    fld_status build_clusters()
    {
        for (void *q : defl_allocs)
            hipFree(q);
        defl_allocs.clear();
        use_defl = false;
        ncl_total = 0;
        n_ctasks = n_rtasks = 0;
        if (!mg || !defl_enabled)
            return FLD_OK;
        auto dal = [&](void **q, size_t bytes) -> fld_status {
            hipError_t er = hipMalloc(q, bytes ? bytes : 8);
            if (er != hipSuccess)
                return hip_fail(er, "hipMalloc clusters");
            defl_allocs.push_back(*q);
            return FLD_OK;
        };
        std::vector<int> vK(vols.size());
        std::vector<int *> vlabel(vols.size()), vpos(vols.size()), vrim(vols.size());
        std::vector<unsigned short *> vmask(vols.size());
        std::vector<std::vector<int>> vstart(vols.size()), vrstart(vols.size());
        for (size_t v = 0; v < vols.size(); ++v) {
            const Vol &V = vols[v];
            std::vector<double> sh(V.n);
            HK(hipMemcpy(sh.data(), V.sig_hat, 8 * V.n, hipMemcpyDeviceToHost), "sig_hat D2H");
            std::vector<int> label;
            const int K = label_clusters(V, sh, opt.deflate_tau, label);
            vK[v] = K;
            // every channel of a volume has the same storage layout
            bool split = false;
            for (const Prob &P : probs)
                if (P.vol == (int)v)
                    split = P.fine.split != 0;
            // voxels of every cluster, cluster by cluster, index order inside
            std::vector<int> start(K + 1, 0), cells;
            for (long long c = 0; c < V.n; ++c)
                if (label[c] >= 0)
                    ++start[label[c] + 1];
            for (int q = 0; q < K; ++q)
                start[q + 1] += start[q];
            cells.resize(start[K]);
            std::vector<int> fill(start.begin(), start.end() - 1);
            for (long long c = 0; c < V.n; ++c)
                if (label[c] >= 0)
                    cells[fill[label[c]]++] = (int)c;
            // their storage positions in the precision-T fields, and the rim
            // voxels with the faces leaving the cluster (x-, x+, y-, y+, z-, z+)
            std::vector<int> pos(cells.size()), rim, rstart(K + 1, 0);
            std::vector<unsigned short> mask;
            const long long sx = (long long)V.ny * V.nz, sy = V.nz;
            for (int q = 0; q < K; ++q) {
                for (int e = start[q]; e < start[q + 1]; ++e) {
                    const long long c = cells[e];
                    const int k = (int)(c % V.nz), j = (int)((c / V.nz) % V.ny), i = (int)(c / sx);
                    pos[e] = split ? (int)(((c >> 6) << 6) + (((i + j + k) & 1) << 5) + ((c >> 1) & 31))
                                   : (int)c;
                    const bool in[6] = {i > 0, i < V.nx - 1, j > 0, j < V.ny - 1, k > 0,
                                        k < V.nz - 1};
                    const long long off[6] = {-sx, sx, -sy, sy, -1, 1};
                    unsigned short mk = 0;
                    for (int d = 0; d < 6; ++d) {
                        if (!in[d])
                            mk |= (unsigned short)((1u << d) | (1u << (d + 6)));
                        else if (label[c + off[d]] != label[c])
                            mk |= (unsigned short)(1u << d);
                    }
                    if (mk) {
                        rim.push_back((int)c);
                        mask.push_back(mk);
                    }
                }
                rstart[q + 1] = (int)rim.size();
            }
            CK(dal((void **)&vlabel[v], sizeof(int) * V.n));
            CK(dal((void **)&vpos[v], sizeof(int) * pos.size()));
            CK(dal((void **)&vrim[v], sizeof(int) * rim.size()));
            CK(dal((void **)&vmask[v], sizeof(unsigned short) * mask.size()));
            HK(hipMemcpy(vlabel[v], label.data(), sizeof(int) * V.n, hipMemcpyHostToDevice), "labels");
            if (!pos.empty())
                HK(hipMemcpy(vpos[v], pos.data(), sizeof(int) * pos.size(), hipMemcpyHostToDevice),
                   "cluster positions");
            if (!rim.empty()) {
                HK(hipMemcpy(vrim[v], rim.data(), sizeof(int) * rim.size(), hipMemcpyHostToDevice),
                   "rim cells");
                HK(hipMemcpy(vmask[v], mask.data(), sizeof(unsigned short) * mask.size(),
                             hipMemcpyHostToDevice), "rim masks");
            }
            vstart[v] = start;
            vrstart[v] = rstart;
        }
        std::vector<CTask> ct, rt;
        std::vector<int> crange(1, 0), rrange(1, 0), cprob;
        std::vector<Fine> hf(nprob);
        for (int p = 0; p < nprob; ++p) {
            Fine &f = probs[p].fine;
            const int v = probs[p].vol;
            f.label = vlabel[v];
            f.cpos = vpos[v];
            f.rcells = vrim[v];
            f.rmask = vmask[v];
            f.cbase = ncl_total;
            f.ncl = vK[v];
            for (int q = 0; q < vK[v]; ++q) {
                for (int s0 = vstart[v][q]; s0 < vstart[v][q + 1]; s0 += kTaskCells)
                    ct.push_back(CTask{p, ncl_total + q, s0,
                                       std::min(kTaskCells, vstart[v][q + 1] - s0)});
                // rim voxels gather neighbour coefficients: short tasks keep
                // enough of them in flight
                for (int s0 = vrstart[v][q]; s0 < vrstart[v][q + 1]; s0 += kRimTaskCells)
                    rt.push_back(CTask{p, ncl_total + q, s0,
                                       std::min(kRimTaskCells, vrstart[v][q + 1] - s0)});
                crange.push_back((int)ct.size());
                rrange.push_back((int)rt.size());
                cprob.push_back(p);
            }
            ncl_total += vK[v];
            hf[p] = f;
        }
        HK(hipMemcpy(d_fines, hf.data(), sizeof(Fine) * nprob, hipMemcpyHostToDevice), "fines");
        if (ncl_total == 0)
            return FLD_OK;
        n_ctasks = (int)ct.size();
        n_rtasks = (int)rt.size();
        CK(dal((void **)&d_ctasks, sizeof(CTask) * ct.size()));
        CK(dal((void **)&d_rtasks, sizeof(CTask) * std::max<size_t>(rt.size(), 1)));
        CK(dal((void **)&d_crange, sizeof(int) * crange.size()));
        CK(dal((void **)&d_rrange, sizeof(int) * rrange.size()));
        CK(dal((void **)&d_cprob, sizeof(int) * cprob.size()));
        CK(dal((void **)&d_alpha, sizeof(double) * ncl_total));
        CK(dal((void **)&d_csa, sizeof(double) * ncl_total));
        CK(dal((void **)&d_cpd, sizeof(double) * std::max<size_t>(rt.size(), 1)));
        CK(dal((void **)&d_cps, sizeof(double) * ct.size()));
        HK(hipMemcpy(d_ctasks, ct.data(), sizeof(CTask) * ct.size(), hipMemcpyHostToDevice), "ctasks");
        if (!rt.empty())
            HK(hipMemcpy(d_rtasks, rt.data(), sizeof(CTask) * rt.size(), hipMemcpyHostToDevice),
               "rtasks");
        HK(hipMemcpy(d_crange, crange.data(), sizeof(int) * crange.size(), hipMemcpyHostToDevice), "crange");
        HK(hipMemcpy(d_rrange, rrange.data(), sizeof(int) * rrange.size(), hipMemcpyHostToDevice), "rrange");
        HK(hipMemcpy(d_cprob, cprob.data(), sizeof(int) * cprob.size(), hipMemcpyHostToDevice), "cprob");
        // the clusters' absorption sums, fixed for this medium
        launch_defl_sum_sa(stream, d_fines, d_ctasks, n_ctasks, d_cps, mixed);
        launch_defl_finish(stream, ncl_total, d_crange, d_rrange, d_cprob, d_cps, d_cpd, d_csa,
                           d_alpha, nullptr, 1);
        HK(hipGetLastError(), "cluster absorption");
        use_defl = true;
        return FLD_OK;
    }

    fld_status finish_medium()
    {
        HK(hipStreamSynchronize(stream), "medium sync");
        drop_graphs();
        CK(build_clusters());
        if (mg) {
            for (int l = 0; l + 1 < max_levels; ++l) {
                if (!coarse_cells[l].n)
                    continue;
                if (mixed)
                    launch_mean8_sa<float>(stream, d_grids[0], coarse_cells[l].d, coarse_cells[l].n);
                else
                    launch_mean8_sa<double>(stream, d_grids[0], coarse_cells[l].d,
                                            coarse_cells[l].n);
            }
        }
        HK(hipGetLastError(), "medium launch");
        HK(hipStreamSynchronize(stream), "medium sync");
        k_state = 0;
        solved_once = false;
        return FLD_OK;
    }

    // Validate on the device-resident copies; returns the first bad index or -1.
    static long long first_bad(const double *st, const double *al, const double *q, long long n,
                               int *which)
    {
        for (long long c = 0; c < n; ++c) {
            if (!(std::isfinite(st[c]) && st[c] >= 0.0)) { *which = 0; return c; }
            if (!(std::isfinite(al[c]) && al[c] >= 0.0 && al[c] <= 1.0)) { *which = 1; return c; }
            if (!(std::isfinite(q[c]) && q[c] >= 0.0)) { *which = 2; return c; }
        }
        return -1;
    }

    fld_status check_host_medium(const double *st, const double *al, const double *q, long long n)
    {
        int which = 0;
        const long long bad = first_bad(st, al, q, n, &which);
        if (bad >= 0) {
            static const char *names[3] = {"sigma_t", "albedo", "Q"};
            const double *arr[3] = {st, al, q};
            return fail(FLD_ERR_INVALID_ARGUMENT, "%s[%lld] = %g is out of range", names[which],
                        bad, arr[which][bad]);
        }
        return FLD_OK;
    }

    // ---- multigrid cycle --------------------------------------------------

    template <typename T>
    void coarsen()
    {
        Grid *G = d_grids[0];
        for (int l = 0; l + 1 < max_levels; ++l)
            if (gal[l].n)
                launch_galerkin<T>(stream, G, gal[l].d, gal[l].n, d_active, lsp);
        // fork: the coarsest factorisations on the second stream
        note(hipEventRecord(ev_fork, stream), "hipEventRecord");
        note(hipStreamWaitEvent(side, ev_fork, 0), "hipStreamWaitEvent");
        launch_coarse_factor<T>(side, G, d_factor_ids, n_factor, d_active, d_fail, max_coarse_n);
        note(hipEventRecord(ev_join, side), "hipEventRecord");
    }

    // One finest-level half-sweep must move, per cell of the grid, the other
    // colour's e (half), all of D, this colour's b and sa (half each) and its
    // new e (half): 3 values of precision T; with over-relaxation (omega_s !=
    // 1) also this colour's old e (half).
    template <typename T>
    void smooth(Grid *G, int l, int colour)
    {
        if (l > 0 && nprob == 1) {
            // one problem: the coarse level by value, no task or activity loads
            // (a solve stops launching once its only problem has converged)
            launch_smooth_one<T>(stream, h_grids[probs[0].gid0 + l], mid_cells[l], colour,
                                 opt.omega_s);
            return;
        }
        hipEvent_t a = l == 0 ? tic() : nullptr;
        launch_smooth<T>(stream, G, mid[l].d, mid[l].n, d_active, colour, opt.omega_s, l == 0);
        if (l == 0)
            toc(a, 0, (opt.omega_s != 1.0 ? 3.5 : 3.0) * sizeof(T));
    }

    // One finest-level sweep in one pass (first colour, then the other), out
    // of place (dir 0: e -> e2, 1: back): e, D, b and sa read, e written.
    template <typename T>
    void smooth_rb(Grid *G, int first, int dir)
    {
        hipEvent_t a = tic();
        launch_smooth_rb<T>(stream, G, d_rbtiles, n_rbtiles, d_active, first, dir, opt.omega_s, lsp);
        toc(a, 0, 5.0 * sizeof(T));
    }

    double active_fine_cells() const
    {
        double c = 0.0;
        for (int p = 0; p < nprob; ++p)
            if (h_active[p])
                c += (double)probs[p].fine.n;
        return c;
    }

    // par: parity of the level-0 right-hand side buffer.  With deflation the
    // finest level starts from the cluster step e0 = alpha[label], every
    // other level from zero.
    template <typename T>
    void vcycle(int par)
    {
        Grid *G = d_grids[par];
        for (int l = 0; l < max_levels; ++l) {
            if (mid[l].n) {
                if (l == 0 && use_defl)
                    launch_defl_init(stream, d_fines, fine_tasks.d, fine_tasks.n, d_active,
                                     d_alpha, kmode);
                else
                    launch_zero<T>(stream, G, mid[l].d, mid[l].n, d_active);
                int s = 0;
                if (l == 0 && fuse_rb)
                    for (; s + 1 < opt.nu1; s += 2) {
                        smooth_rb<T>(G, 0, 0);
                        smooth_rb<T>(G, 0, 1);
                    }
                for (; s < sweeps(l, true); ++s) {
                    smooth<T>(G, l, 0);
                    smooth<T>(G, l, 1);
                }
                launch_restrict<T>(stream, G, rest[l].d, rest[l].n, d_active, lsp);
            }
        }
        // join: the coarsest factors are complete
        note(hipStreamWaitEvent(stream, ev_join, 0), "hipStreamWaitEvent");
        launch_tail<T>(stream, G, d_tail_roots, n_tail, d_active, d_fail, opt.omega_s,
                       (int)tail_lds);
        launch_deep<T>(stream, G, d_deep_roots, n_deep, d_active, opt.omega_s, true);
        launch_coarse_solve<T>(stream, G, d_coarse_ids, n_coarse, d_active, d_fail, max_coarse_n,
                               max_coarse_bw);
        launch_deep<T>(stream, G, d_deep_roots, n_deep, d_active, opt.omega_s, false);
        for (int l = max_levels - 2; l >= 0; --l) {
            if (!mid[l].n)
                continue;
            launch_prolong<T>(stream, G, mid[l].d, mid[l].n, d_active, lsp,
                              l == 0 ? opt.corr_scale : 1.0);
            int s = 0;
            if (l == 0 && fuse_rb)
                for (; s + 1 < opt.nu2; s += 2) {
                    smooth_rb<T>(G, 1, 0);
                    smooth_rb<T>(G, 1, 1);
                }
            for (; s < sweeps(l, false); ++s) {
                smooth<T>(G, l, 1);
                smooth<T>(G, l, 0);
            }
        }
    }

    double vcycle_updates() const
    {
        double u = 0.0;
        for (const Prob &P : probs)
            for (int l = 0; l + 1 < P.nlev; ++l)
                u += (double)P.lv[l].n * (sweeps(l, true) + sweeps(l, false));
        return u;
    }

    // ---- solves -----------------------------------------------------------

    // The active mask goes to the device only when it changed (or when forced
    // at the start of a solve); both directions of the per-iteration scalar
    // traffic use pinned host buffers.
    fld_status sync_active(bool force = false)
    {
        if (!force && h_active == uploaded_active)
            return FLD_OK;
        std::copy(h_active.begin(), h_active.end(), h_active_pin);
        HK(hipMemcpyAsync(d_active, h_active_pin, sizeof(int) * nprob, hipMemcpyHostToDevice,
                          stream), "active upload");
        uploaded_active = h_active;
        return FLD_OK;
    }

    fld_status read_scalars(std::vector<double> &s)
    {
        HK(hipMemcpyAsync(h_scal_pin, d_scal, sizeof(double) * S_COUNT * nprob,
                          hipMemcpyDeviceToHost, stream), "scalars D2H");
        HK(hipStreamSynchronize(stream), "sync");
        s.assign(h_scal_pin, h_scal_pin + (size_t)S_COUNT * nprob);
        return FLD_OK;
    }

    // Limiter and residual passes of outer iteration k (D^k, r^k, rel_k); for
    // k past the first iteration of a call, phi^k = phi^{k-1} + theta p^{k-1}
    // is formed on the fly.
    void head(int k, bool first)
    {
        const int N = nprob;
        hipEvent_t ta = tic();
        // with Anderson acceleration the update pass has written phi^k already
        if (opt.aa_m > 0)
            first = true;
        if (first && fuse) {
            // D (FP64 as well when a conjugate-direction pass will read it) and
            // r in one pass; phi, sig_hat, sa, j read
            const bool d64 = !mixed || opt.aa_m == 0;
            launch_lim_res(stream, d_fines, d_lrtiles, n_lrtiles, d_active, d_scal, k & 1, k & 1,
                           d64 ? 1 : 0, d_lrpart, kmode);
            toc(ta, 1, 32.0 + tsz + (mixed ? 4.0 : lsp != 0 ? 8.0 : 0.0) + (d64 ? 8.0 : 0.0));
            launch_sum_partials(stream, N, d_lr_range, d_lrpart, d_scal, S_RES2, d_active);
            launch_rel(stream, N, d_scal, d_active);
            return;
        }
        if (first)
            launch_limiter(stream, d_fines, fine_tasks.d, fine_tasks.n, d_active, d_scal, k & 1,
                           k & 1, 0, 0, 0, kmode, opt.limiter);
        else
            launch_limiter(stream, d_fines, fine_tasks.d, fine_tasks.n, d_active, d_scal,
                           (k - 1) & 1, k & 1, 1, (k - 1) & 1, 0, kmode, opt.limiter);
        // limiter: phi and sig_hat read, D written (FP64, plus the smoother's
        // copy: FP32 in the mixed form, colour-split FP64 in the FP64 form);
        // with the direction update also p read, phi written
        toc(ta, 2, 24.0 + (mixed ? 4.0 : lsp != 0 ? 8.0 : 0.0) + (first ? 0.0 : tsz + 8.0));
        ta = tic();
        launch_residual(stream, d_fines, fine_tasks.d, fine_tasks.n, d_active, k & 1, 0, k & 1,
                        nullptr, d_part[0], kmode);
        // residual: phi, D, sa, j read (FP64), r written in precision T
        toc(ta, 1, 32.0 + tsz);
        launch_sum_partials(stream, N, d_fine_range, d_part[0], d_scal, S_RES2, d_active);
        launch_rel(stream, N, d_scal, d_active);
    }

    // Preconditioner and conjugate-gradient step of outer iteration k.
    void body(int k)
    {
        const int N = nprob;
        if (use_defl) {
            launch_defl_sum_b(stream, d_fines, d_ctasks, n_ctasks, d_active, k & 1, d_cps, mixed);
            launch_defl_rim(stream, d_fines, d_rtasks, n_rtasks, d_active, d_cpd, kmode);
            launch_defl_finish(stream, ncl_total, d_crange, d_rrange, d_cprob, d_cps, d_cpd, d_csa,
                               d_alpha, d_active, 0);
        }
        if (mixed) {
            coarsen<float>();
            vcycle<float>(k & 1);
        } else {
            coarsen<double>();
            vcycle<double>(k & 1);
        }
        if (opt.aa_m > 0) {
            const int m = opt.aa_m;
            launch_aa_dots(stream, d_fines, aa_tasks.d, aa_tasks.n, d_active, d_aai, d_aad, m,
                           d_aapart, kmode);
            launch_aa_sums(stream, N, d_aa_range, d_aapart, aa_tasks.n, d_aai, d_aad, m,
                           d_active);
            launch_aa_solve(stream, N, d_scal, d_aai, d_aad, m, opt.aa_reg, opt.restart_growth,
                            d_active);
            hipEvent_t tu = tic();
            launch_aa_update(stream, d_fines, fine_tasks.d, fine_tasks.n, d_active, d_aai, d_aad,
                             k & 1, (k + 1) & 1, kmode);
            // update: phi, e0 and the window's dG read, phi and one dG written
            toc(tu, 3, 16.0 + (2.0 + 1.0 * m) * tsz);
            return;
        }
        launch_npcg_dots(stream, d_fines, fine_tasks.d, fine_tasks.n, d_active, k & 1, d_part[0],
                         d_part[1], kmode);
        launch_sum_partials(stream, N, d_fine_range, d_part[0], d_scal, S_GAMMA, d_active);
        launch_sum_partials(stream, N, d_fine_range, d_part[1], d_scal, S_SIGMA, d_active);
        launch_npcg_beta(stream, N, d_scal, d_active, k == 0 ? 1 : 0, opt.restart_growth);
        hipEvent_t td = tic();
        launch_npcg_dir(stream, d_fines, fine_tasks.d, fine_tasks.n, d_active, d_scal, k & 1,
                        (k - 1) & 1, k & 1, d_part[2], d_part[3], kmode);
        // direction: e, p_old, r (precision T) and D, sa (FP64) read, p_new written
        toc(td, 3, 16.0 + 4.0 * tsz);
        launch_sum_partials(stream, N, d_fine_range, d_part[2], d_scal, S_RP, d_active);
        launch_sum_partials(stream, N, d_fine_range, d_part[3], d_scal, S_PAP, d_active);
        launch_npcg_theta(stream, N, d_scal, d_active);
    }

    // Capture body(k) + head(k+1) for the parity of k (k >= 1); false when
    // the runtime refuses, after which iterations run without graphs.
    bool capture(int k)
    {
        const int par = k & 1;
        reserve_graph_events();
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        capturing = true;
        timed_sink = &graph_timed[par];
        body(k);
        head(k + 1, false);
        capturing = false;
        timed_sink = &timed;
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(stream, &g);
        if (e != hipSuccess || !g) {
            (void)hipGetLastError();
            graph_timed[par].clear();
            return false;
        }
        e = hipGraphInstantiate(&graph_exec[par], g, nullptr, nullptr, 0);
        hipGraphDestroy(g);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            graph_exec[par] = nullptr;
            graph_timed[par].clear();
            return false;
        }
        return true;
    }

    // Multigrid solve of every problem.  start: 0 paper init / 1 given phi
    // already in phi[0] / 2 resume.
    fld_status solve_mg(int start, double *updates)
    {
        const int N = nprob;
        int k = 0;
        if (start == 2) {
            k = k_state;
        } else {
            if (start == 0)
                launch_init_phi(stream, d_fines, fine_tasks.d, fine_tasks.n, d_scal, 1, mixed);
            else
                launch_init_phi_dirs_only();
            for (Prob &P : probs) {
                P.hist.clear();
                P.status = FLD_ERR_NOT_CONVERGED;
                P.final_k = 0;
            }
        }
        std::vector<double> sc;
        HK(hipMemsetAsync(d_fail, 0, sizeof(int) * N, stream), "memset");
        if (opt.aa_m > 0 && start != 2)
            launch_aa_reset(stream, N, d_aai);
        std::fill(h_active.begin(), h_active.end(), 1);
        CK(sync_active(true));
        const int first_k = k;
        *updates = 0.0;
        head(k, true);
        int replayed = -1;        // parity of the graph whose events the last sync covers
        for (;;) {
            if (pending != hipSuccess) {
                const hipError_t e = pending;
                pending = hipSuccess;
                (void)hipGetLastError();
                return hip_fail(e, pending_what);
            }
            HK(hipGetLastError(), "launch");
            CK(read_scalars(sc));
            if (replayed >= 0)
                harvest(graph_timed[replayed], false);
            int n_active = 0;
            for (int p = 0; p < N; ++p) {
                if (!h_active[p])
                    continue;
                Prob &P = probs[p];
                const double rel = sc[(size_t)p * S_COUNT + S_REL];
                P.hist.push_back(rel);
                P.final_k = k;
                if (log_iters)
                    std::fprintf(stderr, "{\"fld_iteration\": %d, \"problem\": %d, \"rel\": %.17g}\n",
                                 k, p, rel);
                if (!std::isfinite(rel)) {
                    P.status = FLD_ERR_DIVERGED;
                    h_active[p] = 0;
                } else if (rel <= opt.tol) {
                    P.status = FLD_OK;
                    h_active[p] = 0;
                } else if (k - first_k >= opt.max_iters) {
                    P.status = FLD_ERR_NOT_CONVERGED;
                    h_active[p] = 0;
                } else {
                    ++n_active;
                }
            }
            if (!n_active)
                break;
            CK(sync_active());
            if (opt.debug_nan_iter > 0 && k == opt.debug_nan_iter)
                launch_poison(stream, d_fines, N, k & 1);
            for (int p = 0; p < N; ++p)
                if (h_active[p])
                    for (int l = 0; l + 1 < probs[p].nlev; ++l)
                        *updates += (double)probs[p].lv[l].n *
                                    (sweeps(l, true) + sweeps(l, false));
            replayed = -1;
            const int par = k & 1;
            const bool use_graph = k >= 1 && opt.graph && graphs_ok;
            if (use_graph && !graph_exec[par])
                graphs_ok = capture(k);
            if (use_graph && graphs_ok && graph_exec[par]) {
                HK(hipGraphLaunch(graph_exec[par], stream), "hipGraphLaunch");
                replayed = par;
            } else {
                body(k);
                head(k + 1, false);
            }
            ++k;
        }
        k_state = k;
        return FLD_OK;
    }

    void launch_init_phi_dirs_only()
    {
        // phi[0] already holds the start; zero the direction/rhs ping-pongs.
        for (Prob &P : probs) {
            const size_t NT = tsz * P.fine.n;
            const size_t NS = P.fine.split ? tsz * (size_t)((P.fine.n + 63) / 64 * 64) : NT;
            hipMemsetAsync(P.fine.p[0], 0, NT, stream);
            hipMemsetAsync(P.fine.p[1], 0, NT, stream);
            hipMemsetAsync(P.fine.b0[0], 0, NS, stream);
            hipMemsetAsync(P.fine.b0[1], 0, NS, stream);
        }
    }

    // Algorithm 1 (single problem).  start as in solve_mg.
    fld_status solve_alg1(int start, double *updates, double *rel_sweep)
    {
        Prob &P = probs[0];
        const int every = opt.check_every > 0 ? opt.check_every : 1;
        int it = 0;
        if (start == 2) {
            it = k_state;
        } else {
            if (start == 0)
                launch_init_phi(stream, d_fines, fine_tasks.d, fine_tasks.n, d_scal, 0, 0);
            else
                launch_init_d_only();
            P.hist.clear();
        }
        const int first = it;
        std::vector<double> sc;
        *updates = 0.0;
        *rel_sweep = NAN;
        bool swept = false;
        for (;;) {
            if ((it - first) % every == 0 || it - first == opt.max_iters) {
                launch_limiter(stream, d_fines, fine_tasks.d, fine_tasks.n, nullptr, d_scal, 0, 0, 0,
                               0, 1, 0, opt.limiter);
                launch_residual(stream, d_fines, fine_tasks.d, fine_tasks.n, nullptr, 0, 1, 0,
                                nullptr, d_part[0], 0);
                launch_sum_partials(stream, 1, d_fine_range, d_part[0], d_scal, S_RES2, nullptr);
                launch_rel(stream, 1, d_scal, nullptr);
                HK(hipGetLastError(), "residual launch");
                CK(read_scalars(sc));
                const double rel = sc[S_REL];
                P.hist.push_back(rel);
                if (swept)
                    *rel_sweep = std::sqrt((sc[S_SWEEP2] + sc[S_AUX]) / (double)P.fine.n) /
                                 sc[S_JBAR];
                if (!std::isfinite(rel)) { P.status = FLD_ERR_DIVERGED; break; }
                if (rel <= opt.tol) { P.status = FLD_OK; break; }
                if (it - first >= opt.max_iters) { P.status = FLD_ERR_NOT_CONVERGED; break; }
            }
            launch_alg1_pass(stream, d_fines, fine_tasks.d, fine_tasks.n, d_scal, 0, opt.omega,
                             d_part[0]);
            launch_sum_partials(stream, 1, d_fine_range, d_part[0], d_scal, S_SWEEP2, nullptr);
            launch_alg1_pass(stream, d_fines, fine_tasks.d, fine_tasks.n, d_scal, 1, opt.omega,
                             d_part[1]);
            launch_sum_partials(stream, 1, d_fine_range, d_part[1], d_scal, S_AUX, nullptr);
            *updates += (double)P.fine.n;
            swept = true;
            ++it;
        }
        P.final_k = it;
        k_state = it;
        return FLD_OK;
    }

    void launch_init_d_only()
    {
        // phi[0] holds the caller's start; D takes the paper's initial value.
        std::vector<double> d((size_t)probs[0].fine.n, opt.eps * probs[0].fine.h);
        hipMemcpyAsync(probs[0].fine.D64, d.data(), sizeof(double) * d.size(),
                       hipMemcpyHostToDevice, stream);
        hipStreamSynchronize(stream);
    }

    const double *current_phi(int p) const
    {
        const Prob &P = probs[p];
        return mg ? P.fine.phi[P.final_k & 1] : P.fine.phi[0];
    }

#undef CK
#undef HK
};

struct fld_context {
    fld_engine_impl eng;
    bool has_medium = false;
    // grid sequencing: the 2:1 coarser problem and its medium arrays
    fld_context *nested = nullptr;
    double *d_nested_medium = nullptr;   // sigma_t, albedo, Q of the coarse grid
    ~fld_context();
};

struct fld_batch {
    fld_engine_impl eng;
    int nvol = 0, nchan = 0;
    std::vector<int> has_medium;
    fld_batch *nested = nullptr;   // grid sequencing: the 2:1 coarser batch
    ~fld_batch();
};

namespace {

fld_status validate_options(const fld_options *o, std::string &err)
{
    if (!o) { err = "options is NULL"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->struct_size != sizeof(fld_options)) { err = "options.struct_size mismatch"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->limiter < FLD_LIMITER_CDA || o->limiter > FLD_LIMITER_LARSEN) { err = "limiter out of range"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->limiter == FLD_LIMITER_LARSEN && !(o->larsen_n > 0.0 && std::isfinite(o->larsen_n))) { err = "larsen_n must be > 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(o->eps > 0.0 && std::isfinite(o->eps))) { err = "eps must be > 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!std::isfinite(o->sigma_eps)) { err = "sigma_eps must be finite"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(std::isfinite(o->phi_b) && o->phi_b >= 0.0)) { err = "phi_b must be finite and >= 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->boundary_d != FLD_BOUNDARY_D_PAPER && o->boundary_d != FLD_BOUNDARY_D_MIRROR) { err = "boundary_d out of range"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->method != FLD_METHOD_RBSOR && o->method != FLD_METHOD_MG) { err = "method out of range"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->precision != FLD_PRECISION_FP64 && o->precision != FLD_PRECISION_MIXED) { err = "precision out of range"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->method == FLD_METHOD_RBSOR && o->precision != FLD_PRECISION_FP64) { err = "Algorithm 1 runs in FP64 only"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(o->omega > 0.0 && o->omega < 2.0)) { err = "omega must lie in (0,2)"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(o->omega_s > 0.0 && o->omega_s < 2.0)) { err = "omega_s must lie in (0,2)"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 + o->nu2 < 1 || o->nu1 > 64 || o->nu2 > 64) { err = "nu1/nu2 out of range"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->max_coarsest < 1 || o->max_coarsest > 4096) { err = "max_coarsest must lie in [1,4096]"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->max_iters < 0) { err = "max_iters must be >= 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(o->tol >= 0.0 && std::isfinite(o->tol))) { err = "tol must be finite and >= 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->check_every < 1) { err = "check_every must be >= 1"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->device < 0) { err = "device must be >= 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!std::isfinite(o->deflate_tau)) { err = "deflate_tau must be finite"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->task_cells0 < 512 || o->task_cells0 > 65536 || (o->task_cells0 & (o->task_cells0 - 1))) { err = "task_cells0 must be a power of two in [512,65536]"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->coarse_blocks < 64 || o->coarse_blocks > 65536) { err = "coarse_blocks must lie in [64,65536]"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->colour_split != 0 && o->colour_split != 1) { err = "colour_split must be 0 or 1"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!std::isfinite(o->restart_growth)) { err = "restart_growth must be finite"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(o->corr_scale > 0.0 && o->corr_scale <= 4.0)) { err = "corr_scale must lie in (0,4]"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(o->anisotropy_g >= 0.0 && o->anisotropy_g < 1.0)) { err = "anisotropy_g must lie in [0,1)"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->deep_cells < 0) { err = "deep_cells must be >= 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(o->nested_tol >= 0.0 && std::isfinite(o->nested_tol))) { err = "nested_tol must be finite and >= 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->nested_tol > 0.0 && o->method != FLD_METHOD_MG) { err = "nested_tol needs the multigrid method"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->nested_tol > 0.0 && o->anisotropy_g != 0.0) { err = "nested_tol needs anisotropy_g = 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->aa_m < 0 || o->aa_m > aa_max_window()) { err = "aa_m must lie in [0,16]"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->fuse_lr != 0 && o->fuse_lr != 1) { err = "fuse_lr must be 0 or 1"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->fuse_rb != 0 && o->fuse_rb != 1) { err = "fuse_rb must be 0 or 1"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->debug_nan_iter < 0) { err = "debug_nan_iter must be >= 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->nu_coarse < 0 || o->nu_coarse > 64) { err = "nu_coarse must lie in [0,64]"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->coarse_from < 1) { err = "coarse_from must be >= 1"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->nested_inherit != 0 && o->nested_inherit != 1) { err = "nested_inherit must be 0 or 1"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(o->aa_reg >= 0.0 && std::isfinite(o->aa_reg))) { err = "aa_reg must be finite and >= 0"; return FLD_ERR_INVALID_ARGUMENT; }
    return FLD_OK;
}

fld_status validate_grid(const fld_options *o, int nx, int ny, int nz, double h, std::string &err)
{
    if (nx < 1 || ny < 1 || nz < 1) { err = "grid dimensions must be >= 1"; return FLD_ERR_INVALID_ARGUMENT; }
    if ((long long)nx * ny * nz > (1LL << 31)) { err = "grid exceeds 2^31 cells"; return FLD_ERR_INVALID_ARGUMENT; }
    if (!(h > 0.0 && std::isfinite(h))) { err = "h must be finite and > 0"; return FLD_ERR_INVALID_ARGUMENT; }
    if (o->method == FLD_METHOD_MG) {
        int a = nx, b = ny, c = nz;
        while (!((a % 2) || (b % 2) || (c % 2) || a / 2 < 4 || b / 2 < 4 || c / 2 < 4)) {
            a /= 2; b /= 2; c /= 2;
        }
        if ((long long)a * b * c > o->max_coarsest) {
            char buf[200];
            snprintf(buf, sizeof buf, "multigrid: coarsest level %dx%dx%d exceeds max_coarsest=%d",
                     a, b, c, o->max_coarsest);
            err = buf;
            return FLD_ERR_INVALID_ARGUMENT;
        }
    }
    return FLD_OK;
}

void fill_report(fld_report *rep, fld_engine_impl &E, int p, int status, double ms,
                 double updates, double rel_sweep)
{
    double kms[4], kl[4], kb[4];
    E.collect_timing(kms, kl, kb);
    if (!rep || rep->struct_size != sizeof(fld_report))
        return;
    double tb = 0.0;
    for (int q = 0; q < 4; ++q) {
        rep->kernel_ms[q] = kms[q];
        rep->kernel_launches[q] = kl[q];
        rep->kernel_bytes[q] = kb[q];
        tb += kb[q];
    }
    const auto &P = E.probs[p];
    rep->status = status;
    rep->iterations = P.final_k;
    rep->rel = P.hist.empty() ? NAN : P.hist.back();
    rep->rel_sweep = rel_sweep;
    rep->history_len = (int)P.hist.size();
    if (rep->history && rep->history_cap > 0)
        for (int q = 0; q < std::min<int>(rep->history_cap, (int)P.hist.size()); ++q)
            rep->history[q] = P.hist[q];
    rep->time_ms = ms;
    rep->voxel_updates = updates;
    rep->bytes = tb;
}

}  // namespace

extern "C" {

fld_status fld_device_arch(int device, char *buf, int len)
{
    if (!buf || len < 2 || device < 0)
        return FLD_ERR_INVALID_ARGUMENT;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess)
        return FLD_ERR_DEVICE;
    if (device >= count)
        return FLD_ERR_INVALID_ARGUMENT;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return FLD_ERR_DEVICE;
    int k = 0;
    for (; k + 1 < len && prop.gcnArchName[k] && prop.gcnArchName[k] != ':'; ++k)
        buf[k] = prop.gcnArchName[k];
    buf[k] = 0;
    return FLD_OK;
}

fld_status fld_default_options(fld_options *o)
{
    if (!o)
        return FLD_ERR_INVALID_ARGUMENT;
    memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(fld_options);
    o->limiter = FLD_LIMITER_LP;
    o->larsen_n = 2.0;
    o->eps = 1e-20;
    o->sigma_eps = -1.0;
    o->phi_b = 0.0;
    o->boundary_d = FLD_BOUNDARY_D_PAPER;
    o->method = FLD_METHOD_MG;
    o->precision = FLD_PRECISION_FP64;
    o->omega = 1.0;
    o->omega_s = 1.0;
    o->nu1 = 2;
    o->nu2 = 2;
    o->max_coarsest = 512;
    o->max_iters = 10000;
    o->tol = 1e-6;
    o->check_every = 1;
    o->device = 0;
    o->stream = nullptr;
    o->timing = 0;
    o->deflate_tau = 1.0;
    o->graph = 1;
    o->task_cells0 = 4096;
    o->coarse_blocks = 2048;
    o->colour_split = 1;
    o->restart_growth = 2.0;
    o->corr_scale = 1.0;
    o->anisotropy_g = 0.0;
    o->deep_cells = 4096;
    o->nested_tol = 0.0;
    o->aa_m = 0;
    o->aa_reg = 1e-10;
    o->fuse_lr = 0;
    o->fuse_rb = 0;
    o->debug_nan_iter = 0;
    o->nu_coarse = 0;
    o->coarse_from = 2;
    o->nested_inherit = 0;
    return FLD_OK;
}

static thread_local std::string g_create_err;

// Options of the 2:1 coarser problem of grid sequencing: the same physics and
// precision, default launch shapes and schedule, solved to nested_tol (at most
// 10000 iterations, not the fine cap, so chunked solves stay nested) without
// timing.
static fld_options nested_options(const fld_options *o)
{
    fld_options co;
    fld_default_options(&co);
    co.limiter = o->limiter;
    co.larsen_n = o->larsen_n;
    co.eps = o->eps;
    co.sigma_eps = o->sigma_eps;
    co.phi_b = o->phi_b;
    co.boundary_d = o->boundary_d;
    co.precision = o->precision;
    co.max_coarsest = o->max_coarsest;
    co.max_iters = 10000;
    co.tol = o->nested_tol;
    co.device = o->device;
    co.stream = o->stream;
    co.deflate_tau = o->deflate_tau;
    co.graph = o->graph;
    co.colour_split = o->colour_split;
    if (o->nested_inherit) {
        // the fine solve's schedule; the coarse grid's level l is the fine
        // grid's level l + 1
        co.nu1 = o->nu1;
        co.nu2 = o->nu2;
        co.omega_s = o->omega_s;
        co.corr_scale = o->corr_scale;
        co.restart_growth = o->restart_growth;
        co.aa_m = o->aa_m;
        co.aa_reg = o->aa_reg;
        co.nu_coarse = o->nu_coarse;
        co.coarse_from = std::max(1, o->coarse_from - 1);
    }
    return co;
}

fld_context::~fld_context()
{
    if (nested)
        delete nested;
    if (d_nested_medium)
        hipFree(d_nested_medium);
}

fld_batch::~fld_batch()
{
    if (nested)
        delete nested;
}

fld_status fld_create(const fld_options *o, int nx, int ny, int nz, double h, fld_context **out)
{
    if (!out)
        return FLD_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    std::string err;
    fld_status s = validate_options(o, err);
    if (s == FLD_OK)
        s = validate_grid(o, nx, ny, nz, h, err);
    if (s == FLD_OK && o->nested_tol > 0.0 && ((nx | ny | nz) & 1)) {
        err = "nested_tol needs every axis even";
        s = FLD_ERR_INVALID_ARGUMENT;
    }
    if (s != FLD_OK) {
        g_create_err = err;
        return s;
    }
    fld_context *c = new (std::nothrow) fld_context;
    if (!c)
        return FLD_ERR_OUT_OF_MEMORY;
    int dims[3] = {nx, ny, nz};
    s = c->eng.build(*o, 1, dims, &h, 1);
    if (s != FLD_OK) {
        g_create_err = c->eng.err;
        delete c;
        return s;
    }
    if (o->nested_tol > 0.0) {
        const fld_options co = nested_options(o);
        s = fld_create(&co, nx / 2, ny / 2, nz / 2, 2.0 * h, &c->nested);
        if (s == FLD_OK) {
            const size_t nc = (size_t)(nx / 2) * (ny / 2) * (nz / 2);
            if (hipMalloc((void **)&c->d_nested_medium, 3 * 8 * nc) != hipSuccess) {
                g_create_err = "grid sequencing: coarse medium allocation failed";
                s = FLD_ERR_OUT_OF_MEMORY;
            }
        } else {
            g_create_err = "grid sequencing: " + g_create_err;
        }
        if (s != FLD_OK) {
            delete c;
            return s;
        }
    }
    *out = c;
    return FLD_OK;
}

static fld_status set_medium_impl(fld_context *c, const double *st, const double *al,
                                  const double *q, bool device, void *hs)
{
    if (!c)
        return FLD_ERR_INVALID_ARGUMENT;
    if (!st || !al || !q)
        return c->eng.fail(FLD_ERR_INVALID_ARGUMENT, "medium pointer is NULL");
    auto &E = c->eng;
    const long long n = E.vols[0].n;
    if (hs && hs != E.stream) {
        // order the caller's stream before ours
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess)
            return E.fail(FLD_ERR_DEVICE, "hipEventCreate failed");
        hipEventRecord(ev, (hipStream_t)hs);
        hipStreamWaitEvent(E.stream, ev, 0);
        hipEventDestroy(ev);
    }
    std::vector<double> hst, hal, hq;
    const double *pst = st, *pal = al, *pq = q;
    if (device) {
        hst.resize(n); hal.resize(n); hq.resize(n);
        if (hipMemcpyAsync(hst.data(), st, 8 * n, hipMemcpyDeviceToHost, E.stream) != hipSuccess ||
            hipMemcpyAsync(hal.data(), al, 8 * n, hipMemcpyDeviceToHost, E.stream) != hipSuccess ||
            hipMemcpyAsync(hq.data(), q, 8 * n, hipMemcpyDeviceToHost, E.stream) != hipSuccess ||
            hipStreamSynchronize(E.stream) != hipSuccess)
            return E.fail(FLD_ERR_DEVICE, "reading device medium failed");
        pst = hst.data(); pal = hal.data(); pq = hq.data();
    }
    fld_status s = E.check_host_medium(pst, pal, pq, n);
    if (s != FLD_OK)
        return s;
    double *dst = nullptr, *dal = nullptr, *dq = nullptr;
    const double *ust = st, *ual = al, *uq = q;
    if (!device) {
        if (hipMalloc(&dst, 8 * n) != hipSuccess || hipMalloc(&dal, 8 * n) != hipSuccess ||
            hipMalloc(&dq, 8 * n) != hipSuccess) {
            hipFree(dst); hipFree(dal); hipFree(dq);
            return E.fail(FLD_ERR_OUT_OF_MEMORY, "staging allocation failed");
        }
        hipMemcpyAsync(dst, st, 8 * n, hipMemcpyHostToDevice, E.stream);
        hipMemcpyAsync(dal, al, 8 * n, hipMemcpyHostToDevice, E.stream);
        hipMemcpyAsync(dq, q, 8 * n, hipMemcpyHostToDevice, E.stream);
        ust = dst; ual = dal; uq = dq;
    }
    s = E.set_problem_medium(0, ust, ual, uq);
    if (s == FLD_OK)
        s = E.finish_medium();
    if (!device) {
        hipFree(dst); hipFree(dal); hipFree(dq);
    }
    if (s == FLD_OK && c->nested) {
        // the coarse problem's medium, averaged from the finest set-up fields
        const Vol &V = E.vols[0];
        const Fine &f = E.probs[0].fine;
        const size_t nc = (size_t)(V.nx / 2) * (V.ny / 2) * (V.nz / 2);
        double *cst = c->d_nested_medium, *cal = cst + nc, *cq = cal + nc;
        launch_nested_coarsen(E.stream, f.sig_hat, f.sa64, f.j, V.nx, V.ny, V.nz, cst, cal, cq);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return E.hip_fail(e, "grid sequencing: coarsen launch");
        s = set_medium_impl(c->nested, cst, cal, cq, true, E.stream);
        if (s != FLD_OK)
            return E.fail(s, "grid sequencing: coarse medium: %s", c->nested->eng.err.c_str());
    }
    if (s == FLD_OK)
        c->has_medium = true;
    return s;
}

fld_status fld_set_medium(fld_context *c, const double *sigma_t, const double *albedo,
                          const double *Q)
{
    return set_medium_impl(c, sigma_t, albedo, Q, false, nullptr);
}

fld_status fld_set_medium_device(fld_context *c, const double *d_sigma_t, const double *d_albedo,
                                 const double *d_Q, void *hip_stream)
{
    return set_medium_impl(c, d_sigma_t, d_albedo, d_Q, true, hip_stream);
}

static fld_status solve_impl(fld_context *c, const double *phi_init, bool init_device,
                             double *phi_out, bool out_device, int resume, fld_report *rep)
{
    if (!c)
        return FLD_ERR_INVALID_ARGUMENT;
    auto &E = c->eng;
    if (!c->has_medium)
        return E.fail(FLD_ERR_STATE, "fld_solve before a medium was set");
    if (resume && !E.solved_once)
        return E.fail(FLD_ERR_STATE, "resume before any solve");
    const long long n = E.vols[0].n;
    std::vector<double> sc;
    auto t0 = std::chrono::steady_clock::now();
    fld_status s = E.read_scalars(sc);
    if (s != FLD_OK)
        return s;
    if (sc[S_JN2] == 0.0) {
        // No emission: the fluence is the boundary value (nothing to solve).
        std::vector<double> v((size_t)n, E.opt.phi_b);
        if (phi_out) {
            hipError_t e = hipMemcpy(phi_out, v.data(), 8 * n,
                                     out_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost);
            if (e != hipSuccess)
                return E.hip_fail(e, "phi_out copy");
        }
        hipMemcpy(E.probs[0].fine.phi[0], v.data(), 8 * n, hipMemcpyHostToDevice);
        E.probs[0].final_k = 0;
        E.probs[0].hist.assign(1, 0.0);
        E.solved_once = true;
        fill_report(rep, E, 0, FLD_OK, 0.0, 0.0, NAN);
        if (rep && rep->struct_size == sizeof(fld_report))
            rep->nested_iterations = 0;
        return FLD_OK;
    }
    int start = resume ? 2 : (phi_init ? 1 : 0);
    int nested_its = 0;
    double nested_updates = 0.0;
    if (start == 0 && c->nested) {
        // grid sequencing: solve the coarse problem, start from its fluence
        fld_report cr;
        std::memset(&cr, 0, sizeof cr);
        cr.struct_size = sizeof cr;
        s = solve_impl(c->nested, nullptr, false, nullptr, false, 0, &cr);
        if (s != FLD_OK && s != FLD_ERR_NOT_CONVERGED && s != FLD_ERR_DIVERGED)
            return E.fail(s, "grid sequencing: coarse solve: %s", c->nested->eng.err.c_str());
        nested_its = cr.iterations;
        nested_updates = cr.voxel_updates;
        if (s != FLD_ERR_DIVERGED) {
            const Vol &V = E.vols[0];
            launch_nested_prolong(E.stream, c->nested->eng.current_phi(0), V.nx, V.ny, V.nz,
                                  E.probs[0].fine.phi[0]);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess)
                return E.hip_fail(e, "grid sequencing: prolong launch");
            start = 1;
        }
    }
    if (start == 1 && phi_init) {
        hipError_t e = hipMemcpyAsync(E.probs[0].fine.phi[0], phi_init, 8 * n,
                                      init_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                      E.stream);
        if (e != hipSuccess)
            return E.hip_fail(e, "phi_init copy");
    }
    double updates = 0.0, rel_sweep = NAN;
    s = E.mg ? E.solve_mg(start, &updates) : E.solve_alg1(start, &updates, &rel_sweep);
    if (s != FLD_OK)
        return s;
    E.solved_once = true;
    if (phi_out) {
        hipError_t e = hipMemcpyAsync(phi_out, E.current_phi(0), 8 * n,
                                      out_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                      E.stream);
        if (e != hipSuccess)
            return E.hip_fail(e, "phi_out copy");
    }
    hipError_t e = hipStreamSynchronize(E.stream);
    if (e != hipSuccess)
        return E.hip_fail(e, "solve sync");
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const int st = E.probs[0].status;
    fill_report(rep, E, 0, st, ms, updates + nested_updates, rel_sweep);
    if (rep && rep->struct_size == sizeof(fld_report))
        rep->nested_iterations = nested_its;
    if (st == FLD_ERR_NOT_CONVERGED)
        E.fail(FLD_ERR_NOT_CONVERGED, "not converged after %d iterations (rel %g)",
               E.probs[0].final_k, E.probs[0].hist.empty() ? NAN : E.probs[0].hist.back());
    if (st == FLD_ERR_DIVERGED)
        E.fail(FLD_ERR_DIVERGED, "residual became non-finite at iteration %d", E.probs[0].final_k);
    return (fld_status)st;
}

fld_status fld_solve(fld_context *c, const double *phi_init, double *phi_out, fld_report *rep)
{
    return solve_impl(c, phi_init, false, phi_out, false, 0, rep);
}

fld_status fld_solve_device(fld_context *c, const double *d_phi_init, double *d_phi_out,
                            int resume, fld_report *rep)
{
    return solve_impl(c, d_phi_init, true, d_phi_out, true, resume, rep);
}

fld_status fld_solve_resume(fld_context *c, double *phi_out, fld_report *rep)
{
    return solve_impl(c, nullptr, false, phi_out, false, 1, rep);
}

// Nonlinear residual of phi (NULL: the context's current fluence), D
// recomputed from phi for every voxel.  Without a workspace the temporaries
// are allocated here and phi / r_out are host pointers unless dev.  With a
// workspace (device memory of the caller) nothing is allocated: phi and
// r_out are device pointers, phi is read in place, and the problem
// descriptor is written by a kernel.
static fld_status residual_impl(fld_context *c, const double *phi, bool dev, double *r_out,
                                double *rel_out, const ResidualWork *ws)
{
    if (!c)
        return FLD_ERR_INVALID_ARGUMENT;
    auto &E = c->eng;
    if (!c->has_medium)
        return E.fail(FLD_ERR_STATE, "fld_residual before a medium was set");
    if (!rel_out)
        return E.fail(FLD_ERR_INVALID_ARGUMENT, "rel_out is NULL");
    const long long n = E.vols[0].n;
    Fine f = E.probs[0].fine;
    if (ws) {
        if (n > ws->max_cells)
            return E.fail(FLD_ERR_INVALID_ARGUMENT,
                          "grid of %lld cells exceeds the workspace of %lld cells", n,
                          ws->max_cells);
        f.phi[0] = f.phi[1] = const_cast<double *>(phi ? phi : E.current_phi(0));
        f.Dtmp = ws->D;
        f.b0[0] = f.b0[1] = ws->b;
        launch_put_fine(E.stream, f, ws->fine);
        launch_limiter(E.stream, ws->fine, E.fine_tasks.d, E.fine_tasks.n, nullptr, E.d_scal, 0,
                       0, 0, 0, 1, 0, E.opt.limiter);
        launch_residual(E.stream, ws->fine, E.fine_tasks.d, E.fine_tasks.n, nullptr, 0, 1, 0,
                        r_out, E.d_part[0], 0);
        launch_sum_partials(E.stream, 1, E.d_fine_range, E.d_part[0], E.d_scal, S_AUX, nullptr);
        double sc[S_COUNT];
        hipError_t e = hipGetLastError();
        if (e == hipSuccess)
            e = hipMemcpyAsync(sc, E.d_scal, sizeof sc, hipMemcpyDeviceToHost, E.stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(E.stream);
        if (e != hipSuccess)
            return E.hip_fail(e, "residual");
        *rel_out = sc[S_JNORM] > 0.0 ? std::sqrt(sc[S_AUX]) / sc[S_JNORM] : 0.0;
        return FLD_OK;
    }
    double *tphi = nullptr, *tD = nullptr, *tr = nullptr;
    void *tb = nullptr;
    Fine *dfine = nullptr;
    auto cleanup = [&]() { hipFree(tphi); hipFree(tD); hipFree(tr); hipFree(tb); hipFree(dfine); };
    if (hipMalloc(&tphi, 8 * n) != hipSuccess || hipMalloc(&tD, 8 * n) != hipSuccess ||
        hipMalloc(&tr, 8 * n) != hipSuccess || hipMalloc(&tb, 8 * n) != hipSuccess ||
        hipMalloc(&dfine, sizeof(Fine)) != hipSuccess) {
        cleanup();
        return E.fail(FLD_ERR_OUT_OF_MEMORY, "residual scratch allocation failed");
    }
    const double *src = phi ? phi : E.current_phi(0);
    hipMemcpyAsync(tphi, src, 8 * n,
                   (phi && !dev) ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, E.stream);
    f.phi[0] = f.phi[1] = tphi;
    f.Dtmp = tD;
    f.b0[0] = f.b0[1] = tb;
    hipMemcpyAsync(dfine, &f, sizeof(Fine), hipMemcpyHostToDevice, E.stream);
    launch_limiter(E.stream, dfine, E.fine_tasks.d, E.fine_tasks.n, nullptr, E.d_scal, 0, 0, 0, 0,
                   1, 0, E.opt.limiter);
    launch_residual(E.stream, dfine, E.fine_tasks.d, E.fine_tasks.n, nullptr, 0, 1, 0, tr,
                    E.d_part[0], 0);
    launch_sum_partials(E.stream, 1, E.d_fine_range, E.d_part[0], E.d_scal, S_AUX, nullptr);
    std::vector<double> sc;
    fld_status s = E.read_scalars(sc);
    if (s == FLD_OK) {
        *rel_out = sc[S_JNORM] > 0.0 ? std::sqrt(sc[S_AUX]) / sc[S_JNORM] : 0.0;
        if (r_out) {
            hipError_t e = hipMemcpy(r_out, tr, 8 * n, dev ? hipMemcpyDeviceToDevice
                                                            : hipMemcpyDeviceToHost);
            if (e != hipSuccess)
                s = E.hip_fail(e, "r_out copy");
        }
    }
    hipStreamSynchronize(E.stream);
    cleanup();
    return s;
}

fld_status fld_residual(fld_context *c, const double *phi, double *r_out, double *rel_out)
{
    return residual_impl(c, phi, false, r_out, rel_out, nullptr);
}

fld_status fld_residual_device(fld_context *c, const double *d_phi, double *d_r_out,
                               double *rel_out)
{
    return residual_impl(c, d_phi, true, d_r_out, rel_out, nullptr);
}

void fld_destroy(fld_context *c) { delete c; }

const char *fld_status_string(fld_status s)
{
    switch (s) {
    case FLD_OK: return "ok";
    case FLD_ERR_INVALID_ARGUMENT: return "invalid argument";
    case FLD_ERR_OUT_OF_MEMORY: return "out of memory";
    case FLD_ERR_DEVICE: return "device error";
    case FLD_ERR_NOT_CONVERGED: return "not converged";
    case FLD_ERR_DIVERGED: return "diverged";
    case FLD_ERR_STATE: return "invalid call order";
    }
    return "unknown status";
}

const char *fld_last_error(const fld_context *c)
{
    if (!c)
        return g_create_err.empty() ? "invalid context" : g_create_err.c_str();
    return c->eng.err.c_str();
}

// ---- batch ------------------------------------------------------------------

fld_status fld_batch_create(const fld_options *o, int nvol, const int *dims3, const double *h,
                            int nchan, fld_batch **out)
{
    if (!out)
        return FLD_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    std::string err;
    if (nvol < 1 || nchan < 1 || !dims3 || !h) {
        g_create_err = "batch: nvol/nchan must be >= 1 and dims3/h non-NULL";
        return FLD_ERR_INVALID_ARGUMENT;
    }
    fld_status s = validate_options(o, err);
    if (s == FLD_OK && o->method != FLD_METHOD_MG) {
        err = "batched solves use the multigrid method";
        s = FLD_ERR_INVALID_ARGUMENT;
    }
    for (int v = 0; s == FLD_OK && o->nested_tol > 0.0 && v < nvol; ++v)
        if ((dims3[3 * v] | dims3[3 * v + 1] | dims3[3 * v + 2]) & 1) {
            err = "nested_tol needs every axis of every volume even";
            s = FLD_ERR_INVALID_ARGUMENT;
        }
    if (s == FLD_OK && o->anisotropy_g != 0.0 && nchan > 1) {
        // the reduced extinction depends on each channel's albedo, while the
        // channels of a volume share one extinction field
        err = "batch: anisotropy_g != 0 needs one channel per volume";
        s = FLD_ERR_INVALID_ARGUMENT;
    }
    for (int v = 0; s == FLD_OK && v < nvol; ++v)
        s = validate_grid(o, dims3[3 * v], dims3[3 * v + 1], dims3[3 * v + 2], h[v], err);
    if (s != FLD_OK) {
        g_create_err = err;
        return s;
    }
    fld_batch *b = new (std::nothrow) fld_batch;
    if (!b)
        return FLD_ERR_OUT_OF_MEMORY;
    s = b->eng.build(*o, nvol, dims3, h, nchan);
    if (s != FLD_OK) {
        g_create_err = b->eng.err;
        delete b;
        return s;
    }
    b->nvol = nvol;
    b->nchan = nchan;
    b->has_medium.assign(nvol, 0);
    if (o->nested_tol > 0.0) {
        const fld_options co = nested_options(o);
        std::vector<int> cd(3 * (size_t)nvol);
        std::vector<double> ch(nvol);
        for (int v = 0; v < nvol; ++v) {
            for (int a = 0; a < 3; ++a)
                cd[3 * v + a] = dims3[3 * v + a] / 2;
            ch[v] = 2.0 * h[v];
        }
        s = fld_batch_create(&co, nvol, cd.data(), ch.data(), nchan, &b->nested);
        if (s != FLD_OK) {
            g_create_err = "grid sequencing: " + g_create_err;
            delete b;
            return s;
        }
    }
    *out = b;
    return FLD_OK;
}

fld_status fld_batch_set_volume(fld_batch *b, int v, const double *sigma_t,
                                const double *const *albedo, const double *const *Q)
{
    if (!b)
        return FLD_ERR_INVALID_ARGUMENT;
    auto &E = b->eng;
    if (v < 0 || v >= b->nvol || !sigma_t || !albedo || !Q)
        return E.fail(FLD_ERR_INVALID_ARGUMENT, "bad volume index or NULL pointer");
    const long long n = E.vols[v].n;
    for (int ch = 0; ch < b->nchan; ++ch) {
        if (!albedo[ch] || !Q[ch])
            return E.fail(FLD_ERR_INVALID_ARGUMENT, "channel %d pointer is NULL", ch);
        fld_status s = E.check_host_medium(sigma_t, albedo[ch], Q[ch], n);
        if (s != FLD_OK)
            return s;
    }
    double *dst = nullptr, *dal = nullptr, *dq = nullptr;
    if (hipMalloc(&dst, 8 * n) != hipSuccess || hipMalloc(&dal, 8 * n) != hipSuccess ||
        hipMalloc(&dq, 8 * n) != hipSuccess) {
        hipFree(dst); hipFree(dal); hipFree(dq);
        return E.fail(FLD_ERR_OUT_OF_MEMORY, "staging allocation failed");
    }
    hipMemcpyAsync(dst, sigma_t, 8 * n, hipMemcpyHostToDevice, E.stream);
    fld_status s = FLD_OK;
    for (int ch = 0; ch < b->nchan && s == FLD_OK; ++ch) {
        hipMemcpyAsync(dal, albedo[ch], 8 * n, hipMemcpyHostToDevice, E.stream);
        hipMemcpyAsync(dq, Q[ch], 8 * n, hipMemcpyHostToDevice, E.stream);
        s = E.set_problem_medium(v * b->nchan + ch, dst, dal, dq);
        hipStreamSynchronize(E.stream);
    }
    hipFree(dst); hipFree(dal); hipFree(dq);
    if (s != FLD_OK)
        return s;
    if (b->nested) {
        // the coarse volume: sigma_t (shared) and each channel's albedo and Q,
        // averaged from the finest set-up fields of every channel
        const Vol &V = E.vols[v];
        const size_t nc = (size_t)(V.nx / 2) * (V.ny / 2) * (V.nz / 2);
        double *dc = nullptr;
        if (hipMalloc(&dc, 3 * 8 * nc) != hipSuccess)
            return E.fail(FLD_ERR_OUT_OF_MEMORY, "grid sequencing: staging allocation failed");
        std::vector<double> cst(nc);
        std::vector<std::vector<double>> cal(b->nchan, std::vector<double>(nc)),
            cq(b->nchan, std::vector<double>(nc));
        hipError_t e = hipSuccess;
        for (int ch = 0; ch < b->nchan && e == hipSuccess; ++ch) {
            const Fine &f = E.probs[v * b->nchan + ch].fine;
            launch_nested_coarsen(E.stream, f.sig_hat, f.sa64, f.j, V.nx, V.ny, V.nz, dc, dc + nc,
                                  dc + 2 * nc);
            e = hipGetLastError();
            if (e == hipSuccess && ch == 0)
                e = hipMemcpyAsync(cst.data(), dc, 8 * nc, hipMemcpyDeviceToHost, E.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(cal[ch].data(), dc + nc, 8 * nc, hipMemcpyDeviceToHost,
                                   E.stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(cq[ch].data(), dc + 2 * nc, 8 * nc, hipMemcpyDeviceToHost,
                                   E.stream);
            if (e == hipSuccess)
                e = hipStreamSynchronize(E.stream);
        }
        hipFree(dc);
        if (e != hipSuccess)
            return E.hip_fail(e, "grid sequencing: coarse medium");
        std::vector<const double *> pal(b->nchan), pq(b->nchan);
        for (int ch = 0; ch < b->nchan; ++ch) {
            pal[ch] = cal[ch].data();
            pq[ch] = cq[ch].data();
        }
        s = fld_batch_set_volume(b->nested, v, cst.data(), pal.data(), pq.data());
        if (s != FLD_OK)
            return E.fail(s, "grid sequencing: coarse volume: %s", b->nested->eng.err.c_str());
    }
    b->has_medium[v] = 1;
    for (int q = 0; q < b->nvol; ++q)
        if (!b->has_medium[q])
            return FLD_OK;
    return E.finish_medium();
}

fld_status fld_batch_solve(fld_batch *b, double *const *phi_out, int *iters_out, fld_report *rep)
{
    if (!b)
        return FLD_ERR_INVALID_ARGUMENT;
    auto &E = b->eng;
    for (int q = 0; q < b->nvol; ++q)
        if (!b->has_medium[q])
            return E.fail(FLD_ERR_STATE, "volume %d has no medium", q);
    auto t0 = std::chrono::steady_clock::now();
    double updates = 0.0;
    int start = 0, nested_its = 0;
    if (b->nested) {
        // grid sequencing: solve the coarse batch, start every problem from
        // its coarse fluence (the paper's state where the coarse one diverged)
        fld_report cr;
        std::memset(&cr, 0, sizeof cr);
        cr.struct_size = sizeof cr;
        fld_status cs = fld_batch_solve(b->nested, nullptr, nullptr, &cr);
        if (cs != FLD_OK && cs != FLD_ERR_NOT_CONVERGED && cs != FLD_ERR_DIVERGED)
            return E.fail(cs, "grid sequencing: coarse solve: %s", b->nested->eng.err.c_str());
        nested_its = cr.iterations;
        updates += cr.voxel_updates;
        const auto &CE = b->nested->eng;
        for (int p = 0; p < E.nprob; ++p) {
            const Vol &V = E.vols[E.probs[p].vol];
            if (CE.probs[p].status != FLD_ERR_DIVERGED)
                launch_nested_prolong(E.stream, CE.current_phi(p), V.nx, V.ny, V.nz,
                                      E.probs[p].fine.phi[0]);
            else
                launch_init_phi(E.stream, E.d_fines, E.fine_tasks.d + E.fine_range[p],
                                E.fine_range[p + 1] - E.fine_range[p], E.d_scal, 0, E.mixed);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return E.hip_fail(e, "grid sequencing: prolong launch");
        start = 1;
    }
    double fine_updates = 0.0;
    fld_status s = E.solve_mg(start, &fine_updates);
    if (s != FLD_OK)
        return s;
    updates += fine_updates;
    E.solved_once = true;
    if (phi_out)
        for (int p = 0; p < E.nprob; ++p)
            if (phi_out[p]) {
                hipError_t e = hipMemcpyAsync(phi_out[p], E.current_phi(p),
                                              8 * E.vols[E.probs[p].vol].n, hipMemcpyDeviceToHost,
                                              E.stream);
                if (e != hipSuccess)
                    return E.hip_fail(e, "phi_out copy");
            }
    hipError_t e = hipStreamSynchronize(E.stream);
    if (e != hipSuccess)
        return E.hip_fail(e, "batch sync");
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int worst = 0, status = FLD_OK;
    for (int p = 0; p < E.nprob; ++p) {
        if (iters_out)
            iters_out[p] = E.probs[p].final_k;
        if (E.probs[p].final_k > E.probs[worst].final_k)
            worst = p;
        if (E.probs[p].status != FLD_OK && status == FLD_OK)
            status = E.probs[p].status;
    }
    fill_report(rep, E, worst, status, ms, updates, NAN);
    if (rep && rep->struct_size == sizeof(fld_report))
        rep->nested_iterations = nested_its;
    return (fld_status)status;
}

void fld_batch_destroy(fld_batch *b) { delete b; }

const char *fld_batch_last_error(const fld_batch *b)
{
    if (!b)
        return g_create_err.empty() ? "invalid batch" : g_create_err.c_str();
    return b->eng.err.c_str();
}

}  // extern "C"

namespace fld {

fld_status residual_with_workspace(fld_context *c, const double *d_phi, double *d_r_out,
                                   double *rel_out, const ResidualWork *ws)
{
    return residual_impl(c, d_phi, true, d_r_out, rel_out, ws);
}

int context_device(const fld_context *c) { return c ? c->eng.opt.device : -1; }

}  // namespace fld
