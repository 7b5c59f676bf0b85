// Runtime entry points: bind, the batched sign solve, write-back.
//
// One call of nolsm_sign_batch runs, for every chunk of submatrices that fits
// the workspace: gather -> Cholesky -> substitution -> bounds -> X_0 ->
// max_iter Newton-Schulz iteration slots (two GEMM launches each; finished
// submatrices drop out inside the kernels) -> finishing products ->
// extraction / traces / write-back. With NOLSM_SCHED_GRAPH on a non-null
// stream the whole sequence is captured once into a hipGraph and replayed by
// later calls with the same buffers and options.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"
#include "plan.h"

static int hip_fail(hipError_t e, const char *where) {
    nolsm_set_last_error(std::string(where) + ": " + hipGetErrorString(e));
    return NOLSM_E_HIP;
}

static void drop_graph(nolsm_plan *pl) {
    if (pl->graph_exec) {
        (void)hipGraphExecDestroy((hipGraphExec_t)pl->graph_exec);
        pl->graph_exec = nullptr;
    }
}

extern "C" int nolsm_plan_bind(nolsm_plan *pl, void *d_meta, size_t bytes, void *stream) {
    if (!pl || !d_meta) { nolsm_set_last_error("bind: null argument"); return NOLSM_E_ARG; }
    if (!pl->configured) { nolsm_set_last_error("bind: plan not configured"); return NOLSM_E_STATE; }
    if (bytes < pl->image.size()) { nolsm_set_last_error("bind: metadata buffer too small"); return NOLSM_E_WORKSPACE; }
    if (((uintptr_t)d_meta) & 255) { nolsm_set_last_error("bind: d_meta must be 256-byte aligned"); return NOLSM_E_ARG; }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = nolsm_kernels_init();
    if (e != hipSuccess) return hip_fail(e, "kernel attributes");
    e = hipMemcpyAsync(d_meta, pl->image.data(), pl->image.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "metadata upload");
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "metadata upload sync");
    drop_graph(pl);
    pl->d_meta = d_meta;
    pl->bound = true;
    (void)hipGetDevice(&pl->device);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device) != hipSuccess || cus < 1)
        cus = 256;
    pl->pgrid = 2 * cus;   // two 256-thread workgroups per CU (LDS-limited)
    return NOLSM_OK;
}

static ChunkDev chunk_dev(const nolsm_plan *pl, const HostChunk &ch, char *ws) {
    const char *base = (const char *)pl->d_meta;
    ChunkDev cd;
    cd.meta = (const SubMeta *)(base + ch.o_meta);
    cd.t_subst = (const uint32_t *)(base + ch.o_subst);
    cd.t_conv = (const uint32_t *)(base + ch.o_conv);
    cd.t_ns = (const uint32_t *)(base + ch.o_ns);
    cd.t_ns64 = (const uint32_t *)(base + ch.o_ns64);
    cd.t_rows = (const uint32_t *)(base + ch.o_rows);
    cd.ctl = (SubCtl *)(ws + ch.off_ctl);
    cd.ictl = ch.off_ictl ? (InvCtl *)(ws + ch.off_ictl) : nullptr;
    cd.queues = (int32_t *)(ws + ch.off_q);
    cd.nqueue = pl->max_iter * 2 * 2 * 8;
    cd.nsub = (int32_t)ch.meta.size();
    cd.n_subst = (int32_t)ch.t_subst.size();
    cd.n_conv = (int32_t)ch.t_conv.size();
    // lists without real entries are not launched
    cd.n_ns = ch.n_ns_real ? (int32_t)ch.t_ns.size() : 0;
    cd.n_ns64 = ch.n_ns64_real ? (int32_t)ch.t_ns64.size() : 0;
    cd.n_rows = (int32_t)ch.t_rows.size();
    cd.max_m = ch.max_m;
    cd.max_np = ch.max_np;
    cd.max_own = ch.max_own;
    return cd;
}

struct BatchArgs {
    const double *dK, *dS;
    double mu;
    const nolsm_solve_opts *o;
    char *ws;
    double *dDcols, *dD;
    void *dstats;
};

enum { PH_GATHER, PH_CHOL, PH_SUBST, PH_BOUNDS, PH_NS, PH_FINISH, PH_EXTRACT, PH_WMAT, PH_INV, PH_END };

// HIP events recorded on the call's stream between phases
struct PhaseEvents {
    hipStream_t st;
    std::vector<hipEvent_t> ev;
    std::vector<int> ph;
    int n_ns = 0, n_fin = 0;
    void mark(int phase) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        (void)hipEventRecord(e, st);
        ev.push_back(e);
        ph.push_back(phase);
    }
    ~PhaseEvents() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

struct LaunchArgs {
    GatherArgs ga;
    BoundsArgs ba;
    NsArgs na;
    InvArgs ia;
    FinishArgs fa;
    ExtractArgs ea;
};

static LaunchArgs make_args(const nolsm_plan *pl, const BatchArgs &b) {
    LaunchArgs A;
    const char *base = (const char *)pl->d_meta;
    const nolsm_solve_opts &o = *b.o;
    GatherArgs &ga = A.ga;
    ga.Krp = (const int32_t *)(base + pl->o_Krp);
    ga.Kci = (const int32_t *)(base + pl->o_Kci);
    ga.Srp = (const int32_t *)(base + pl->o_Srp);
    ga.Sci = (const int32_t *)(base + pl->o_Sci);
    ga.grp_blk = (const int32_t *)(base + pl->o_grp_blk);
    ga.own_pos = (const int32_t *)(base + pl->o_own_pos);
    ga.own_J = (const int32_t *)(base + pl->o_own_J);
    ga.s_fp32 = o.inverse == NOLSM_INV_CHOLESKY_FP32;
    ga.Kval = b.dK;
    ga.Sval = b.dS;
    ga.bs = pl->bs;
    ga.poison_J = o.debug_poison_mol;
    // the Cholesky reads T_J(S) only on and below its diagonal tiles; the
    // symmetric route's substitutions read T_J(K) only on and above them
    ga.s_lower = o.inverse != NOLSM_INV_COUPLED_NS;
    ga.k_upper = o.sym_sign ? 1 : 0;
    ga.pad_ = 0;
    BoundsArgs &ba = A.ba;
    ba.d_mlp = o.d_mlp;
    ba.d_norm = o.d_mlp_norm;
    ba.d_features = o.d_features;
    ba.own_J = (const int32_t *)(base + pl->o_own_J);
    ba.safety = o.mlp_safety > 0 ? o.mlp_safety : 1.05f;
    ba.learned = o.bounds == NOLSM_BOUNDS_LEARNED;
    ba.scale_mult = o.debug_scale_mult;
    ba.sym = o.sym_sign ? 1 : 0;
    ba.pad_ = 0;
    NsArgs &na = A.na;
    na.prec = o.prec;
    na.max_iter = o.max_iter;
    na.fixed_iters = o.fixed_iters;
    na.allow_restart = 1;
    na.tol = nolsm_switch_tol(o.prec, o.n_final_fp32, o.tol);
    na.theta = o.switch_theta > 0 ? o.switch_theta : 0.7;
    na.rmax = o.switch_rmax > 0 ? o.switch_rmax : 0.5;
    na.persistent = o.sched == NOLSM_SCHED_PERSISTENT;
    na.pgrid = pl->pgrid;
    na.sym = o.sym_sign ? 1 : 0;
    na.force_stall = o.debug_force_stall;
    InvArgs &ia = A.ia;
    ia.prec = o.prec;
    ia.max_iter = o.inv_max_iter;
    ia.theta = na.theta;
    ia.rmax = na.rmax;
    ia.own_pos = ga.own_pos;
    ia.bs = pl->bs;
    FinishArgs &fa = A.fa;
    fa.prec = o.prec;
    fa.nfinal = (o.prec == NOLSM_FP16 || o.prec == NOLSM_BF16) ? o.n_final_fp32 : 0;
    fa.rows = o.finish_rows ? 1 : 0;
    fa.pad_ = 0;
    ExtractArgs &ea = A.ea;
    ea.Krp = ga.Krp; ea.Kci = ga.Kci; ea.Srp = ga.Srp; ea.Sci = ga.Sci;
    ea.sub_blk = (const int32_t *)(base + pl->o_sub_blk);
    ea.sub_ptr = (const int32_t *)(base + pl->o_sub_ptr);
    ea.rowpos = (const int32_t *)(base + pl->o_rowpos);
    ea.own_J = (const int32_t *)(base + pl->o_own_J);
    ea.own_pos = ga.own_pos;
    ea.grp_blk = ga.grp_blk;
    ea.scatter_pos = (const int32_t *)(base + pl->o_scatter);
    ea.Kval = b.dK;
    ea.Sval = b.dS;
    ea.Dcols = b.dDcols;
    ea.Dval = b.dD;
    ea.Wcols = o.d_wcols;
    ea.stats = b.dstats;
    ea.bs = pl->bs;
    ea.prec = o.prec;
    ea.nfinal = fa.nfinal;
    ea.sym = o.sym_sign ? 1 : 0;
    ea.L_fp32 = o.inverse == NOLSM_INV_CHOLESKY_FP32;
    return A;
}

// gather, factor / inverse, substitution, bounds and X_0 of one chunk
static int enqueue_setup(const nolsm_plan *pl, const BatchArgs &b, const LaunchArgs &A, const HostChunk &ch,
                         hipStream_t st, PhaseEvents *prof) {
    const nolsm_solve_opts &o = *b.o;
    char *ws = b.ws + ch.base;
    const ChunkDev cd = chunk_dev(pl, ch, ws);
    hipError_t e;
    if (prof) prof->mark(PH_GATHER);
    if ((e = launch_gather(cd, ws, A.ga, st)) != hipSuccess) return hip_fail(e, "gather launch");
    // the FP32 route factors and applies in FP32; the mixed one factors in
    // FP64 and applies the FP32 copy of the factor
    const bool fp32 = o.inverse == NOLSM_INV_CHOLESKY_FP32;
    const bool apply32 = fp32 || o.inverse == NOLSM_INV_CHOLESKY_APPLY_FP32;
    if (o.inverse == NOLSM_INV_COUPLED_NS) {
        if (prof) prof->mark(PH_INV);
        if ((e = launch_inverse(cd, ws, A.ia, st)) != hipSuccess) return hip_fail(e, "inverse launch");
    } else {
        if (prof) prof->mark(PH_CHOL);
        if ((e = launch_chol(cd, ws, fp32, st)) != hipSuccess) return hip_fail(e, "Cholesky launch");
        if (prof) prof->mark(PH_SUBST);
        e = o.sym_sign ? launch_subst_sym(cd, ws, apply32, o.subst_fp32 == 0, st)
                       : launch_subst(cd, ws, apply32, st);
        if (e != hipSuccess) return hip_fail(e, "substitution launch");
    }
    if (prof) prof->mark(PH_BOUNDS);
    if ((e = launch_bounds(cd, ws, A.ba, o.prec, st)) != hipSuccess) return hip_fail(e, "bounds launch");
    return NOLSM_OK;
}

// sign iteration, finishing, extraction and W of one chunk
static int enqueue_solve(const nolsm_plan *pl, const BatchArgs &b, const LaunchArgs &A, const HostChunk &ch,
                         hipStream_t st, PhaseEvents *prof) {
    const nolsm_solve_opts &o = *b.o;
    char *ws = b.ws + ch.base;
    const ChunkDev cd = chunk_dev(pl, ch, ws);
    hipError_t e;
    if (prof) prof->mark(PH_NS);
    for (int it = 0; it < o.max_iter; ++it) {
        e = launch_ns_iter(cd, ws, A.na, it, st);
        if (e != hipSuccess) return hip_fail(e, "Newton-Schulz launch");
    }
    if (prof) prof->mark(PH_FINISH);
    if ((e = launch_finish(cd, ws, A.fa, st)) != hipSuccess) return hip_fail(e, "finish launch");
    if (prof) prof->mark(PH_EXTRACT);
    if ((e = launch_extract(cd, ws, A.ea, st)) != hipSuccess) return hip_fail(e, "extract launch");
    if (A.ea.Wcols) {
        if (prof) prof->mark(PH_WMAT);
        if ((e = launch_wcols(cd, ws, A.ea, st)) != hipSuccess) return hip_fail(e, "W launch");
    }
    if (prof) {
        prof->n_ns += 2 * o.max_iter;
        prof->n_fin += finish_launches(A.fa);
    }
    return NOLSM_OK;
}

// every chunk in turn on one stream
static int enqueue(nolsm_plan *pl, const BatchArgs &b, hipStream_t st, PhaseEvents *prof = nullptr) {
    const LaunchArgs A = make_args(pl, b);
    for (const HostChunk &ch : pl->chunks) {
        int rc = enqueue_setup(pl, b, A, ch, st, prof);
        if (rc == NOLSM_OK) rc = enqueue_solve(pl, b, A, ch, st, prof);
        if (rc != NOLSM_OK) return rc;
    }
    if (prof) prof->mark(PH_END);
    return NOLSM_OK;
}

// Pipeline schedule: the chunks alternate between two workspace regions.
// The setups run in order on the library's stream s2 and the solves in
// order on the call's stream st; solve(c) waits for setup(c), and setup(c)
// for solve(c - 2), the last user of its region. The two streams fork from
// and join back into st, so a capture of st holds all of it.
static int pipe_resources(nolsm_plan *pl) {
    const size_t need = 2 * pl->chunks.size() + 2;
    if (!pl->aux_stream) {
        hipStream_t s2 = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "pipeline stream");
        pl->aux_stream = s2;
    }
    while (pl->events.size() < need) {
        hipEvent_t ev = nullptr;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "pipeline event");
        pl->events.push_back(ev);
    }
    return NOLSM_OK;
}

static int enqueue_pipe(nolsm_plan *pl, const BatchArgs &b, hipStream_t st) {
    int rc = pipe_resources(pl);
    if (rc != NOLSM_OK) return rc;
    const LaunchArgs A = make_args(pl, b);
    hipStream_t s2 = (hipStream_t)pl->aux_stream;
    const size_t nc = pl->chunks.size();
    auto ev = [&](size_t i) { return (hipEvent_t)pl->events[i]; };
    // events: [0, nc) setup done, [nc, 2 nc) solve done, 2 nc fork, 2 nc + 1 join
    hipError_t e;
    if ((e = hipEventRecord(ev(2 * nc), st)) != hipSuccess) return hip_fail(e, "pipeline fork");
    if ((e = hipStreamWaitEvent(s2, ev(2 * nc), 0)) != hipSuccess) return hip_fail(e, "pipeline fork");
    for (size_t c = 0; c < nc; ++c) {
        const HostChunk &ch = pl->chunks[c];
        if (c >= 2 && (e = hipStreamWaitEvent(s2, ev(nc + c - 2), 0)) != hipSuccess) return hip_fail(e, "pipeline wait");
        if ((rc = enqueue_setup(pl, b, A, ch, s2, nullptr)) != NOLSM_OK) return rc;
        if ((e = hipEventRecord(ev(c), s2)) != hipSuccess) return hip_fail(e, "pipeline record");
        if ((e = hipStreamWaitEvent(st, ev(c), 0)) != hipSuccess) return hip_fail(e, "pipeline wait");
        if ((rc = enqueue_solve(pl, b, A, ch, st, nullptr)) != NOLSM_OK) return rc;
        if ((e = hipEventRecord(ev(nc + c), st)) != hipSuccess) return hip_fail(e, "pipeline record");
    }
    if ((e = hipEventRecord(ev(2 * nc + 1), s2)) != hipSuccess) return hip_fail(e, "pipeline join");
    if ((e = hipStreamWaitEvent(st, ev(2 * nc + 1), 0)) != hipSuccess) return hip_fail(e, "pipeline join");
    return NOLSM_OK;
}

static bool same_opts(const nolsm_solve_opts &a, const nolsm_solve_opts &b) {
    return std::memcmp(&a, &b, sizeof(a)) == 0;
}

// argument checks shared by the batch entry points
static int check_batch(const nolsm_plan *pl, const double *dK_val, const double *dS_val,
                       const nolsm_solve_opts *opts, const void *d_ws, size_t ws_bytes, const double *dDcols,
                       const nolsm_mol_stats *dstats) {
    if (!pl || !dK_val || !dS_val || !opts || !d_ws || !dDcols || !dstats) {
        nolsm_set_last_error("sign_batch: null argument");
        return NOLSM_E_ARG;
    }
    if (!pl->bound) { nolsm_set_last_error("sign_batch: plan not bound"); return NOLSM_E_STATE; }
    if (opts->prec != pl->prec || opts->max_iter != pl->max_iter || opts->inverse != pl->inverse ||
        (opts->sym_sign != 0) != (pl->sym != 0) ||
        (pl->inverse == NOLSM_INV_COUPLED_NS && opts->inv_max_iter != pl->inv_max_iter) ||
        ((opts->sched == NOLSM_SCHED_PER_BUCKET) != (pl->sched == NOLSM_SCHED_PER_BUCKET))) {
        nolsm_set_last_error("sign_batch: options differ from the configured ones");
        return NOLSM_E_STATE;
    }
    if (opts->d_wcols && (pl->bs & 1)) {
        nolsm_set_last_error("sign_batch: the energy-weighted output needs an even block size");
        return NOLSM_E_ARG;
    }
    if (opts->sym_sign && opts->d_wcols) {
        nolsm_set_last_error("sign_batch: the energy-weighted output is formed from A_J: it needs sym_sign = 0");
        return NOLSM_E_ARG;
    }
    if (opts->bounds == NOLSM_BOUNDS_LEARNED && (!opts->d_mlp || !opts->d_mlp_norm)) {
        nolsm_set_last_error("sign_batch: learned bounds need d_mlp and d_mlp_norm");
        return NOLSM_E_ARG;
    }
    if (opts->prec != NOLSM_FP64 && opts->prec != NOLSM_FP32 && (opts->n_final_fp32 < 0 || opts->n_final_fp32 > 2)) {
        nolsm_set_last_error("sign_batch: n_final_fp32 must be 0..2");
        return NOLSM_E_ARG;
    }
    if (ws_bytes < pl->ws_bytes) { nolsm_set_last_error("sign_batch: workspace smaller than configured"); return NOLSM_E_WORKSPACE; }
    if (((uintptr_t)d_ws) & 255) { nolsm_set_last_error("sign_batch: workspace must be 256-byte aligned"); return NOLSM_E_ARG; }
    return NOLSM_OK;
}

// mu lives in the workspace header (outside any captured graph), so a
// captured batch serves every mu; the pipeline's second region has a header
// of its own
static int write_headers(const nolsm_plan *pl, char *ws, double mu, hipStream_t st) {
    hipError_t e = launch_set_header(ws, mu, st);
    if (e != hipSuccess) return hip_fail(e, "header launch");
    for (const HostChunk &ch : pl->chunks)
        if (ch.base) {
            e = launch_set_header(ws + ch.base, mu, st);
            if (e != hipSuccess) return hip_fail(e, "header launch");
            break;
        }
    return NOLSM_OK;
}

extern "C" int nolsm_sign_batch(nolsm_plan *pl, const double *dK_val, const double *dS_val, double mu,
                                const nolsm_solve_opts *opts, void *d_ws, size_t ws_bytes, double *dDcols,
                                double *dD_val, nolsm_mol_stats *dstats, void *stream) {
    int rc = check_batch(pl, dK_val, dS_val, opts, d_ws, ws_bytes, dDcols, dstats);
    if (rc != NOLSM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    BatchArgs b{dK_val, dS_val, mu, opts, (char *)d_ws, dDcols, dD_val, (void *)dstats};
    if ((rc = write_headers(pl, (char *)d_ws, mu, st)) != NOLSM_OK) return rc;
    if (opts->profile) {
        PhaseEvents pe;
        pe.st = st;
        rc = enqueue(pl, b, st, &pe);
        if (rc != NOLSM_OK) return rc;
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "profile sync");
        nolsm_profile p = {};
        double *slot[] = {&p.ms_gather, &p.ms_chol,   &p.ms_subst, &p.ms_bounds,  &p.ms_ns,
                          &p.ms_finish, &p.ms_extract, &p.ms_wmat, &p.ms_inverse};
        for (size_t i = 0; i + 1 < pe.ev.size(); ++i) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pe.ev[i], pe.ev[i + 1]) == hipSuccess && pe.ph[i] < PH_END) *slot[pe.ph[i]] += ms;
        }
        float tot = 0.f;
        if (pe.ev.size() >= 2) (void)hipEventElapsedTime(&tot, pe.ev.front(), pe.ev.back());
        p.ms_total = tot;
        p.valid = 1;
        p.nchunks = (int32_t)pl->chunks.size();
        p.n_ns_launches = pe.n_ns;
        p.n_fin_launches = pe.n_fin;
        pl->prof = p;
    } else if ((opts->sched == NOLSM_SCHED_GRAPH || opts->sched == NOLSM_SCHED_PERSISTENT ||
                opts->sched == NOLSM_SCHED_PIPELINE) && st != nullptr) {
        const void *key[6] = {dK_val, dS_val, d_ws, dDcols, dD_val, dstats};
        bool hit = pl->graph_exec && pl->g_stream == stream && same_opts(pl->g_opts, *opts);
        for (int i = 0; i < 6 && hit; ++i) hit = pl->g_key[i] == key[i];
        if (!hit) {
            drop_graph(pl);
            hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return hip_fail(e, "graph capture begin");
            rc = opts->sched == NOLSM_SCHED_PIPELINE ? enqueue_pipe(pl, b, st) : enqueue(pl, b, st);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(st, &g);
            if (rc != NOLSM_OK) {
                if (g) (void)hipGraphDestroy(g);
                return rc;
            }
            if (e != hipSuccess) return hip_fail(e, "graph capture end");
            hipGraphExec_t ex = nullptr;
            e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return hip_fail(e, "graph instantiate");
            pl->graph_exec = ex;
            for (int i = 0; i < 6; ++i) pl->g_key[i] = key[i];
            pl->g_mu = mu;
            pl->g_opts = *opts;
            pl->g_stream = stream;
        }
        hipError_t e = hipGraphLaunch((hipGraphExec_t)pl->graph_exec, st);
        if (e != hipSuccess) return hip_fail(e, "graph launch");
        rc = NOLSM_OK;
    } else {
        rc = enqueue(pl, b, st);
        if (rc != NOLSM_OK) return rc;
    }
    if (opts->sync_errors) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "sync");
        std::vector<nolsm_mol_stats> hs(pl->nb);
        e = hipMemcpy(hs.data(), dstats, sizeof(nolsm_mol_stats) * pl->nb, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "stats read-back");
        for (const auto &s : hs) {
            if (s.status == NOLSM_MOL_NOT_SPD) { nolsm_set_last_error("molecule not SPD"); return NOLSM_E_NOT_SPD; }
        }
        for (const auto &s : hs) {
            if (s.status == NOLSM_MOL_NOCONV) { nolsm_set_last_error("molecule did not converge"); return NOLSM_E_NOCONV; }
        }
    }
    return NOLSM_OK;
}

// ------------------------------------------------- allocation-free variant
// The workspace of nolsm_sign_batch_noalloc: a device array of the library.
// Every GPU the library runs on holds its own copy, at its own address, from
// the load of the library's code until the process ends. In host code the
// name is a stand-in, not a device address: kernels get the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) char scratch[NOLSM_NOALLOC_WS_BYTES];

#define NOLSM_NOALLOC_MAX_DEVICES 64
static std::mutex scratch_mu;
static char *scratch_ptr[NOLSM_NOALLOC_MAX_DEVICES];

// device address of `scratch` on device `dev`, looked up once per device with
// that device current
static int scratch_address(int dev, char **out) {
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch symbol address");
        if (!p || ((uintptr_t)p & 255)) {
            nolsm_set_last_error("sign_batch_noalloc: scratch address not 256-byte aligned");
            return NOLSM_E_HIP;
        }
        scratch_ptr[dev] = (char *)p;
    }
    *out = scratch_ptr[dev];
    return NOLSM_OK;
}

extern "C" int nolsm_sign_batch_noalloc(nolsm_plan *pl, const double *dK_val, const double *dS_val, double mu,
                                        const nolsm_solve_opts *opts, double *dDcols, double *dD_val,
                                        nolsm_mol_stats *dstats, void *stream) {
    if (!pl || !opts) {
        nolsm_set_last_error("sign_batch_noalloc: null argument");
        return NOLSM_E_ARG;
    }
    if (pl->configured && pl->ws_bytes > (size_t)NOLSM_NOALLOC_WS_BYTES) {
        nolsm_set_last_error("sign_batch_noalloc: the plan is configured for a workspace of " +
                             std::to_string((unsigned long long)pl->ws_bytes) + " bytes, above the " +
                             std::to_string((unsigned long long)NOLSM_NOALLOC_WS_BYTES) +
                             " bytes of the library's scratch array");
        return NOLSM_E_WORKSPACE;
    }
    if (opts->sched == NOLSM_SCHED_PIPELINE || opts->profile || opts->sync_errors) {
        nolsm_set_last_error("sign_batch_noalloc: launches directly on the call's stream only "
                             "(no pipeline schedule, profile or sync_errors)");
        return NOLSM_E_ARG;
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    if (dev < 0 || dev >= NOLSM_NOALLOC_MAX_DEVICES) {
        nolsm_set_last_error("sign_batch_noalloc: device index out of range");
        return NOLSM_E_ARG;
    }
    if (pl->bound && dev != pl->device) {
        nolsm_set_last_error("sign_batch_noalloc: current device differs from the one the plan is bound on");
        return NOLSM_E_STATE;
    }
    char *ws = nullptr;
    int rc = scratch_address(dev, &ws);
    if (rc != NOLSM_OK) return rc;
    rc = check_batch(pl, dK_val, dS_val, opts, ws, (size_t)NOLSM_NOALLOC_WS_BYTES, dDcols, dstats);
    if (rc != NOLSM_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    BatchArgs b{dK_val, dS_val, mu, opts, ws, dDcols, dD_val, (void *)dstats};
    if ((rc = write_headers(pl, ws, mu, st)) != NOLSM_OK) return rc;
    // every kernel initialises the workspace state it reads (control blocks,
    // queue counters, residual partials) within the call, so contents left by
    // an earlier call are never read
    return enqueue(pl, b, st);
}

extern "C" int nolsm_trace_sums(const nolsm_plan *pl, const nolsm_mol_stats *dstats, void *d_ws,
                                double *sums_out, void *stream) {
    if (!pl || !dstats || !d_ws || !sums_out) return NOLSM_E_ARG;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = launch_trace_sums(dstats, pl->nb, (char *)d_ws, st);
    if (e != hipSuccess) return hip_fail(e, "trace-sum launch");
    WsHeader h;
    e = hipMemcpyAsync(&h, d_ws, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "trace-sum read-back");
    sums_out[0] = h.sumN;
    sums_out[1] = h.sumE;
    sums_out[2] = (double)h.n_bad;
    return NOLSM_OK;
}

// Chemical-potential bisection: the paper fixes mu for charge neutrality by
// a bisection-like outer loop (Sec. IV-A, simulation details). Each step is a
// full batched solve (the same captured graph, mu from the workspace header)
// followed by the FP64 trace sum sum_J N_J; the interval halves towards
// sum_J N_J = n_target.
extern "C" int nolsm_mu_bisect(nolsm_plan *pl, const double *dK_val, const double *dS_val, double mu_lo,
                               double mu_hi, double n_target, double tol_count, int32_t max_steps,
                               const nolsm_solve_opts *opts, void *d_ws, size_t ws_bytes, double *dDcols,
                               double *dD_val, nolsm_mol_stats *dstats, void *stream, double *mu_out,
                               double *count_out, int32_t *steps_out) {
    if (!pl || !mu_out || !count_out || !(mu_hi > mu_lo) || max_steps < 1 || !(tol_count > 0)) {
        nolsm_set_last_error("mu_bisect: bad argument");
        return NOLSM_E_ARG;
    }
    double lo = mu_lo, hi = mu_hi, mu = 0.5 * (lo + hi), cnt = 0.0, n_bad = 0.0;
    int32_t step = 0;
    for (step = 1; step <= max_steps; ++step) {
        mu = 0.5 * (lo + hi);
        int rc = nolsm_sign_batch(pl, dK_val, dS_val, mu, opts, d_ws, ws_bytes, dDcols, dD_val, dstats, stream);
        if (rc != NOLSM_OK) return rc;
        double sums[3];
        rc = nolsm_trace_sums(pl, dstats, d_ws, sums, stream);
        if (rc != NOLSM_OK) return rc;
        cnt = sums[0];
        n_bad = sums[2];
        if (std::fabs(cnt - n_target) <= tol_count) break;
        if (cnt < n_target) lo = mu; else hi = mu;
    }
    *mu_out = mu;
    *count_out = cnt;
    if (steps_out) *steps_out = step > max_steps ? max_steps : step;
    if (std::fabs(cnt - n_target) > tol_count) {
        nolsm_set_last_error("mu_bisect: electron count not reached within max_steps");
        return NOLSM_E_NOCONV;
    }
    // the count of the final solve includes molecules whose sign iteration
    // did not meet its stop rule (a mu inside a band converges slowly): the
    // result is returned, but not as a converged one
    if (n_bad > 0.0) {
        nolsm_set_last_error("mu_bisect: " + std::to_string((long long)n_bad) +
                             " molecules not converged (or not SPD) at the final mu");
        return NOLSM_E_NOCONV;
    }
    return NOLSM_OK;
}

extern "C" int nolsm_assemble_D(const nolsm_plan *pl, const double *dDcols, double *dD_val, void *stream) {
    if (!pl || !dDcols || !dD_val) return NOLSM_E_ARG;
    if (!pl->bound) return NOLSM_E_STATE;
    const int32_t *sp = (const int32_t *)((const char *)pl->d_meta + pl->o_scatter);
    hipError_t e = launch_assemble(dDcols, dD_val, sp, (int64_t)pl->sub_blk.size(), pl->bs, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "assemble launch");
    return NOLSM_OK;
}

extern "C" int nolsm_profile_last(const nolsm_plan *pl, nolsm_profile *out) {
    if (!pl || !out) return NOLSM_E_ARG;
    *out = pl->prof;
    return NOLSM_OK;
}

extern "C" void nolsm_plan_destroy(nolsm_plan *pl) {
    if (!pl) return;
    drop_graph(pl);
    for (void *ev : pl->events) (void)hipEventDestroy((hipEvent_t)ev);
    if (pl->aux_stream) (void)hipStreamDestroy((hipStream_t)pl->aux_stream);
    delete pl;
}
