// Batched marches: many independent instances of Eq. (1), each with its own
// grid (Nx, D, Delta) and packet, advanced together.  Launch k of the batch
// runs launch k of every instance that still needs one (block_rows), so one
// kernel launch carries hundreds of instances; the whole launch sequence is
// captured once in a HIP graph and replayed.  The instances can be dealt to
// up to MAXG groups marched concurrently on their own streams, each its own
// launch sequence and graph, so that one group's launches fill the tails of
// the others'.  The autotuner below picks the row-block cap, the workgroup width
// and the number of groups by timing a prefix of the march.

#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "fdtd_common.h"

constexpr int MAXG = 4;              // concurrently marched groups (streams) at most

struct fdtd_batch {
    int n = 0;
    std::vector<fdtd_ctx*> c;        // per instance, in the caller's order
    std::vector<int> order;          // instance ids, most launches first
    int G = 1;                       // groups marched concurrently (1 .. MAXG)
    std::vector<int> grp;            // per instance: its group
    int gbeg[MAXG + 1] = {};         // group g holds table entries gbeg[g] .. gbeg[g+1]-1
    std::vector<BInst> h_tab;        // device table contents (by group, each sorted by launches)
    BInst* d_tab = nullptr;          // in the workspace
    OdeInst* d_ode = nullptr;        // delay-equation boundary records of those instances that use it
    int n_ode = 0;
    OdeTab* d_otab = nullptr;        // every instance's delay-equation step weights
    int* d_stat = nullptr;           // every instance's status word, gathered for one copy
    ChiJob* d_jobs = nullptr;        // chi snapshots, by group, sorted by the launch after which they are taken
    int* d_status = nullptr;         // the batch's status word (non-finite values in any instance's march)
    std::vector<int> job_begin[MAXG];    // per group and launch k: first job, one past the last at k+1
    int job_off[MAXG] = {};          // the group's first job in d_jobs
    int64_t chi_ntau = 0;
    std::vector<int> n_active[MAXG];     // per group and launch k: instances still marching
    std::vector<int> nb[MAXG];       // per group and launch k: workgroups launched (multiple of 8)
    int64_t L[MAXG] = {};            // launches of each group
    int64_t Lmax = 0;                // launches of the longest group
    hipStream_t stream = nullptr;    // the caller's stream (group 0)
    hipStream_t side[MAXG] = {};     // private streams of groups 1 .. G-1 (default priority)
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[MAXG] = {};
    hipStream_t cap[MAXG] = {};      // private streams the graphs are captured on
    hipGraph_t graph[MAXG] = {};
    hipGraphExec_t exec[MAXG] = {};
    fdtd_batch_opts o;
    int state = 0;                   // 0: no boundary, 1: ready to march, 2: marched
    char err[512];
};

static char g_berr[512];

static int bfail(fdtd_batch* b, int code, const char* fmt, ...)
{
    char* dst = b ? b->err : g_berr;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(dst, 512, fmt, ap);
    va_end(ap);
    return code;
}

static int64_t al256(int64_t n) { return (n + 255) & ~(int64_t)255; }

static int opts_check(const fdtd_batch_opts* o, fdtd_batch_opts* out, char* why, size_t n)
{
    fdtd_batch_opts d;
    memset(&d, 0, sizeof d);
    d.struct_size = sizeof(fdtd_batch_opts);
    d.tmax = BM_TMAX;
    d.wmax = BM_CAP;
    d.use_graph = 1;
    d.groups = 1;
    if (o) {
        if (o->struct_size != sizeof(fdtd_batch_opts)) {
            snprintf(why, n, "opts struct_size %u, expected %zu", o->struct_size, sizeof(fdtd_batch_opts));
            return FDTD_EINVAL;
        }
        if (o->tmax < 0 || o->tmax > BM_TMAX) { snprintf(why, n, "tmax must be 0..%d", BM_TMAX); return FDTD_EINVAL; }
        if (o->wmax < 0) { snprintf(why, n, "wmax must be >= 0"); return FDTD_EINVAL; }
        if (o->use_graph != 0 && o->use_graph != 1) { snprintf(why, n, "use_graph must be 0 or 1"); return FDTD_EINVAL; }
        if (o->groups < 0 || o->groups > MAXG) { snprintf(why, n, "groups must be 0..%d", MAXG); return FDTD_EINVAL; }
        if (o->tmax) d.tmax = o->tmax;
        if (o->wmax) d.wmax = o->wmax < BM_CAP ? o->wmax : BM_CAP;
        d.use_graph = o->use_graph;
        if (o->groups) d.groups = o->groups;
    }
    *out = d;
    return FDTD_OK;
}

static PlanKnobs knobs_of(const fdtd_batch_opts& o)
{
    PlanKnobs k;
    k.ncu = 1;              // the widest workgroups: the batch, not one instance, fills the chip
    k.tmax = o.tmax;
    k.wmax = o.wmax;
    k.stream_ok = 0;        // measured: ordinary ring stores are faster for batches of small instances
    return k;
}

static int batch_bytes(const fdtd_params* p, int32_t n, const fdtd_batch_opts& o, int64_t* total, char* why,
                       size_t nwhy)
{
    const PlanKnobs kn = knobs_of(o);
    int64_t t = al256((int64_t)n * (int64_t)sizeof(BInst)) + al256((int64_t)n * (int64_t)sizeof(OdeInst)) +
                al256((int64_t)n * (int64_t)sizeof(ChiJob)) + 256 + al256((int64_t)n * (int64_t)sizeof(OdeTab)) +
                al256((int64_t)n * (int64_t)sizeof(int));
    for (int i = 0; i < n; ++i) {
        int rc = ctx_validate(&p[i], kn, why, nwhy);
        if (!rc && p[i].identical_photons == 0) {
            snprintf(why, nwhy, "two different photons (identical_photons = 0) are marched one instance at a time");
            rc = FDTD_EINVAL;
        }
        if (!rc && p[i].read_mode != FDTD_READ_EXACT) {
            snprintf(why, nwhy, "FDTD_READ_PAPER_DIAG is marched one instance at a time");
            rc = FDTD_EINVAL;
        }
        if (rc) {
            char tmp[256];
            snprintf(tmp, sizeof tmp, "instance %d: %s", i, why);
            snprintf(why, nwhy, "%s", tmp);
            return rc;
        }
        t += al256(ctx_bytes(&p[i], kn));
    }
    *total = t;
    return FDTD_OK;
}

static void destroy(fdtd_batch* b)
{
    if (!b) return;
    for (int g = 0; g < MAXG; ++g) {
        if (b->exec[g]) (void)hipGraphExecDestroy(b->exec[g]);
        if (b->graph[g]) (void)hipGraphDestroy(b->graph[g]);
        if (b->cap[g]) (void)hipStreamDestroy(b->cap[g]);
        if (b->side[g]) (void)hipStreamDestroy(b->side[g]);
        if (b->ev_join[g]) (void)hipEventDestroy(b->ev_join[g]);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (fdtd_ctx* c : b->c) fdtd_destroy(c);
    delete b;
}

// launches k0 .. k1-1 of group g on stream s, each followed by the chi
// snapshots whose row it completes; a march that reaches the group's last
// launch ends with the non-finite check of its instances
static int enqueue_group(fdtd_batch* b, int g, int64_t k0, int64_t k1, hipStream_t s)
{
    const BInst* tab = b->d_tab + b->gbeg[g];
    for (int64_t k = k0; k < k1 && k < b->L[g]; ++k) {
        int rc = launch_block_batch(tab, b->n_active[g][k], k, b->nb[g][k], s);
        if (rc) return rc;
        if (!b->job_begin[g].empty()) {
            const int j0 = b->job_begin[g][k], j1 = b->job_begin[g][k + 1];
            rc = launch_chi_batch(b->d_jobs + b->job_off[g] + j0, j1 - j0, b->chi_ntau, s);
            if (rc) return rc;
        }
    }
    if (k1 >= b->L[g]) return launch_check_batch(tab, b->gbeg[g + 1] - b->gbeg[g], b->d_status, s);
    return FDTD_OK;
}

// groups 1 .. G-1 on their private streams, forked from s and joined back into it
static int fork_side(fdtd_batch* b, hipStream_t s)
{
    if (b->G == 1) return FDTD_OK;
    if (hipEventRecord(b->ev_fork, s) != hipSuccess) return FDTD_EDEVICE;
    for (int g = 1; g < b->G; ++g)
        if (hipStreamWaitEvent(b->side[g], b->ev_fork, 0) != hipSuccess) return FDTD_EDEVICE;
    return FDTD_OK;
}

static int join_side(fdtd_batch* b, hipStream_t s)
{
    int rc = FDTD_OK;
    for (int g = 1; g < b->G; ++g) {
        if (hipEventRecord(b->ev_join[g], b->side[g]) != hipSuccess ||
            hipStreamWaitEvent(s, b->ev_join[g], 0) != hipSuccess)
            rc = FDTD_EDEVICE;
    }
    return rc;
}

// launches k0 .. k1-1 of every group, plain launches
static int enqueue(fdtd_batch* b, int64_t k0, int64_t k1, hipStream_t s)
{
    int rc = fork_side(b, s);
    if (rc) return rc;
    for (int g = b->G - 1; g >= 1 && !rc; --g) rc = enqueue_group(b, g, k0, k1, b->side[g]);
    if (!rc) rc = enqueue_group(b, 0, k0, k1, s);
    const int rj = join_side(b, s);
    return rc ? rc : rj;
}

static void drop_graph(fdtd_batch* b)
{
    for (int g = 0; g < MAXG; ++g) {
        if (b->exec[g]) (void)hipGraphExecDestroy(b->exec[g]);
        if (b->graph[g]) (void)hipGraphDestroy(b->graph[g]);
        b->exec[g] = nullptr;
        b->graph[g] = nullptr;
    }
}

extern "C" {

int fdtd_batch_workspace_size(const fdtd_params* p, int32_t n, const fdtd_batch_opts* opts, size_t* bytes)
{
    char why[320];
    if (!p || n < 1 || !bytes) return bfail(nullptr, FDTD_EINVAL, "params, n >= 1 and bytes are required");
    fdtd_batch_opts o;
    int rc = opts_check(opts, &o, why, sizeof why);
    if (rc) return bfail(nullptr, rc, "%s", why);
    int64_t t = 0;
    rc = batch_bytes(p, n, o, &t, why, sizeof why);
    if (rc) return bfail(nullptr, rc, "%s", why);
    *bytes = (size_t)t;
    return FDTD_OK;
}

int fdtd_batch_init(const fdtd_params* p, int32_t n, const fdtd_batch_opts* opts, void* d_workspace, size_t bytes,
                    void* hip_stream, fdtd_batch** out)
{
    char why[320];
    if (!out) return bfail(nullptr, FDTD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p || n < 1 || n > 65535) return bfail(nullptr, FDTD_EINVAL, "params and 1 <= n <= 65535 are required");
    fdtd_batch_opts o;
    int rc = opts_check(opts, &o, why, sizeof why);
    if (rc) return bfail(nullptr, rc, "%s", why);
    int64_t total = 0;
    rc = batch_bytes(p, n, o, &total, why, sizeof why);
    if (rc) return bfail(nullptr, rc, "%s", why);
    if (!d_workspace || bytes < (size_t)total)
        return bfail(nullptr, FDTD_ESIZE, "workspace of %zu bytes is smaller than the %lld needed", bytes,
                     (long long)total);
    if (((uintptr_t)d_workspace) & 255) return bfail(nullptr, FDTD_EINVAL, "workspace must be 256-byte aligned");

    fdtd_batch* b = new fdtd_batch();
    b->n = n;
    b->o = o;
    b->stream = (hipStream_t)hip_stream;
    const PlanKnobs kn = knobs_of(o);
    char* base = (char*)d_workspace;
    b->d_tab = (BInst*)base;
    int64_t off = al256((int64_t)n * (int64_t)sizeof(BInst));
    b->d_ode = (OdeInst*)(base + off);
    off += al256((int64_t)n * (int64_t)sizeof(OdeInst));
    b->d_jobs = (ChiJob*)(base + off);
    off += al256((int64_t)n * (int64_t)sizeof(ChiJob));
    b->d_status = (int*)(base + off);
    off += 256;
    b->d_otab = (OdeTab*)(base + off);
    off += al256((int64_t)n * (int64_t)sizeof(OdeTab));
    b->d_stat = (int*)(base + off);
    off += al256((int64_t)n * (int64_t)sizeof(int));
    // contexts set up on the host only; the device side follows in bulk
    std::vector<OdeTab> otab(n);
    std::vector<OdeInst> oinst(n);
    for (int i = 0; i < n; ++i) {
        const int64_t sz = ctx_bytes(&p[i], kn);
        fdtd_ctx* c = nullptr;
        const CtxDefer df = {b->d_otab + i, &otab[i], &oinst[i]};
        rc = ctx_create(&p[i], kn, base + off, (size_t)sz, b->stream, &c, why, sizeof why, &df);
        if (rc) {
            destroy(b);
            return bfail(nullptr, rc, "instance %d: %s", i, why);
        }
        b->c.push_back(c);
        off += al256(sz);
    }

    // sort by launch count, most first: the instances active in launch k are then a prefix
    std::vector<int64_t> L(n);
    for (int i = 0; i < n; ++i) {
        const int64_t T = b->c[i]->plan.T, Nt = b->c[i]->p.Nt;
        L[i] = 1 + (Nt + T - 1) / T;
        b->order.push_back(i);
    }
    std::stable_sort(b->order.begin(), b->order.end(), [&](int x, int y) { return L[x] > L[y]; });
    // groups: instance q of that order goes to group q mod G, so each group
    // stays sorted and the groups carry alike work
    b->G = o.groups < n ? o.groups : n;
    b->grp.assign(n, 0);
    std::vector<int> tab_order;
    for (int g = 0; g < b->G; ++g) {
        b->gbeg[g] = (int)tab_order.size();
        for (int q = g; q < n; q += b->G) {
            tab_order.push_back(b->order[q]);
            b->grp[b->order[q]] = g;
        }
    }
    b->gbeg[b->G] = n;
    for (int g = 0; g < b->G; ++g) {
        const int q0 = b->gbeg[g], q1 = b->gbeg[g + 1];
        int64_t wg = 0;
        std::vector<int64_t> wg_end;
        for (int q = q0; q < q1; ++q) {
            const fdtd_ctx* c = b->c[tab_order[q]];
            BInst e;
            memset(&e, 0, sizeof e);
            e.g = c->g;
            e.b = c->b;
            e.P = c->plan;
            e.wg_begin = wg;
            e.launches = L[tab_order[q]];
            e.index = tab_order[q];
            wg += c->plan.nwg;
            wg_end.push_back(wg);
            b->h_tab.push_back(e);
        }
        b->L[g] = b->h_tab[q0].launches;
        b->n_active[g].resize(b->L[g]);
        b->nb[g].resize(b->L[g]);
        int q = q1 - q0;
        for (int64_t k = 0; k < b->L[g]; ++k) {
            while (q > 0 && b->h_tab[q0 + q - 1].launches <= k) --q;
            b->n_active[g][k] = q;
            const int64_t w = wg_end[q - 1];
            if (w > (int64_t)0x7fffffff - 8) {
                destroy(b);
                return bfail(nullptr, FDTD_EINVAL, "too many workgroups in one launch");
            }
            b->nb[g][k] = (int)(((w + 7) / 8) * 8);
        }
    }
    b->Lmax = b->L[0];
    if (b->G > 1) {
        hipError_t he = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
        for (int g = 1; g < b->G && he == hipSuccess; ++g) {
            he = hipStreamCreateWithFlags(&b->side[g], hipStreamNonBlocking);
            if (he == hipSuccess) he = hipEventCreateWithFlags(&b->ev_join[g], hipEventDisableTiming);
        }
        if (he != hipSuccess) {
            destroy(b);
            return bfail(nullptr, FDTD_EDEVICE, "stream or event creation failed: %s", hipGetErrorString(he));
        }
    }
    // delay-equation boundaries: one workgroup each in one launch, longest first
    std::vector<OdeInst> ode;
    for (int q2 = 0; q2 < n; ++q2) {
        const int i = b->order[q2];
        if (b->c[i]->p.boundary != FDTD_E_DELAY_ODE) continue;
        b->c[i]->d_ode = b->d_ode + ode.size();
        ode.push_back(oinst[i]);
    }
    b->n_ode = (int)ode.size();
    hipError_t e = hipMemcpyAsync(b->d_tab, b->h_tab.data(), (size_t)n * sizeof(BInst), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_otab, otab.data(), (size_t)n * sizeof(OdeTab), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess && b->n_ode)
        e = hipMemcpyAsync(b->d_ode, ode.data(), ode.size() * sizeof(OdeInst), hipMemcpyHostToDevice, b->stream);
    // rows before t = 0 are read as zeros: every ring and diagonal copy cleared
    if (e == hipSuccess && launch_clear_batch(b->d_tab, n, b->stream)) e = hipErrorLaunchFailure;
    if (e == hipSuccess && launch_clear_status(b->d_status, b->stream)) e = hipErrorLaunchFailure;
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        destroy(b);
        return bfail(nullptr, FDTD_EDEVICE, "copy of the instance table failed: %s", hipGetErrorString(e));
    }
    *out = b;
    return FDTD_OK;
}

int fdtd_batch_set_boundary(fdtd_batch* b)
{
    if (!b) return bfail(nullptr, FDTD_EINVAL, "batch is NULL");
    b->state = 0;
    if (launch_clear_status(b->d_status, b->stream)) return bfail(b, FDTD_EDEVICE, "status clear failed");
    for (int i = 0; i < b->n; ++i) {
        fdtd_ctx* c = b->c[i];
        c->boundary_ready = 0;
        if (c->p.boundary == FDTD_E_DELAY_ODE) continue;
        int rc = ctx_boundary_enqueue(c);
        if (rc) return bfail(b, rc, "instance %d: %s", i, fdtd_last_error(c));
    }
    // the delay-equation boundaries of all instances at once; e0 and mu of
    // stimulated emission instance by instance after them
    if (b->n_ode && launch_boundary_batch(b->d_ode, b->n_ode, b->stream))
        return bfail(b, FDTD_EDEVICE, "delay-equation boundary launch failed");
    for (int i = 0; i < b->n; ++i) {
        fdtd_ctx* c = b->c[i];
        if (c->p.boundary != FDTD_E_DELAY_ODE || !c->E0) continue;
        if (launch_e0(c) || launch_mu_rows(c, 0, 0, c->stream))
            return bfail(b, FDTD_EDEVICE, "instance %d: boundary launch failed", i);
    }
    std::vector<int> st(b->n, 0);
    if (launch_gather_status(b->d_tab, b->n, b->d_stat, b->stream))
        return bfail(b, FDTD_EDEVICE, "status gather failed");
    hipError_t e = hipMemcpyAsync(st.data(), b->d_stat, (size_t)b->n * sizeof(int), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, "boundary kernels failed: %s", hipGetErrorString(e));
    for (int i = 0; i < b->n; ++i) {
        int rc = ctx_boundary_status(b->c[i], st[i]);
        if (rc) return bfail(b, rc, "instance %d: %s", i, fdtd_last_error(b->c[i]));
    }
    b->state = 1;
    return FDTD_OK;
}

int fdtd_batch_march(fdtd_batch* b)
{
    if (!b) return bfail(nullptr, FDTD_EINVAL, "batch is NULL");
    if (b->state != 1) return bfail(b, FDTD_ESTATE, "march needs a fresh boundary (fdtd_batch_set_boundary)");
    if (b->o.use_graph) {
        for (int g = 0; g < b->G; ++g) {
            if (b->exec[g]) continue;
            hipError_t e = b->cap[g] ? hipSuccess : hipStreamCreateWithFlags(&b->cap[g], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipStreamBeginCapture(b->cap[g], hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
            int rc = enqueue_group(b, g, 0, b->L[g], b->cap[g]);
            e = hipStreamEndCapture(b->cap[g], &b->graph[g]);
            if (rc || e != hipSuccess)
                return bfail(b, FDTD_EDEVICE, "graph capture failed: %s", hipGetErrorString(hipGetLastError()));
            e = hipGraphInstantiate(&b->exec[g], b->graph[g], nullptr, nullptr, 0);
            if (e != hipSuccess) {
                b->exec[g] = nullptr;
                return bfail(b, FDTD_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
            }
        }
        int rc = fork_side(b, b->stream);
        hipError_t e = rc ? hipErrorLaunchFailure : hipSuccess;
        for (int g = b->G - 1; g >= 1 && e == hipSuccess; --g) e = hipGraphLaunch(b->exec[g], b->side[g]);
        if (e == hipSuccess) e = hipGraphLaunch(b->exec[0], b->stream);
        if (join_side(b, b->stream) && e == hipSuccess) e = hipErrorLaunchFailure;
        if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, "graph launch failed: %s", hipGetErrorString(e));
    } else {
        int rc = enqueue(b, 0, b->Lmax, b->stream);
        if (rc) return bfail(b, rc, "march launch failed: %s", hipGetErrorString(hipGetLastError()));
    }
    for (fdtd_ctx* c : b->c) {
        c->row = c->p.Nt;
        c->strip_row = c->p.Nt;
    }
    b->state = 2;
    return FDTD_OK;
}

int fdtd_batch_readout(fdtd_batch* b, int32_t i, int32_t what, int64_t arg, void* dst, int64_t count,
                       int32_t dst_on_device)
{
    if (!b) return bfail(nullptr, FDTD_EINVAL, "batch is NULL");
    if (i < 0 || i >= b->n) return bfail(b, FDTD_EINVAL, "instance %d out of 0..%d", i, b->n - 1);
    int rc = fdtd_readout(b->c[i], what, arg, dst, count, dst_on_device);
    if (rc) return bfail(b, rc, "instance %d: %s", i, fdtd_last_error(b->c[i]));
    return FDTD_OK;
}

int fdtd_batch_set_chi(fdtd_batch* b, const int64_t* rows, const int64_t* strides, int64_t n_tau, void* d_out)
{
    if (!b) return bfail(nullptr, FDTD_EINVAL, "batch is NULL");
    drop_graph(b);
    for (int g = 0; g < MAXG; ++g) b->job_begin[g].clear();
    b->chi_ntau = 0;
    if (!rows) return FDTD_OK;                        // snapshots off
    if (!strides || n_tau < 1 || !d_out) return bfail(b, FDTD_EINVAL, "strides, n_tau >= 1 and d_out are required");
    std::vector<ChiJob> jobs;
    std::vector<int64_t> kstar;
    std::vector<int> jg;
    for (int i = 0; i < b->n; ++i) {
        const fdtd_ctx* c = b->c[i];
        if (rows[i] < 0) continue;
        if (rows[i] > c->p.Nt || strides[i] < 1)
            return bfail(b, FDTD_EINVAL, "instance %d: snapshot row %lld outside 0..Nt or stride < 1", i,
                         (long long)rows[i]);
        ChiJob j;
        memset(&j, 0, sizeof j);
        j.g = c->g;
        j.b = c->b;
        j.c0 = chi0_coefficient(&c->p);
        j.row = rows[i];
        j.stride = strides[i];
        j.n_tau = n_tau;
        j.dst = (cd*)d_out + (int64_t)i * n_tau;
        jobs.push_back(j);
        // the first launch after which row `row` is complete in every column
        kstar.push_back(rows[i] == 0 ? 0 : (rows[i] + c->plan.T - 1) / c->plan.T);
        jg.push_back(b->grp[i]);
    }
    // by group, then by the launch after which the snapshot is taken
    std::vector<int> idx(jobs.size());
    for (size_t q = 0; q < idx.size(); ++q) idx[q] = (int)q;
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
        return jg[x] != jg[y] ? jg[x] < jg[y] : kstar[x] < kstar[y];
    });
    std::vector<ChiJob> sorted;
    for (int q : idx) sorted.push_back(jobs[q]);
    int off = 0;
    for (int g = 0; g < b->G; ++g) {
        b->job_off[g] = off;
        b->job_begin[g].assign(b->L[g] + 1, 0);
        for (int q : idx)
            if (jg[q] == g) b->job_begin[g][kstar[q] + 1]++;
        for (int64_t k = 0; k < b->L[g]; ++k) b->job_begin[g][k + 1] += b->job_begin[g][k];
        off += b->job_begin[g][b->L[g]];
    }
    b->chi_ntau = n_tau;
    if (!sorted.empty()) {
        hipError_t e = hipMemcpyAsync(b->d_jobs, sorted.data(), sorted.size() * sizeof(ChiJob),
                                      hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, "copy of the snapshot table failed: %s", hipGetErrorString(e));
    }
    return FDTD_OK;
}

int fdtd_batch_sample_pe(fdtd_batch* b, int64_t n_samples, const double* d_t_end, double* d_out)
{
    if (!b) return bfail(nullptr, FDTD_EINVAL, "batch is NULL");
    if (b->state != 2) return bfail(b, FDTD_ESTATE, "sample P_e after a march");
    if (n_samples < 1 || !d_out) return bfail(b, FDTD_EINVAL, "n_samples >= 1 and d_out are required");
    int rc = launch_pe_sample_batch(b->d_tab, b->n, n_samples, d_t_end, d_out, b->stream);
    return rc ? bfail(b, rc, "launch failed") : FDTD_OK;
}

int fdtd_batch_info(const fdtd_batch* b, int64_t* launches, int64_t* max_workgroups)
{
    if (!b) return FDTD_EINVAL;
    if (launches) *launches = b->Lmax;
    if (max_workgroups) {
        int64_t w = 0;
        for (int g = 0; g < b->G; ++g) w += b->nb[g].empty() ? 0 : b->nb[g][0];
        *max_workgroups = w;
    }
    return FDTD_OK;
}

int fdtd_batch_sync(fdtd_batch* b)
{
    if (!b) return bfail(nullptr, FDTD_EINVAL, "batch is NULL");
    int st = 0;
    hipError_t e = hipMemcpyAsync(&st, b->d_status, sizeof(int), hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, FDTD_EDEVICE, "%s", hipGetErrorString(e));
    if (st & STATUS_MARCH_NONFINITE)
        return bfail(b, FDTD_ERANGE, "non-finite value (NaN or infinity) in the march of an instance "
                     "(fdtd_batch_readout names it)");
    return FDTD_OK;
}

int fdtd_batch_destroy(fdtd_batch* b)
{
    destroy(b);
    return FDTD_OK;
}

const char* fdtd_batch_last_error(const fdtd_batch* b) { return b ? b->err : g_berr; }

// Autotuner: for each candidate (row-block cap, workgroup width cap, groups)
// that fits the workspace, set up the batch, march its first probe_rows rows
// with plain launches and time them with events; the candidate with the most
// cell updates per second wins (graph capture is switched on in the result).
int fdtd_batch_autotune(const fdtd_params* p, int32_t n, void* d_workspace, size_t bytes, void* hip_stream,
                        int64_t probe_rows, fdtd_batch_opts* best, double* best_rate)
{
    if (!p || n < 1 || !best || probe_rows < 1) return bfail(nullptr, FDTD_EINVAL, "bad arguments");
    static const int tmaxes[] = {32, 16, 8};
    static const int64_t wmaxes[] = {BM_CAP, 768};
    static const int groupss[] = {1, 2};
    double top = -1.0;
    fdtd_batch_opts win;
    memset(&win, 0, sizeof win);
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return bfail(nullptr, FDTD_EDEVICE, "event creation failed");
    int rc = FDTD_OK;
    for (int tm : tmaxes) {
        for (int64_t wm : wmaxes) {
          for (int gr : groupss) {
            fdtd_batch_opts o;
            memset(&o, 0, sizeof o);
            o.struct_size = sizeof o;
            o.tmax = tm;
            o.wmax = wm;
            o.use_graph = 0;
            o.groups = gr;
            size_t need = 0;
            if (fdtd_batch_workspace_size(p, n, &o, &need) != FDTD_OK || need > bytes) continue;
            fdtd_batch* b = nullptr;
            rc = fdtd_batch_init(p, n, &o, d_workspace, bytes, hip_stream, &b);
            if (rc) break;
            rc = fdtd_batch_set_boundary(b);
            if (rc) { destroy(b); break; }
            // launches that cover probe_rows rows of every instance, and the cells they update
            int64_t k1 = 0;
            double cells = 0.0;
            for (const BInst& e : b->h_tab) {
                const int64_t rows = probe_rows < e.g.Nt ? probe_rows : e.g.Nt;
                const int64_t k = 1 + (rows + e.P.T - 1) / e.P.T;
                if (k > k1) k1 = k;
            }
            if (k1 > b->Lmax) k1 = b->Lmax;
            for (const BInst& e : b->h_tab) {
                for (int64_t k = 0; k < k1 && k < e.launches; ++k) {
                    int64_t m0, m1, s0, s1;
                    block_rows(e.P.T, e.g.Nt, k, &m0, &m1, &s0, &s1);
                    if (m1 >= m0) cells += (double)(m1 - m0 + 1) * (double)(e.g.Nx - e.g.D);
                    if (s1 >= s0) cells += (double)(s1 - s0 + 1) * (double)e.g.D;
                }
            }
            (void)hipEventRecord(e0, s);
            rc = enqueue(b, 0, k1, s);
            (void)hipEventRecord(e1, s);
            hipError_t he = hipEventSynchronize(e1);
            float ms = 0.f;
            if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            destroy(b);
            if (rc || he != hipSuccess) { rc = FDTD_EDEVICE; break; }
            const double rate = cells / (ms * 1e-3);
            if (rate > top) {
                top = rate;
                win = o;
            }
          }
          if (rc) break;
        }
        if (rc) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return bfail(nullptr, rc, "autotune failed: %s", g_berr[0] ? g_berr : "device error");
    if (top < 0.0) return bfail(nullptr, FDTD_ESIZE, "no candidate fits the workspace");
    win.use_graph = 1;
    *best = win;
    if (best_rate) *best_rate = top;
    return FDTD_OK;
}

}  // extern "C"
