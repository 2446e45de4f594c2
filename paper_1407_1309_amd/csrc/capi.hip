// capi.hip -- the extern "C" boundary of libmpdata (declared in mpdata.h).
//
// Host-side validation, workspace carving, the step loop (ping-pong between
// the caller's psi and a workspace buffer), kernel selection and the
// synchronous diagnostics.  No exception crosses the boundary; failures set a
// thread-local message and return a negative status.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/mpdata.h"
#include "adjoint.hpp"
#include "common.hpp"
#include "kernels.hpp"

namespace {

thread_local std::string g_err;

// Named range around an entry point's work in rocprofv3's marker trace
// (--marker-trace): pushed on entry, popped on return.
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    // the status code carries the failure; clear HIP's sticky last error so
    // the caller's next runtime call does not report it again
    (void)hipGetLastError();
    return fail(MPDATA_EHIP, "%s: %s", what, hipGetErrorString(e));
}

constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Bump allocator over the caller's workspace (offsets only; no allocation).
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base((char *)b) {}
    void *take(size_t bytes)
    {
        void *p = base ? base + used : nullptr;
        used += align_up(bytes);
        return p;
    }
};

int64_t cells_of(const mp::Geom &g) { return g.n[0] * g.n[1] * g.n[2]; }

int64_t walls_of(const mp::Geom &g, int d)
{
    int64_t e[3] = {g.n[0], g.n[1], g.n[2]};
    e[d] += 1;
    return e[0] * e[1] * e[2];
}

size_t dsize(int dtype) { return dtype == MPDATA_F64 ? 8 : 4; }

int check_desc(const mpdata_desc *d, mp::Geom *g)
{
    if (!d) return fail(MPDATA_EINVAL, "desc is NULL");
    if (d->n_dims < 1 || d->n_dims > 3) return fail(MPDATA_EINVAL, "n_dims %d not in 1..3", d->n_dims);
    if (d->dtype != MPDATA_F32 && d->dtype != MPDATA_F64)
        return fail(MPDATA_EINVAL, "unknown dtype %d", d->dtype);
    if (d->n_iters < 1 || d->n_iters > 8)
        return fail(MPDATA_EINVAL, "n_iters %d not in 1..8", d->n_iters);
    if ((d->opts & MPDATA_OPT_ABS) && (d->opts & MPDATA_OPT_IGA))
        return fail(MPDATA_EINVAL, "abs and iga are alternative variable-sign options");
    if (d->opts & ~(uint32_t)(MPDATA_OPT_FCT | MPDATA_OPT_IGA | MPDATA_OPT_TOT | MPDATA_OPT_ABS |
                              MPDATA_OPT_DFL | MPDATA_OPT_KAHAN))
        return fail(MPDATA_EINVAL, "unknown option bits 0x%x", d->opts);
    g->nd = d->n_dims;
    for (int k = 0; k < 3; k++) {
        if (k < d->n_dims) {
            if (d->bc[k] != MPDATA_BC_PERIODIC && d->bc[k] != MPDATA_BC_OPEN)
                return fail(MPDATA_EINVAL, "unknown bc %d in dimension %d", d->bc[k], k);
            int64_t lo = d->bc[k] == MPDATA_BC_PERIODIC ? 3 : 1;
            if (d->shape[k] < lo)
                return fail(MPDATA_EINVAL, "shape[%d] = %lld below %lld", k,
                            (long long)d->shape[k], (long long)lo);
            // kernels index cells and walls of one dimension in 32 bits,
            // with halo offsets of a few cells on either side
            if (d->shape[k] >= (int64_t)1 << 30)
                return fail(MPDATA_EINVAL, "shape[%d] = %lld is 2^30 or more", k,
                            (long long)d->shape[k]);
            g->n[k] = d->shape[k];
            g->bc[k] = d->bc[k];
        } else {
            g->n[k] = 1;
            g->bc[k] = MPDATA_BC_PERIODIC;
        }
    }
    if (cells_of(*g) > ((int64_t)1 << 40)) return fail(MPDATA_EINVAL, "grid too large");
    if ((d->opts & MPDATA_OPT_IGA) && d->n_iters > 2)
        return fail(MPDATA_EUNSUPPORTED,
                    "the infinite gauge is defined for n_iters <= 2 (got %d)", d->n_iters);
    return MPDATA_OK;
}

// Workspace layout of a single-grid plan.
struct Layout {
    void *psi_alt;
    void *tmp[2];
    void *faces[2][3];
    void *bup, *bdn;
    double *part;   // diag partials (5 per block)
    double *out;    // diag result (4) + courant result (1)
    double *spart;  // step diagnostics: partials written by the fused 2-D step
    double *sdiag;  // step diagnostics: result (4)
    size_t bytes;
};

// fused 2-D chunks shorter than this run without the in-kernel diagnostics
// (the partial buffer is sized for chunks of at least this many rows)
constexpr int SDIAG_MIN_ROWS = 16;

Layout carve(const mp::Geom &g, int dtype, void *base, int n_iters = 1, unsigned opts = 0)
{
    Layout L;
    memset(&L, 0, sizeof L);
    Carver c(base);
    size_t es = dsize(dtype);
    int64_t N = cells_of(g);
    L.part = (double *)c.take(sizeof(double) * 5 * mp::diag_max_blocks());
    L.out = (double *)c.take(sizeof(double) * 8);
    L.sdiag = (double *)c.take(sizeof(double) * 8);
    if (g.nd == 2)
        L.spart = (double *)c.take(
            sizeof(double) * 5 * mp::fused2d_max_parts(g.n[0], g.n[1], n_iters, opts, SDIAG_MIN_ROWS));
    L.psi_alt = c.take(es * N);
    L.tmp[0] = c.take(es * N);
    L.tmp[1] = c.take(es * N);
    for (int s = 0; s < 2; s++)
        for (int d = 0; d < g.nd; d++) L.faces[s][d] = c.take(es * walls_of(g, d));
    L.bup = c.take(es * N);
    L.bdn = c.take(es * N);
    L.bytes = c.used;
    return L;
}

}  // namespace

struct mpdata_plan {
    mpdata_desc desc;
    mp::Geom g;
    void *ws;
    size_t ws_bytes;
    hipStream_t stream;
    int kernel;
    int tile_rows = 0;   // fused kernel rows per wavefront chunk (0 = default)
    Layout L;
    // batched plans
    bool batched = false;
    std::vector<mp::BatchGrid> grids;
    mp::BatchGrid *grids_dev = nullptr;
    void *batch_alt = nullptr;
    int64_t batch_psi_total = 0, batch_c0_total = 0, batch_c1_total = 0;
    int batch_tiles = 0;
    int batch_xcd = 0;   // tile order: 0 grid by grid, 1 grouped per XCD
    // graph cache (batched); graphs are captured on a library-owned stream
    // (capture is not allowed on the legacy default stream) and launched on
    // the plan's stream
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    const void *g_key[3] = {nullptr, nullptr, nullptr};
    int g_steps = -1;
    // timing window of the step kernels (mpdata_timing): an event before the
    // first timed launch, one after the latest, and the launch count
    bool timing = false;
    hipEvent_t tev[2] = {nullptr, nullptr};
    int t_launches = 0, t_limit = 0;
    const char *tname = "";
    // stop flag (host memory, caller-owned) and the last call's step count
    const volatile int *cancel = nullptr;
    int64_t steps_done = 0;
    // diagnostics of each mpdata_step call's result (mpdata_set_step_diag)
    bool step_diag = false;
    bool sdiag_ready = false;
};

namespace {

// Brackets of a timed launch: timer_begin records the window's start event
// before the first timed launch; timer_end records the stop event after the
// last one the window holds (no event between the launches, so the window
// covers the same back-to-back launches as an untimed run).  Launches beyond
// the limit are not timed.
bool timer_begin(mpdata_plan *p, const char *name)
{
    if (!p->timing || p->t_launches >= p->t_limit) return false;
    if (p->t_launches == 0) (void)hipEventRecord(p->tev[0], p->stream);
    p->tname = name;
    return true;
}

void timer_end(mpdata_plan *p)
{
    p->t_launches++;
    if (p->t_launches == p->t_limit) (void)hipEventRecord(p->tev[1], p->stream);
}

// kernels of one step: stage by stage, the whole-step fused kernels, or the
// donor pass plus one launch per corrective pass (2-D)
enum { PATH_STAGED = 0, PATH_FUSED = 1, PATH_PASS2D = 2 };

template <typename T>
int one_step(mpdata_plan *p, const T *psi_n, T *psi_out, const T *G, const T *c0, const T *c1,
             const T *c2, int path, bool timed = false, int *dparts = nullptr)
{
    hipError_t e = hipSuccess;
    const bool fused = path == PATH_FUSED;
    const char *name = path == PATH_PASS2D ? "k_pass2d"
                       : !fused            ? "staged step"
                       : p->desc.n_dims == 3
                           ? (p->desc.n_iters == 1 ? "k_donor3d" : "k_step3d")
                           : "k_fused2d";
    bool tm = timed && timer_begin(p, name);
    if (path == PATH_PASS2D) {
        // one launch per corrective pass, the first with the donor pass
        // folded in (psi_out != psi_n: the passes read psi^n)
        const T *x = psi_n;
        const T *c[3] = {c0, c1, nullptr};
        int set = 0;
        for (int it = 2; it <= p->desc.n_iters && e == hipSuccess; it++) {
            const bool last = it == p->desc.n_iters;
            T *y = last ? psi_out : (T *)p->L.tmp[(it - 1) & 1];
            T *w0 = last ? nullptr : (T *)p->L.faces[set][0];
            T *w1 = last ? nullptr : (T *)p->L.faces[set][1];
            e = mp::pass2d_launch<T>(p->g, p->desc.opts, x, c[0], c[1], it == 2 ? nullptr : psi_n,
                                     G, y, w0, w1, p->stream, mp::PassRecord<T>(),
                                     p->tile_rows);
            c[0] = w0;
            c[1] = w1;
            set ^= 1;
            x = y;
        }
    } else if (fused && p->desc.n_dims == 3) {
        mp::Fused3DWork<T> w;
        for (int k = 0; k < 2; k++) {
            w.cell[k] = (T *)p->L.tmp[k];
            for (int d = 0; d < 3; d++) w.wall[k][d] = (T *)p->L.faces[k][d];
        }
        w.bup = (T *)p->L.bup;
        w.bdn = (T *)p->L.bdn;
        e = mp::fused3d_step<T>(p->g, p->desc.n_iters, p->desc.opts, psi_n, psi_out, c0, c1, c2,
                                G, p->tile_rows, p->stream, w);
    } else if (fused) {
        mp::Fused2DShape sh{p->g.n[0], p->g.n[1], p->g.bc[0], p->g.bc[1], p->tile_rows};
        e = mp::fused2d_step<T>(sh, p->desc.n_iters, p->desc.opts, psi_n, psi_out, c0, c1, G,
                                p->stream, dparts ? p->L.spart : nullptr, dparts);
    } else {
        mp::StagedArgs<T> a;
        a.g = p->g;
        a.n_iters = p->desc.n_iters;
        a.opts = p->desc.opts;
        a.psi_n = psi_n;
        a.psi_out = psi_out;
        a.c[0] = c0;
        a.c[1] = c1;
        a.c[2] = c2;
        a.G = G;
        a.tmp[0] = (T *)p->L.tmp[0];
        a.tmp[1] = (T *)p->L.tmp[1];
        for (int s = 0; s < 2; s++)
            for (int d = 0; d < 3; d++) a.faces[s][d] = (T *)p->L.faces[s][d];
        a.bup = (T *)p->L.bup;
        a.bdn = (T *)p->L.bdn;
        e = mp::staged_step<T>(a, p->stream);
    }
    if (tm) timer_end(p);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    return MPDATA_OK;
}

bool fused_available(const mpdata_plan *p)
{
    return mp::fused2d_supported(p->desc.n_dims, p->desc.n_iters, p->desc.opts, p->desc.has_g,
                                 p->g.bc[0], p->g.bc[1]) ||
           mp::fused3d_supported(p->desc.n_dims, p->desc.n_iters, p->desc.opts, p->g.n, p->g.bc);
}

bool resident_available(const mpdata_plan *p)
{
    return mp::resident1d_supported(p->desc.n_dims, p->g.n[0], p->desc.dtype == MPDATA_F64,
                                    p->desc.has_g);
}

bool use_fused(const mpdata_plan *p)
{
    return (p->kernel == MPDATA_KERNEL_AUTO || p->kernel == MPDATA_KERNEL_FUSED) &&
           fused_available(p);
}

bool use_pass2d(const mpdata_plan *p)
{
    return p->kernel != MPDATA_KERNEL_STAGED && !use_fused(p) &&
           mp::pass2d_supported(p->desc.n_dims, p->desc.n_iters, p->desc.opts, p->desc.has_g,
                                p->g.n);
}

int step_path(const mpdata_plan *p)
{
    return use_fused(p) ? PATH_FUSED : use_pass2d(p) ? PATH_PASS2D : PATH_STAGED;
}

bool use_resident(const mpdata_plan *p)
{
    return p->kernel != MPDATA_KERNEL_STAGED && resident_available(p);
}

// Diagnostics of a step call's result (mpdata_set_step_diag): the final merge
// of the partials the fused 2-D step's last launch wrote (dparts > 0), else
// a diagnostics pass over psi.
template <typename T>
int step_diag_finish(mpdata_plan *p, const T *psi, const T *G, int dparts)
{
    hipError_t e = dparts > 0 ? mp::diag_final_launch(p->L.spart, dparts, p->L.sdiag, p->stream)
                              : mp::diag_launch<T>(psi, G, cells_of(p->g), p->L.part,
                                                   p->L.sdiag, p->stream);
    if (e != hipSuccess) return hip_fail(e, "step diagnostics launch");
    p->sdiag_ready = true;
    return MPDATA_OK;
}

// true when the fused 2-D step can write the diagnostics partials itself
bool step_diag_in_kernel(const mpdata_plan *p, int path)
{
    return p->step_diag && path == PATH_FUSED && p->desc.n_dims == 2 &&
           (p->tile_rows == 0 || p->tile_rows >= SDIAG_MIN_ROWS);
}

// Step loop with a stop flag: every step runs to completion (stream
// synchronisation) before the flag is read and the next step launched; the
// state alternates between psi and the workspace buffer and is copied back
// to psi if the run stops on the workspace side.
template <typename T>
int run_steps_polled(mpdata_plan *p, T *psi, const T *G, const T *c0, const T *c1,
                     const T *c2, int n_steps)
{
    const bool resident = use_resident(p);
    const int path = step_path(p);
    T *cur = psi, *nxt = (T *)p->L.psi_alt;
    int done = 0, rc = MPDATA_OK;
    while (done < n_steps) {
        if (*p->cancel) {
            rc = fail(MPDATA_ECANCELLED, "cancelled after %d of %d steps", done, n_steps);
            break;
        }
        hipError_t e;
        if (resident) {
            e = mp::resident1d_steps<T>(p->g.n[0], p->g.bc[0], p->desc.n_iters, p->desc.opts,
                                        cur, c0, G, n_steps, p->stream);
            if (e != hipSuccess) return hip_fail(e, "resident 1-D launch");
            done = n_steps;
        } else if (path == PATH_STAGED && p->desc.n_iters >= 2) {
            int r = one_step<T>(p, cur, cur, G, c0, c1, c2, PATH_STAGED, true);
            if (r) return r;
            done++;
        } else {
            int r = one_step<T>(p, cur, nxt, G, c0, c1, c2, path, true);
            if (r) return r;
            T *t = cur;
            cur = nxt;
            nxt = t;
            done++;
        }
        e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return hip_fail(e, "step synchronisation");
        p->steps_done = done;
    }
    if (cur != psi) {
        hipError_t e = hipMemcpyAsync(psi, cur, sizeof(T) * cells_of(p->g),
                                      hipMemcpyDeviceToDevice, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return hip_fail(e, "copy of the last completed step");
    }
    if (p->step_diag) {
        int r = step_diag_finish<T>(p, psi, G, 0);
        if (r) return r;
    }
    return rc;
}

template <typename T>
int run_steps(mpdata_plan *p, T *psi, const T *G, const T *c0, const T *c1, const T *c2,
              int n_steps)
{
    p->steps_done = 0;
    p->sdiag_ready = false;
    if (n_steps == 0) return p->step_diag ? step_diag_finish<T>(p, psi, G, 0) : MPDATA_OK;
    if (p->cancel) return run_steps_polled<T>(p, psi, G, c0, c1, c2, n_steps);
    if (use_resident(p)) {
        bool tm = timer_begin(p, "k_resident1d");
        hipError_t e = mp::resident1d_steps<T>(p->g.n[0], p->g.bc[0], p->desc.n_iters,
                                               p->desc.opts, psi, c0, G, n_steps, p->stream);
        if (tm) timer_end(p);
        if (e != hipSuccess) return hip_fail(e, "resident 1-D launch");
        p->steps_done = n_steps;
        return p->step_diag ? step_diag_finish<T>(p, psi, G, 0) : MPDATA_OK;
    }
    const int path = step_path(p);
    if (path == PATH_STAGED && p->desc.n_iters >= 2) {
        // staged passes: psi^n is last read before the final corrective pass,
        // which reads only the previous pass's result, so the step may
        // overwrite psi in place (no ping-pong, no copy)
        for (int s = 0; s < n_steps; s++) {
            int rc = one_step<T>(p, psi, psi, G, c0, c1, c2, PATH_STAGED, true);
            if (rc) return rc;
        }
        p->steps_done = n_steps;
        return p->step_diag ? step_diag_finish<T>(p, psi, G, 0) : MPDATA_OK;
    }
    int64_t N = cells_of(p->g);
    T *alt = (T *)p->L.psi_alt;
    T *cur = psi, *nxt = alt;
    if (n_steps & 1) {
        hipError_t e = hipMemcpyAsync(alt, psi, sizeof(T) * N, hipMemcpyDeviceToDevice, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        cur = alt;
        nxt = psi;
    }
    // the last launch of the call also writes the diagnostics partials when
    // the fused 2-D step can (dparts receives their number)
    int dparts = 0;
    const bool in_kernel = step_diag_in_kernel(p, path);
    for (int s = 0; s < n_steps; s++) {
        int rc = one_step<T>(p, cur, nxt, G, c0, c1, c2, path, true,
                             in_kernel && s == n_steps - 1 ? &dparts : nullptr);
        if (rc) return rc;
        T *t = cur;
        cur = nxt;
        nxt = t;
    }
    p->steps_done = n_steps;
    return p->step_diag ? step_diag_finish<T>(p, psi, G, dparts) : MPDATA_OK;
}

}  // namespace

extern "C" {

const char *mpdata_last_error(void) { return g_err.c_str(); }

size_t mpdata_workspace_bytes(const mpdata_desc *desc)
{
    mp::Geom g;
    if (check_desc(desc, &g) != MPDATA_OK) return 0;
    return carve(g, desc->dtype, nullptr, desc->n_iters, desc->opts).bytes;
}

int mpdata_init(const mpdata_desc *desc, void *workspace, size_t ws_bytes, void *hip_stream,
                mpdata_plan **out)
{
    if (!out) return fail(MPDATA_EINVAL, "out is NULL");
    *out = nullptr;
    mp::Geom g;
    int rc = check_desc(desc, &g);
    if (rc) return rc;
    size_t need = carve(g, desc->dtype, nullptr, desc->n_iters, desc->opts).bytes;
    if (!workspace) return fail(MPDATA_EWORKSPACE, "workspace is NULL (need %zu bytes)", need);
    if ((uintptr_t)workspace % ALIGN) return fail(MPDATA_EWORKSPACE, "workspace not 256-byte aligned");
    if (ws_bytes < need)
        return fail(MPDATA_EWORKSPACE, "workspace has %zu bytes, need %zu", ws_bytes, need);
    mpdata_plan *p = new (std::nothrow) mpdata_plan();
    if (!p) return fail(MPDATA_EINVAL, "out of host memory");
    p->desc = *desc;
    p->g = g;
    p->ws = workspace;
    p->ws_bytes = ws_bytes;
    p->stream = (hipStream_t)hip_stream;
    p->kernel = MPDATA_KERNEL_AUTO;
    p->L = carve(g, desc->dtype, workspace, desc->n_iters, desc->opts);
    *out = p;
    return MPDATA_OK;
}

int mpdata_set_kernel(mpdata_plan *plan, int kernel)
{
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    if (kernel < MPDATA_KERNEL_AUTO || kernel > MPDATA_KERNEL_PASS)
        return fail(MPDATA_EINVAL, "unknown kernel %d", kernel);
    if (kernel == MPDATA_KERNEL_FUSED && !fused_available(plan) && !resident_available(plan))
        return fail(MPDATA_EUNSUPPORTED, "no fused kernel for this plan");
    if (kernel == MPDATA_KERNEL_PASS &&
        !mp::pass2d_supported(plan->desc.n_dims, plan->desc.n_iters, plan->desc.opts,
                              plan->desc.has_g, plan->g.n))
        return fail(MPDATA_EUNSUPPORTED, "no single-pass kernel for this plan");
    plan->kernel = kernel;
    return MPDATA_OK;
}

int mpdata_set_stream(mpdata_plan *plan, void *hip_stream)
{
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    plan->stream = (hipStream_t)hip_stream;
    return MPDATA_OK;
}

size_t mpdata_tlm_workspace_bytes(const mpdata_desc *desc)
{
    mp::Geom g;
    if (check_desc(desc, &g) != MPDATA_OK) return 0;
    return mp::tlm_workspace_bytes(g, desc->dtype == MPDATA_F64, desc->has_g);
}

int mpdata_tlm_step(mpdata_plan *plan, void *psi, void *dpsi, const void *g, const void *c0,
                    const void *c1, const void *c2, const void *dc0, const void *dc1,
                    const void *dc2, int n_steps)
{
    TraceRange trace_range("mpdata_tlm_step");
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    if (plan->batched) return fail(MPDATA_EINVAL, "the tangent-linear step needs a single-grid plan");
    if (!psi || !dpsi) return fail(MPDATA_EINVAL, "psi or dpsi is NULL");
    if (psi == dpsi) return fail(MPDATA_EINVAL, "psi and dpsi must be distinct buffers");
    if (n_steps < 0) return fail(MPDATA_EINVAL, "n_steps < 0");
    const void *c[3] = {c0, c1, c2}, *dc[3] = {dc0, dc1, dc2};
    for (int d = 0; d < 3; d++) {
        if (d < plan->desc.n_dims && !c[d]) return fail(MPDATA_EINVAL, "c%d is NULL", d);
        if (d >= plan->desc.n_dims && (c[d] || dc[d]))
            return fail(MPDATA_EINVAL, "c%d / dc%d given for a %d-D plan", d, d,
                        plan->desc.n_dims);
    }
    if ((g != nullptr) != (plan->desc.has_g != 0)) return fail(MPDATA_EINVAL, "g / has_g mismatch");
    const bool f64 = plan->desc.dtype == MPDATA_F64;
    const size_t need = mp::tlm_workspace_bytes(plan->g, f64, plan->desc.has_g);
    if (plan->ws_bytes < need)
        return fail(MPDATA_EWORKSPACE, "workspace has %zu bytes, the tangent-linear step needs %zu",
                    plan->ws_bytes, need);
    if (n_steps == 0) return MPDATA_OK;
    hipError_t e;
    if (f64) {
        const double *cc[3], *dd[3];
        for (int d = 0; d < 3; d++) {
            cc[d] = (const double *)c[d];
            dd[d] = (const double *)dc[d];
        }
        e = mp::tlm_steps<double>(plan->g, plan->desc.n_iters, plan->desc.opts, (double *)psi,
                                  (double *)dpsi, (const double *)g, cc, dd, n_steps, plan->ws,
                                  plan->stream);
    } else {
        const float *cc[3], *dd[3];
        for (int d = 0; d < 3; d++) {
            cc[d] = (const float *)c[d];
            dd[d] = (const float *)dc[d];
        }
        e = mp::tlm_steps<float>(plan->g, plan->desc.n_iters, plan->desc.opts, (float *)psi,
                                 (float *)dpsi, (const float *)g, cc, dd, n_steps, plan->ws,
                                 plan->stream);
    }
    return e == hipSuccess ? MPDATA_OK : hip_fail(e, "tangent-linear launch");
}

int mpdata_set_cancel_flag(mpdata_plan *plan, const volatile int *flag)
{
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    plan->cancel = flag;
    return MPDATA_OK;
}

int mpdata_steps_done(const mpdata_plan *plan, int64_t *out)
{
    if (!plan || !out) return fail(MPDATA_EINVAL, "NULL argument");
    *out = plan->steps_done;
    return MPDATA_OK;
}

int mpdata_set_tile_rows(mpdata_plan *plan, int rows)
{
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    if (rows < 0 || rows > (1 << 20)) return fail(MPDATA_EINVAL, "tile rows %d out of range", rows);
    plan->tile_rows = rows;
    return MPDATA_OK;
}

int mpdata_autotune(mpdata_plan *plan, const void *psi, const void *g, const void *c0,
                    const void *c1, const void *c2, int *out_tile_rows)
{
    TraceRange trace_range("mpdata_autotune");
    if (!plan || !psi || !out_tile_rows) return fail(MPDATA_EINVAL, "NULL argument");
    if (plan->batched) return fail(MPDATA_EINVAL, "autotune needs a single-grid plan");
    *out_tile_rows = plan->tile_rows;
    if (!use_fused(plan)) return MPDATA_OK;   // staged path: nothing to tune
    const void *c[3] = {c0, c1, c2};
    for (int d = 0; d < plan->desc.n_dims; d++)
        if (!c[d]) return fail(MPDATA_EINVAL, "c%d is NULL", d);
    static const int cand[] = {16, 24, 32, 40, 48, 64, 80, 96, 128, 160, 192, 256, 384, 512};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(MPDATA_EHIP, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(MPDATA_EHIP, "hipEventCreate");
    }
    int saved = plan->tile_rows, best = 0;
    float best_ms = 0.0f;
    int rc = MPDATA_OK;
    const int ncand = (int)(sizeof cand / sizeof cand[0]);
    // two sweeps over the candidates; the minimum time of each counts
    for (int kk = 0; kk < 2 * ncand && rc == MPDATA_OK; kk++) {
        int k = kk % ncand;
        int th = cand[k];
        if (th > plan->g.n[0] && k > 0) continue;
        plan->tile_rows = th;
        const int reps = 5;
        for (int r = 0; r <= reps && rc == MPDATA_OK; r++) {
            if (r == 1) (void)hipEventRecord(e0, plan->stream);
            if (plan->desc.dtype == MPDATA_F64)
                rc = one_step<double>(plan, (const double *)psi, (double *)plan->L.psi_alt,
                                      (const double *)g, (const double *)c0, (const double *)c1,
                                      (const double *)c2, PATH_FUSED);
            else
                rc = one_step<float>(plan, (const float *)psi, (float *)plan->L.psi_alt,
                                     (const float *)g, (const float *)c0, (const float *)c1,
                                     (const float *)c2, PATH_FUSED);
        }
        if (rc) break;
        (void)hipEventRecord(e1, plan->stream);
        hipError_t e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = hip_fail(e, "autotune timing");
            break;
        }
        if (best == 0 || ms < best_ms) {
            best = th;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan->tile_rows = rc == MPDATA_OK ? best : saved;
    *out_tile_rows = plan->tile_rows;
    return rc;
}

int mpdata_step(mpdata_plan *plan, void *psi, const void *g, const void *c0, const void *c1,
                const void *c2, int n_steps)
{
    TraceRange trace_range("mpdata_step");
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    if (plan->batched) return fail(MPDATA_EINVAL, "batched plan: use mpdata_step_batched");
    if (!psi) return fail(MPDATA_EINVAL, "psi is NULL");
    if (n_steps < 0) return fail(MPDATA_EINVAL, "n_steps < 0");
    const void *c[3] = {c0, c1, c2};
    for (int d = 0; d < 3; d++) {
        if (d < plan->desc.n_dims && !c[d]) return fail(MPDATA_EINVAL, "c%d is NULL", d);
        if (d >= plan->desc.n_dims && c[d])
            return fail(MPDATA_EINVAL, "c%d given for a %d-D plan", d, plan->desc.n_dims);
    }
    if ((g != nullptr) != (plan->desc.has_g != 0))
        return fail(MPDATA_EINVAL, plan->desc.has_g ? "plan has_g but g is NULL"
                                                    : "g given but plan was made without has_g");
    if (plan->desc.dtype == MPDATA_F64)
        return run_steps<double>(plan, (double *)psi, (const double *)g, (const double *)c0,
                                 (const double *)c1, (const double *)c2, n_steps);
    return run_steps<float>(plan, (float *)psi, (const float *)g, (const float *)c0,
                            (const float *)c1, (const float *)c2, n_steps);
}

int mpdata_set_step_diag(mpdata_plan *plan, int on)
{
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    if (plan->batched) return fail(MPDATA_EINVAL, "step diagnostics need a single-grid plan");
    plan->step_diag = on != 0;
    plan->sdiag_ready = false;
    return MPDATA_OK;
}

int mpdata_step_diag(mpdata_plan *plan, double out[3], int64_t *n_nonfinite)
{
    TraceRange trace_range("mpdata_step_diag");
    if (!plan || !out || !n_nonfinite) return fail(MPDATA_EINVAL, "NULL argument");
    if (!plan->sdiag_ready)
        return fail(MPDATA_EINVAL, "no mpdata_step call with step diagnostics on since they were "
                                   "switched on");
    double h[4];
    hipError_t e = hipMemcpyAsync(h, plan->L.sdiag, sizeof h, hipMemcpyDeviceToHost, plan->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "step diagnostics copy");
    out[0] = h[0];
    out[1] = h[1];
    out[2] = h[2];
    *n_nonfinite = (int64_t)h[3];
    if (*n_nonfinite > 0)
        return fail(MPDATA_ENONFINITE, "%lld non-finite values", (long long)*n_nonfinite);
    return MPDATA_OK;
}

int mpdata_step_rhs(mpdata_plan *plan, void *psi, const void *g, const void *c0,
                    const void *c1, const void *c2, const void *r_pre, double a_pre,
                    const void *r_post, double a_post)
{
    TraceRange trace_range("mpdata_step_rhs");
    if (!plan || !psi) return fail(MPDATA_EINVAL, "NULL argument");
    if (plan->batched) return fail(MPDATA_EINVAL, "source terms need a single-grid plan");
    const int64_t N = cells_of(plan->g);
    const bool f64 = plan->desc.dtype == MPDATA_F64;
    hipError_t e = hipSuccess;
    if (r_pre)
        e = f64 ? mp::axpy_launch<double>((double *)psi, (const double *)r_pre, a_pre, N,
                                          plan->stream)
                : mp::axpy_launch<float>((float *)psi, (const float *)r_pre, a_pre, N,
                                         plan->stream);
    if (e != hipSuccess) return hip_fail(e, "source term launch");
    int rc = mpdata_step(plan, psi, g, c0, c1, c2, 1);
    if (rc) return rc;
    if (r_post)
        e = f64 ? mp::axpy_launch<double>((double *)psi, (const double *)r_post, a_post, N,
                                          plan->stream)
                : mp::axpy_launch<float>((float *)psi, (const float *)r_post, a_post, N,
                                         plan->stream);
    if (e != hipSuccess) return hip_fail(e, "source term launch");
    return MPDATA_OK;
}

int mpdata_osc_step(mpdata_plan *plan, void *psi, void *phi, const void *g, const void *c0,
                    const void *c1, const void *c2, double a, int n_steps)
{
    TraceRange trace_range("mpdata_osc_step");
    if (!plan || !psi || !phi) return fail(MPDATA_EINVAL, "NULL argument");
    if (psi == phi) return fail(MPDATA_EINVAL, "psi and phi must be distinct buffers");
    if (plan->batched) return fail(MPDATA_EINVAL, "the oscillator needs a single-grid plan");
    if (n_steps < 0) return fail(MPDATA_EINVAL, "n_steps < 0");
    const int64_t N = cells_of(plan->g);
    const bool f64 = plan->desc.dtype == MPDATA_F64;
    if (n_steps == 0) return MPDATA_OK;
    if (plan->kernel != MPDATA_KERNEL_STAGED &&
        mp::resident1d_supported(plan->desc.n_dims, plan->g.n[0], f64, plan->desc.has_g, 1)) {
        // 1-D pair resident in LDS: every step of the call in one launch
        bool tm = timer_begin(plan, "k_resident1d");
        hipError_t e =
            f64 ? mp::resident1d_osc<double>(plan->g.n[0], plan->g.bc[0], plan->desc.n_iters,
                                             plan->desc.opts, (double *)psi, (double *)phi,
                                             (const double *)c0, (const double *)g, a, n_steps,
                                             plan->stream)
                : mp::resident1d_osc<float>(plan->g.n[0], plan->g.bc[0], plan->desc.n_iters,
                                            plan->desc.opts, (float *)psi, (float *)phi,
                                            (const float *)c0, (const float *)g, a, n_steps,
                                            plan->stream);
        if (tm) timer_end(plan);
        return e == hipSuccess ? MPDATA_OK : hip_fail(e, "resident oscillator launch");
    }
    for (int st = 0; st < n_steps; st++) {
        hipError_t e = f64 ? mp::osc_couple_launch<double>((double *)psi, (double *)phi, a, 0,
                                                           N, plan->stream)
                           : mp::osc_couple_launch<float>((float *)psi, (float *)phi, a, 0, N,
                                                          plan->stream);
        if (e != hipSuccess) return hip_fail(e, "oscillator coupling launch");
        int rc = mpdata_step(plan, psi, g, c0, c1, c2, 1);
        if (rc) return rc;
        rc = mpdata_step(plan, phi, g, c0, c1, c2, 1);
        if (rc) return rc;
        e = f64 ? mp::osc_couple_launch<double>((double *)psi, (double *)phi, a, 1, N,
                                                plan->stream)
                : mp::osc_couple_launch<float>((float *)psi, (float *)phi, a, 1, N,
                                               plan->stream);
        if (e != hipSuccess) return hip_fail(e, "oscillator coupling launch");
    }
    return MPDATA_OK;
}

}  // extern "C"

namespace {

// checks shared by the prognosed-velocity entry points: spacing, eps, the
// per-dimension pointers of a plan of n_dims dimensions
int vip_args(const mpdata_plan *plan, double dt, const double dx[3], double eps)
{
    if (!dx) return fail(MPDATA_EINVAL, "dx is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(MPDATA_EINVAL, "dt must be finite and > 0");
    for (int d = 0; d < plan->desc.n_dims; d++)
        if (!(dx[d] > 0.0) || !std::isfinite(dx[d]))
            return fail(MPDATA_EINVAL, "dx[%d] must be finite and > 0", d);
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(MPDATA_EINVAL, "eps must be finite and >= 0");
    return MPDATA_OK;
}

int ptr_set(const mpdata_plan *plan, const void *const a[3], const char *name)
{
    if (!a) return fail(MPDATA_EINVAL, "%s is NULL", name);
    for (int d = 0; d < plan->desc.n_dims; d++)
        if (!a[d]) return fail(MPDATA_EINVAL, "%s[%d] is NULL", name, d);
    return MPDATA_OK;
}

// true if two of the n non-NULL pointers are equal
bool any_alias(const void *const *p, int n)
{
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++)
            if (p[i] && p[i] == p[j]) return true;
    return false;
}

template <typename T> const T *const *cpp(const void *const a[3], const T *out[3], int nd)
{
    for (int d = 0; d < 3; d++) out[d] = d < nd ? (const T *)a[d] : nullptr;
    return out;
}

template <typename T> T *const *mpp(void *const a[3], T *out[3], int nd)
{
    for (int d = 0; d < 3; d++) out[d] = d < nd ? (T *)a[d] : nullptr;
    return out;
}

template <typename T>
hipError_t vip_run(mpdata_plan *plan, const void *const num[3], const void *den,
                   const void *const nump[3], const void *denp, double dt, const double dx[3],
                   double eps, void *const c[3])
{
    const int nd = plan->desc.n_dims;
    const T *a[3], *b[3];
    T *o[3];
    double k[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < nd; d++) k[d] = dt / dx[d];
    return mp::vip_launch<T>(plan->g, cpp<T>(num, a, nd), (const T *)den, cpp<T>(nump, b, nd),
                             (const T *)denp, eps, k, mpp<T>(c, o, nd), plan->stream);
}

template <typename T>
int sw_run(mpdata_plan *plan, void *h, void *const q[3], void *h_prev, void *const q_prev[3],
           void *const c[3], double dt, const double dx[3], double grav, double eps, int n_steps)
{
    const int nd = plan->desc.n_dims;
    T *qq[3], *qp[3], *cc[3];
    mpp<T>(q, qq, nd);
    mpp<T>(q_prev, qp, nd);
    mpp<T>(c, cc, nd);
    const void *qc[3] = {qq[0], qq[1], qq[2]}, *qpc[3] = {qp[0], qp[1], qp[2]};
    double sp[3] = {1.0, 1.0, 1.0};
    for (int d = 0; d < nd; d++) sp[d] = dx[d];
    for (int st = 0; st < n_steps; st++) {
        // advector at n+1/2 from levels n and n-1
        hipError_t e = vip_run<T>(plan, qc, h, qpc, h_prev, dt, sp, eps, c);
        if (e != hipSuccess) return hip_fail(e, "prognosed-velocity launch");
        int rc;
        if (use_resident(plan)) {
            // the LDS-resident 1-D kernel steps in place: level n becomes the
            // previous level and the explicit half of the forcing is added in
            // place, then every field is stepped
            e = mp::sw_force_launch<T>(plan->g, (const T *)h, (T *)h_prev, qq, qp, grav, sp, dt,
                                       1, plan->stream);
            if (e != hipSuccess) return hip_fail(e, "shallow-water forcing launch");
            rc = mpdata_step(plan, h, nullptr, cc[0], cc[1], cc[2], 1);
            for (int d = 0; d < nd && !rc; d++)
                rc = mpdata_step(plan, qq[d], nullptr, cc[0], cc[1], cc[2], 1);
            if (rc) return rc;
        } else {
            // per momentum component: level n saved to q_prev, the explicit
            // half of the forcing written to the workspace's alternate buffer,
            // the step from there into q[d] (h still at level n throughout);
            // the first launch also saves h to h_prev, from which the depth
            // is then stepped into h.  No field is copied into the workspace.
            T *alt = (T *)plan->L.psi_alt;
            const int path = step_path(plan);
            for (int d = 0; d < nd; d++) {
                e = mp::sw_force1_launch<T>(plan->g, d, (const T *)h, d == 0 ? (T *)h_prev : nullptr,
                                            qq[d], qp[d], alt, grav, sp, dt, plan->stream);
                if (e != hipSuccess) return hip_fail(e, "shallow-water forcing launch");
                rc = one_step<T>(plan, alt, qq[d], nullptr, cc[0], cc[1], cc[2], path, false);
                if (rc) return rc;
            }
            rc = one_step<T>(plan, (const T *)h_prev, (T *)h, nullptr, cc[0], cc[1], cc[2], path,
                             false);
            if (rc) return rc;
        }
        // forcing at n+1 from the advected depth
        e = mp::sw_force_launch<T>(plan->g, (const T *)h, (T *)h_prev, qq, qp, grav, sp, dt, 0,
                                   plan->stream);
        if (e != hipSuccess) return hip_fail(e, "shallow-water forcing launch");
    }
    return MPDATA_OK;
}

}  // namespace

extern "C" {

int mpdata_vip_advector(mpdata_plan *plan, const void *const num[3], const void *den,
                        const void *const num_prev[3], const void *den_prev, double dt,
                        const double dx[3], double eps, void *const c[3])
{
    TraceRange trace_range("mpdata_vip_advector");
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    if (plan->batched) return fail(MPDATA_EINVAL, "prognosed velocity needs a single-grid plan");
    int rc = vip_args(plan, dt, dx, eps);
    if (!rc) rc = ptr_set(plan, num, "num");
    if (!rc) rc = ptr_set(plan, num_prev, "num_prev");
    if (!rc) rc = ptr_set(plan, (const void *const *)c, "c");
    if (rc) return rc;
    if ((den != nullptr) != (den_prev != nullptr))
        return fail(MPDATA_EINVAL, "den and den_prev must both be given or both be NULL");
    const int nd = plan->desc.n_dims;
    const void *all[11] = {den, den_prev};
    int k = 2;
    for (int d = 0; d < nd; d++) {
        all[k++] = num[d];
        all[k++] = num_prev[d];
    }
    for (int d = 0; d < nd; d++)
        for (int j = 0; j < k; j++)
            if (all[j] == c[d]) return fail(MPDATA_EINVAL, "c[%d] aliases an input", d);
    if (any_alias((const void *const *)c, nd)) return fail(MPDATA_EINVAL, "c components alias");
    hipError_t e = plan->desc.dtype == MPDATA_F64
                       ? vip_run<double>(plan, num, den, num_prev, den_prev, dt, dx, eps, c)
                       : vip_run<float>(plan, num, den, num_prev, den_prev, dt, dx, eps, c);
    return e == hipSuccess ? MPDATA_OK : hip_fail(e, "prognosed-velocity launch");
}

int mpdata_sw_step(mpdata_plan *plan, void *h, void *const q[3], void *h_prev,
                   void *const q_prev[3], void *const c[3], double dt, const double dx[3],
                   double grav, double eps, int n_steps)
{
    TraceRange trace_range("mpdata_sw_step");
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    if (plan->batched) return fail(MPDATA_EINVAL, "shallow water needs a single-grid plan");
    if (plan->desc.has_g)
        return fail(MPDATA_EUNSUPPORTED, "prognosed velocity is defined for G = 1 only");
    if (!h || !h_prev) return fail(MPDATA_EINVAL, "h or h_prev is NULL");
    if (n_steps < 0) return fail(MPDATA_EINVAL, "n_steps < 0");
    if (!std::isfinite(grav)) return fail(MPDATA_EINVAL, "grav must be finite");
    int rc = vip_args(plan, dt, dx, eps);
    if (!rc) rc = ptr_set(plan, (const void *const *)q, "q");
    if (!rc) rc = ptr_set(plan, (const void *const *)q_prev, "q_prev");
    if (!rc) rc = ptr_set(plan, (const void *const *)c, "c");
    if (rc) return rc;
    const int nd = plan->desc.n_dims;
    const void *all[11] = {h, h_prev};
    int k = 2;
    for (int d = 0; d < nd; d++) {
        all[k++] = q[d];
        all[k++] = q_prev[d];
        all[k++] = c[d];
    }
    if (any_alias(all, k)) return fail(MPDATA_EINVAL, "state and advector buffers must be distinct");
    if (n_steps == 0) return MPDATA_OK;
    return plan->desc.dtype == MPDATA_F64
               ? sw_run<double>(plan, h, q, h_prev, q_prev, c, dt, dx, grav, eps, n_steps)
               : sw_run<float>(plan, h, q, h_prev, q_prev, c, dt, dx, grav, eps, n_steps);
}

int mpdata_diag(mpdata_plan *plan, const void *psi, const void *g, double out[3],
                int64_t *n_nonfinite)
{
    TraceRange trace_range("mpdata_diag");
    if (!plan || !psi || !out || !n_nonfinite) return fail(MPDATA_EINVAL, "NULL argument");
    if (plan->batched) return fail(MPDATA_EINVAL, "diag needs a single-grid plan");
    int64_t N = cells_of(plan->g);
    hipError_t e;
    if (plan->desc.dtype == MPDATA_F64)
        e = mp::diag_launch<double>((const double *)psi, (const double *)g, N, plan->L.part,
                                    plan->L.out, plan->stream);
    else
        e = mp::diag_launch<float>((const float *)psi, (const float *)g, N, plan->L.part,
                                   plan->L.out, plan->stream);
    if (e != hipSuccess) return hip_fail(e, "diag launch");
    double h[4];
    e = hipMemcpyAsync(h, plan->L.out, sizeof h, hipMemcpyDeviceToHost, plan->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "diag copy");
    out[0] = h[0];
    out[1] = h[1];
    out[2] = h[2];
    *n_nonfinite = (int64_t)h[3];
    if (*n_nonfinite > 0)
        return fail(MPDATA_ENONFINITE, "%lld non-finite values", (long long)*n_nonfinite);
    return MPDATA_OK;
}

int mpdata_courant_max(mpdata_plan *plan, const void *g, const void *c0, const void *c1,
                       const void *c2, double *out)
{
    if (!plan || !out) return fail(MPDATA_EINVAL, "NULL argument");
    if (plan->batched) return fail(MPDATA_EINVAL, "courant check needs a single-grid plan");
    const void *c[3] = {c0, c1, c2};
    for (int d = 0; d < plan->desc.n_dims; d++)
        if (!c[d]) return fail(MPDATA_EINVAL, "c%d is NULL", d);
    hipError_t e;
    if (plan->desc.dtype == MPDATA_F64)
        e = mp::courant_launch<double>(plan->g, (const double *)c0, (const double *)c1,
                                       (const double *)c2, (const double *)g, plan->L.part,
                                       plan->L.out + 4, plan->stream);
    else
        e = mp::courant_launch<float>(plan->g, (const float *)c0, (const float *)c1,
                                      (const float *)c2, (const float *)g, plan->L.part,
                                      plan->L.out + 4, plan->stream);
    if (e != hipSuccess) return hip_fail(e, "courant launch");
    double h[2];
    e = hipMemcpyAsync(h, plan->L.out + 4, sizeof h, hipMemcpyDeviceToHost, plan->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "courant copy");
    *out = h[0];
    if (h[1] > 0)
        return fail(MPDATA_ENONFINITE, "%lld cells with a non-finite advector or G",
                    (long long)h[1]);
    return MPDATA_OK;
}

// ------------------------------------------------------------------ adjoint
size_t mpdata_adj_workspace_bytes(const mpdata_desc *desc, int n_steps, int ckpt_every)
{
    mp::Geom g;
    if (check_desc(desc, &g) != MPDATA_OK) return 0;
    if (n_steps < 1 || ckpt_every < 1 || ckpt_every > n_steps) return 0;
    size_t base = carve(g, desc->dtype, nullptr, desc->n_iters, desc->opts).bytes;
    return base + mp::adj_extra_bytes(g, desc->dtype == MPDATA_F64 ? 8 : 4, desc->n_iters,
                                      desc->opts, n_steps, ckpt_every);
}

}  // extern "C"

namespace {

// forward step without records for the adjoint's state sweeps
struct AdjStepCtx {
    mpdata_plan *p;
    const void *G, *c[3];
};

template <typename T> hipError_t adj_plain_step(void *ctx, const T *in, T *out)
{
    const AdjStepCtx *x = (const AdjStepCtx *)ctx;
    int rc = one_step<T>(x->p, in, out, (const T *)x->G, (const T *)x->c[0], (const T *)x->c[1],
                         (const T *)x->c[2], step_path(x->p));
    return rc == MPDATA_OK ? hipSuccess : hipErrorLaunchFailure;
}

}  // namespace

extern "C" {

int mpdata_adv_adj(mpdata_plan *plan, const void *psi0, const void *g, const void *c0,
                   const void *c1, const void *c2, int n_steps, int ckpt_every,
                   const void *lambda_T, void *grad_psi0, void *grad_c0, void *grad_c1,
                   void *grad_c2)
{
    TraceRange trace_range("mpdata_adv_adj");
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    if (plan->batched) return fail(MPDATA_EINVAL, "adjoint needs a single-grid plan");
    if (plan->desc.opts & (MPDATA_OPT_ABS | MPDATA_OPT_DFL))
        return fail(MPDATA_EUNSUPPORTED, "the reverse mode does not cover the abs / dfl options");
    if (!psi0 || !lambda_T || !grad_psi0) return fail(MPDATA_EINVAL, "NULL argument");
    if (n_steps < 1 || ckpt_every < 1 || ckpt_every > n_steps)
        return fail(MPDATA_EINVAL, "need 1 <= ckpt_every <= n_steps (got %d, %d)", ckpt_every,
                    n_steps);
    const void *c[3] = {c0, c1, c2};
    void *gc[3] = {grad_c0, grad_c1, grad_c2};
    for (int d = 0; d < 3; d++) {
        bool want = d < plan->desc.n_dims;
        if (want && (!c[d] || !gc[d])) return fail(MPDATA_EINVAL, "c%d / grad_c%d is NULL", d, d);
        if (!want && (c[d] || gc[d])) return fail(MPDATA_EINVAL, "c%d given for a %d-D plan", d,
                                                  plan->desc.n_dims);
    }
    if ((g != nullptr) != (plan->desc.has_g != 0)) return fail(MPDATA_EINVAL, "g / has_g mismatch");
    size_t need = mpdata_adj_workspace_bytes(&plan->desc, n_steps, ckpt_every);
    if (plan->ws_bytes < need)
        return fail(MPDATA_EWORKSPACE, "adjoint needs %zu workspace bytes, plan has %zu", need,
                    plan->ws_bytes);
    char *extra = (char *)plan->ws + plan->L.bytes;
    AdjStepCtx sc{plan, g, {c0, c1, c2}};
    hipError_t e;
    if (plan->desc.dtype == MPDATA_F64) {
        mp::AdjArgs<double> a;
        mp::adj_fill_args<double>(a, plan->g, plan->desc.n_iters, plan->desc.opts,
                                  (const double *)psi0, (const double *)g,
                                  (const double *const *)c, n_steps, ckpt_every,
                                  (const double *)lambda_T, (double *)grad_psi0, (double **)gc,
                                  extra);
        a.plain_step = adj_plain_step<double>;
        a.plain_ctx = &sc;
        e = mp::adjoint_run<double>(a, plan->stream);
    } else {
        mp::AdjArgs<float> a;
        mp::adj_fill_args<float>(a, plan->g, plan->desc.n_iters, plan->desc.opts,
                                 (const float *)psi0, (const float *)g, (const float *const *)c,
                                 n_steps, ckpt_every, (const float *)lambda_T,
                                 (float *)grad_psi0, (float **)gc, extra);
        a.plain_step = adj_plain_step<float>;
        a.plain_ctx = &sc;
        e = mp::adjoint_run<float>(a, plan->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(plan->stream);
    if (e != hipSuccess) return hip_fail(e, "adjoint");
    return MPDATA_OK;
}

}  // extern "C"

namespace {

void drop_graph(mpdata_plan *p)
{
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->gexec = nullptr;
    p->graph = nullptr;
    p->g_steps = -1;
}

// (Re)build the batched work list for chunks of `rows` rows and upload it to
// the workspace (waits for the upload).  Cached graphs refer to the old list
// and are dropped.
int batched_table(mpdata_plan *p, int rows)
{
    if (rows < 1 || rows > (1 << 20)) return fail(MPDATA_EINVAL, "tile rows %d out of range", rows);
    int tc = mp::fused2d_strip_cols(p->desc.n_iters, p->desc.opts);
    int64_t tiles = 0;
    for (mp::BatchGrid &G : p->grids) {
        G.tiles_w = (int)mp::cdiv(G.n1, tc);
        G.tile_begin = (int)tiles;
        tiles += (int64_t)G.tiles_w * mp::cdiv(G.n0, rows);
        if (tiles > (int64_t)1 << 30) return fail(MPDATA_EINVAL, "too many tiles");
    }
    hipError_t e = hipStreamSynchronize(p->stream);   // no launch may still read the old list
    if (e == hipSuccess)
        e = hipMemcpyAsync(p->grids_dev, p->grids.data(), sizeof(mp::BatchGrid) * p->grids.size(),
                           hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "batched table upload");
    p->batch_tiles = (int)tiles;
    p->tile_rows = rows;
    drop_graph(p);
    return MPDATA_OK;
}

}  // namespace

extern "C" {

// ------------------------------------------------------------------ batched
size_t mpdata_batched_workspace_bytes(int n_grids, const int64_t *shapes, int dtype, int n_iters,
                                      uint32_t opts, int bc)
{
    (void)n_iters;
    (void)opts;
    (void)bc;
    if (n_grids < 1 || !shapes || (dtype != MPDATA_F32 && dtype != MPDATA_F64)) return 0;
    int64_t tot = 0;
    for (int i = 0; i < n_grids; i++) {
        if (shapes[2 * i] < 3 || shapes[2 * i + 1] < 3) return 0;
        tot += shapes[2 * i] * shapes[2 * i + 1];
    }
    return align_up(sizeof(mp::BatchGrid) * (size_t)n_grids) + align_up(dsize(dtype) * tot);
}

int mpdata_batched_init(int n_grids, const int64_t *shapes, int dtype, int n_iters, uint32_t opts,
                        int bc, void *workspace, size_t ws_bytes, void *hip_stream,
                        mpdata_plan **out)
{
    if (!out) return fail(MPDATA_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_grids < 1 || !shapes) return fail(MPDATA_EINVAL, "need n_grids >= 1 and shapes");
    mpdata_desc d;
    memset(&d, 0, sizeof d);
    d.n_dims = 2;
    d.dtype = dtype;
    d.n_iters = n_iters;
    d.opts = opts;
    d.bc[0] = d.bc[1] = bc;
    mp::Geom g;
    for (int i = 0; i < n_grids; i++) {
        d.shape[0] = shapes[2 * i];
        d.shape[1] = shapes[2 * i + 1];
        int rc = check_desc(&d, &g);
        if (rc) return fail(rc, "grid %d: %s", i, g_err.c_str());
    }
    if (!mp::fused2d_supported(2, n_iters, opts, 0, bc, bc))
        return fail(MPDATA_EUNSUPPORTED, "no batched kernel for these options");
    size_t need = mpdata_batched_workspace_bytes(n_grids, shapes, dtype, n_iters, opts, bc);
    if (!workspace || ws_bytes < need || (uintptr_t)workspace % ALIGN)
        return fail(MPDATA_EWORKSPACE, "batched workspace: need %zu aligned bytes", need);
    mpdata_plan *p = new (std::nothrow) mpdata_plan();
    if (!p) return fail(MPDATA_EINVAL, "out of host memory");
    p->desc = d;
    p->batched = true;
    p->ws = workspace;
    p->ws_bytes = ws_bytes;
    p->stream = (hipStream_t)hip_stream;
    p->kernel = MPDATA_KERNEL_FUSED;
    memset(&p->L, 0, sizeof p->L);
    p->grids.resize(n_grids);
    int64_t op = 0, o0 = 0, o1 = 0;
    for (int i = 0; i < n_grids; i++) {
        mp::BatchGrid &G = p->grids[i];
        G.n0 = shapes[2 * i];
        G.n1 = shapes[2 * i + 1];
        G.off_psi = op;
        G.off_c0 = o0;
        G.off_c1 = o1;
        op += G.n0 * G.n1;
        o0 += (G.n0 + 1) * G.n1;
        o1 += G.n0 * (G.n1 + 1);
    }
    p->batch_psi_total = op;
    p->batch_c0_total = o0;
    p->batch_c1_total = o1;
    Carver c(workspace);
    p->grids_dev = (mp::BatchGrid *)c.take(sizeof(mp::BatchGrid) * n_grids);
    p->batch_alt = c.take(dsize(dtype) * op);
    int rc = batched_table(p, mp::fused2d_tile_rows());
    if (rc) {
        delete p;
        return rc;
    }
    *out = p;
    return MPDATA_OK;
}

}  // extern "C"

namespace {

template <typename T>
hipError_t batched_launches(mpdata_plan *p, T *psi, const T *c0, const T *c1, int n_steps)
{
    T *alt = (T *)p->batch_alt;
    T *cur = psi, *nxt = alt;
    hipError_t e = hipSuccess;
    if (n_steps & 1) {
        e = hipMemcpyAsync(alt, psi, sizeof(T) * p->batch_psi_total, hipMemcpyDeviceToDevice,
                           p->stream);
        if (e != hipSuccess) return e;
        cur = alt;
        nxt = psi;
    }
    for (int s = 0; s < n_steps; s++) {
        e = mp::fused2d_batched_step<T>(p->grids_dev, (int)p->grids.size(), p->batch_tiles,
                                        p->desc.bc[0], p->desc.n_iters, p->desc.opts,
                                        p->tile_rows, p->batch_xcd, cur, nxt, c0, c1, p->stream);
        if (e != hipSuccess) return e;
        T *t = cur;
        cur = nxt;
        nxt = t;
    }
    return e;
}

template <typename T>
hipError_t per_grid_launches(mpdata_plan *p, T *psi, const T *c0, const T *c1, int n_steps)
{
    T *alt = (T *)p->batch_alt;
    hipError_t e = hipSuccess;
    for (const mp::BatchGrid &G : p->grids) {
        T *gp = psi + G.off_psi, *ga = alt + G.off_psi;
        const T *g0 = c0 + G.off_c0, *g1 = c1 + G.off_c1;
        T *cur = gp, *nxt = ga;
        if (n_steps & 1) {
            e = hipMemcpyAsync(ga, gp, sizeof(T) * G.n0 * G.n1, hipMemcpyDeviceToDevice, p->stream);
            if (e != hipSuccess) return e;
            cur = ga;
            nxt = gp;
        }
        mp::Fused2DShape sh{G.n0, G.n1, p->desc.bc[0], p->desc.bc[1], 0};
        for (int s = 0; s < n_steps; s++) {
            e = mp::fused2d_step<T>(sh, p->desc.n_iters, p->desc.opts, cur, nxt, g0, g1, nullptr,
                                    p->stream);
            if (e != hipSuccess) return e;
            T *t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    return e;
}

}  // namespace

extern "C" {

int mpdata_step_batched(mpdata_plan *plan, void *psi, const void *c0, const void *c1,
                        int n_steps, int use_graph)
{
    TraceRange trace_range("mpdata_step_batched");
    if (!plan || !plan->batched) return fail(MPDATA_EINVAL, "not a batched plan");
    if (!psi || !c0 || !c1) return fail(MPDATA_EINVAL, "NULL buffer");
    if (n_steps < 0) return fail(MPDATA_EINVAL, "n_steps < 0");
    if (n_steps == 0) return MPDATA_OK;
    bool f64 = plan->desc.dtype == MPDATA_F64;
    auto launch = [&]() -> hipError_t {
        return f64 ? batched_launches<double>(plan, (double *)psi, (const double *)c0,
                                              (const double *)c1, n_steps)
                   : batched_launches<float>(plan, (float *)psi, (const float *)c0,
                                             (const float *)c1, n_steps);
    };
    if (!use_graph) {
        hipError_t e = launch();
        return e == hipSuccess ? MPDATA_OK : hip_fail(e, "batched launch");
    }
    bool hit = plan->gexec && plan->g_key[0] == psi && plan->g_key[1] == c0 &&
               plan->g_key[2] == c1 && plan->g_steps == n_steps;
    if (!hit) {
        drop_graph(plan);
        if (!plan->cap_stream) {
            hipError_t e = hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking);
            if (e != hipSuccess) {
                plan->cap_stream = nullptr;
                return hip_fail(e, "hipStreamCreateWithFlags");
            }
        }
        hipStream_t user = plan->stream;
        plan->stream = plan->cap_stream;
        hipError_t e = hipStreamBeginCapture(plan->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            plan->stream = user;
            return hip_fail(e, "hipStreamBeginCapture");
        }
        hipError_t le = launch();
        hipGraph_t gr = nullptr;
        e = hipStreamEndCapture(plan->stream, &gr);
        plan->stream = user;
        if (le != hipSuccess) {
            if (gr) (void)hipGraphDestroy(gr);
            return hip_fail(le, "batched launch under capture");
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&plan->gexec, gr, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(gr);
            return hip_fail(e, "hipGraphInstantiate");
        }
        plan->graph = gr;
        plan->g_key[0] = psi;
        plan->g_key[1] = c0;
        plan->g_key[2] = c1;
        plan->g_steps = n_steps;
    }
    hipError_t e = hipGraphLaunch(plan->gexec, plan->stream);
    return e == hipSuccess ? MPDATA_OK : hip_fail(e, "hipGraphLaunch");
}

int mpdata_set_batched_tiling(mpdata_plan *plan, int tile_rows, int xcd_order)
{
    if (!plan || !plan->batched) return fail(MPDATA_EINVAL, "not a batched plan");
    if (tile_rows < 0) return fail(MPDATA_EINVAL, "tile rows %d < 0", tile_rows);
    plan->batch_xcd = xcd_order ? 1 : 0;
    drop_graph(plan);
    return batched_table(plan, tile_rows ? tile_rows : mp::fused2d_tile_rows());
}

int mpdata_autotune_batched(mpdata_plan *plan, const void *psi, const void *c0, const void *c1,
                            int *out_tile_rows, int *out_xcd_order)
{
    TraceRange trace_range("mpdata_autotune_batched");
    if (!plan || !plan->batched) return fail(MPDATA_EINVAL, "not a batched plan");
    if (!psi || !c0 || !c1 || !out_tile_rows || !out_xcd_order)
        return fail(MPDATA_EINVAL, "NULL argument");
    static const int cand[] = {16, 24, 32, 48, 64, 96, 128, 192, 256};
    const bool f64 = plan->desc.dtype == MPDATA_F64;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    int best_rows = plan->tile_rows, best_x = plan->batch_xcd, rc = MPDATA_OK;
    float best = 0.0f;
    // one step from psi into the workspace buffer (psi itself is not written)
    auto one = [&]() -> hipError_t {
        return f64 ? mp::fused2d_batched_step<double>(
                         plan->grids_dev, (int)plan->grids.size(), plan->batch_tiles,
                         plan->desc.bc[0], plan->desc.n_iters, plan->desc.opts, plan->tile_rows,
                         plan->batch_xcd, (const double *)psi, (double *)plan->batch_alt,
                         (const double *)c0, (const double *)c1, plan->stream)
                   : mp::fused2d_batched_step<float>(
                         plan->grids_dev, (int)plan->grids.size(), plan->batch_tiles,
                         plan->desc.bc[0], plan->desc.n_iters, plan->desc.opts, plan->tile_rows,
                         plan->batch_xcd, (const float *)psi, (float *)plan->batch_alt,
                         (const float *)c0, (const float *)c1, plan->stream);
    };
    for (int x = 0; x < 2 && e == hipSuccess && rc == MPDATA_OK; x++)
        for (int rows : cand) {
            plan->batch_xcd = x;
            rc = batched_table(plan, rows);
            if (rc) break;
            e = one();                                   // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, plan->stream);
            for (int r = 0; r < 3 && e == hipSuccess; r++) e = one();
            if (e == hipSuccess) e = hipEventRecord(e1, plan->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) break;
            if (best == 0.0f || ms < best) {
                best = ms;
                best_rows = rows;
                best_x = x;
            }
        }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) rc = hip_fail(e, "batched autotune");
    plan->batch_xcd = best_x;
    int rc2 = batched_table(plan, best_rows);
    if (rc == MPDATA_OK) rc = rc2;
    *out_tile_rows = plan->tile_rows;
    *out_xcd_order = plan->batch_xcd;
    return rc;
}

int mpdata_step_per_grid(mpdata_plan *plan, void *psi, const void *c0, const void *c1,
                         int n_steps)
{
    TraceRange trace_range("mpdata_step_per_grid");
    if (!plan || !plan->batched) return fail(MPDATA_EINVAL, "not a batched plan");
    if (!psi || !c0 || !c1) return fail(MPDATA_EINVAL, "NULL buffer");
    if (n_steps < 0) return fail(MPDATA_EINVAL, "n_steps < 0");
    if (n_steps == 0) return MPDATA_OK;
    hipError_t e = plan->desc.dtype == MPDATA_F64
                       ? per_grid_launches<double>(plan, (double *)psi, (const double *)c0,
                                                   (const double *)c1, n_steps)
                       : per_grid_launches<float>(plan, (float *)psi, (const float *)c0,
                                                  (const float *)c1, n_steps);
    return e == hipSuccess ? MPDATA_OK : hip_fail(e, "per-grid launch");
}

int mpdata_timing(mpdata_plan *plan, int max_launches)
{
    if (!plan) return fail(MPDATA_EINVAL, "plan is NULL");
    if (max_launches < 0) return fail(MPDATA_EINVAL, "max_launches %d < 0", max_launches);
    if (plan->batched) return fail(MPDATA_EINVAL, "timing needs a single-grid plan");
    plan->t_launches = 0;
    plan->t_limit = max_launches;
    plan->tname = "";
    plan->timing = false;
    if (max_launches == 0) return MPDATA_OK;
    for (int i = 0; i < 2; i++) {
        if (plan->tev[i]) continue;
        hipError_t e = hipEventCreate(&plan->tev[i]);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    plan->timing = true;
    return MPDATA_OK;
}

int mpdata_timing_read(mpdata_plan *plan, double *total_ms, int *launches, const char **kernel)
{
    if (!plan || !total_ms || !launches) return fail(MPDATA_EINVAL, "NULL argument");
    *total_ms = 0.0;
    *launches = plan->t_launches;
    if (kernel) *kernel = plan->tname;
    if (plan->t_launches == 0) return MPDATA_OK;
    hipError_t e = hipSuccess;
    if (plan->t_launches < plan->t_limit) {
        // the window is not full: close it now, after the launches made
        e = hipEventRecord(plan->tev[1], plan->stream);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    e = hipEventSynchronize(plan->tev[1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0.0f;
    e = hipEventElapsedTime(&ms, plan->tev[0], plan->tev[1]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    *total_ms = ms;
    return MPDATA_OK;
}

void mpdata_destroy(mpdata_plan *plan)
{
    if (!plan) return;
    for (hipEvent_t ev : plan->tev)
        if (ev) (void)hipEventDestroy(ev);
    if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    delete plan;
}

}  // extern "C"

// ------------------------------------------------- allocation-free diagnostics
// mpdata_diag_noalloc keeps the block partials and the result in `scratch`, a
// file-scope device array of fixed size, instead of a plan's workspace.  In
// host code the array's name stands for a host-side shadow, not device
// memory: its device address is looked up once per device, with that device
// current, and only that address is passed to kernels and copies.
namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
// partials of at most 1024 blocks (5 doubles each) and the result (4 doubles)
constexpr int NOALLOC_PART = 5 * 1024;
constexpr int NOALLOC_DOUBLES = NOALLOC_PART + 8;

static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

std::mutex g_scratch_mu;
double *g_scratch_ptr[NOALLOC_MAX_DEVICES];

// device address of the current device's scratch array
int scratch_ptr(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(MPDATA_EUNSUPPORTED, "device %d beyond the %d the library keeps scratch for",
                    dev, NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress");
        if (!p) return fail(MPDATA_EHIP, "hipGetSymbolAddress returned NULL");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return MPDATA_OK;
}

}  // namespace

extern "C" {

int mpdata_diag_noalloc(int dtype, int64_t n_cells, const void *psi, const void *g,
                        void *hip_stream, double out_sum_min_max[3], int64_t *n_nonfinite)
{
    TraceRange trace_range("mpdata_diag_noalloc");
    if (!psi || !out_sum_min_max || !n_nonfinite) return fail(MPDATA_EINVAL, "NULL argument");
    if (dtype != MPDATA_F32 && dtype != MPDATA_F64)
        return fail(MPDATA_EINVAL, "unknown dtype %d", dtype);
    if (n_cells < 1 || n_cells > ((int64_t)1 << 40))
        return fail(MPDATA_EINVAL, "n_cells %lld outside 1..2^40", (long long)n_cells);
    if (mp::diag_max_blocks() * 5 > NOALLOC_PART)
        return fail(MPDATA_EINVAL, "the scratch array holds fewer partials than one call makes");
    double *base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    double *part = base, *res = base + NOALLOC_PART;
    hipError_t e = dtype == MPDATA_F64
                       ? mp::diag_launch<double>((const double *)psi, (const double *)g, n_cells,
                                                 part, res, s)
                       : mp::diag_launch<float>((const float *)psi, (const float *)g, n_cells,
                                                part, res, s);
    if (e != hipSuccess) return hip_fail(e, "diag launch");
    double h[4];
    e = hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "diag copy");
    out_sum_min_max[0] = h[0];
    out_sum_min_max[1] = h[1];
    out_sum_min_max[2] = h[2];
    *n_nonfinite = (int64_t)h[3];
    if (*n_nonfinite > 0)
        return fail(MPDATA_ENONFINITE, "%lld non-finite values", (long long)*n_nonfinite);
    return MPDATA_OK;
}

}  // extern "C"
