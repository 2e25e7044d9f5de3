// shweno_api.cpp -- host side of the C ABI declared in include/shweno.h:
// argument checking, the device workspace layout, launches and error
// reporting.  All arithmetic of the scheme runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/shweno.h"
#include "api_host.h"
#include "shw_kernels.h"

using namespace shw;

using namespace shw::host;

struct shw_ctx {
    int n_inst = 0, dim = 1, m = 1;
    shw_params params{};
    DevParams dp{};
    std::vector<shw_mesh> meshes;
    std::vector<long long> off, cell_off;
    double *state = nullptr;
    char *ws = nullptr;
    Layout lay;
    hipStream_t stream = nullptr;
    int grid1d = 1;
    int variant = -1;                   // tile variant in use (set at create)
    int tiles2d[N_TILE_VARIANTS][2] = {};
    bool gate_loaded = false;
    int bad_instance = -1;
    std::vector<int> order_host;        // 1D: the last launch's instance order (kept
                                        // alive for its asynchronous upload)
    std::string msg;
    // 2D: a chunk of steps captured once as a HIP graph and replayed
    bool use_graphs = true;
    hipGraphExec_t chunk_exec = nullptr;
    hipStream_t capture_stream = nullptr;   // capture cannot run on the null stream

    ~shw_ctx()
    {
        if (chunk_exec) (void)hipGraphExecDestroy(chunk_exec);
        if (capture_stream) (void)hipStreamDestroy(capture_stream);
    }

    template <class T> T *at(size_t o) { return reinterpret_cast<T *>(ws + o); }
    double *alt() { return at<double>(lay.alt); }
    InstState *ist() { return at<InstState>(lay.ist); }

    shw_status fail(shw_status s, const std::string &m_) { msg = m_; return s; }
    shw_status hip(hipError_t e, const char *what)
    {
        if (e == hipSuccess) return SHW_OK;
        msg = std::string(what) + ": " + hipGetErrorString(e);
        return SHW_EDEVICE;
    }
};

extern "C" {

const char *shw_version(void) { return "shweno-gfx950 0.1"; }

size_t shw_state_doubles(const shw_mesh *mesh, const shw_params *params)
{
    if (!valid_mesh(mesh) || !valid_params(params)) return 0;
    return state_doubles(mesh, params->eq);
}

size_t shw_workspace_bytes(const shw_mesh *meshes, int n_inst, const shw_params *params)
{
    if (!valid_batch(meshes, n_inst, params)) return 0;
    return make_layout(meshes, n_inst, params).total;
}

shw_status shw_create(const shw_mesh *meshes, int n_inst, const shw_params *params,
                      double *d_state, void *d_workspace, void *hip_stream, shw_ctx **out)
{
    if (!out) return SHW_EINVAL;
    *out = nullptr;
    if (!valid_batch(meshes, n_inst, params) || !d_state || !d_workspace) return SHW_EINVAL;
    shw_ctx *c = new (std::nothrow) shw_ctx;
    if (!c) return SHW_ENOMEM;
    c->n_inst = n_inst;
    c->dim = meshes[0].dim;
    c->m = ncomp(params->eq, c->dim);
    c->params = *params;
    c->meshes.assign(meshes, meshes + n_inst);
    c->state = d_state;
    c->ws = static_cast<char *>(d_workspace);
    c->lay = make_layout(meshes, n_inst, params);
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->dp = make_devparams(params);

    long long o = 0, co = 0, fo = 0;
    std::vector<Inst1D> i1;
    std::vector<Inst2D> i2;
    std::vector<int> toff[N_TILE_VARIANTS][2];
    for (auto &tv : toff) tv[0] = tv[1] = std::vector<int>(1, 0);
    for (int i = 0; i < n_inst; ++i) {
        const shw_mesh &m = meshes[i];
        c->off.push_back(o);
        c->cell_off.push_back(co);
        if (c->dim == 1) {
            Inst1D d{};
            d.off = o;
            d.cell_off = co;
            d.n = m.nx;
            d.bc_lo = m.bc[0];
            d.bc_hi = m.bc[1];
            d.dx = (m.x1 - m.x0) / m.nx;
            i1.push_back(d);
        } else {
            Inst2D d{};
            d.off = o;
            d.cell_off = co;
            d.face_off = fo;
            fo += 20LL * ((long long)m.ny * (m.nx + 1) + (long long)(m.ny + 1) * m.nx);
            d.nx = m.nx;
            d.ny = m.ny;
            for (int k = 0; k < 4; ++k) d.bc[k] = m.bc[k];
            d.dx = (m.x1 - m.x0) / m.nx;
            d.dy = (m.y1 - m.y0) / m.ny;
            i2.push_back(d);
            for (int v = 0; v < N_TILE_VARIANTS; ++v) {
                toff[v][0].push_back(toff[v][0].back() + sweep2d_tiles(m.nx, m.ny, lines2d(v)));
                toff[v][1].push_back(toff[v][1].back() + sweep2d_tiles(m.ny, m.nx, lines2d(v)));
            }
        }
        o += (long long)state_doubles(&m, params->eq);
        co += (long long)m.nx * m.ny;
    }
    // largest instances first: a greedy schedule of the persistent loop
    std::vector<int> order(n_inst);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        double wa = (double)meshes[a].nx * meshes[a].ny, wb = (double)meshes[b].nx * meshes[b].ny;
        return wa * wa > wb * wb;
    });
    shw_status s = SHW_OK;
    if (c->dim == 1) {
        s = c->hip(hipMemcpyAsync(c->ws + c->lay.inst, i1.data(), i1.size() * sizeof(Inst1D),
                                  hipMemcpyHostToDevice, c->stream), "copy instances");
        c->variant = 1;
        c->grid1d = loop1d_max_blocks(params->eq, c->variant, params->weights == SHW_W_LEARNED,
                                      params->positivity != 0);
    } else {
        s = c->hip(hipMemcpyAsync(c->ws + c->lay.inst, i2.data(), i2.size() * sizeof(Inst2D),
                                  hipMemcpyHostToDevice, c->stream), "copy instances");
        const size_t per = (size_t)(n_inst + 1);
        for (int v = 0; v < N_TILE_VARIANTS && s == SHW_OK; ++v) {
            s = c->hip(hipMemcpyAsync(c->ws + c->lay.tiles0 + v * per * sizeof(int), toff[v][0].data(),
                                      per * sizeof(int), hipMemcpyHostToDevice, c->stream),
                       "copy tiles");
            if (s == SHW_OK)
                s = c->hip(hipMemcpyAsync(c->ws + c->lay.tiles1 + v * per * sizeof(int),
                                          toff[v][1].data(), per * sizeof(int),
                                          hipMemcpyHostToDevice, c->stream), "copy tiles");
            c->tiles2d[v][0] = toff[v][0].back();
            c->tiles2d[v][1] = toff[v][1].back();
        }
        c->variant = 2;
    }
    if (s == SHW_OK)
        s = c->hip(hipMemsetAsync(c->ws + c->lay.parity, 0, n_inst * sizeof(int), c->stream),
                   "clear parity");
    if (s == SHW_OK)
        s = c->hip(hipMemsetAsync(c->ws + c->lay.bad, 0, n_inst * sizeof(int), c->stream),
                   "clear flags");
    if (s == SHW_OK)
        s = c->hip(hipMemcpyAsync(c->ws + c->lay.order, order.data(), n_inst * sizeof(int),
                                  hipMemcpyHostToDevice, c->stream), "copy order");
    if (s == SHW_OK)
        s = c->hip(hipMemsetAsync(c->ws + c->lay.ist, 0, n_inst * sizeof(InstState), c->stream),
                   "clear instance state");
    if (s == SHW_OK)
        s = c->hip(hipMemsetAsync(c->ws + c->lay.flags, 1, (size_t)co, c->stream), "set flags");
    if (s == SHW_OK) s = c->hip(hipStreamSynchronize(c->stream), "create");
    if (s != SHW_OK) {
        delete c;
        return s;
    }
    *out = c;
    return SHW_OK;
}

void shw_destroy(shw_ctx *ctx) { delete ctx; }

shw_status shw_set_state(shw_ctx *c, int inst, const double *src, int on_device)
{
    if (!c || !src || inst < 0 || inst >= c->n_inst) return SHW_EINVAL;
    size_t n = state_doubles(&c->meshes[inst], c->params.eq);
    shw_status s = c->hip(hipMemcpyAsync(c->state + c->off[inst], src, n * sizeof(double),
                                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                         c->stream), "set_state");
    if (s != SHW_OK) return s;
    // clear the sticky non-physical flag of this instance
    s = c->hip(hipMemsetAsync(reinterpret_cast<char *>(c->ist() + inst) + offsetof(InstState, code),
                              0, sizeof(int), c->stream), "set_state flag");
    if (s != SHW_OK) return s;
    s = c->hip(hipMemsetAsync(c->ws + c->lay.bad + inst * sizeof(int), 0, sizeof(int), c->stream),
               "set_state flag");
    if (s != SHW_OK) return s;
    if (!on_device) return c->hip(hipStreamSynchronize(c->stream), "set_state sync");
    return SHW_OK;
}

shw_status shw_get_state(shw_ctx *c, int inst, double *dst, int on_device)
{
    if (!c || !dst || inst < 0 || inst >= c->n_inst) return SHW_EINVAL;
    size_t n = state_doubles(&c->meshes[inst], c->params.eq);
    shw_status s = c->hip(hipMemcpyAsync(dst, c->state + c->off[inst], n * sizeof(double),
                                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                         c->stream), "get_state");
    if (s != SHW_OK || on_device) return s;
    return c->hip(hipStreamSynchronize(c->stream), "get_state sync");
}

static shw_status read_ist(shw_ctx *c, std::vector<InstState> &h)
{
    h.resize(c->n_inst);
    shw_status s = c->hip(hipMemcpyAsync(h.data(), c->ist(), c->n_inst * sizeof(InstState),
                                         hipMemcpyDeviceToHost, c->stream), "read times");
    if (s != SHW_OK) return s;
    return c->hip(hipStreamSynchronize(c->stream), "read times sync");
}

shw_status shw_get_time(shw_ctx *c, double *t, long long *steps)
{
    if (!c) return SHW_EINVAL;
    std::vector<InstState> h;
    shw_status s = read_ist(c, h);
    if (s != SHW_OK) return s;
    for (int i = 0; i < c->n_inst; ++i) {
        if (t) t[i] = h[i].t;
        if (steps) steps[i] = h[i].steps;
    }
    return SHW_OK;
}

shw_status shw_instance_status(shw_ctx *c, int *codes)
{
    if (!c || !codes) return SHW_EINVAL;
    std::vector<InstState> h;
    shw_status s = read_ist(c, h);
    if (s != SHW_OK) return s;
    for (int i = 0; i < c->n_inst; ++i) codes[i] = h[i].code ? SHW_ENONPHYS : SHW_OK;
    return SHW_OK;
}

shw_status shw_set_time(shw_ctx *c, const double *t)
{
    if (!c || !t) return SHW_EINVAL;
    std::vector<InstState> h;
    shw_status s = read_ist(c, h);
    if (s != SHW_OK) return s;
    for (int i = 0; i < c->n_inst; ++i) h[i].t = t[i];
    s = c->hip(hipMemcpyAsync(c->ist(), h.data(), c->n_inst * sizeof(InstState),
                              hipMemcpyHostToDevice, c->stream), "set_time");
    if (s != SHW_OK) return s;
    return c->hip(hipStreamSynchronize(c->stream), "set_time sync");
}

static Step2D step2d_args(shw_ctx *c);

shw_status shw_compute_dt(shw_ctx *c, double *dt)
{
    if (!c || !dt) return SHW_EINVAL;
    double *d_dt = c->at<double>(c->lay.dt);
    shw_status s;
    if (c->dim == 1) {
        s = c->hip(launch_dt1d(c->params.eq, c->at<Inst1D>(c->lay.inst), c->n_inst, c->state,
                               c->dp, d_dt, c->stream), "dt1d");
    } else {
        Step2D S = step2d_args(c);
        s = c->hip(launch_speed2d(c->params.eq, S, c->dp, 0, c->stream), "speed2d");
        if (s != SHW_OK) return s;
        std::vector<double> smax(c->n_inst);
        std::vector<int> bad(c->n_inst);
        s = c->hip(hipMemcpyAsync(smax.data(), S.smax, c->n_inst * sizeof(double),
                                  hipMemcpyDeviceToHost, c->stream), "smax copy");
        if (s == SHW_OK)
            s = c->hip(hipMemcpyAsync(bad.data(), S.bad, c->n_inst * sizeof(int),
                                      hipMemcpyDeviceToHost, c->stream), "bad copy");
        if (s == SHW_OK) s = c->hip(hipStreamSynchronize(c->stream), "dt sync");
        if (s != SHW_OK) return s;
        for (int i = 0; i < c->n_inst; ++i)
            dt[i] = bad[i] ? -1.0 : c->params.cfl / smax[i];
    }
    if (c->dim == 1) {
        if (s != SHW_OK) return s;
        s = c->hip(hipMemcpyAsync(dt, d_dt, c->n_inst * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream), "dt copy");
        if (s != SHW_OK) return s;
        s = c->hip(hipStreamSynchronize(c->stream), "dt sync");
        if (s != SHW_OK) return s;
    }
    for (int i = 0; i < c->n_inst; ++i)
        if (!(dt[i] > 0.0)) {
            c->bad_instance = i;
            return c->fail(SHW_ENONPHYS, "non-physical cell average");
        }
    return SHW_OK;
}

static Step2D step2d_args(shw_ctx *c)
{
    Step2D S{};
    S.inst = c->at<Inst2D>(c->lay.inst);
    S.n_inst = c->n_inst;
    S.tile_off[0] = c->at<int>(c->lay.tiles0) + (size_t)c->variant * (c->n_inst + 1);
    S.tile_off[1] = c->at<int>(c->lay.tiles1) + (size_t)c->variant * (c->n_inst + 1);
    S.act_inst = c->at<int>(c->lay.act_inst);
    S.act_off[0] = c->at<int>(c->lay.act_off0);
    S.act_off[1] = c->at<int>(c->lay.act_off1);
    S.act_n = c->at<int>(c->lay.act_n);
    S.state = c->state;
    S.alt = c->alt();
    S.parity = c->at<int>(c->lay.parity);
    S.dt = c->at<double>(c->lay.dt);
    S.last = c->at<int>(c->lay.last);
    S.dt_fixed = c->at<double>(c->lay.dt_fixed);
    S.t_end = c->at<double>(c->lay.t_end);
    S.steps_left = c->at<long long>(c->lay.steps_left);
    S.smax = c->at<double>(c->lay.smax);
    S.bad = c->at<int>(c->lay.bad);
    S.active = c->at<int>(c->lay.active);
    S.ist = c->ist();
    S.flags = c->at<uint8_t>(c->lay.flags);
    S.gate = c->at<GateLane>(c->lay.gate);
    const double th = c->params.gate_threshold;
    S.gate_logit_min = (th > 0.0 && th < 1.0) ? (float)std::log(th / (1.0 - th)) : 0.0f;
    if (c->params.positivity) {
        S.faces = c->at<double>(c->lay.faces);
        S.trouble = c->at<uint8_t>(c->lay.trouble);
        S.guard = c->at<int>(c->lay.guard);
    }
    return S;
}

static Loop1D loop_args(shw_ctx *c)
{
    Loop1D L{};
    L.inst = c->at<Inst1D>(c->lay.inst);
    L.n_inst = c->n_inst;
    L.order = c->at<int>(c->lay.order);
    L.queue = c->at<int>(c->lay.queue);
    L.state = c->state;
    L.alt = c->alt();
    L.ist = c->ist();
    L.flags = c->at<uint8_t>(c->lay.flags);
    L.gate = c->at<GateLane>(c->lay.gate);
    const double th = c->params.gate_threshold;
    L.gate_logit_min = (th > 0.0 && th < 1.0) ? (float)std::log(th / (1.0 - th)) : 0.0f;
    L.gate_every = c->params.gate_every > 0 ? c->params.gate_every : 1;
    if (c->params.positivity) {
        L.faces = c->at<double>(c->lay.faces);
        L.trouble = c->at<uint8_t>(c->lay.trouble);
    }
    return L;
}

shw_status shw_step(shw_ctx *c, const double *dt)
{
    if (!c || !dt) return SHW_EINVAL;
    for (int i = 0; i < c->n_inst; ++i)
        if (!std::isfinite(dt[i])) return SHW_EINVAL;
    if (c->params.weights == SHW_W_LEARNED && !c->gate_loaded)
        return c->fail(SHW_ESTATE, "learned gate not loaded");
    if (c->dim == 2) {
        Step2D S = step2d_args(c);
        shw_status s = c->hip(hipMemcpyAsync(const_cast<double *>(S.dt_fixed), dt,
                                             c->n_inst * sizeof(double), hipMemcpyHostToDevice,
                                             c->stream), "step dt");
        if (s != SHW_OK) return s;
        s = c->hip(launch_step2d(c->params.eq, S, c->dp, 1, c->tiles2d[c->variant],
                                 lines2d(c->variant), c->stream), "step2d");
        if (s != SHW_OK) return s;
        return c->hip(launch_settle2d(S, c->m, c->stream), "settle");
    }
    double *d_dt = c->at<double>(c->lay.dt);
    shw_status s = c->hip(hipMemcpyAsync(d_dt, dt, c->n_inst * sizeof(double),
                                         hipMemcpyHostToDevice, c->stream), "step dt");
    if (s != SHW_OK) return s;
    Loop1D L = loop_args(c);
    L.dt_fixed = d_dt;
    L.t_end = nullptr;
    L.max_steps = 1;
    int grid = std::min(c->grid1d, c->n_inst);
    return c->hip(launch_loop1d(c->params.eq, L, c->dp, grid, c->variant, c->stream), "step");
}

// 2D time loop: steps run on the device in chunks; the host only polls the
// number of instances still running between chunks.  A full chunk is one
// replay, on the context's stream, of a HIP graph captured on the first call
// on a private stream (its kernels take only device pointers fixed for the
// context, so every replay does the same as launching them; the graph holds
// kernels only).
constexpr int CHUNK_STEPS = 8;

static shw_status chunk_graph(shw_ctx *c, const Step2D &S)
{
    if (c->chunk_exec) return SHW_OK;
    shw_status s = SHW_OK;
    if (!c->capture_stream)
        s = c->hip(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking),
                   "capture stream");
    if (s == SHW_OK)
        s = c->hip(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal),
                   "begin capture");
    if (s != SHW_OK) return s;
    hipError_t launch = hipSuccess;
    for (int j = 0; j < CHUNK_STEPS && launch == hipSuccess; ++j)
        launch = launch_step2d(c->params.eq, S, c->dp, 0, c->tiles2d[c->variant], lines2d(c->variant),
                               c->capture_stream);
    hipGraph_t g = nullptr;
    s = c->hip(hipStreamEndCapture(c->capture_stream, &g), "end capture");
    if (s == SHW_OK) s = c->hip(launch, "capture step2d");
    if (s == SHW_OK) s = c->hip(hipGraphInstantiate(&c->chunk_exec, g, nullptr, nullptr, 0),
                                "instantiate");
    if (g) (void)hipGraphDestroy(g);
    if (s != SHW_OK) c->chunk_exec = nullptr;
    return s;
}

static shw_status advance2d(shw_ctx *c, long long max_steps)
{
    Step2D S = step2d_args(c);
    std::vector<long long> budget(c->n_inst, max_steps);
    shw_status s = c->hip(hipMemcpyAsync(S.steps_left, budget.data(), c->n_inst * sizeof(long long),
                                         hipMemcpyHostToDevice, c->stream), "budget");
    if (s != SHW_OK) return s;
    s = c->hip(launch_speed2d(c->params.eq, S, c->dp, 1, c->stream), "speed2d");
    if (s != SHW_OK) return s;
    for (long long done = 0; done < max_steps;) {
        const int k = (int)std::min<long long>(CHUNK_STEPS, max_steps - done);
        if (k == CHUNK_STEPS && c->use_graphs) {
            s = chunk_graph(c, S);
            if (s == SHW_OK) s = c->hip(hipGraphLaunch(c->chunk_exec, c->stream), "graph launch");
            if (s != SHW_OK) return s;
        } else {
            for (int j = 0; j < k; ++j) {
                s = c->hip(launch_step2d(c->params.eq, S, c->dp, 0, c->tiles2d[c->variant],
                                         lines2d(c->variant), c->stream), "step2d");
                if (s != SHW_OK) return s;
            }
        }
        done += k;
        int active = 0;
        s = c->hip(hipMemcpyAsync(&active, S.active, sizeof(int), hipMemcpyDeviceToHost, c->stream),
                   "active");
        if (s == SHW_OK) s = c->hip(hipStreamSynchronize(c->stream), "active sync");
        if (s != SHW_OK) return s;
        if (active == 0) break;
    }
    return c->hip(launch_settle2d(S, c->m, c->stream), "settle");
}

static shw_status run_to(shw_ctx *c, const double *T, long long max_steps);

shw_status shw_set_tile(shw_ctx *c, int variant)
{
    if (!c || variant < 0 || variant >= N_TILE_VARIANTS) return SHW_EINVAL;
    if (variant == c->variant) return SHW_OK;
    if (c->chunk_exec) {                  // the captured chunk holds the old tiles
        (void)hipGraphExecDestroy(c->chunk_exec);
        c->chunk_exec = nullptr;
    }
    c->variant = variant;
    if (c->dim == 1)
        c->grid1d = loop1d_max_blocks(c->params.eq, variant, c->params.weights == SHW_W_LEARNED,
                                          c->params.positivity != 0);
    return SHW_OK;
}

shw_status shw_get_tile(shw_ctx *c, int *variant)
{
    if (!c || !variant) return SHW_EINVAL;
    *variant = c->variant;
    return SHW_OK;
}

shw_status shw_autotune(shw_ctx *c, double *d_scratch, int steps, int *best, float *ms)
{
    if (!c || !d_scratch || steps < 1 || steps > 100000) return SHW_EINVAL;
    if (c->params.weights == SHW_W_LEARNED && !c->gate_loaded)
        return c->fail(SHW_ESTATE, "learned gate not loaded");
    size_t nd = 0;
    for (const auto &m : c->meshes) nd += state_doubles(&m, c->params.eq);
    std::vector<InstState> saved;
    std::vector<int> saved_bad(c->n_inst);
    shw_status s = read_ist(c, saved);
    // the per-instance non-physical flags (2D reads them at the next step)
    if (s == SHW_OK)
        s = c->hip(hipMemcpyAsync(saved_bad.data(), c->ws + c->lay.bad, c->n_inst * sizeof(int),
                                  hipMemcpyDeviceToHost, c->stream), "save flags");
    if (s == SHW_OK) s = c->hip(hipStreamSynchronize(c->stream), "save flags sync");
    if (s == SHW_OK)
        s = c->hip(hipMemcpyAsync(d_scratch, c->state, nd * sizeof(double), hipMemcpyDeviceToDevice,
                                  c->stream), "save state");
    if (s != SHW_OK) return s;
    auto restore = [&]() {
        shw_status r = c->hip(hipMemcpyAsync(c->state, d_scratch, nd * sizeof(double),
                                             hipMemcpyDeviceToDevice, c->stream), "restore state");
        if (r == SHW_OK)
            r = c->hip(hipMemcpyAsync(c->ist(), saved.data(), c->n_inst * sizeof(InstState),
                                      hipMemcpyHostToDevice, c->stream), "restore times");
        if (r == SHW_OK)
            r = c->hip(hipMemcpyAsync(c->ws + c->lay.bad, saved_bad.data(), c->n_inst * sizeof(int),
                                      hipMemcpyHostToDevice, c->stream), "restore flags");
        return r;
    };
    // every instance steps: no end time within reach
    const std::vector<double> far(c->n_inst, 1e300);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    s = c->hip(hipEventCreate(&e0), "event");
    if (s == SHW_OK) s = c->hip(hipEventCreate(&e1), "event");
    const int start = c->variant;
    float t_best = 0.0f;
    int v_best = start;
    float t_v[N_TILE_VARIANTS] = {};
    for (int v = 0; v < N_TILE_VARIANTS && s == SHW_OK; ++v) {
        s = shw_set_tile(c, v);
        float t = 0.0f;
        for (int rep = 0; rep < 2 && s == SHW_OK; ++rep) {       // warm (and capture), timed
            s = restore();
            if (s == SHW_OK) s = c->hip(hipEventRecord(e0, c->stream), "event");
            if (s == SHW_OK) s = run_to(c, far.data(), steps);
            if (s == SHW_OK) s = c->hip(hipEventRecord(e1, c->stream), "event");
            if (s == SHW_OK) s = c->hip(hipEventSynchronize(e1), "event sync");
            if (s == SHW_OK) s = c->hip(hipEventElapsedTime(&t, e0, e1), "event time");
        }
        if (s != SHW_OK) break;
        if (ms) ms[v] = t;
        t_v[v] = t;
        if (v == 0 || t < t_best) {
            t_best = t;
            v_best = v;
        }
    }
    // 1D: the probe keeps every instance busy, but a whole run ends on its
    // longest instance, which finishes sooner the more threads advance it;
    // so among the variants within 3 % of the fastest the one with the most
    // threads per instance is kept
    if (s == SHW_OK && c->dim == 1)
        for (int v = N_TILE_VARIANTS - 1; v > v_best; --v)
            if (t_v[v] <= 1.03f * t_best) {
                v_best = v;
                break;
            }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    shw_status r = restore();
    if (s == SHW_OK) s = r;
    if (s == SHW_OK) s = c->hip(hipStreamSynchronize(c->stream), "autotune sync");
    const shw_status t = shw_set_tile(c, s == SHW_OK ? v_best : start);
    if (s == SHW_OK) s = t;
    if (s == SHW_OK && best) *best = v_best;
    return s;
}

shw_status shw_set_graphs(shw_ctx *c, int enable)
{
    if (!c) return SHW_EINVAL;
    c->use_graphs = enable != 0;
    return SHW_OK;
}

// 1D schedule of a CFL launch towards T: each instance's work is estimated as
// its cells times the steps its current CFL step size needs to reach T (at
// most max_steps); the persistent workgroups take instances heaviest first,
// and share is the work per workgroup if it were spread evenly (the kernel's
// wave priorities are set against it).
static shw_status schedule1d(shw_ctx *c, const double *T, long long max_steps, int grid,
                             double &share)
{
    const int n = c->n_inst;
    double *d_dt = c->at<double>(c->lay.dt);
    shw_status s = c->hip(launch_dt1d(c->params.eq, c->at<Inst1D>(c->lay.inst), n, c->state,
                                      c->dp, d_dt, c->stream), "schedule dt");
    std::vector<double> dt(n);
    if (s == SHW_OK)
        s = c->hip(hipMemcpyAsync(dt.data(), d_dt, n * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream), "schedule dt copy");
    std::vector<InstState> ist;
    if (s == SHW_OK) s = read_ist(c, ist);
    if (s != SHW_OK) return s;
    std::vector<double> work(n, 0.0);
    double total = 0.0;
    for (int i = 0; i < n; ++i) {
        if (ist[i].code != 0 || !(dt[i] > 0.0) || !(T[i] > ist[i].t)) continue;
        const double steps = std::min((double)max_steps, std::ceil((T[i] - ist[i].t) / dt[i]));
        work[i] = (double)c->meshes[i].nx * steps;
        total += work[i];
    }
    c->order_host.resize(n);
    std::iota(c->order_host.begin(), c->order_host.end(), 0);
    std::stable_sort(c->order_host.begin(), c->order_host.end(),
                     [&](int a, int b) { return work[a] > work[b]; });
    share = total / std::max(grid, 1);
    return c->hip(hipMemcpyAsync(c->ws + c->lay.order, c->order_host.data(), n * sizeof(int),
                                 hipMemcpyHostToDevice, c->stream), "schedule order");
}

// CFL steps towards the end times T (host array) with the current tile
// variant; asynchronous except for the 2D chunk polls and the 1D schedule.
static shw_status run_to(shw_ctx *c, const double *T, long long max_steps)
{
    double *d_T = c->at<double>(c->lay.t_end);
    shw_status s = c->hip(hipMemcpyAsync(d_T, T, c->n_inst * sizeof(double), hipMemcpyHostToDevice,
                                         c->stream), "advance T");
    if (s != SHW_OK) return s;
    if (c->dim == 2) return advance2d(c, max_steps);
    Loop1D L = loop_args(c);
    L.dt_fixed = nullptr;
    L.t_end = d_T;
    L.max_steps = max_steps;
    int grid = std::min(c->grid1d, c->n_inst);
    s = schedule1d(c, T, max_steps, grid, L.share);
    if (s != SHW_OK) return s;
    return c->hip(launch_loop1d(c->params.eq, L, c->dp, grid, c->variant, c->stream), "advance");
}

shw_status shw_advance_to(shw_ctx *c, const double *T, long long max_steps, long long *steps_out)
{
    if (!c || !T || max_steps < 0) return SHW_EINVAL;
    for (int i = 0; i < c->n_inst; ++i)
        if (!std::isfinite(T[i])) return SHW_EINVAL;
    if (c->params.weights == SHW_W_LEARNED && !c->gate_loaded)
        return c->fail(SHW_ESTATE, "learned gate not loaded");
    std::vector<InstState> before;
    shw_status s = read_ist(c, before);
    if (s != SHW_OK) return s;
    s = run_to(c, T, max_steps);
    if (s != SHW_OK) return s;
    std::vector<InstState> after;
    s = read_ist(c, after);
    if (s != SHW_OK) return s;
    shw_status r = SHW_OK;
    for (int i = 0; i < c->n_inst; ++i) {
        if (steps_out) steps_out[i] = after[i].steps - before[i].steps;
        if (after[i].code != 0 && r == SHW_OK) {
            c->bad_instance = i;
            r = c->fail(SHW_ENONPHYS, "non-physical cell average in instance " + std::to_string(i));
        }
    }
    return r;
}

shw_status shw_step_cfl(shw_ctx *c)
{
    if (!c) return SHW_EINVAL;
    // an end time no instance reaches in one step
    const std::vector<double> far(c->n_inst, 1e300);
    return shw_advance_to(c, far.data(), 1, nullptr);
}

shw_status shw_set_flags(shw_ctx *c, int inst, const uint8_t *flags)
{
    if (!c || !flags || inst < 0 || inst >= c->n_inst) return SHW_EINVAL;
    size_t n = (size_t)c->meshes[inst].nx * c->meshes[inst].ny;
    shw_status s = c->hip(hipMemcpyAsync(c->ws + c->lay.flags + c->cell_off[inst], flags, n,
                                         hipMemcpyHostToDevice, c->stream), "set_flags");
    if (s != SHW_OK) return s;
    return c->hip(hipStreamSynchronize(c->stream), "set_flags sync");
}

shw_status shw_get_flags(shw_ctx *c, int inst, uint8_t *flags)
{
    if (!c || !flags || inst < 0 || inst >= c->n_inst) return SHW_EINVAL;
    const size_t n = (size_t)c->meshes[inst].nx * c->meshes[inst].ny;
    shw_status s = c->hip(hipMemcpyAsync(flags, c->ws + c->lay.flags + c->cell_off[inst], n,
                                         hipMemcpyDeviceToHost, c->stream), "get_flags");
    if (s != SHW_OK) return s;
    return c->hip(hipStreamSynchronize(c->stream), "get_flags sync");
}

static unsigned short host_bf16(float f)
{
    unsigned u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

static_assert(GATE_NPAR == SHW_GATE_NPARAMS && GATE_NF == SHW_GATE_NFEATURES,
              "gate sizes of the header and the kernels differ");
static_assert(sizeof(GateLane) == 256, "packed gate lane is 256 bytes");

size_t shw_gate_packed_bytes(void) { return 64 * sizeof(GateLane); }

shw_status shw_gate_pack(const float *p, void *packed)
{
    if (!p || !packed) return SHW_EINVAL;
    const float *W1 = p, *b1 = W1 + GATE_H * GATE_NF, *W2 = b1 + GATE_H, *b2 = W2 + GATE_H * GATE_H;
    const float *w3 = b2 + GATE_H, *b3 = w3 + GATE_H;
    GateLane *out = static_cast<GateLane *>(packed);
    std::memset(out, 0, 64 * sizeof(GateLane));
    for (int lane = 0; lane < 64; ++lane) {
        GateLane &L = out[lane];
        const int r = lane % 32, h = lane / 32;
        for (int i = 0; i < 4; ++i) {
            // BF16 pair (elements 2i, 2i + 1) in one word, element 2i low
            auto pair = [](float a, float b) {
                return (unsigned)host_bf16(a) | ((unsigned)host_bf16(b) << 16);
            };
            L.w1[i] = pair(W1[r * GATE_NF + 8 * h + 2 * i], W1[r * GATE_NF + 8 * h + 2 * i + 1]);
            for (int q = 0; q < 2; ++q)
                L.w2[q][i] = pair(W2[r * GATE_H + gate_hidden(q, h, 2 * i)],
                                  W2[r * GATE_H + gate_hidden(q, h, 2 * i + 1)]);
        }
        for (int v = 0; v < 16; ++v) {
            const int row = mfma_row(lane, v);
            L.b1[v] = b1[row];
            L.b2[v] = b2[row];
            L.w3[v] = w3[row];
        }
        L.b3 = b3[0];
    }
    return SHW_OK;
}

shw_status shw_gate_load(shw_ctx *c, const float *params)
{
    if (!c || !params) return SHW_EINVAL;
    std::vector<GateLane> packed(64);
    shw_gate_pack(params, packed.data());
    shw_status s = c->hip(hipMemcpyAsync(c->ws + c->lay.gate, packed.data(), 64 * sizeof(GateLane),
                                         hipMemcpyHostToDevice, c->stream), "gate load");
    if (s != SHW_OK) return s;
    s = c->hip(hipStreamSynchronize(c->stream), "gate load sync");
    if (s == SHW_OK) c->gate_loaded = true;
    return s;
}

shw_status shw_gate_data(shw_ctx *c, double level, float *d_features, uint8_t *d_labels)
{
    if (!c || !d_features || !d_labels) return SHW_EINVAL;
    if (c->dim != 1 || c->params.eq != SHW_EULER)
        return c->fail(SHW_EINVAL, "gate data: 1D Euler only");
    if (!(level > 0.0 && level <= 1.0))
        return c->fail(SHW_EINVAL, "gate data: label level must lie in (0, 1]");
    int max_n = 0;
    for (const auto &m : c->meshes) max_n = std::max(max_n, m.nx);
    return c->hip(launch_gate_data1d(c->at<Inst1D>(c->lay.inst), c->n_inst, max_n, c->state, c->dp,
                                     level, d_features, d_labels, c->stream), "gate data");
}

shw_status shw_mlp_logits(const float *d_X, int n, const void *d_packed, float *d_logits,
                          void *stream)
{
    if (!d_X || n < 1 || !d_packed || !d_logits) return SHW_EINVAL;
    return launch_mlp_logits(d_X, n, static_cast<const GateLane *>(d_packed), d_logits,
                             static_cast<hipStream_t>(stream)) == hipSuccess ? SHW_OK : SHW_EDEVICE;
}

shw_status shw_mlp_grad(const float *d_X, const float *d_y, int n, const float *d_params,
                        float pos_weight, float *d_grad, float *d_loss, void *stream)
{
    if (!d_X || !d_y || n < 1 || !d_params || !d_grad || !d_loss || !(pos_weight > 0.0f))
        return SHW_EINVAL;
    return launch_mlp_grad(d_X, d_y, n, d_params, pos_weight, d_grad, d_loss,
                           static_cast<hipStream_t>(stream)) == hipSuccess ? SHW_OK : SHW_EDEVICE;
}

shw_status shw_mlp_adam(float *d_params, const float *d_grad, float *d_m, float *d_v, int step,
                        float lr, void *stream)
{
    if (!d_params || !d_grad || !d_m || !d_v || step < 1 || !(lr > 0.0f)) return SHW_EINVAL;
    return launch_adam(d_params, d_grad, d_m, d_v, step, lr, static_cast<hipStream_t>(stream)) ==
                   hipSuccess ? SHW_OK : SHW_EDEVICE;
}

shw_status shw_status_detail(shw_ctx *c, int *bad_instance, char *msg, size_t msg_len)
{
    if (!c) return SHW_EINVAL;
    if (bad_instance) *bad_instance = c->bad_instance;
    if (msg && msg_len) {
        std::strncpy(msg, c->msg.c_str(), msg_len - 1);
        msg[msg_len - 1] = 0;
    }
    return SHW_OK;
}

} // extern "C"
