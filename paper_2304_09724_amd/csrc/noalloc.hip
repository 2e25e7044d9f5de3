// noalloc.hip -- the batched 1D time loop for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops, harnesses
// that forbid hipMalloc): shw_advance1d_static runs the kernels of
// shw_create + shw_advance_to with every device buffer beyond the caller's
// state carved out of a static array that the library keeps on each GPU.
//
// The array is a file-scope __device__ variable.  In host code its name is a
// host-side stand-in, not a device address: each device's address is looked
// up once, with that device current, by hipGetSymbolAddress, and only that
// address is ever handed to kernels.  Host-side staging lives in static
// arrays too, so a call allocates nothing on the host either.  Calls share
// the array (and the staging, under a mutex): calls that overlap on one GPU
// race on the device array and must be serialised by the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "api_host.h"
#include "shw_kernels.h"

using namespace shw;
using namespace shw::host;

static_assert(SHW_STATIC_SCRATCH_BYTES % 256 == 0, "scratch size is a multiple of 256");

namespace {

__device__ __align__(256) unsigned char scratch[SHW_STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
void *g_scratch[MAX_DEVICES];                 // per device: the address of `scratch`
std::mutex g_lock;                            // guards the host staging below

// host staging (static: no allocation per call)
Inst1D h_inst[SHW_STATIC_MAX_INSTANCES];
int h_order[SHW_STATIC_MAX_INSTANCES];
double h_T[SHW_STATIC_MAX_INSTANCES];
InstState h_ist[SHW_STATIC_MAX_INSTANCES];

// The device address of this device's copy of `scratch` (looked up once per
// device, the device being current).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// zero the per-instance time-loop state (kernels, not memsets: the call may
// sit in code that a caller captures)
__global__ void clear_ist_kernel(InstState *ist, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ist[i] = InstState{};
}

} // namespace

extern "C" shw_status shw_advance1d_static(const shw_mesh *meshes, int n_inst,
                                           const shw_params *params, double *d_state,
                                           const double *T, long long max_steps,
                                           long long *steps_out, void *hip_stream)
{
    if (!valid_batch(meshes, n_inst, params) || !d_state || !T || max_steps < 0)
        return SHW_EINVAL;
    if (meshes[0].dim != 1) return SHW_EINVAL;
    if (params->weights != SHW_W_NONLINEAR && params->weights != SHW_W_LINEAR) return SHW_EINVAL;
    for (int i = 0; i < n_inst; ++i)
        if (!std::isfinite(T[i])) return SHW_EINVAL;
    if (n_inst > SHW_STATIC_MAX_INSTANCES) return SHW_ESCRATCH;
    const Layout lay = make_layout(meshes, n_inst, params);
    if (lay.total > (size_t)SHW_STATIC_SCRATCH_BYTES) return SHW_ESCRATCH;

    std::lock_guard<std::mutex> guard(g_lock);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    void *base = nullptr;
    if (scratch_address(&base) != hipSuccess) return SHW_EDEVICE;
    char *ws = static_cast<char *>(base);

    // descriptors; processing order largest first (the workgroups take
    // instances from a counter, so only the time to solution depends on it)
    long long off = 0, cell = 0;
    for (int i = 0; i < n_inst; ++i) {
        Inst1D d{};
        d.off = off;
        d.cell_off = cell;
        d.n = meshes[i].nx;
        d.bc_lo = meshes[i].bc[0];
        d.bc_hi = meshes[i].bc[1];
        d.dx = (meshes[i].x1 - meshes[i].x0) / meshes[i].nx;
        h_inst[i] = d;
        h_order[i] = i;
        h_T[i] = T[i];
        off += (long long)state_doubles(&meshes[i], params->eq);
        cell += meshes[i].nx;
    }
    std::sort(h_order, h_order + n_inst, [&](int a, int b) {
        return meshes[a].nx != meshes[b].nx ? meshes[a].nx > meshes[b].nx : a < b;
    });
    hipError_t e = hipMemcpyAsync(ws + lay.inst, h_inst, n_inst * sizeof(Inst1D),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + lay.order, h_order, n_inst * sizeof(int), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ws + lay.t_end, h_T, n_inst * sizeof(double), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return SHW_EDEVICE;
    InstState *ist = reinterpret_cast<InstState *>(ws + lay.ist);
    clear_ist_kernel<<<(n_inst + 255) / 256, 256, 0, st>>>(ist, n_inst);
    if (hipGetLastError() != hipSuccess) return SHW_EDEVICE;

    Loop1D L{};
    L.inst = reinterpret_cast<const Inst1D *>(ws + lay.inst);
    L.n_inst = n_inst;
    L.order = reinterpret_cast<const int *>(ws + lay.order);
    L.queue = reinterpret_cast<int *>(ws + lay.queue);
    L.state = d_state;
    L.alt = reinterpret_cast<double *>(ws + lay.alt);
    L.t_end = reinterpret_cast<const double *>(ws + lay.t_end);
    L.dt_fixed = nullptr;
    L.max_steps = max_steps;
    L.ist = ist;
    L.flags = reinterpret_cast<uint8_t *>(ws + lay.flags);
    L.gate = nullptr;
    L.gate_every = 1;
    L.share = 0.0;
    if (params->positivity) {
        L.faces = reinterpret_cast<double *>(ws + lay.faces);
        L.trouble = reinterpret_cast<uint8_t *>(ws + lay.trouble);
    }
    const DevParams dp = make_devparams(params);
    const int variant = 1;
    const int grid = std::min(loop1d_max_blocks(params->eq, variant, false, params->positivity != 0),
                              n_inst);
    e = launch_loop1d(params->eq, L, dp, grid, variant, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_ist, ist, n_inst * sizeof(InstState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return SHW_EDEVICE;
    shw_status r = SHW_OK;
    for (int i = 0; i < n_inst; ++i) {
        if (steps_out) steps_out[i] = h_ist[i].steps;
        if (h_ist[i].code != 0) r = SHW_ENONPHYS;
    }
    return r;
}
