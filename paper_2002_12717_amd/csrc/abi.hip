// C-ABI entry points of the G1-G2 library (declared in include/g1g2.h).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <new>
#include <vector>

#include "ctx.h"

g1g2_status set_error(g1g2_ctx* c, g1g2_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

void prof_mark(g1g2_ctx* c, const char* name) {
    if (!c->prof) return;
    if (c->prof_used == c->prof_ev.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        c->prof_ev.push_back(e);
        c->prof_name.push_back(name);
    }
    c->prof_name[c->prof_used] = name;
    (void)hipEventRecord(c->prof_ev[c->prof_used], c->stream);
    ++c->prof_used;
}

namespace {

struct HostCopy {
    std::vector<cd> v;
    const cd* p = nullptr;
};

// Bring an input array to the host (it may be a device pointer).
g1g2_status fetch(g1g2_ctx* c, const void* src, size_t n, HostCopy& out) {
    if (!src) {
        out.p = nullptr;
        return G1G2_OK;
    }
    if (c->d.flags & G1G2_PTR_DEVICE) {
        out.v.resize(n);
        HIP_OK(c, hipMemcpyAsync(out.v.data(), src, n * sizeof(cd), hipMemcpyDeviceToHost, c->stream));
        HIP_OK(c, hipStreamSynchronize(c->stream));
        out.p = out.v.data();
    } else {
        out.p = (const cd*)src;
    }
    return G1G2_OK;
}

size_t g1_count(const g1g2_ctx* c) {
    const size_t nb = c->d.nb;
    if (c->d.basis == G1G2_JELLIUM) return 2 * nb;
    return c->d.basis == G1G2_HUBBARD ? 2 * nb * nb : nb * nb;
}
// Channels of the stored G2: Hubbard GW and DSL keep up-down-up-down,
// up-up-up-up and down-down-down-down; every other closure one block.
size_t g2_channels(const g1g2_desc& d) {
    return d.basis == G1G2_HUBBARD && (d.selfenergy == G1G2_GW || d.selfenergy == G1G2_DSL) ? 3 : 1;
}
size_t g2_count(const g1g2_ctx* c) {
    const size_t nb = c->d.nb;
    if (c->d.basis == G1G2_JELLIUM) return 3 * nb * nb * nb;   // up-up, up-down, down-down blocks
    return g2_channels(c->d) * nb * nb * nb * nb;
}

g1g2_status alloc_regs(g1g2_ctx* c, Regs& r) {
    HIP_OK(c, hipMalloc(&r.g1, c->n1 * sizeof(cd)));
    HIP_OK(c, hipMalloc(&r.g2, c->n2 * sizeof(cd)));
    HIP_OK(c, hipMemsetAsync(r.g1, 0, c->n1 * sizeof(cd), c->stream));
    HIP_OK(c, hipMemsetAsync(r.g2, 0, c->n2 * sizeof(cd), c->stream));
    return G1G2_OK;
}

void free_regs(Regs& r) {
    if (r.g1) (void)hipFree(r.g1);
    if (r.g2) (void)hipFree(r.g2);
    r = Regs();
}

// Copy an ABI-layout array (host or device as given by `device`) into an
// internal register component.
g1g2_status load_component(g1g2_ctx* c, const void* src, bool device, cd* dst, int rank) {
    const size_t n = rank == 2 ? g1_count(c) : g2_count(c);
    const hipMemcpyKind kind = device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (c->d.basis != G1G2_GENERAL) {   // internal layout = ABI layout
        HIP_OK(c, hipMemcpyAsync(dst, src, n * sizeof(cd), kind, c->stream));
        return G1G2_OK;
    }
    cd* tmp = (rank == 2) ? c->io.g1 : c->io.g2;  // unpadded staging in scratch
    HIP_OK(c, hipMemcpyAsync(tmp, src, n * sizeof(cd), kind, c->stream));
    return gen_pad(c, tmp, dst, rank);
}

g1g2_status store_component(g1g2_ctx* c, const cd* src, void* dst, bool device, int rank) {
    const size_t n = rank == 2 ? g1_count(c) : g2_count(c);
    const hipMemcpyKind kind = device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (c->d.basis != G1G2_GENERAL) {
        HIP_OK(c, hipMemcpyAsync(dst, src, n * sizeof(cd), kind, c->stream));
        return G1G2_OK;
    }
    cd* tmp = (rank == 2) ? c->io.g1 : c->io.g2;
    g1g2_status s = gen_unpad(c, src, tmp, rank);
    if (s != G1G2_OK) return s;
    HIP_OK(c, hipMemcpyAsync(dst, tmp, n * sizeof(cd), kind, c->stream));
    return G1G2_OK;
}

g1g2_status stage(g1g2_ctx* c, int mode, double t, const Regs& in, const Regs& y, const Regs& acc,
                  const Regs& out, double cb, double cc) {
    if (c->d.basis == G1G2_HUBBARD) return hub_stage(c, mode, t, in, y, acc, out, cb, cc);
    if (c->d.basis == G1G2_JELLIUM) return jel_stage(c, mode, in, y, acc, out, cb, cc);
    return gen_stage(c, mode, t, in, y, acc, out, cb, cc);
}

// One classical RK4 step on the registers (y, acc, s0, s1).
g1g2_status rk4_step(g1g2_ctx* c, double t, double dt) {
    g1g2_status s;
    if ((s = stage(c, RK_FIRST, t, c->y, c->y, c->acc, c->s0, dt / 6.0, dt / 2.0)) != G1G2_OK) return s;
    if ((s = stage(c, RK_MID, t + 0.5 * dt, c->s0, c->y, c->acc, c->s1, dt / 3.0, dt / 2.0)) != G1G2_OK)
        return s;
    if ((s = stage(c, RK_MID, t + 0.5 * dt, c->s1, c->y, c->acc, c->s0, dt / 3.0, dt)) != G1G2_OK) return s;
    return stage(c, RK_LAST, t + dt, c->s0, c->y, c->acc, c->y, dt / 6.0, 0.0);
}

__global__ void guard_count_kernel(unsigned long long* div, unsigned long long steps) { div[0] = steps; }

// Allocate the divergence guard of n clusters, all clear.
g1g2_status guard_alloc(g1g2_ctx* c, int n) {
    HIP_OK(c, hipMalloc(&c->dflag, sizeof(int)));
    HIP_OK(c, hipMalloc(&c->ddiv, (size_t)(n + 1) * sizeof(unsigned long long)));
    c->nguard = n;
    return G1G2_OK;
}

// Clear the guard: no cluster has diverged.
g1g2_status guard_clear(g1g2_ctx* c) {
    HIP_OK(c, hipMemsetAsync(c->dflag, 0, sizeof(int), c->stream));
    HIP_OK(c, hipMemsetAsync(c->ddiv, 0xff, (size_t)(c->nguard + 1) * sizeof(unsigned long long), c->stream));
    return G1G2_OK;
}

// First diverged step of every cluster (-1: none); synchronizes the stream.
g1g2_status guard_read(g1g2_ctx* c, std::vector<long long>& first) {
    std::vector<unsigned long long> h((size_t)c->nguard + 1);
    HIP_OK(c, hipMemcpyAsync(h.data(), c->ddiv, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                             c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    first.assign(c->nguard, -1);
    for (int q = 0; q < c->nguard; ++q)
        if (h[q + 1] != ~0ull) first[q] = (long long)h[q + 1];
    return G1G2_OK;
}

void drop_graph(g1g2_ctx* c) {
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
    c->graph_steps = 0;
}

// Steps per captured graph: g1g2_step_rk4 replays it for every whole group of
// that many steps and launches the rest one by one.
constexpr int GRAPH_STEPS = 8;

// Kernel arguments of a step do not depend on t unless a drive or a switching
// ramp is set, so a captured sequence of steps can be replayed for any t.
bool can_capture(const g1g2_ctx* c) {
    return c->graphs && c->stream != nullptr && !c->prof &&
           !c->has_switch() && !(c->d.basis == G1G2_HUBBARD && c->hub.has_drive());
}

g1g2_status capture(g1g2_ctx* c, double dt, int gsteps) {
    drop_graph(c);
    HIP_OK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    g1g2_status s = G1G2_OK;
    for (int n = 0; n < gsteps && s == G1G2_OK; ++n) s = rk4_step(c, 0.0, dt);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (s != G1G2_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    HIP_OK(c, e);
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_OK(c, e);
    c->graph_dt = dt;
    c->graph_steps = gsteps;
    return G1G2_OK;
}

}  // namespace

extern "C" {

const char* g1g2_strerror(g1g2_status s) {
    switch (s) {
        case G1G2_OK: return "ok";
        case G1G2_EINVAL: return "invalid argument";
        case G1G2_ENOMEM: return "out of device memory";
        case G1G2_EDEVICE: return "HIP device error";
        case G1G2_EUNSUPPORTED: return "unsupported configuration";
        case G1G2_EDIVERGED: return "propagation diverged";
        case G1G2_ESTATE: return "invalid state";
    }
    return "unknown status";
}

const char* g1g2_last_error(const g1g2_ctx* c) { return c ? c->err.c_str() : "null context"; }

void g1g2_destroy(g1g2_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_regs(c->y);
    free_regs(c->acc);
    free_regs(c->s0);
    free_regs(c->s1);
    free_regs(c->io);
    if (c->dflag) (void)hipFree(c->dflag);
    if (c->ddiv) (void)hipFree(c->ddiv);
    if (c->dscratch) (void)hipFree(c->dscratch);
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    adj_free(c);
    hub_free(c);
    gen_free(c);
    jel_free(c);
    delete c;
}

g1g2_status g1g2_init(g1g2_ctx** out, const g1g2_desc* d, const void* h0, const void* w,
                      const void* G1_0, const void* G2_0, void* hip_stream) {
    if (!out || !d || !h0 || !G1_0) return G1G2_EINVAL;
    *out = nullptr;
    if (d->nb <= 0) return G1G2_EINVAL;
    if (d->basis != G1G2_GENERAL && d->basis != G1G2_HUBBARD) return G1G2_EINVAL;   // jellium: g1g2_jellium_init
    if (d->selfenergy < G1G2_SOA || d->selfenergy > G1G2_DSL) return G1G2_EINVAL;
    if (d->precision != G1G2_FP64 && d->precision != G1G2_MIXED) return G1G2_EINVAL;
    if (d->basis == G1G2_GENERAL && !w) return G1G2_EINVAL;
    if (d->basis == G1G2_GENERAL && d->nb > 64) return G1G2_EUNSUPPORTED;
    if ((d->flags & G1G2_DSL_EXCHANGE) && !(d->basis == G1G2_GENERAL && d->selfenergy == G1G2_DSL))
        return G1G2_EUNSUPPORTED;
    if (d->basis == G1G2_HUBBARD && (long long)d->nb * d->nb * d->nb * d->nb > (1LL << 30))
        return G1G2_EUNSUPPORTED;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return G1G2_EDEVICE;

    g1g2_ctx* c = new (std::nothrow) g1g2_ctx();
    if (!c) return G1G2_ENOMEM;
    c->d = *d;
    c->stream = (hipStream_t)hip_stream;
    {
        const char* ng = std::getenv("G1G2_NO_GRAPH");
        c->graphs = !(ng && ng[0] == '1');
    }
    (void)hipGetDevice(&c->device);
    g1g2_status s = G1G2_OK;
    const size_t nb = d->nb;
    if (d->basis == G1G2_HUBBARD) {
        c->n1 = 2 * nb * nb;
        c->n2 = g2_channels(*d) * nb * nb * nb * nb;
    } else {
        const size_t nbp = ((nb + 15) / 16) * 16;
        c->n1 = nbp * nbp;
        c->n2 = nbp * nbp * nbp * nbp;
    }
    auto fail = [&](g1g2_status st) {
        std::string e = c->err;
        g1g2_destroy(c);
        (void)e;
        return st;
    };
    for (Regs* r : {&c->y, &c->acc, &c->s0, &c->s1, &c->io})
        if ((s = alloc_regs(c, *r)) != G1G2_OK) return fail(s);
    if ((s = guard_alloc(c, 1)) != G1G2_OK || (s = guard_clear(c)) != G1G2_OK) return fail(s);
    if (d->basis == G1G2_HUBBARD && (s = hub_noalloc_setup(c)) != G1G2_OK) return fail(s);
    c->nscratch = 8 + 3 * 256 + 3 * (int)nb + 64;
    if (hipMalloc(&c->dscratch, c->nscratch * sizeof(double)) != hipSuccess) return fail(G1G2_ENOMEM);

    HostCopy hh0, hw;
    const size_t nh0 = g1_count(c);
    if ((s = fetch(c, h0, nh0, hh0)) != G1G2_OK) return fail(s);
    if (d->basis == G1G2_HUBBARD) {
        const int ns = d->nb;
        const double U = d->U;
        const cd* h0p = hh0.p;
        if ((s = hub_setup(c, 1, &ns, &U, &h0p, nullptr)) != G1G2_OK) return fail(s);
    } else {
        if ((s = fetch(c, w, g2_count(c), hw)) != G1G2_OK) return fail(s);
        if ((s = gen_setup(c, hh0.p, hw.p)) != G1G2_OK) return fail(s);
    }
    const bool dev = d->flags & G1G2_PTR_DEVICE;
    if ((s = load_component(c, G1_0, dev, c->y.g1, 2)) != G1G2_OK) return fail(s);
    if (G2_0) {
        if ((s = load_component(c, G2_0, dev, c->y.g2, 4)) != G1G2_OK) return fail(s);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(G1G2_EDEVICE);
    *out = c;
    return G1G2_OK;
}

g1g2_status g1g2_jellium_init(g1g2_ctx** out, const g1g2_desc* d, const int32_t* dims, const double* eps,
                              const double* v, const void* G1_0, const void* G2_0, void* hip_stream) {
    if (!out || !d || !dims || !eps || !v || !G1_0) return G1G2_EINVAL;
    *out = nullptr;
    if (d->basis != G1G2_JELLIUM) return G1G2_EINVAL;
    if (d->selfenergy < G1G2_SOA || d->selfenergy > G1G2_DSL) return G1G2_EINVAL;
    if (d->precision != G1G2_FP64 && d->precision != G1G2_MIXED) return G1G2_EINVAL;
    if (d->flags & ~(G1G2_PTR_DEVICE | G1G2_GW_EXCHANGE | G1G2_JEL_LAD_ROWS2)) return G1G2_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (dims[k] < 1 || dims[k] > 1024) return G1G2_EINVAL;
    const long long nbl = (long long)dims[0] * dims[1] * dims[2];
    if (nbl != d->nb) return G1G2_EINVAL;
    if (d->selfenergy == G1G2_DSL) return G1G2_EUNSUPPORTED;
    if (nbl > jel_max_nb()) return G1G2_EUNSUPPORTED;
    if (v[0] != 0.0) return G1G2_EINVAL;   // the neutralizing background removes v_0
    for (long long q = 0; q < nbl; ++q)
        if (!std::isfinite(v[q]) || !std::isfinite(eps[q]) || !std::isfinite(eps[nbl + q])) return G1G2_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return G1G2_EDEVICE;
    g1g2_ctx* c = new (std::nothrow) g1g2_ctx();
    if (!c) return G1G2_ENOMEM;
    c->d = *d;
    c->stream = (hipStream_t)hip_stream;
    {
        const char* ng = std::getenv("G1G2_NO_GRAPH");
        c->graphs = !(ng && ng[0] == '1');
    }
    (void)hipGetDevice(&c->device);
    const size_t nb = (size_t)nbl;
    c->n1 = 2 * nb;
    c->n2 = 3 * nb * nb * nb;
    auto fail = [&](g1g2_status st) {
        g1g2_destroy(c);
        return st;
    };
    g1g2_status s;
    for (Regs* r : {&c->y, &c->acc, &c->s0, &c->s1, &c->io})
        if ((s = alloc_regs(c, *r)) != G1G2_OK) return fail(s);
    if ((s = guard_alloc(c, 1)) != G1G2_OK || (s = guard_clear(c)) != G1G2_OK) return fail(s);
    c->nscratch = 64;
    if (hipMalloc(&c->dscratch, c->nscratch * sizeof(double)) != hipSuccess) return fail(G1G2_ENOMEM);
    const int dd[3] = {dims[0], dims[1], dims[2]};
    if ((s = jel_setup(c, dd, eps, v)) != G1G2_OK) return fail(s);
    const bool dev = d->flags & G1G2_PTR_DEVICE;
    if ((s = load_component(c, G1_0, dev, c->y.g1, 2)) != G1G2_OK) return fail(s);
    if (G2_0 && (s = load_component(c, G2_0, dev, c->y.g2, 4)) != G1G2_OK) return fail(s);
    if ((s = jel_state_changed(c)) != G1G2_OK) return fail(s);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(G1G2_EDEVICE);
    *out = c;
    return G1G2_OK;
}

g1g2_status g1g2_rhs(g1g2_ctx* c, double t, const void* G1, const void* G2, void* dG1, void* dG2) {
    if (!c || !G1 || !G2 || !dG1 || !dG2) return G1G2_EINVAL;
    if (c->d.basis == G1G2_HUBBARD && c->hub.ncl != 1)
        return set_error(c, G1G2_ESTATE, "single-cluster call on a batch");
    g1g2_status s;
    if (c->d.basis != G1G2_GENERAL) {   // caller buffers in the internal layout
        Regs in{(cd*)G1, (cd*)G2};
        Regs out{(cd*)dG1, (cd*)dG2};
        s = c->d.basis == G1G2_HUBBARD ? hub_stage(c, RK_RHS, t, in, in, in, out, 0.0, 0.0)
                                       : jel_stage(c, RK_RHS, in, in, in, out, 0.0, 0.0);
        if (s != G1G2_OK) return s;
        HIP_OK(c, hipStreamSynchronize(c->stream));
        return G1G2_OK;
    }
    // general: pad into s0 (dead between steps), evaluate into s1, unpad
    if ((s = load_component(c, G1, true, c->s0.g1, 2)) != G1G2_OK) return s;
    if ((s = load_component(c, G2, true, c->s0.g2, 4)) != G1G2_OK) return s;
    if ((s = gen_stage(c, RK_RHS, t, c->s0, c->s0, c->s0, c->s1, 0.0, 0.0)) != G1G2_OK) return s;
    if ((s = store_component(c, c->s1.g1, dG1, true, 2)) != G1G2_OK) return s;
    if ((s = store_component(c, c->s1.g2, dG2, true, 4)) != G1G2_OK) return s;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return G1G2_OK;
}

g1g2_status g1g2_step_rk4(g1g2_ctx* c, double dt, int64_t nsteps) {
    if (!c || nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return G1G2_EINVAL;
    const double t0 = c->t;
    const int64_t step0 = c->step;
    g1g2_status s;
    int64_t n = 0;
    if (nsteps > 0) {   // the steps of this call are numbered from the completed ones
        hipLaunchKernelGGL(guard_count_kernel, dim3(1), dim3(1), 0, c->stream, c->ddiv,
                           (unsigned long long)step0);
        HIP_OK(c, hipGetLastError());
        prof_mark(c, "guard_count");
    }
    if (c->d.basis == G1G2_HUBBARD && hub_persistent_ok(c)) {
        if ((s = hub_step_persistent(c, dt, nsteps)) != G1G2_OK) return s;
        n = nsteps;
    }
    if (n < nsteps && can_capture(c) && nsteps >= GRAPH_STEPS) {
        // one graph of GRAPH_STEPS steps per dt, captured on first use and kept
        if (!c->graph || c->graph_dt != dt)
            if ((s = capture(c, dt, GRAPH_STEPS)) != G1G2_OK) return s;
        for (; n + GRAPH_STEPS <= nsteps; n += GRAPH_STEPS) HIP_OK(c, hipGraphLaunch(c->graph, c->stream));
    }
    for (; n < nsteps; ++n)
        if ((s = rk4_step(c, t0 + (double)n * dt, dt)) != G1G2_OK) return s;
    c->t = t0 + (double)nsteps * dt;
    c->step = step0 + nsteps;
    int flag = 0;
    HIP_OK(c, hipMemcpyAsync(&flag, c->dflag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (flag) {
        std::vector<long long> first;
        if ((s = guard_read(c, first)) != G1G2_OK) return s;
        int q0 = -1, nbad = 0;
        for (int q = 0; q < c->nguard; ++q)
            if (first[q] >= 0) {
                ++nbad;
                if (q0 < 0 || first[q] < first[q0]) q0 = q;
            }
        std::string msg = "non-finite state or occupation outside [-0.5, 1.5]";
        if (q0 >= 0) {
            msg += " after step " + std::to_string(first[q0]);
            if (c->nguard > 1)
                msg += " in cluster " + std::to_string(q0) + " (" + std::to_string(nbad) + " of " +
                       std::to_string(c->nguard) + " clusters flagged; see g1g2_batch_observables)";
        }
        return set_error(c, G1G2_EDIVERGED, msg);
    }
    return G1G2_OK;
}

g1g2_status g1g2_step_path(const g1g2_ctx* c, int32_t* path) {
    if (!c || !path) return G1G2_EINVAL;
    if (c->d.basis == G1G2_GENERAL) *path = G1G2_PATH_GENERAL;
    else if (c->d.basis == G1G2_JELLIUM) *path = G1G2_PATH_JELLIUM;
    else if (hub_persistent_ok(c)) *path = G1G2_PATH_HUB_PERSISTENT;
    else if (c->hub.slices) *path = G1G2_PATH_HUB_SLICE;
    else if (c->hub.rows) *path = G1G2_PATH_HUB_ROW;
    else *path = G1G2_PATH_HUB_ELEMENT;
    return G1G2_OK;
}

g1g2_status g1g2_prepare_graph(g1g2_ctx* c, double dt) {
    if (!c || !(dt > 0.0) || !std::isfinite(dt)) return G1G2_EINVAL;
    if (c->d.basis == G1G2_HUBBARD && hub_persistent_ok(c)) return G1G2_OK;
    if (!can_capture(c) || (c->graph && c->graph_dt == dt)) return G1G2_OK;
    return capture(c, dt, GRAPH_STEPS);
}

g1g2_status g1g2_observables(g1g2_ctx* c, g1g2_obs* o) {
    if (!c || !o) return G1G2_EINVAL;
    if (c->d.basis == G1G2_HUBBARD && c->hub.ncl != 1)
        return set_error(c, G1G2_ESTATE, "use g1g2_batch_observables on a batch");
    std::memset(o, 0, sizeof(*o));
    g1g2_status s = c->d.basis == G1G2_HUBBARD   ? hub_observables(c, c->y, c->t, o)
                    : c->d.basis == G1G2_JELLIUM ? jel_observables(c, c->y, o)
                                                 : gen_observables(c, c->y, c->t, o);
    if (s != G1G2_OK) return s;
    std::vector<long long> first;
    if ((s = guard_read(c, first)) != G1G2_OK) return s;
    o->t = c->t;
    o->step = c->step;
    o->diverged = first[0] >= 0;
    o->diverged_step = first[0];
    return G1G2_OK;
}

g1g2_status g1g2_site_observables(g1g2_ctx* c, double* nu, double* nd, double* docc) {
    if (!c) return G1G2_EINVAL;
    if (c->d.basis != G1G2_HUBBARD) return set_error(c, G1G2_EUNSUPPORTED, "Hubbard basis only");
    if (c->hub.ncl != 1) return set_error(c, G1G2_ESTATE, "single-cluster call on a batch");
    return hub_site_observables(c, c->y, nu, nd, docc);
}

g1g2_status g1g2_get_state(g1g2_ctx* c, void* G1, void* G2, double* t) {
    if (!c || !G1) return G1G2_EINVAL;
    if (c->d.basis == G1G2_HUBBARD && c->hub.ncl != 1)
        return set_error(c, G1G2_ESTATE, "single-cluster call on a batch");
    const bool dev = c->d.flags & G1G2_PTR_DEVICE;
    g1g2_status s;
    if ((s = store_component(c, c->y.g1, G1, dev, 2)) != G1G2_OK) return s;
    if (G2 && (s = store_component(c, c->y.g2, G2, dev, 4)) != G1G2_OK) return s;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (t) *t = c->t;
    return G1G2_OK;
}

g1g2_status g1g2_set_state(g1g2_ctx* c, const void* G1, const void* G2, double t) {
    if (!c || !G1) return G1G2_EINVAL;
    if (c->d.basis == G1G2_HUBBARD && c->hub.ncl != 1)
        return set_error(c, G1G2_ESTATE, "single-cluster call on a batch");
    const bool dev = c->d.flags & G1G2_PTR_DEVICE;
    g1g2_status s;
    if ((s = load_component(c, G1, dev, c->y.g1, 2)) != G1G2_OK) return s;
    if (G2) {
        if ((s = load_component(c, G2, dev, c->y.g2, 4)) != G1G2_OK) return s;
    } else {
        HIP_OK(c, hipMemsetAsync(c->y.g2, 0, c->n2 * sizeof(cd), c->stream));
    }
    if ((s = guard_clear(c)) != G1G2_OK) return s;
    if (c->d.basis == G1G2_JELLIUM && (s = jel_state_changed(c)) != G1G2_OK) return s;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->t = t;
    return G1G2_OK;
}

g1g2_status g1g2_set_h0(g1g2_ctx* c, const void* h0) {
    if (!c || !h0) return G1G2_EINVAL;
    if (c->d.basis == G1G2_JELLIUM) return set_error(c, G1G2_EUNSUPPORTED, "jellium: energies are set at init");
    HostCopy hh;
    g1g2_status s = fetch(c, h0, g1_count(c), hh);
    if (s != G1G2_OK) return s;
    HIP_OK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    if (c->d.basis == G1G2_HUBBARD) {
        if (c->hub.ncl != 1) return set_error(c, G1G2_ESTATE, "set_h0 applies to a single cluster");
        const int ns = c->d.nb;
        const double U = c->d.U;
        const cd* h0p = hh.p;
        return hub_setup(c, 1, &ns, &U, &h0p, nullptr);
    }
    return gen_set_h0(c, hh.p);
}

g1g2_status g1g2_set_U(g1g2_ctx* c, double U) {
    if (!c || !std::isfinite(U)) return G1G2_EINVAL;
    if (c->d.basis != G1G2_HUBBARD) return set_error(c, G1G2_EUNSUPPORTED, "Hubbard basis only");
    if (c->hub.ncl != 1) return set_error(c, G1G2_ESTATE, "set_U applies to a single cluster");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->d.U = U;
    c->hub.hdesc[0].U = U;
    HIP_OK(c, hipMemcpy(c->hub.desc, c->hub.hdesc.data(), sizeof(ClusterDesc), hipMemcpyHostToDevice));
    return G1G2_OK;
}

g1g2_status g1g2_set_drive(g1g2_ctx* c, const double* x, int32_t M, const double* cm,
                           const double* tc, double tau) {
    if (!c || M < 0) return G1G2_EINVAL;
    if (c->d.basis != G1G2_HUBBARD) return set_error(c, G1G2_EUNSUPPORTED, "Hubbard basis only");
    HubbardData& H = c->hub;
    if (H.ncl != 1) return set_error(c, G1G2_ESTATE, "set_drive applies to a single cluster");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    if (M == 0) {
        H.drive_c.clear();
        H.drive_tc.clear();
        return G1G2_OK;
    }
    if (!x || !cm || !tc || !(tau > 0.0)) return G1G2_EINVAL;
    H.drive_c.assign(cm, cm + M);
    H.drive_tc.assign(tc, tc + M);
    H.drive_x.assign(x, x + c->d.nb);
    H.drive_tau = tau;
    HIP_OK(c, hipMemcpy(H.xdrv, x, c->d.nb * sizeof(double), hipMemcpyHostToDevice));
    return G1G2_OK;
}

g1g2_status g1g2_set_switch(g1g2_ctx* c, double t_on, double tau) {
    if (!c || !std::isfinite(t_on) || !std::isfinite(tau) || tau < 0.0) return G1G2_EINVAL;
    if (c->d.basis == G1G2_JELLIUM) return set_error(c, G1G2_EUNSUPPORTED, "jellium: no switching ramp");
    HIP_OK(c, hipStreamSynchronize(c->stream));
    drop_graph(c);
    c->switch_t_on = t_on;
    c->switch_tau = tau;
    return G1G2_OK;
}

double g1g2_ctx::switch_value(double t) const {
    if (switch_tau <= 0.0) return 1.0;
    const double x = (t - switch_t_on) / switch_tau;
    if (x <= 0.0) return 0.0;
    if (x >= 1.0) return 1.0;
    const double s = std::sin(0.5 * M_PI * x);
    return s * s;
}

g1g2_status g1g2_batch_init(g1g2_ctx** out, const g1g2_desc* d, int32_t n, const int32_t* ns,
                            const double* U, const void* const* h0, const void* const* G1_0,
                            const int32_t* chunk, void* hip_stream) {
    if (!out || !d || n < 1 || !ns || !U || !h0 || !G1_0) return G1G2_EINVAL;
    *out = nullptr;
    if (d->basis != G1G2_HUBBARD) return G1G2_EINVAL;
    if (d->selfenergy < G1G2_SOA || d->selfenergy > G1G2_DSL) return G1G2_EINVAL;
    if (d->precision != G1G2_FP64 && d->precision != G1G2_MIXED) return G1G2_EINVAL;
    long long n1 = 0, n2 = 0;
    int nsmax = 0;
    const long long nch = (long long)g2_channels(*d);
    for (int c = 0; c < n; ++c) {
        if (ns[c] < 1 || !h0[c] || !G1_0[c]) return G1G2_EINVAL;
        n1 += 2LL * ns[c] * ns[c];
        n2 += nch * ns[c] * ns[c] * ns[c] * ns[c];
        nsmax = std::max(nsmax, (int)ns[c]);
    }
    if (n2 > (1LL << 31) - 1) return G1G2_EUNSUPPORTED;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return G1G2_EDEVICE;
    g1g2_ctx* c = new (std::nothrow) g1g2_ctx();
    if (!c) return G1G2_ENOMEM;
    c->d = *d;
    c->d.flags &= ~G1G2_PTR_DEVICE;
    c->d.nb = nsmax;
    c->stream = (hipStream_t)hip_stream;
    {
        const char* ng = std::getenv("G1G2_NO_GRAPH");
        c->graphs = !(ng && ng[0] == '1');
    }
    (void)hipGetDevice(&c->device);
    c->n1 = (size_t)n1;
    c->n2 = (size_t)n2;
    g1g2_status s;
    auto fail = [&](g1g2_status st) {
        g1g2_destroy(c);
        return st;
    };
    for (Regs* r : {&c->y, &c->acc, &c->s0, &c->s1})
        if ((s = alloc_regs(c, *r)) != G1G2_OK) return fail(s);
    if ((s = guard_alloc(c, n)) != G1G2_OK || (s = guard_clear(c)) != G1G2_OK) return fail(s);
    if ((s = hub_noalloc_setup(c)) != G1G2_OK) return fail(s);
    c->nscratch = 8 + 3 * 256 + 3 * nsmax + 64;
    if (hipMalloc(&c->dscratch, c->nscratch * sizeof(double)) != hipSuccess) return fail(G1G2_ENOMEM);
    std::vector<int> nsv(ns, ns + n), ch(n, 0);
    if (chunk)
        for (int q = 0; q < n; ++q) ch[q] = chunk[q];
    std::vector<double> Uv(U, U + n);
    std::vector<const cd*> hp(n);
    for (int q = 0; q < n; ++q) hp[q] = (const cd*)h0[q];
    if ((s = hub_setup(c, n, nsv.data(), Uv.data(), hp.data(), ch.data())) != G1G2_OK) return fail(s);
    for (int q = 0; q < n; ++q) {
        const ClusterDesc& cd0 = c->hub.hdesc[q];
        if (hipMemcpyAsync(c->y.g1 + cd0.g1off, G1_0[q], 2ULL * ns[q] * ns[q] * sizeof(cd),
                           hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return fail(G1G2_EDEVICE);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(G1G2_EDEVICE);
    *out = c;
    return G1G2_OK;
}

g1g2_status g1g2_batch_observables(g1g2_ctx* c, g1g2_obs* o) {
    if (!c || !o) return G1G2_EINVAL;
    if (c->d.basis != G1G2_HUBBARD) return set_error(c, G1G2_EUNSUPPORTED, "Hubbard batches only");
    const int n = c->hub.ncl;
    std::memset(o, 0, n * sizeof(g1g2_obs));
    g1g2_status s = hub_batch_observables(c, c->y, c->t, o);
    if (s != G1G2_OK) return s;
    std::vector<long long> first;
    if ((s = guard_read(c, first)) != G1G2_OK) return s;
    for (int q = 0; q < n; ++q) {
        o[q].t = c->t;
        o[q].step = c->step;
        o[q].diverged = first[q] >= 0;
        o[q].diverged_step = first[q];
    }
    return G1G2_OK;
}

g1g2_status g1g2_batch_get_state(g1g2_ctx* c, int32_t cluster, void* G1, void* G2) {
    if (!c || !G1) return G1G2_EINVAL;
    if (c->d.basis != G1G2_HUBBARD || cluster < 0 || cluster >= c->hub.ncl) return G1G2_EINVAL;
    const ClusterDesc& d = c->hub.hdesc[cluster];
    const size_t ns = d.ns;
    HIP_OK(c, hipMemcpyAsync(G1, c->y.g1 + d.g1off, 2 * ns * ns * sizeof(cd), hipMemcpyDeviceToHost,
                             c->stream));
    if (G2)   // the cluster's channels are stored one after another
        HIP_OK(c, hipMemcpyAsync(G2, c->y.g2 + d.g2off, g2_channels(c->d) * ns * ns * ns * ns * sizeof(cd),
                                 hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return G1G2_OK;
}

}  // extern "C"

namespace {

// Per-kernel timing: prof_begin turns on an event after every kernel launch
// (prof_mark), prof_end sums the time between consecutive events per kernel.
g1g2_status prof_begin(g1g2_ctx* c) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->prof = true;
    c->prof_used = 0;
    prof_mark(c, "start");
    return G1G2_OK;
}

g1g2_status prof_end(g1g2_ctx* c, int32_t max_kernels, double* ms_total, int32_t* launches, int32_t* count) {
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->prof_kernels.clear();
    std::vector<double> tot;
    std::vector<int> cnt;
    for (size_t k = 1; k < c->prof_used; ++k) {
        const char* nm = c->prof_name[k];
        if (std::strcmp(nm, "start") == 0) continue;
        float m = 0.f;
        HIP_OK(c, hipEventElapsedTime(&m, c->prof_ev[k - 1], c->prof_ev[k]));
        size_t q = 0;
        while (q < c->prof_kernels.size() && std::strcmp(c->prof_kernels[q], nm) != 0) ++q;
        if (q == c->prof_kernels.size()) {
            c->prof_kernels.push_back(nm);
            tot.push_back(0.0);
            cnt.push_back(0);
        }
        tot[q] += m;
        cnt[q] += 1;
    }
    *count = (int32_t)c->prof_kernels.size();
    for (size_t q = 0; q < c->prof_kernels.size() && (int)q < max_kernels; ++q) {
        ms_total[q] = tot[q];
        launches[q] = cnt[q];
    }
    return G1G2_OK;
}

}  // namespace

extern "C" {

g1g2_status g1g2_profile(g1g2_ctx* c, double dt, int64_t nsteps, int32_t max_kernels,
                         double* ms_total, int32_t* launches, int32_t* count) {
    if (!c || nsteps < 0 || max_kernels < 1 || !ms_total || !launches || !count) return G1G2_EINVAL;
    if (nsteps > 0 && !(dt > 0.0)) return G1G2_EINVAL;
    g1g2_status s;
    if ((s = prof_begin(c)) != G1G2_OK) return s;
    if (nsteps == 0) {
        s = stage(c, RK_RHS, c->t, c->y, c->y, c->y, c->s1, 0.0, 0.0);
    } else {
        s = g1g2_step_rk4(c, dt, nsteps);
    }
    c->prof = false;
    if (s != G1G2_OK) return s;
    return prof_end(c, max_kernels, ms_total, launches, count);
}

g1g2_status g1g2_profile_adjoint(g1g2_ctx* c, const double* a, const double* b, int32_t max_kernels,
                                 double* ms_total, int32_t* launches, int32_t* count) {
    if (!c || !a || !b || max_kernels < 1 || !ms_total || !launches || !count) return G1G2_EINVAL;
    g1g2_status s;
    if ((s = prof_begin(c)) != G1G2_OK) return s;
    s = g1g2_adjoint(c, a, b, nullptr, nullptr, nullptr);
    c->prof = false;
    if (s != G1G2_OK) return s;
    return prof_end(c, max_kernels, ms_total, launches, count);
}

const char* g1g2_profile_name(const g1g2_ctx* c, int32_t k) {
    if (!c || k < 0 || (size_t)k >= c->prof_kernels.size()) return "";
    return c->prof_kernels[k];
}

}  // extern "C"
