// Continuous-batching request pool: solve requests of different sizes,
// parameters and storage types are admitted by a fixed device-memory budget,
// keep their state resident, advance together in fused batched launches one
// 100-step bundle per tick, and leave when their residual falls below the
// requested tolerance or their step cap is reached.  Requests that arrive
// while others run join at the next bundle boundary.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/axlb.h"
#include "axlb_internal.h"

namespace {

struct Req {
    axlb_request r{};
    std::vector<double> init[5];
    int state = AXLB_REQ_QUEUED;
    axlb_lattice *lat = nullptr;
    size_t bytes = 0;
    double residual = INFINITY;
    long steps = 0;
    int rc = AXLB_OK;
    std::string err;
    std::vector<double> out[5];
    double nu[3] = {0, 0, 0};
    int has_nu = 0;
};

}  // namespace

struct axlb_pool {
    size_t budget = 0, used = 0;
    int device = 0, max_members = 0;
    int order = AXLB_POOL_FIFO;
    long long node_window = 0;  // 0: no cap on resident nodes
    long long nodes = 0;        // fluid nodes resident now
    long next_id = 1;
    std::deque<long> queue;
    std::map<long, Req> reqs;
    axlb_batch *batch[3] = {nullptr, nullptr, nullptr};
    bool dirty[3] = {false, false, false};
    long long node_steps = 0;  // node updates done so far
    std::string err;
};

static thread_local std::string g_pool_error;

static int pfail(axlb_pool *p, int code, const std::string &m) {
    if (p) p->err = m;
    else g_pool_error = m;
    return code;
}

// Layout of a request's lattice: FP32 requests take two steps per launch on
// two buffers (AXLB_LAYOUT_AB2, the faster batch in FP32: 26.9k against
// 23.5k MLUPS over 256 uneven annuli); 16-bit requests keep the single
// buffer, whose step is faster than the two-step one with 16-bit storage
// (binary16 at 1024 x 2048: 40.6 us against 45.8 us per step).
static int pool_layout(int storage) {
    return storage == AXLB_F32 ? AXLB_LAYOUT_AB2 : AXLB_LAYOUT_AA;
}

static int make_lattice(Req &q, int device) {
    const axlb_request &r = q.r;
    axlb_options o;
    std::memset(&o, 0, sizeof(o));
    o.storage = r.storage;
    o.layout = pool_layout(r.storage);
    o.T_ref = r.T_ref;
    o.device = device;
    axlb_lattice *L = nullptr;
    int rc = axlb_lattice_create(r.Nr, r.Nz, &r.geo, r.nu, r.alpha, r.Pr, r.Ra, r.Omega, nullptr,
                                 &o, &L);
    if (rc != AXLB_OK) {
        q.err = axlb_last_error(nullptr);
        return rc;
    }
    for (int f = 0; f < 4 && rc == AXLB_OK; ++f)
        for (int d = 0; d < 3 && rc == AXLB_OK; ++d) {
            const int k = r.bc_kind[f][d];
            if (k == AXLB_MIRROR && r.geo.kind == AXLB_CYLINDER && f == AXLB_R_IN) continue;
            rc = axlb_set_bc(L, f, d, k, r.bc_value[f][d]);
        }
    if (rc == AXLB_OK) rc = axlb_set_body_force(L, r.g_axial, r.T0);
    const double *in[5];
    for (int c = 0; c < 5; ++c) in[c] = q.init[c].empty() ? nullptr : q.init[c].data();
    if (rc == AXLB_OK) rc = axlb_set_fields(L, in[0], in[1], in[2], in[3], in[4]);
    if (rc != AXLB_OK) {
        q.err = axlb_last_error(L);
        axlb_destroy(L);
        return rc;
    }
    q.lat = L;
    return AXLB_OK;
}

static int rebuild(axlb_pool *p, int s) {
    if (p->batch[s]) {
        axlb_batch_destroy(p->batch[s]);
        p->batch[s] = nullptr;
    }
    std::vector<axlb_lattice *> m;
    for (auto &kv : p->reqs)
        if (kv.second.state == AXLB_REQ_RUNNING && kv.second.r.storage == s) m.push_back(kv.second.lat);
    p->dirty[s] = false;
    if (m.empty()) return AXLB_OK;
    const int rc = axlb_batch_create(m.data(), (int)m.size(), &p->batch[s]);
    if (rc != AXLB_OK) return pfail(p, rc, axlb_batch_last_error(nullptr));
    return AXLB_OK;
}

static void finish(Req &q, int state) {
    axlb_lattice *L = q.lat;
    q.steps = axlb_steps_done(L);
    const size_t N = (size_t)q.r.Nr * q.r.Nz;
    if (state == AXLB_REQ_DONE) {
        for (int c = 0; c < 5; ++c) q.out[c].assign(N, 0.0);
        int rc = axlb_get_moments(L, q.out[0].data(), q.out[1].data(), q.out[2].data(),
                                  q.out[3].data(), q.out[4].data());
        if (rc != AXLB_OK) {
            state = AXLB_REQ_FAILED;
            q.rc = rc;
            q.err = axlb_last_error(L);
        } else {
            q.has_nu = axlb_nusselt(L, &q.nu[0], &q.nu[1], &q.nu[2]) == AXLB_OK;
        }
    }
    q.state = state;
}

extern "C" {

int axlb_pool_create(size_t budget_bytes, int device, int max_members, axlb_pool **out) {
    if (!out) return pfail(nullptr, AXLB_EINVAL, "out is NULL");
    *out = nullptr;
    if (budget_bytes == 0 || max_members <= 0) return pfail(nullptr, AXLB_EINVAL, "bad pool limits");
    axlb_pool *p = new (std::nothrow) axlb_pool();
    if (!p) return pfail(nullptr, AXLB_ENOMEM, "host allocation failed");
    p->budget = budget_bytes;
    p->max_members = max_members;
    if (device < 0 && hipGetDevice(&device) != hipSuccess) {
        delete p;
        return pfail(nullptr, AXLB_EDEVICE, "hipGetDevice failed");
    }
    p->device = device;
    *out = p;
    return AXLB_OK;
}

int axlb_pool_set_policy(axlb_pool *p, int order, long long node_window) {
    if (!p) return pfail(nullptr, AXLB_EINVAL, "pool is NULL");
    if ((order != AXLB_POOL_FIFO && order != AXLB_POOL_SMALLEST_FIRST) || node_window < 0)
        return pfail(p, AXLB_EINVAL, "bad pool policy");
    p->order = order;
    p->node_window = node_window;
    return AXLB_OK;
}

int axlb_pool_submit(axlb_pool *p, const axlb_request *r, long *id) {
    if (!p || !r || !id) return pfail(p, AXLB_EINVAL, "NULL argument");
    size_t bytes = 0;
    int rc = axlb_state_bytes(r->Nr, r->Nz, r->storage, pool_layout(r->storage), &bytes);
    if (rc != AXLB_OK) return pfail(p, rc, axlb_last_error(nullptr));
    if (bytes > p->budget) return pfail(p, AXLB_ENOMEM, "request larger than the pool budget");
    if (!(r->tol >= 0.0) || r->max_steps <= 0) return pfail(p, AXLB_EINVAL, "bad stop rule");
    Req q;
    q.r = *r;
    const size_t N = (size_t)r->Nr * r->Nz;
    for (int c = 0; c < 5; ++c) {
        if (r->init[c]) q.init[c].assign(r->init[c], r->init[c] + N);
        q.r.init[c] = nullptr;
    }
    q.bytes = bytes;
    *id = p->next_id++;
    p->reqs.emplace(*id, std::move(q));
    p->queue.push_back(*id);
    return AXLB_OK;
}

int axlb_pool_tick(axlb_pool *p, int *running, int *queued) {
    if (!p) return pfail(nullptr, AXLB_EINVAL, "pool is NULL");
    if (hipSetDevice(p->device) != hipSuccess) return pfail(p, AXLB_EDEVICE, "hipSetDevice failed");
    // 1. admission in the pool's order while the budget, the member limit
    //    and the node window allow; the request next in order that does not
    //    fit blocks the ones behind it
    int members = 0;
    for (auto &kv : p->reqs) members += kv.second.state == AXLB_REQ_RUNNING;
    while (!p->queue.empty()) {
        auto next = p->queue.begin();
        if (p->order == AXLB_POOL_SMALLEST_FIRST) {
            // least nodes x max_steps; the queue is in arrival order, so the
            // first minimum breaks ties by arrival
            double best = INFINITY;
            for (auto it = p->queue.begin(); it != p->queue.end(); ++it) {
                const axlb_request &r = p->reqs[*it].r;
                const double work = (double)r.Nr * r.Nz * (double)r.max_steps;
                if (work < best) {
                    best = work;
                    next = it;
                }
            }
        }
        Req &q = p->reqs[*next];
        const long long qn = (long long)q.r.Nr * q.r.Nz;
        if (p->used + q.bytes > p->budget || members >= p->max_members) break;
        if (p->node_window > 0 && p->nodes > 0 && p->nodes + qn > p->node_window) break;
        p->queue.erase(next);
        const int rc = make_lattice(q, p->device);
        if (rc != AXLB_OK) {
            q.rc = rc;
            q.state = AXLB_REQ_FAILED;
            continue;
        }
        q.state = AXLB_REQ_RUNNING;
        p->used += q.bytes;
        p->nodes += qn;
        p->dirty[q.r.storage] = true;
        ++members;
    }
    // 2. one bundle for every resident request, one fused batch per storage
    //    type, each batch on its own stream so that they overlap
    for (int s = 0; s < 3; ++s) {
        if (p->dirty[s]) {
            const int rc = rebuild(p, s);
            if (rc != AXLB_OK) return rc;
        }
        if (p->batch[s]) {
            const int rc = axlb_batch_step(p->batch[s], axlb::BUNDLE);
            if (rc != AXLB_OK) return pfail(p, rc, axlb_batch_last_error(p->batch[s]));
        }
    }
    for (int s = 0; s < 3; ++s)
        if (p->batch[s]) {
            const int rc = axlb_batch_sync(p->batch[s]);
            if (rc != AXLB_OK) return pfail(p, rc, axlb_batch_last_error(p->batch[s]));
        }
    // 3. residuals and retirement
    std::vector<long> leaving;
    for (auto &kv : p->reqs) {
        Req &q = kv.second;
        if (q.state != AXLB_REQ_RUNNING) continue;
        p->node_steps += (long long)q.r.Nr * q.r.Nz * axlb::BUNDLE;
        double r = INFINITY;
        const int rc = axlb_residual(q.lat, &r);
        q.residual = r;
        if (rc == AXLB_EUNSTABLE) {
            q.rc = rc;
            q.err = "non-finite state";
            leaving.push_back(kv.first);
        } else if (rc != AXLB_OK) {
            return pfail(p, rc, axlb_last_error(q.lat));
        } else if (r < q.r.tol || axlb_steps_done(q.lat) >= q.r.max_steps) {
            leaving.push_back(kv.first);
        }
    }
    for (long id : leaving) {
        Req &q = p->reqs[id];
        finish(q, q.rc == AXLB_OK ? AXLB_REQ_DONE : AXLB_REQ_FAILED);
        p->dirty[q.r.storage] = true;
    }
    if (!leaving.empty()) {
        // members leave their batch before they are destroyed
        for (int s = 0; s < 3; ++s)
            if (p->dirty[s] && p->batch[s]) {
                axlb_batch_destroy(p->batch[s]);
                p->batch[s] = nullptr;
            }
        for (long id : leaving) {
            Req &q = p->reqs[id];
            axlb_destroy(q.lat);
            q.lat = nullptr;
            p->used -= q.bytes;
            p->nodes -= (long long)q.r.Nr * q.r.Nz;
        }
    }
    int run = 0;
    for (auto &kv : p->reqs) run += kv.second.state == AXLB_REQ_RUNNING;
    if (running) *running = run;
    if (queued) *queued = (int)p->queue.size();
    return AXLB_OK;
}

int axlb_pool_status(const axlb_pool *p, long id, int *state, long *steps, double *residual) {
    if (!p) return pfail(nullptr, AXLB_EINVAL, "pool is NULL");
    auto it = p->reqs.find(id);
    if (it == p->reqs.end()) return pfail(nullptr, AXLB_EINVAL, "unknown request");
    const Req &q = it->second;
    if (state) *state = q.state;
    if (steps) *steps = q.lat ? axlb_steps_done(q.lat) : q.steps;
    if (residual) *residual = q.residual;
    return AXLB_OK;
}

int axlb_pool_result(axlb_pool *p, long id, double *rho, double *ur, double *uz, double *uth,
                     double *T, double *nusselt3) {
    if (!p) return pfail(nullptr, AXLB_EINVAL, "pool is NULL");
    auto it = p->reqs.find(id);
    if (it == p->reqs.end()) return pfail(p, AXLB_EINVAL, "unknown request");
    Req &q = it->second;
    if (q.state == AXLB_REQ_FAILED) {
        const int rc = q.rc ? q.rc : AXLB_EDEVICE;
        p->err = q.err;
        p->reqs.erase(it);
        return rc;
    }
    if (q.state != AXLB_REQ_DONE) return pfail(p, AXLB_ESTATE, "request not finished");
    double *dst[5] = {rho, ur, uz, uth, T};
    for (int c = 0; c < 5; ++c)
        if (dst[c]) std::memcpy(dst[c], q.out[c].data(), q.out[c].size() * sizeof(double));
    if (nusselt3) {
        for (int k = 0; k < 3; ++k) nusselt3[k] = q.has_nu ? q.nu[k] : NAN;
    }
    p->reqs.erase(it);
    return AXLB_OK;
}

int axlb_pool_usage(const axlb_pool *p, size_t *used_bytes, long long *node_updates) {
    if (!p) return pfail(nullptr, AXLB_EINVAL, "pool is NULL");
    if (used_bytes) *used_bytes = p->used;
    if (node_updates) *node_updates = p->node_steps;
    return AXLB_OK;
}

void axlb_pool_destroy(axlb_pool *p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    for (int s = 0; s < 3; ++s)
        if (p->batch[s]) axlb_batch_destroy(p->batch[s]);
    for (auto &kv : p->reqs)
        if (kv.second.lat) axlb_destroy(kv.second.lat);
    delete p;
}

const char *axlb_pool_last_error(const axlb_pool *p) {
    return p ? p->err.c_str() : g_pool_error.c_str();
}

}  // extern "C"
