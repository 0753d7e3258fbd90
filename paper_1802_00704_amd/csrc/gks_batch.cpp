// Batched steps: one step of Eq. fvm3 for several mesh handles at once, in
// one sequence of grouped launches (gks_batch_step).
//
// Each handle keeps its own device state (mesh, factors, Krylov basis,
// solution history); a grouped launch runs a kernel for every handle of the
// batch with the arguments and grid of that handle's own launch, so each
// handle does exactly the arithmetic of its own eager gks_step.  The
// restarted GMRES cycles of the handles run in lockstep: Arnoldi step k is
// one grouped launch sequence over the handles whose cycle is still running
// (a handle leaves once its columns converge, its cycle reaches the restart
// length or its solve reaches max_iter), and the handles whose cycle ended
// wait for the others before their end-of-cycle and next cycle start.  One
// status read back per Arnoldi step serves the whole batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gks_internal.h"

using namespace gks;

struct gks_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;
    BatchSlot* slots = nullptr;   // pinned, GKS_BATCH_MAX entries, written by the device
    std::string err;
};

namespace {

struct BFail {
    int code;
    std::string msg;
};

#define BHIP(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) throw BFail{GKS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

bool converged(const Status& s) {
    for (int c = 0; c < NC; ++c)
        if (!s.conv[c]) return false;
    return true;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Status words of the handles idx (positions in the batch) read back into
// their slots.
void read_slots(gks_batch* b, const std::vector<gks_mesh*>& ms, const std::vector<int>& idx, bool counters) {
    std::vector<gks_mesh*> sub;
    std::vector<BatchSlot*> out;
    for (int r : idx) {
        sub.push_back(ms[r]);
        out.push_back(b->slots + r);
    }
    glaunch_gather(b->stream, sub, out, counters);
    BHIP(hipStreamSynchronize(b->stream));
}

template <class T>
std::vector<T> pick(const std::vector<T>& v, const std::vector<int>& idx) {
    std::vector<T> o;
    for (int r : idx) o.push_back(v[r]);
    return o;
}

}  // namespace

extern "C" {

int gks_batch_create(void* hip_stream, gks_batch** out) {
    if (!out) return GKS_EINVAL;
    *out = nullptr;
    gks_batch* b = new (std::nothrow) gks_batch();
    if (!b) return GKS_ENOMEM;
    b->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return GKS_EHIP;
    }
    if (!b->stream) {
        if (hipStreamCreate(&b->stream) != hipSuccess) {
            delete b;
            return GKS_EHIP;
        }
        b->own_stream = true;
    }
    if (hipHostMalloc((void**)&b->slots, sizeof(BatchSlot) * GKS_BATCH_MAX, hipHostMallocCoherent) != hipSuccess) {
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return GKS_ENOMEM;
    }
    std::memset(b->slots, 0, sizeof(BatchSlot) * GKS_BATCH_MAX);
    *out = b;
    return GKS_OK;
}

int gks_batch_step(gks_batch* b, int32_t n, gks_mesh* const* meshes, double* const* W, const double* dt,
                   double* dt_used, gks_solve_info* info, int32_t* status) {
    if (!b) return GKS_EINVAL;
    const auto t_call = std::chrono::steady_clock::now();
    if (n < 1 || n > GKS_BATCH_MAX || !meshes || !W || !status) {
        b->err = "gks_batch_step needs 1 <= n <= GKS_BATCH_MAX, meshes, W and status";
        return GKS_EINVAL;
    }
    std::vector<gks_mesh*> ms(meshes, meshes + n);
    std::vector<double*> Wv(W, W + n);
    for (int r = 0; r < n; ++r) {
        gks_mesh* m = ms[r];
        if (!m || !Wv[r]) {
            b->err = "gks_batch_step: null handle or W at position " + std::to_string(r);
            return GKS_EINVAL;
        }
        for (int q = 0; q < r; ++q)
            if (ms[q] == m) {
                b->err = "gks_batch_step: a handle appears twice";
                return GKS_EINVAL;
            }
        if (m->device != b->device) {
            b->err = "gks_batch_step: handle " + std::to_string(r) + " belongs to another device";
            return GKS_EINVAL;
        }
        if (m->prm.precision != ms[0]->prm.precision) {
            b->err = "gks_batch_step: the handles of a batch share one precision";
            return GKS_EINVAL;
        }
        if (m->prm.precision == GKS_MIXED && !m->d.split) {
            b->err = "gks_batch_step: mixed-form handles need the split-form sweeps (a cell graph without 3-cycles)";
            return GKS_EINVAL;
        }
        if (m->prm.limiter) {
            b->err = "gks_batch_step: handles with the limiter on are not batched";
            return GKS_EINVAL;
        }
        if (m->prm.precision == GKS_MIXED && m->prm.inner_solver != GKS_INNER_RICHARDSON) {
            b->err = "gks_batch_step: mixed-form handles with inner GMRES are not batched";
            return GKS_EINVAL;
        }
    }
    hipStream_t st = b->stream;
    std::vector<int> hist(n), all(n), q1(n);
    for (int r = 0; r < n; ++r) {
        q1[r] = ms[r]->prm.precision == GKS_MIXED ? outer_step_sweeps(ms[r], 0) : 0;
        hist[r] = ms[r]->hist;
        ms[r]->hist = 0;   // until the step has succeeded
        all[r] = r;
        status[r] = GKS_OK;
    }
    try {
        // the handles' own streams hold no work of this step; earlier work
        // on them must be complete
        for (gks_mesh* m : ms)
            if (m->stream != st) BHIP(hipStreamSynchronize(m->stream));
        std::vector<const double*> Wc(Wv.begin(), Wv.end());
        // time step: the caller's, or the CFL rule's; counters cleared
        std::vector<double> dtv(n, 0.0);
        std::vector<int> cfl;
        for (int r = 0; r < n; ++r) {
            dtv[r] = dt ? dt[r] : 0.0;
            if (!(dtv[r] > 0.0)) cfl.push_back(r);
        }
        glaunch_zero_counters(st, ms, dtv);
        if (!cfl.empty()) glaunch_cfl(st, pick(ms, cfl), pick(Wc, cfl));
        // initial guesses from the solution histories
        glaunch_extrap(st, ms, hist);
        // reconstruction: right-hand sides, then lockstep GMRES cycles
        const auto t_solve = std::chrono::steady_clock::now();
        glaunch_rhs(st, ms, Wc);
        glaunch_ctl(st, ms, 0);
        glaunch_mask_cols(st, ms);
        std::vector<int> start = all, ok, failed;
        while (!start.empty()) {
            glaunch_cycle_start(st, pick(ms, start));
            read_slots(b, ms, start, false);
            std::vector<int> running;
            for (int r : start) {
                const Status& s = b->slots[r].st;
                if (converged(s))
                    ok.push_back(r);
                else if (s.total >= ms[r]->prm.max_iter)
                    failed.push_back(r);
                else
                    running.push_back(r);
            }
            std::vector<int> ended, nvec;
            for (int k = 0; !running.empty(); ++k) {
                glaunch_arnoldi(st, pick(ms, running), k);
                read_slots(b, ms, running, false);
                std::vector<int> next;
                for (int r : running) {
                    const Status& s = b->slots[r].st;
                    if (converged(s) || k + 1 >= ms[r]->prm.restart || s.total >= ms[r]->prm.max_iter) {
                        ended.push_back(r);
                        nvec.push_back(k + 1);
                    } else {
                        next.push_back(r);
                    }
                }
                running.swap(next);
            }
            if (!ended.empty()) glaunch_end_cycle(st, pick(ms, ended), nvec);
            start = ended;
        }
        const double solve_ms = ms_since(t_solve);
        for (int r : failed) {
            status[r] = GKS_ENOCONV;
            ms[r]->err = "GMRES did not converge within max_iter";
        }
        std::sort(ok.begin(), ok.end());
        // fluxes and updates of the converged handles, then their counters
        if (!ok.empty()) {
            glaunch_flux_update(st, pick(ms, ok), pick(Wc, ok));
            read_slots(b, ms, ok, true);
            std::vector<int> commit;
            for (int r : ok) {
                const BatchSlot& sl = b->slots[r];
                if ((sl.counters[0] > 0 && !ms[r]->prm.nonphys_fallback) || sl.counters[1] > 0) {
                    status[r] = GKS_ENONPHYS;
                    ms[r]->err = "non-physical state (" + std::to_string(sl.counters[0]) + " Gauss points, " +
                                 std::to_string(sl.counters[1]) + " updated cells)";
                } else {
                    commit.push_back(r);
                }
            }
            if (!commit.empty()) {
                glaunch_commit(st, pick(ms, commit), pick(Wv, commit));
                BHIP(hipStreamSynchronize(st));
            }
            for (int r : commit) {
                ms[r]->hist = std::min(hist[r], ring_slots(ms[r]->prm)) + 1;
                push_step(ms[r], b->slots[r].dt);
                adapt_first_sweeps(ms[r], b->slots[r].st.total);
                adapt_points(ms[r], start_resid(b->slots[r].st), ms[r]->last_npts, b->slots[r].st.total);
            }
        }
        const double call_ms = ms_since(t_call);
        for (int r = 0; r < n; ++r) {
            const BatchSlot& sl = b->slots[r];
            if (dt_used) dt_used[r] = status[r] == GKS_ENOCONV ? 0.0 : sl.dt;
            if (info) {
                gks_solve_info& in = info[r];
                for (int c = 0; c < NC; ++c) {
                    in.iters[c] = sl.st.its[c];
                    in.restarts[c] = sl.st.cycles;
                    in.rel_resid[c] = sl.st.bnorm[c] > 0.0 ? sl.st.beta[c] / sl.st.bnorm[c] : 0.0;
                }
                in.nonphys = status[r] == GKS_ENOCONV ? 0 : sl.counters[0];
                in.solve_ms = solve_ms;
                in.call_ms = call_ms;
                in.limited = 0;
                in.reorth = sl.st.reorths;
                in.first_sweeps = q1[r];
                in.start_resid = start_resid(sl.st);
                in.start_points = ms[r]->last_npts;
            }
        }
        return GKS_OK;
    } catch (const BFail& f) {
        b->err = f.msg;
        return f.code;
    } catch (const LaunchError& e) {
        b->err = std::string("launch of ") + e.kernel + " failed: " + hipGetErrorString(e.err);
        return GKS_EHIP;
    }
}

const char* gks_batch_last_error(const gks_batch* b) { return b ? b->err.c_str() : ""; }

void gks_batch_destroy(gks_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->slots) (void)hipHostFree(b->slots);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // extern "C"
