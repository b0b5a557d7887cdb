// Native velocity-Verlet driver (Sec. 3.3): runs whole steps of the path
// without returning to the caller, so no interpreter sits between kernels.
//
// Per step: kick + drift with the rebuild check (the closing half kick of the
// previous step is fused in when steps follow each other), a one-thread
// kernel publishes the step's rebuild flag into pinned host memory, the
// force evaluation of the new positions is queued behind it (gated on the
// device by the same flag), the host polls the flag word, and when some atom
// has moved more than half the skin it rebuilds the lists and evaluates the
// forces again; then it either opens the next step or closes this one with
// a half kick.
#include <chrono>
#include <thread>

#include "md_common.h"

namespace md {

// status[0] == tag: some atom moved more than skin/2 in step `tag`;
// status[1]: error bits.  Written to host memory last-word-last.
__global__ void k_publish(const int32_t *status, int32_t *host, int32_t tag)
{
    volatile int32_t *h = host;
    h[1] = status[0] == tag ? 1 : 0;
    h[2] = status[1];
    __threadfence_system();
    h[0] = tag;
}

// The longest row of the list just built, into host word 3 (which the host
// set negative before queueing this kernel).
__global__ void k_publish_longest(const int32_t *max_count, int32_t *host)
{
    volatile int32_t *h = host;
    h[3] = *max_count;
    __threadfence_system();
}

namespace {

// The rebuild flag of step `tag`, in two halves so that device work can be
// queued between them.  Fast path: the publish kernel writes device-visible
// pinned memory that the host polls; otherwise a copy and a stream
// synchronisation.
int post_flag(md_system_t *sys, int32_t *host_dev, int32_t tag, hipStream_t s)
{
    if (!host_dev) return MD_OK;
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(1), 0, s, sys->status, host_dev, tag);
    MD_HIP_TRY(hipGetLastError());
    return MD_OK;
}

// Waits for the flag posted for step `tag`; sets *moved, *bad.
int read_flag(md_system_t *sys, int32_t *host_dev, int32_t tag, hipStream_t s, bool *moved, bool *bad)
{
    if (host_dev) {
        volatile int32_t *h = sys->host_status;
        const auto t0 = std::chrono::steady_clock::now();
        for (uint64_t spin = 0; h[0] != tag; ++spin) {
            if ((spin & 4095) == 4095) {
                const hipError_t e = hipStreamQuery(s);
                if (e != hipSuccess && e != hipErrorNotReady) return MD_ERR_HIP;
                if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120)) return MD_ERR_HIP;
                std::this_thread::yield();
            }
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        *moved = h[1] != 0;
        *bad = h[2] != 0;
        return MD_OK;
    }
    int32_t st[2];
    MD_HIP_TRY(hipMemcpyAsync(st, sys->status, sizeof(st), hipMemcpyDeviceToHost, s));
    MD_HIP_TRY(hipStreamSynchronize(s));
    *moved = st[0] == tag;
    *bad = st[1] != 0;
    return MD_OK;
}

// Bins, sorts and builds the lists without waiting for the longest row:
// check_build reads it once the force evaluation (gated on the device by the
// same row length) is queued behind the build.
int rebuild(md_system_t *sys, const WsLayout &w, hipStream_t s, int32_t *host_dev)
{
    const int64_t n = sys->n;
    int rc = bin_cells(&sys->grid, n, sys->x, sys->cell, sys->perm, sys->cell_start, sys->ws, w, s);
    if (rc) return rc;
    if (n > 0) {
        // state into the sorted order; xref = the sorted positions
        uint32_t *xs = (sys->flags & MD_PAIR_FP64) ? nullptr : sys->xs;
        if ((rc = reorder_state(n, sys->perm, sys->x, sys->v, sys->ids, sys->xref, sys->scratch, sys->ids_scratch,
                                &sys->box, xs, s)))
            return rc;
        if (sys->potential == MD_POT_TBM) {
            // elements follow their atoms into the new order and into the scaled coordinates
            MD_HIP_TRY(hipMemcpyAsync(sys->types_scratch, sys->types, size_t(n) * 4, hipMemcpyDeviceToDevice, s));
            if ((rc = permute(n, 1, sys->perm, sys->types_scratch, sys->types, 4, s))) return rc;
            if ((rc = set_elements(n, sys->types, sys->xs, s))) return rc;
        }
    }
    rc = build_neighbors(&sys->grid, n, sys->x, sys->cell_start, sys->row_cap, sys->idx, sys->count, sys->max_count,
                         nullptr, sys->ws, w, s);
    if (rc) return rc;
    if (host_dev) {
        reinterpret_cast<volatile int32_t *>(sys->host_status)[3] = -1;
        hipLaunchKernelGGL(k_publish_longest, dim3(1), dim3(1), 0, s, sys->max_count, host_dev);
        MD_HIP_TRY(hipGetLastError());
    }
    return MD_OK;
}

// Waits for the longest row of the last build: MD_ERR_CAPACITY (with
// row_cap_needed) when it exceeds row_cap.
int check_build(md_system_t *sys, int32_t *host_dev, hipStream_t s)
{
    int32_t longest = 0;
    if (host_dev) {
        volatile int32_t *h = sys->host_status;
        const auto t0 = std::chrono::steady_clock::now();
        for (uint64_t spin = 0; h[3] < 0; ++spin) {
            if ((spin & 4095) == 4095) {
                const hipError_t e = hipStreamQuery(s);
                if (e != hipSuccess && e != hipErrorNotReady) return MD_ERR_HIP;
                if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(120)) return MD_ERR_HIP;
                std::this_thread::yield();
            }
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        longest = h[3];
    } else {
        MD_HIP_TRY(hipMemcpyAsync(&longest, sys->max_count, sizeof(longest), hipMemcpyDeviceToHost, s));
        MD_HIP_TRY(hipStreamSynchronize(s));
    }
    if (longest > sys->row_cap) {
        sys->row_cap_needed = longest;
        return MD_ERR_CAPACITY;
    }
    ++sys->builds;
    return MD_OK;
}

// The force evaluation of the current positions; with a gate, the kernels
// do nothing when the gate's flag is set on the device.
int forces(md_system_t *sys, const WsLayout &w, hipStream_t s, Gate gate = {})
{
    if (sys->potential == MD_POT_LJ)
        return forces_lj(&sys->box, sys->n, sys->x, sys->xs, sys->row_cap, sys->idx, sys->count, &sys->lj, sys->f,
                         nullptr, sys->flags & (MD_PAIR_FP64 | MD_NO_COMPENSATE), sys->ws, w, s, gate);
    if (sys->potential == MD_POT_TBM)
        return forces_tbm(&sys->box, sys->n, sys->xs, sys->row_cap, sys->idx, sys->count, &sys->tbm, sys->rho,
                          sys->fprime, static_cast<float *>(sys->f), nullptr, nullptr, sys->flags & MD_NO_COMPENSATE,
                          sys->ws, w, s, gate);
    if (sys->potential == MD_POT_TAB)
        return forces_tab(&sys->box, sys->n, sys->xs, sys->row_cap, sys->idx, sys->count, &sys->tab, sys->tab_table,
                          sys->rho, sys->fprime, static_cast<float *>(sys->f), nullptr, nullptr,
                          sys->flags & MD_NO_COMPENSATE, sys->ws, w, s, gate);
    if (sys->potential == MD_POT_TB)
        return forces_tb(&sys->box, sys->n, sys->xs, sys->row_cap, sys->idx, sys->count, &sys->tb, sys->rho,
                         sys->fprime, static_cast<float *>(sys->f), nullptr, nullptr, sys->flags & MD_NO_COMPENSATE,
                         sys->ws, w, s, gate);
    if (sys->potential == MD_POT_MLP)
        return forces_mlp(&sys->box, sys->n, sys->xs, sys->row_cap, sys->idx, sys->count, &sys->mlp, sys->mlp_w,
                          sys->dEdG, sys->idx_in, sys->cnt_in, nullptr, static_cast<float *>(sys->f), nullptr,
                          sys->flags & MD_NO_COMPENSATE, sys->ws, w, s, gate);
    return forces_eam(&sys->box, sys->n, sys->xs, sys->row_cap, sys->idx, sys->count, &sys->fs, sys->rho,
                      sys->fprime, static_cast<float *>(sys->f), nullptr, nullptr, sys->flags & MD_NO_COMPENSATE,
                      sys->ws, w, s, gate);
}

// Optional timing of the force evaluations: one event pair per evaluation,
// kept in recording order and read back once the stream has passed it.  A
// speculative evaluation that the device skipped is dropped unread.
struct ForceTimer {
    static constexpr int kSlots = 4;
    bool on = false;
    hipEvent_t ev[kSlots][2] = {};
    int queue[kSlots] = {};   // recorded, unread pairs, oldest first
    int queued = 0;
    int next = 0;
    bool init(bool want)
    {
        if (!want) return true;
        for (auto &p : ev)
            for (auto &e : p)
                if (hipEventCreate(&e) != hipSuccess) return false;
        on = true;
        return true;
    }
    ~ForceTimer()
    {
        if (on)
            for (auto &p : ev)
                for (auto &e : p) (void)hipEventDestroy(e);
    }
    void start(hipStream_t s)
    {
        if (on) (void)hipEventRecord(ev[next][0], s);
    }
    void stop(md_system_t *sys, hipStream_t s)
    {
        if (!on) return;
        if (queued == kSlots) collect(sys, true, 0);   // keep a free slot
        (void)hipEventRecord(ev[next][1], s);
        queue[queued++] = next;
        next = (next + 1) % kSlots;
    }
    void drop_last()
    {
        if (on && queued > 0) --queued;
    }
    // Reads back all but the `keep` most recent pairs (waiting for them when
    // `wait`; otherwise the caller knows the stream has passed them).
    void collect(md_system_t *sys, bool wait, int keep)
    {
        if (!on) return;
        int k = 0;
        for (; k < queued - keep; ++k) {
            const int p = queue[k];
            if (wait) (void)hipEventSynchronize(ev[p][1]);
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[p][0], ev[p][1]) == hipSuccess) {
                sys->force_ms += ms;
                ++sys->force_calls;
            }
        }
        for (int j = k; j < queued; ++j) queue[j - k] = queue[j];
        queued -= k;
    }
};

}  // namespace

int run(md_system_t *sys, int64_t steps, hipStream_t s)
{
    const WsLayout w = ws_layout(sys->grid.n_cells, sys->n);
    const bool f64 = sys->flags & MD_PAIR_FP64;
    const double hk = 0.5 * sys->dt * sys->accel;
    uint32_t *xs = f64 ? nullptr : sys->xs;
    int32_t *host_dev = nullptr;
    if (sys->host_status) {
        void *p = nullptr;
        if (hipHostGetDevicePointer(&p, sys->host_status, 0) == hipSuccess) host_dev = static_cast<int32_t *>(p);
        else (void)hipGetLastError();
    }
    int rc = MD_OK;
    bool moved = false, bad = false;
    ForceTimer timer;
    if (!timer.init(sys->timing != 0)) return MD_ERR_HIP;
    // forces of a fresh build, skipped on the device when a row overflowed
    const Gate fits{nullptr, 0, sys->max_count, sys->row_cap};
    if (sys->phase == 0 && sys->need_build) {
        if ((rc = rebuild(sys, w, s, host_dev))) return rc;
        if ((rc = forces(sys, w, s, fits))) return rc;
        if ((rc = check_build(sys, host_dev, s))) return rc;
        sys->need_build = 0;
    }
    int64_t done = 0;
    // Speculative force evaluation: after each drift the forces of the new
    // positions are queued before the host has read the rebuild flag, gated
    // on the device by that flag (status[0] == tag: some atom moved more than
    // half the skin).  When the flag is set the gated kernels do nothing and
    // the host rebuilds and evaluates again; otherwise the evaluation is the
    // step's.
    bool ready = false;   // forces of the in-flight step already queued
    const auto drift = [&](double h, int32_t tag) -> int {
        int r = kick_drift(&sys->box, sys->n, sys->x, sys->v, sys->f, f64, h, sys->dt, sys->xref, sys->half_skin_sq,
                           sys->status, tag, xs, s, sys->potential == MD_POT_TBM);
        if (r || (r = post_flag(sys, host_dev, tag, s))) return r;
        timer.start(s);
        if ((r = forces(sys, w, s, Gate{sys->status, tag}))) return r;
        timer.stop(sys, s);
        if ((r = read_flag(sys, host_dev, tag, s, &moved, &bad))) return r;
        ready = !moved && !bad;
        if (!ready) timer.drop_last();
        // the flag came after every earlier evaluation on the stream
        timer.collect(sys, false, ready ? 1 : 0);
        return MD_OK;
    };
    for (;;) {
        if (sys->phase == 0) {
            if (done >= steps) break;
            if ((rc = drift(hk, int32_t(sys->step + 1)))) return rc;
            sys->phase = 1;
            if (bad) return MD_ERR_NONFINITE;
            sys->need_build |= moved ? 1 : 0;
        }
        // a step is in flight: positions drifted, forces stale unless queued
        const bool built = sys->need_build != 0;
        if (built) {
            ready = false;
            if ((rc = rebuild(sys, w, s, host_dev))) return rc;
        }
        if (!ready) {
            timer.start(s);
            if ((rc = forces(sys, w, s, built ? fits : Gate{}))) return rc;
            timer.stop(sys, s);
        }
        if (built) {
            if ((rc = check_build(sys, host_dev, s))) {
                timer.drop_last();
                return rc;
            }
            sys->need_build = 0;
        }
        ready = false;
        ++sys->step;
        ++done;
        if (done < steps) {
            // closing half kick of this step fused with the opening one of the next
            if ((rc = drift(2.0 * hk, int32_t(sys->step + 1)))) return rc;
            if (bad) return MD_ERR_NONFINITE;
            sys->need_build |= moved ? 1 : 0;
        } else {
            if ((rc = integrate(MD_KICK, &sys->box, sys->n, sys->x, sys->v, sys->f, sys->dt, sys->accel, 1.0, nullptr,
                                0.0, nullptr, 0, nullptr, nullptr, sys->flags & MD_PAIR_FP64, sys->ws, w, s)))
                return rc;
            sys->phase = 0;
        }
    }
    timer.collect(sys, true, 0);
    return MD_OK;
}

}  // namespace md
