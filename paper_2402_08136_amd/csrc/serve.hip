// Serving loop for HHL solves: continuous batching on one GPU.
//
// Requests (A, b, clock bits) arrive from any thread (svs_submit, which copies
// the inputs).  A pool of prep threads builds each request's circuit on the
// host (Sec. III-A steps 1-2 of Zheng et al., PESGM 2024: normalise, pad,
// eigen-decompose; the controlled e^{iAt 2^j} are built later on the device),
// fuses it, waits until the request's device footprint fits the HBM budget
// and a slot is free (admission), then uploads its program so that it is
// resident on the device.  A scheduler thread keeps up to `streams`
// micro-batches in flight: resident requests of up to batch_max_qubits go
// together through the batched persistent kernel (one workgroup per request,
// the state in LDS when it fits, else in HBM), larger requests run alone
// through the whole-GPU sweep kernels.
// New requests are admitted and launched while earlier ones are still on the
// GPU.  When a micro-batch finishes its postselected outputs are copied back,
// x is recovered (step 4), latency is recorded and the memory and slots are
// released.  A request's arithmetic never depends on what else is in flight,
// so its result is the same alone and in the mix.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "device_common.hpp"
#include "hhlsv_batch.hpp"
#include "kernels.hpp"

using namespace hhlsv;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Copy each instance's output block into one contiguous staging buffer.
__global__ __launch_bounds__(256) void k_gather_outputs(const BInst *__restrict__ insts, int count,
                                                        const unsigned long long *__restrict__ offs,
                                                        double *__restrict__ staging)
{
    for (int i = blockIdx.x; i < count; i += gridDim.x) {
        const BInst in = insts[i];
        const int len = 2 + (2 << in.ns);
        for (int j = threadIdx.x; j < len; j += blockDim.x) staging[offs[i] + j] = in.out[j];
    }
}

// Postselected block of a large request: out = [P(anc=1) (already there), 0,
// y_0.re, y_0.im, ...] with y_s = psi[2^{n-1} + s], widened to double.
template <typename R>
__global__ __launch_bounds__(256) void k_copy_y(const typename V2<R>::type *__restrict__ psi, uint64_t half,
                                                int D, double *__restrict__ out)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < D; i += gridDim.x * blockDim.x) {
        const auto y = psi[half + i];
        out[2 + 2 * i] = (double)y.x;
        out[3 + 2 * i] = (double)y.y;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[1] = 0.0;
}

// How a request runs: in a batched launch with its state in LDS, in a
// batched launch with its state in HBM (one workgroup per request), or alone
// through the whole-GPU sweep kernels.
enum { kBatchLds = 0, kBatchHbm = 1, kAlone = 2 };

struct Req {
    uint64_t ticket = 0;
    std::vector<double> A, b;
    int dim = 0, m = 0;
    double t = 0;
    double t_arrive = 0, t_done = 0;
    double t_prep0 = 0, t_admit = 0, t_ready = 0, t_launch = 0;
    bool cancelled = false;
    // prepared
    HHLParams h;
    int n = 0, ns = 0, kmax = 0;
    int kind = 0;                // kBatchLds / kBatchHbm / kAlone
    size_t footprint = 0;
    bool admitted = false;
    void *dmem = nullptr;
    BInst inst;                  // small: its batch instance
    std::vector<DevOp> ops;      // large: its program
    DeviceProgram prog;          // large: dbuf points into dmem
    void *state = nullptr;       // large
    double *partials = nullptr;  // large: reduction scratch (kReducePartials + 1)
    double *out = nullptr;       // device [p1, 0, y...]
    hipEvent_t done = nullptr;   // alone: completion of its launches
    hipStream_t run = nullptr;   // alone: the stream it was launched on
    // result
    sv_status status = SV_OK;
    std::string err;
    std::vector<double> result;  // [p1, 0, y...]
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<std::shared_ptr<Req>> reqs;
    BInst *h_insts = nullptr, *d_insts = nullptr;   // pinned / device
    int *h_order = nullptr, *d_order = nullptr;
    unsigned long long *h_offs = nullptr, *d_offs = nullptr;
    double *h_out = nullptr, *d_out = nullptr;
    size_t out_cap = 0;
};

}  // namespace

struct svs {
    // configuration
    size_t budget = 0;
    int max_slots = 0;
    sv_dtype dtype = SV_C128;
    int device = 0;
    int prep_threads = 8;
    int k_max = 0;
    int max_batch = 256;
    int nstreams = 8;
    int batch_max_qubits = 0;    // 0: batch only LDS-resident requests; larger run alone
    int hhl_flags = 0;           // SV_HHL_SIGNED / _DILATE / _AUTO / _GAUSS_SEIDEL per request
    size_t queue_limit = 1 << 20;
    long fail_alloc_at = 0;   // test hook: the n-th device allocation fails (0 = off)
    // state
    std::mutex mu;
    std::condition_variable cv_prep, cv_budget, cv_sched, cv_done;
    std::deque<std::shared_ptr<Req>> prep_q;
    std::deque<std::shared_ptr<Req>> ready_q;
    std::vector<std::shared_ptr<Req>> alone_inflight;   // launched by prep threads
    std::unordered_map<uint64_t, std::shared_ptr<Req>> all;
    uint64_t next_ticket = 1;
    size_t hbm_used = 0;
    int slots_used = 0;
    std::atomic<long> alloc_count{0};
    bool started = false, stopping = false;
    int preps_alive = 0;
    size_t pending = 0;   // submitted, not yet finished
    std::vector<std::thread> threads;
    std::vector<Slot> slots;
    // statistics
    std::vector<double> latencies;
    double first_arrival = 0, last_done = 0;
    uint64_t n_rejected = 0, n_failed = 0, n_done = 0;
    // phase times summed over successful requests (seconds)
    double sum_queue = 0, sum_prep = 0, sum_admit = 0, sum_upload = 0, sum_ready = 0, sum_gpu = 0;
    uint64_t n_small = 0, n_large = 0;
};

namespace {

void finish(svs *s, const std::shared_ptr<Req> &r, sv_status st, const std::string &err)
{
    // caller holds s->mu
    r->status = st;
    r->err = err;
    r->t_done = now_s();
    if (st == SV_OK) {
        s->latencies.push_back(r->t_done - r->t_arrive);
        s->last_done = std::max(s->last_done, r->t_done);
        ++s->n_done;
        s->sum_queue += r->t_prep0 - r->t_arrive;
        s->sum_prep += r->t_admit - r->t_prep0;
        s->sum_upload += r->t_ready - r->t_admit;
        s->sum_ready += r->t_launch - r->t_ready;
        s->sum_gpu += r->t_done - r->t_launch;
        if (r->kind != kAlone)
            ++s->n_small;
        else
            ++s->n_large;
    } else {
        ++s->n_failed;
    }
    r->A.clear();
    r->A.shrink_to_fit();
    r->b.clear();
    r->b.shrink_to_fit();
    r->h.spec.reset();
    --s->pending;
    s->cv_done.notify_all();
}

void release(svs *s, const std::shared_ptr<Req> &r, hipStream_t st)
{
    // caller holds s->mu
    if (r->dmem) (void)hipFreeAsync(r->dmem, st);
    r->dmem = nullptr;
    if (r->admitted) {
        s->hbm_used -= r->footprint;
        --s->slots_used;
        r->admitted = false;
        s->cv_budget.notify_all();
    }
}

// Prepare one request: build, fuse, admit, upload.  Returns false with
// (st, err) set when the request fails.
bool prepare(svs *s, Req &r, hipStream_t up, sv_status &st, std::string &err)
{
    sv_circuit *c = nullptr, *f = nullptr;
    st = circuit_build_hhl_ex(r.A.data(), r.b.data(), r.dim, r.m, r.t, SV_HHL_DEVICE_EVOLUTIONS | s->hhl_flags,
                              &c);
    if (st != SV_OK) {
        err = sv_last_error();
        return false;
    }
    r.h = c->c.hhl;
    r.n = c->c.n;
    r.ns = r.h.ns;
    int k = s->k_max ? s->k_max : batch_tuned_k(s->dtype, r.ns, r.m);
    if (k == 0) k = kDefaultBatchK;
    st = fuse(c, k, &f);
    circuit_destroy(c);
    if (st != SV_OK) {
        err = sv_last_error();
        return false;
    }
    bool resident = false;
    batch_lds_bytes(r.n, s->dtype, &resident);
    r.kind = resident ? kBatchLds : (r.n <= s->batch_max_qubits ? kBatchHbm : kAlone);
    const size_t out_bytes = sizeof(double) * (2 + (2u << r.ns));
    const size_t asz = s->dtype == SV_C128 ? 16 : 8;
    std::vector<BOp> bops;
    std::vector<unsigned char> tables, image;
    std::vector<EvoJob> jobs;
    int max_D = 0;
    size_t ops_bytes = 0, tab_bytes = 0, state_bytes = 0;
    if (r.kind != kAlone) {
        lower_for_batch(f->c, s->dtype, bops, tables, jobs);
        for (const BOp &op : bops)
            if (op.type == OP_DENSE) r.kmax = std::max(r.kmax, op.k);
        for (EvoJob &jb : jobs) {
            jb.vt_off = 0;
            jb.w_off = (unsigned long long)r.h.spec->D * r.h.spec->D;
            max_D = std::max(max_D, jb.D);
        }
        ops_bytes = align256(bops.size() * sizeof(BOp));
        tab_bytes = align256(tables.size());
        if (r.kind == kBatchHbm) state_bytes = align256(asz << r.n);
    } else {
        st = build_program_image(f->c, s->dtype, r.ops, image, jobs, &max_D);
        if (st != SV_OK) {
            err = sv_last_error();
            circuit_destroy(f);
            return false;
        }
        tab_bytes = align256(image.size());
        state_bytes = align256(asz << r.n) + align256(sizeof(double) * (kReducePartials + 1));
    }
    circuit_destroy(f);
    r.footprint = ops_bytes + tab_bytes + state_bytes + align256(out_bytes);
    // admission: wait for budget and a slot
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (r.footprint > s->budget) {
            st = SV_ERR_OOM;
            err = "svs: request needs " + std::to_string(r.footprint) + " bytes, more than the HBM budget";
            return false;
        }
        s->cv_budget.wait(lk, [&] {
            return r.cancelled || (s->hbm_used + r.footprint <= s->budget && s->slots_used < s->max_slots);
        });
        if (r.cancelled) {
            st = SV_ERR_INVALID;
            err = "svs: request cancelled";
            return false;
        }
        s->hbm_used += r.footprint;
        ++s->slots_used;
        r.admitted = true;
    }
    r.t_admit = now_s();
    const long nth = ++s->alloc_count;
    hipError_t e = (s->fail_alloc_at > 0 && nth == s->fail_alloc_at) ? hipErrorOutOfMemory
                                                                     : hipMallocAsync(&r.dmem, r.footprint, up);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        r.dmem = nullptr;
        st = SV_ERR_OOM;
        err = std::string("svs: device allocation failed: ") + hipGetErrorString(e);
        return false;
    }
    unsigned char *base = static_cast<unsigned char *>(r.dmem);
    if (r.kind != kAlone) {
        BOp *d_ops = reinterpret_cast<BOp *>(base);
        unsigned char *d_tab = base + ops_bytes;
        unsigned char *d_state = r.kind == kBatchHbm ? base + ops_bytes + tab_bytes : nullptr;
        r.out = reinterpret_cast<double *>(base + ops_bytes + tab_bytes + state_bytes);
        e = hipMemcpyAsync(d_ops, bops.data(), bops.size() * sizeof(BOp), hipMemcpyHostToDevice, up);
        if (e == hipSuccess) e = hipMemcpyAsync(d_tab, tables.data(), tables.size(), hipMemcpyHostToDevice, up);
        if (e != hipSuccess) {
            st = SV_ERR_HIP;
            err = std::string("svs: upload: ") + hipGetErrorString(e);
            return false;
        }
        Circuit tmp;   // only its hhl.spec is read by the uploader
        tmp.hhl = r.h;
        st = upload_program_image(tmp, {}, jobs, max_D, d_tab, s->dtype, up);
        if (st != SV_OK) {
            err = sv_last_error();
            return false;
        }
        std::memset(&r.inst, 0, sizeof(r.inst));
        r.inst.n = r.n;
        r.inst.ns = r.ns;
        r.inst.op_count = (int)bops.size();
        r.inst.ops = d_ops;
        r.inst.tables = d_tab;
        r.inst.state = d_state;
        r.inst.out = r.out;
    } else {
        r.prog.dbuf = base;
        r.prog.dtype = s->dtype;
        r.prog.device = s->device;
        r.state = base + tab_bytes;
        r.partials = reinterpret_cast<double *>(base + tab_bytes + align256(asz << r.n));
        r.out = reinterpret_cast<double *>(base + tab_bytes + state_bytes);
        Circuit tmp;
        tmp.hhl = r.h;
        st = upload_program_image(tmp, image, jobs, max_D, r.prog.dbuf, s->dtype, up);
        if (st != SV_OK) {
            err = sv_last_error();
            return false;
        }
        std::memset(&r.inst, 0, sizeof(r.inst));
        r.inst.ns = r.ns;
        r.inst.out = r.out;
    }
    r.h.spec.reset();   // the eigen-decomposition lives on the device now
    return true;
}

// Launch a request that runs alone (init, every op, postselection into its
// device output block) on the calling prep thread's execution stream.
sv_status launch_alone(svs *s, Req &r, hipStream_t run)
{
    sv_status st = launch_init_zero_state(r.state, r.n, s->dtype, run);
    for (const DevOp &op : r.ops) {
        if (st != SV_OK) return st;
        st = launch_op(op, r.prog, r.state, r.n, s->dtype, run);
    }
    const uint64_t half = uint64_t(1) << (r.n - 1);
    if (st == SV_OK) st = launch_norm2_range(r.state, half, half << 1, s->dtype, r.partials, r.out, run);
    if (st != SV_OK) return st;
    const int D = 1 << r.ns;
    if (s->dtype == SV_C128)
        hipLaunchKernelGGL((k_copy_y<double>), dim3((D + 255) / 256), dim3(256), 0, run,
                           static_cast<const V2<double>::type *>(r.state), half, D, r.out);
    else
        hipLaunchKernelGGL((k_copy_y<float>), dim3((D + 255) / 256), dim3(256), 0, run,
                           static_cast<const V2<float>::type *>(r.state), half, D, r.out);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipEventCreateWithFlags(&r.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(r.done, run);
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: launch: ") + hipGetErrorString(e));
    r.run = run;
    return SV_OK;
}

void prep_main(svs *s)
{
    (void)hipSetDevice(s->device);
    hipStream_t up = nullptr, run = nullptr;
    (void)hipStreamCreateWithFlags(&up, hipStreamNonBlocking);
    (void)hipStreamCreateWithFlags(&run, hipStreamNonBlocking);
    for (;;) {
        std::shared_ptr<Req> r;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_prep.wait(lk, [&] { return s->stopping || !s->prep_q.empty(); });
            if (s->prep_q.empty()) break;   // stopping and drained
            r = s->prep_q.front();
            s->prep_q.pop_front();
        }
        sv_status st = SV_OK;
        std::string err;
        r->t_prep0 = now_s();
        bool ok = !r->cancelled && prepare(s, *r, up, st, err);
        r->t_ready = now_s();
        if (!ok && r->cancelled && st == SV_OK) {
            st = SV_ERR_INVALID;
            err = "svs: request cancelled";
        }
        if (ok && r->kind == kAlone) {
            r->t_launch = now_s();
            st = launch_alone(s, *r, run);
            if (st != SV_OK) {
                ok = false;
                err = sv_last_error();
                (void)hipStreamSynchronize(run);
            }
        }
        std::lock_guard<std::mutex> lk(s->mu);
        if (ok && r->kind == kAlone) {
            s->alone_inflight.push_back(r);
            s->cv_sched.notify_all();
        } else if (ok) {
            s->ready_q.push_back(r);
            s->cv_sched.notify_all();
        } else {
            release(s, r, up);
            finish(s, r, st, err);
        }
    }
    (void)hipStreamSynchronize(up);
    (void)hipStreamSynchronize(run);
    (void)hipStreamDestroy(up);
    (void)hipStreamDestroy(run);
    std::lock_guard<std::mutex> lk(s->mu);
    --s->preps_alive;
    s->cv_sched.notify_all();
}

// Launch one micro-batch on a free slot (caller holds s->mu).
sv_status launch_slot(svs *s, Slot &sl)
{
    const int cnt = (int)sl.reqs.size();
    if (cnt == 0) return SV_OK;
    size_t off = 0;
    for (int i = 0; i < cnt; ++i) {
        sl.h_insts[i] = sl.reqs[i]->inst;
        sl.h_offs[i] = off;
        off += 2 + (2u << sl.reqs[i]->ns);
    }
    if (off > sl.out_cap) return fail(SV_ERR_INVALID, "svs: micro-batch output larger than its staging buffer");
    hipError_t e = hipMemcpyAsync(sl.d_insts, sl.h_insts, cnt * sizeof(BInst), hipMemcpyHostToDevice, sl.stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(sl.d_offs, sl.h_offs, cnt * sizeof(unsigned long long), hipMemcpyHostToDevice, sl.stream);
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: launch: ") + hipGetErrorString(e));
    if (sl.reqs[0]->kind != kAlone) {
        // order by n (one launch per size class), longest programs first
        std::vector<int> idx(cnt);
        for (int i = 0; i < cnt; ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            if (sl.reqs[a]->n != sl.reqs[b]->n) return sl.reqs[a]->n < sl.reqs[b]->n;
            return sl.reqs[a]->inst.op_count > sl.reqs[b]->inst.op_count;
        });
        for (int i = 0; i < cnt; ++i) sl.h_order[i] = idx[i];
        e = hipMemcpyAsync(sl.d_order, sl.h_order, cnt * sizeof(int), hipMemcpyHostToDevice, sl.stream);
        if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: launch: ") + hipGetErrorString(e));
        int first = 0;
        while (first < cnt) {
            const int n = sl.reqs[idx[first]]->n;
            int last = first, kmax = 0;
            while (last < cnt && sl.reqs[idx[last]]->n == n) kmax = std::max(kmax, sl.reqs[idx[last++]]->kmax);
            sv_status st = launch_batch_class(sl.d_insts, sl.d_order + first, last - first, n, kmax, s->dtype,
                                              sl.stream);
            if (st != SV_OK) return st;
            first = last;
        }
    } else {
        Req &r = *sl.reqs[0];
        sv_status st = launch_init_zero_state(r.state, r.n, s->dtype, sl.stream);
        for (const DevOp &op : r.ops) {
            if (st != SV_OK) break;
            st = launch_op(op, r.prog, r.state, r.n, s->dtype, sl.stream);
        }
        const uint64_t half = uint64_t(1) << (r.n - 1);
        if (st == SV_OK)
            st = launch_norm2_range(r.state, half, half << 1, s->dtype, r.partials, r.out, sl.stream);
        if (st != SV_OK) return st;
        const int D = 1 << r.ns;
        if (s->dtype == SV_C128)
            hipLaunchKernelGGL((k_copy_y<double>), dim3((D + 255) / 256), dim3(256), 0, sl.stream,
                               static_cast<const V2<double>::type *>(r.state), half, D, r.out);
        else
            hipLaunchKernelGGL((k_copy_y<float>), dim3((D + 255) / 256), dim3(256), 0, sl.stream,
                               static_cast<const V2<float>::type *>(r.state), half, D, r.out);
        if ((e = hipGetLastError()) != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: ") + hipGetErrorString(e));
    }
    hipLaunchKernelGGL(k_gather_outputs, dim3(std::min(cnt, 1024)), dim3(256), 0, sl.stream, sl.d_insts, cnt,
                       sl.d_offs, sl.d_out);
    if ((e = hipGetLastError()) != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: ") + hipGetErrorString(e));
    e = hipMemcpyAsync(sl.h_out, sl.d_out, off * sizeof(double), hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs: launch: ") + hipGetErrorString(e));
    sl.busy = true;
    return SV_OK;
}

void complete_slot(svs *s, Slot &sl)
{
    // caller holds s->mu; the slot's event has completed
    size_t off = 0;
    for (auto &r : sl.reqs) {
        const size_t len = 2 + (2u << r->ns);
        r->result.assign(sl.h_out + off, sl.h_out + off + len);
        off += len;
        release(s, r, sl.stream);
        finish(s, r, SV_OK, "");
    }
    sl.reqs.clear();
    sl.busy = false;
}

void sched_main(svs *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // retire finished micro-batches
        bool any_busy = false;
        for (Slot &sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                complete_slot(s, sl);
            } else if (q != hipErrorNotReady) {
                const std::string msg = std::string("svs: device error: ") + hipGetErrorString(q);
                for (auto &r : sl.reqs) {
                    release(s, r, sl.stream);
                    finish(s, r, SV_ERR_HIP, msg);
                }
                sl.reqs.clear();
                sl.busy = false;
            } else {
                any_busy = true;
            }
        }
        // retire requests that prep threads launched alone
        for (size_t i = 0; i < s->alone_inflight.size();) {
            std::shared_ptr<Req> r = s->alone_inflight[i];
            const hipError_t q = hipEventQuery(r->done);
            if (q == hipErrorNotReady) {
                any_busy = true;
                ++i;
                continue;
            }
            sv_status st = SV_OK;
            std::string msg;
            if (q == hipSuccess) {
                r->result.resize(2 + (2u << r->ns));
                const hipError_t e = hipMemcpy(r->result.data(), r->out, r->result.size() * sizeof(double),
                                               hipMemcpyDeviceToHost);
                if (e != hipSuccess) {
                    st = SV_ERR_HIP;
                    msg = std::string("svs: result copy: ") + hipGetErrorString(e);
                }
            } else {
                st = SV_ERR_HIP;
                msg = std::string("svs: device error: ") + hipGetErrorString(q);
            }
            (void)hipEventDestroy(r->done);
            r->done = nullptr;
            release(s, r, r->run);
            finish(s, r, st, msg);
            s->alone_inflight[i] = s->alone_inflight.back();
            s->alone_inflight.pop_back();
        }
        // launch new micro-batches on free slots
        for (Slot &sl : s->slots) {
            if (sl.busy || s->ready_q.empty()) continue;
            // the oldest ready request decides the kind of this micro-batch
            const int kind = s->ready_q.front()->kind;
            if (kind != kAlone) {
                for (auto it = s->ready_q.begin(); it != s->ready_q.end() && (int)sl.reqs.size() < s->max_batch;) {
                    if ((*it)->kind == kind) {
                        sl.reqs.push_back(*it);
                        it = s->ready_q.erase(it);
                    } else {
                        ++it;
                    }
                }
            } else {
                sl.reqs.push_back(s->ready_q.front());
                s->ready_q.pop_front();
            }
            const double tl = now_s();
            for (auto &r : sl.reqs) r->t_launch = tl;
            const sv_status st = launch_slot(s, sl);
            if (st != SV_OK) {
                const std::string msg = sv_last_error();
                (void)hipStreamSynchronize(sl.stream);
                for (auto &r : sl.reqs) {
                    release(s, r, sl.stream);
                    finish(s, r, st, msg);
                }
                sl.reqs.clear();
                sl.busy = false;
            } else {
                any_busy = true;
            }
        }
        if (s->stopping && s->preps_alive == 0 && s->ready_q.empty() && s->alone_inflight.empty() && !any_busy)
            break;
        if (any_busy)
            s->cv_sched.wait_for(lk, std::chrono::microseconds(50));
        else
            s->cv_sched.wait_for(lk, std::chrono::milliseconds(5));
    }
}

sv_status start_threads(svs *s)
{
    if (s->started) return SV_OK;
    s->slots.resize(s->nstreams);
    const size_t out_cap = (size_t)s->max_batch * (2 + 2 * 4096);
    for (Slot &sl : s->slots) {
        hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_insts, s->max_batch * sizeof(BInst));
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_order, s->max_batch * sizeof(int));
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_offs, s->max_batch * sizeof(unsigned long long));
        if (e == hipSuccess) e = hipHostMalloc((void **)&sl.h_out, out_cap * sizeof(double));
        if (e == hipSuccess) e = hipMalloc((void **)&sl.d_insts, s->max_batch * sizeof(BInst));
        if (e == hipSuccess) e = hipMalloc((void **)&sl.d_order, s->max_batch * sizeof(int));
        if (e == hipSuccess) e = hipMalloc((void **)&sl.d_offs, s->max_batch * sizeof(unsigned long long));
        if (e == hipSuccess) e = hipMalloc((void **)&sl.d_out, out_cap * sizeof(double));
        if (e != hipSuccess) return fail(SV_ERR_HIP, std::string("svs_start: ") + hipGetErrorString(e));
        sl.out_cap = out_cap;
    }
    s->preps_alive = s->prep_threads;
    for (int i = 0; i < s->prep_threads; ++i) s->threads.emplace_back(prep_main, s);
    s->threads.emplace_back(sched_main, s);
    s->started = true;
    return SV_OK;
}

}  // namespace

extern "C" sv_status svs_start(size_t hbm_budget_bytes, int max_slots, sv_dtype dtype, svs **out)
{
    if (!out) return fail(SV_ERR_INVALID, "svs_start: out is NULL");
    *out = nullptr;
    if (dtype != SV_C128 && dtype != SV_C64) return fail(SV_ERR_INVALID, "svs_start: bad dtype");
    if (max_slots < 1) return fail(SV_ERR_INVALID, "svs_start: max_slots must be >= 1");
    auto *s = new (std::nothrow) svs;
    if (!s) return fail(SV_ERR_OOM, "svs_start: out of host memory");
    s->dtype = dtype;
    s->max_slots = max_slots;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(SV_ERR_HIP, "svs_start: hipGetDevice failed");
    }
    if (hbm_budget_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete s;
            return fail(SV_ERR_HIP, "svs_start: hipMemGetInfo failed");
        }
        hbm_budget_bytes = free_b / 2;
    }
    s->budget = hbm_budget_bytes;
    const unsigned hw = std::max(2u, std::thread::hardware_concurrency());
    s->prep_threads = (int)std::max(1u, std::min(12u, hw - 1));
    *out = s;
    return SV_OK;
}

extern "C" sv_status svs_configure(svs *s, int option, double value)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_configure: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->started) return fail(SV_ERR_BUSY, "svs_configure: the server has already started");
    switch (option) {
    case SVS_OPT_PREP_THREADS:
        if (value < 1 || value > 256) return fail(SV_ERR_INVALID, "svs_configure: prep threads in [1, 256]");
        s->prep_threads = (int)value;
        return SV_OK;
    case SVS_OPT_K_MAX:
        if (value < 0 || value > 5) return fail(SV_ERR_INVALID, "svs_configure: k_max in [0, 5]");
        s->k_max = (int)value;
        return SV_OK;
    case SVS_OPT_MAX_BATCH:
        if (value < 1 || value > 65535) return fail(SV_ERR_INVALID, "svs_configure: max batch in [1, 65535]");
        s->max_batch = (int)value;
        return SV_OK;
    case SVS_OPT_STREAMS:
        if (value < 1 || value > 32) return fail(SV_ERR_INVALID, "svs_configure: streams in [1, 32]");
        s->nstreams = (int)value;
        return SV_OK;
    case SVS_OPT_QUEUE_LIMIT:
        if (value < 1) return fail(SV_ERR_INVALID, "svs_configure: queue limit >= 1");
        s->queue_limit = (size_t)value;
        return SV_OK;
    case SVS_OPT_BATCH_MAX_QUBITS:
        if (value < 0 || value > 24) return fail(SV_ERR_INVALID, "svs_configure: batch qubit limit in [0, 24]");
        s->batch_max_qubits = (int)value;
        return SV_OK;
    case SVS_OPT_HHL_FLAGS: {
        const int f = (int)value;
        if (value < 0 || f != value || (f & ~(SV_HHL_SIGNED | SV_HHL_DILATE | SV_HHL_AUTO | SV_HHL_GAUSS_SEIDEL)))
            return fail(SV_ERR_INVALID,
                        "svs_configure: HHL flags must combine SV_HHL_SIGNED, _DILATE, _AUTO, _GAUSS_SEIDEL");
        s->hhl_flags = f;
        return SV_OK;
    }
    case SVS_OPT_FAIL_ALLOC_AT:
        if (value < 0) return fail(SV_ERR_INVALID, "svs_configure: allocation index >= 0");
        s->fail_alloc_at = (long)value;
        return SV_OK;
    default:
        return fail(SV_ERR_INVALID, "svs_configure: unknown option");
    }
}

extern "C" sv_status svs_submit(svs *s, const double *A, const double *b, int dim, int clock_bits, double t,
                                uint64_t *ticket)
{
    if (!s || !A || !b || !ticket) return fail(SV_ERR_INVALID, "svs_submit: NULL argument");
    if (dim < 1 || dim > 4096 || clock_bits < 1 || clock_bits > 16)
        return fail(SV_ERR_INVALID, "svs_submit: dim in [1, 4096], clock_bits in [1, 16]");
    auto r = std::make_shared<Req>();
    r->A.assign(A, A + (size_t)dim * dim);
    r->b.assign(b, b + dim);
    r->dim = dim;
    r->m = clock_bits;
    r->t = t;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return fail(SV_ERR_INVALID, "svs_submit: server is stopping");
    sv_status st = start_threads(s);
    if (st != SV_OK) return st;
    if (s->prep_q.size() >= s->queue_limit) {
        ++s->n_rejected;
        return fail(SV_ERR_BUSY, "svs_submit: queue full");
    }
    r->ticket = s->next_ticket++;
    r->t_arrive = now_s();
    if (s->first_arrival == 0) s->first_arrival = r->t_arrive;
    s->all.emplace(r->ticket, r);
    s->prep_q.push_back(r);
    ++s->pending;
    s->cv_prep.notify_one();
    *ticket = r->ticket;
    return SV_OK;
}

extern "C" sv_status svs_poll(svs *s, uint64_t ticket, double *x_hat, int dim, sv_solution_info *info)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_poll: NULL server");
    std::shared_ptr<Req> r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return fail(SV_ERR_INVALID, "svs_poll: unknown ticket");
        r = it->second;
        if (r->t_done == 0) return SV_PENDING;
        s->all.erase(it);
    }
    if (r->status != SV_OK) return fail(r->status, r->err);
    if (!x_hat) return fail(SV_ERR_INVALID, "svs_poll: x_hat is NULL");
    if (dim != r->h.dim) return fail(SV_ERR_SHAPE, "svs_poll: dim differs from the request's");
    return recover_solution(r->h, r->result.data(), x_hat, dim, info);
}

extern "C" sv_status svs_cancel(svs *s, uint64_t ticket)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_cancel: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return fail(SV_ERR_INVALID, "svs_cancel: unknown ticket");
    std::shared_ptr<Req> r = it->second;
    if (r->t_done != 0 || r->admitted) return fail(SV_ERR_BUSY, "svs_cancel: request already admitted");
    r->cancelled = true;
    auto q = std::find(s->prep_q.begin(), s->prep_q.end(), r);
    if (q != s->prep_q.end()) {
        s->prep_q.erase(q);
        finish(s, r, SV_ERR_INVALID, "svs: request cancelled");
    }
    s->cv_budget.notify_all();
    return SV_OK;
}

extern "C" sv_status svs_drain(svs *s, double timeout_s)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_drain: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto pred = [&] { return s->pending == 0; };
    if (timeout_s <= 0) {
        s->cv_done.wait(lk, pred);
        return SV_OK;
    }
    if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), pred))
        return fail(SV_ERR_BUSY, "svs_drain: timed out with requests pending");
    return SV_OK;
}

extern "C" sv_status svs_stats(svs *s, double *p50_s, double *p99_s, double *solves_per_s, uint64_t *n_rejected)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_stats: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    std::vector<double> l = s->latencies;
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) -> double {
        if (l.empty()) return 0.0;
        // nearest rank on the exact sorted sample
        size_t k = (size_t)std::ceil(p * (double)l.size());
        k = std::max<size_t>(1, std::min(k, l.size()));
        return l[k - 1];
    };
    if (p50_s) *p50_s = pct(0.50);
    if (p99_s) *p99_s = pct(0.99);
    if (solves_per_s) {
        const double span = s->last_done - s->first_arrival;
        *solves_per_s = (span > 0 && s->n_done) ? (double)s->n_done / span : 0.0;
    }
    if (n_rejected) *n_rejected = s->n_rejected;
    return SV_OK;
}

extern "C" sv_status svs_counts(svs *s, uint64_t *done, uint64_t *failed, uint64_t *pending)
{
    if (!s) return fail(SV_ERR_INVALID, "svs_counts: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (done) *done = s->n_done;
    if (failed) *failed = s->n_failed;
    if (pending) *pending = s->pending;
    return SV_OK;
}

extern "C" sv_status svs_profile(svs *s, double *out, int cap)
{
    if (!s || !out || cap < 8) return fail(SV_ERR_INVALID, "svs_profile: need an output array of 8");
    std::lock_guard<std::mutex> lk(s->mu);
    const double n = s->n_done ? (double)s->n_done : 1.0;
    out[0] = s->sum_queue / n;    // submit -> prep start
    out[1] = s->sum_prep / n;     // build + fuse + lower + admission wait
    out[2] = s->sum_upload / n;   // allocation + upload + device evolution tables
    out[3] = s->sum_ready / n;    // resident -> launched
    out[4] = s->sum_gpu / n;      // launched -> results back
    out[5] = (double)s->n_small;
    out[6] = (double)s->n_large;
    out[7] = (double)s->prep_threads;
    return SV_OK;
}

extern "C" sv_status svs_stop(svs *s)
{
    if (!s) return SV_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_prep.notify_all();
        s->cv_budget.notify_all();
        s->cv_sched.notify_all();
    }
    for (auto &t : s->threads) t.join();
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        (void)hipFree(sl.d_insts);
        (void)hipFree(sl.d_order);
        (void)hipFree(sl.d_offs);
        (void)hipFree(sl.d_out);
        if (sl.h_insts) (void)hipHostFree(sl.h_insts);
        if (sl.h_order) (void)hipHostFree(sl.h_order);
        if (sl.h_offs) (void)hipHostFree(sl.h_offs);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s;
    return SV_OK;
}
