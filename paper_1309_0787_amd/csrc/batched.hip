// Batched STGD: many decompositions (uneven k and row counts), each with
// several restarts, in one launch.  A host planner turns the problem table
// into jobs (problem, restart) and groups them by kernel variant (padded k,
// tile layout chosen by the autotuner, view staging), longest job first in
// every group.  A run enqueues, on one stream or into one graph:
//   reset (queue counters, non-finite flag)
//   -> one persistent kernel per group on up to four forked branches (as
//      many as run side by side), groups balanced over the branches by
//      estimated work; a kernel's workgroups pull jobs from its group's
//      counter until it is empty
//   -> selection of the best restart of every problem.
// Each persistent kernel is its own instantiation, so its registers are
// allocated for its variant alone and small-k variants keep more workgroups
// per CU.  Every job ends with a scoring pass (the residual up to a constant).
//
// Variants (FP32 operands): padded k KP = 16, 32, ..., 128; wave grid 4 x 2
// (layout 0) or, layout 1, 8 x 1 for KP <= 32 and 2 x 4 above; batch staging
// for one aliased view or three views.
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "stgd_kernel.h"

namespace otm {
namespace {

constexpr int kClasses = kMaxK / 16;          // KP = 16 (c + 1)
constexpr int kVariants = kClasses * 2 * 2;   // x layout x view staging
constexpr int kMaxBranches = 16;              // most concurrent streams of one run (hardware queues)

__host__ __device__ constexpr int variant_id(int cls, int layout, int three_views) {
    return (cls * 2 + layout) * 2 + three_views;
}

template <int KP, int L>
constexpr int wr_of() { return L == 0 ? 4 : (KP <= 32 ? 8 : 2); }

template <int KP, int L, int V3>
struct Var {
    static constexpr int WR = wr_of<KP, L>();
    static constexpr int NS = staging_for<MmaF32, KP, WR>(V3 == 0);
    using SM = SgdSmem<MmaF32, KP, NS, WR>;
};

struct BatchJob {
    SgdArgs args;
    int32_t r_id;
    int32_t problem;
};

struct BatchProblem {
    double* score;
    int32_t restarts;
    int32_t pad_;
};

// --------------------------------------------------------------- kernels
// Persistent: every workgroup takes the next job of its group from the
// group's counter until the index passes the group's end, so every wave
// reaches the exit.
template <int KP, int L, int V3>
__global__ __launch_bounds__(kThreads) void sgd_persistent_kernel(const BatchJob* __restrict__ jobs, int count,
                                                                  int32_t* counter) {
    using VV = Var<KP, L, V3>;
    __shared__ __attribute__((aligned(16))) typename VV::SM sm;
    __shared__ int s_job;
    for (;;) {
        if (threadIdx.x == 0) s_job = atomicAdd(counter, 1);
        __syncthreads();
        const int j = __builtin_amdgcn_readfirstlane(s_job);
        __syncthreads();   // s_job is rewritten only after every wave has read it
        if (j >= count) break;
        const SgdArgs g = jobs[j].args;
        sgd_body<MmaF32, KP, VV::NS, VV::WR, true, true, KP / 16, V3 == 0 && VV::NS == 0>(g, jobs[j].r_id, sm);
    }
}

using KernelFn = void (*)(const BatchJob*, int, int32_t*);

KernelFn variant_kernel(int v) {
    static const KernelFn table[kVariants] = {
#define OTM_K(KP) sgd_persistent_kernel<KP, 0, 0>, sgd_persistent_kernel<KP, 0, 1>, \
                  sgd_persistent_kernel<KP, 1, 0>, sgd_persistent_kernel<KP, 1, 1>,
        OTM_K(16) OTM_K(32) OTM_K(48) OTM_K(64) OTM_K(80) OTM_K(96) OTM_K(112) OTM_K(128)
#undef OTM_K
    };
    return table[v];
}

__global__ void batched_reset_kernel(int32_t* counters, int n, int32_t* nonfinite) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0;
    if (threadIdx.x == 0 && nonfinite != nullptr) *nonfinite = 0;
}

// best restart of every problem: lowest score, ties to the lower index, a
// non-finite score never wins over a finite one
__global__ void select_best_kernel(const BatchProblem* __restrict__ probs, int n_problems, int32_t* best) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n_problems) return;
    const BatchProblem P = probs[p];
    int b = 0;
    double bv = P.score[0];
    for (int r = 1; r < P.restarts; ++r) {
        const double v = P.score[r];
        if ((v < bv) || (!isfinite(bv) && isfinite(v))) {
            b = r;
            bv = v;
        }
    }
    best[p] = b;
}

// one job descriptor copied `count` times with r_id = index
__global__ void write_jobs_kernel(BatchJob job, int count, BatchJob* out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count) return;
    BatchJob j = job;
    j.r_id = r;
    out[r] = j;
}

// ------------------------------------------------------------- device info
int device_info(int* cus) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
    return e == hipSuccess ? OTM_OK : hip_fail(e, "hipDeviceGetAttribute");
}

int per_cu(int v, int* out) {
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(out, variant_kernel(v), kThreads, 0);
    if (e != hipSuccess) return hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    *out = std::max(1, *out);
    return OTM_OK;
}

// library-owned streams and events for the concurrent branches of a run
// (default priority, non-blocking streams; events without timing), created
// once per device and kept until the process ends.  Runs on one device must
// not be issued from several host threads at once.
// Kernels of one process run side by side on at most as many hardware queues
// as the HIP runtime gives it (GPU_MAX_HW_QUEUES, 4 by default).
int hw_queues() {
    static const int q = [] {
        const char* v = getenv("GPU_MAX_HW_QUEUES");
        const int n = v ? atoi(v) : 4;
        return n < 1 ? 1 : (n > kMaxBranches ? kMaxBranches : n);
    }();
    return q;
}

struct Branches {
    hipStream_t stream[kMaxBranches];
    hipEvent_t fork;
    hipEvent_t join[kMaxBranches];
    bool ready;
};

int branches(Branches** out) {
    static Branches per_dev[64] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    OTM_REQUIRE(dev >= 0 && dev < 64, OTM_EINVAL, "device index out of range");
    Branches& b = per_dev[dev];
    if (!b.ready) {
        for (int i = 0; i < hw_queues(); ++i) {
            if ((e = hipStreamCreateWithFlags(&b.stream[i], hipStreamNonBlocking)) != hipSuccess)
                return hip_fail(e, "hipStreamCreateWithFlags");
            if ((e = hipEventCreateWithFlags(&b.join[i], hipEventDisableTiming)) != hipSuccess)
                return hip_fail(e, "hipEventCreateWithFlags");
        }
        if ((e = hipEventCreateWithFlags(&b.fork, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "hipEventCreateWithFlags");
        b.ready = true;
    }
    *out = &b;
    return OTM_OK;
}

}  // namespace
}  // namespace otm

// ------------------------------------------------------------------ plans
struct otm_plan_s {
    struct Group {
        int variant;
        int first, count;   // jobs [first, first + count) of the image
        double work;        // estimated microseconds of all its jobs
    };
    std::vector<char> image;   // device image: jobs, then problems
    std::vector<Group> groups;
    int n_jobs = 0, n_problems = 0;
    size_t problems_offset = 0;
    int32_t* best = nullptr;
    int32_t* nonfinite = nullptr;
};

namespace otm {
namespace {

// --------------------------------------------------------------- tuning cache
// Lines: "sgd_batched f32 kp=<KP> views=<1|3> layout=<0|1> us_step=<t0>,<t1>"
struct TuneEntry {
    int layout;
    double us0, us1;
};
using TuneMap = std::map<std::pair<int, int>, TuneEntry>;

TuneMap read_cache(const char* path) {
    TuneMap m;
    if (path == nullptr) return m;
    FILE* f = std::fopen(path, "r");
    if (!f) return m;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        int kp = 0, views = 0, layout = 0;
        double a = 0, b = 0;
        if (std::sscanf(line, "sgd_batched f32 kp=%d views=%d layout=%d us_step=%lf,%lf", &kp, &views, &layout, &a,
                        &b) == 5 &&
            kp >= 16 && kp <= kMaxK && kp % 16 == 0 && (views == 1 || views == 3) && (layout == 0 || layout == 1))
            m[{kp, views}] = TuneEntry{layout, a, b};
    }
    std::fclose(f);
    return m;
}

int write_cache(const char* path, const TuneMap& m) {
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return fail(OTM_EINVAL, std::string("cannot write tuning cache ") + path);
    std::fprintf(f, "# batched STGD tile layouts, microseconds per step of each layout\n");
    for (const auto& kv : m)
        std::fprintf(f, "sgd_batched f32 kp=%d views=%d layout=%d us_step=%.4f,%.4f\n", kv.first.first,
                     kv.first.second, kv.second.layout, kv.second.us0, kv.second.us1);
    std::fclose(f);
    if (std::rename(tmp.c_str(), path) != 0) return fail(OTM_EINVAL, std::string("cannot replace ") + path);
    return OTM_OK;
}

// estimated microseconds per step when nothing is tuned: a fixed latency plus
// the k x k and batch products
double model_us_step(int kp, int batch) {
    const double k = kp;
    return 2.0 + (4.0 * k * k * k + 6.0 * batch * k * k) / 2.0e6;
}

int fill_problem_job(const otm_problem& P, const otm_sgd_params* p, int restarts, BatchJob& J) {
    OTM_REQUIRE(P.YA && P.YB && P.YC && P.ybar && P.Phi0 && P.Phi && P.score, OTM_EINVAL,
                "problem has a null pointer");
    std::memset(&J, 0, sizeof J);
    int s = fill_scalars(P.n, P.k, P.ldy, P.alpha0, p, 0, -1, J.args);
    if (s != OTM_OK) return s;
    OTM_REQUIRE(P.perms == nullptr || restarts == 1 || P.perm_stride == 0 ||
                    P.perm_stride >= (int64_t)p->passes * P.n,
                OTM_ESHAPE, "perm_stride must be 0 (shared) or >= passes * n");
    SgdArgs& a = J.args;
    a.YA = P.YA; a.YB = P.YB; a.YC = P.YC; a.ybar = P.ybar; a.perms = P.perms; a.perm_stride = P.perm_stride;
    a.Phi0 = P.Phi0; a.Phi = P.Phi; a.Phi_comp = nullptr; a.snapshots = nullptr; a.score = P.score;
    return OTM_OK;
}

// One run of a plan whose image is at `image` in device memory: reset, the
// groups' persistent kernels on forked branches, then the selection.
int enqueue_plan(const otm_plan_s& P, const void* image, int32_t* counters, hipStream_t st) {
    int cus = 0, s = device_info(&cus);
    if (s != OTM_OK) return s;
    const int ng = static_cast<int>(P.groups.size());
    hipLaunchKernelGGL(batched_reset_kernel, dim3(1), dim3(64), 0, st, counters, ng, P.nonfinite);
    if ((s = check_launch("batched_reset_kernel")) != OTM_OK) return s;
    // Branches: as many as a process's kernels run side by side (its hardware
    // queues).  Groups go to the least loaded branch, largest estimated work
    // first, and run one after another there; each kernel takes its branch's
    // share of the device (its variant's resident workgroups over the number
    // of branches, at most its job count).
    const int nb = std::min(ng, hw_queues());
    // every group on a branch of its own: all start at once and each kernel may
    // take the whole device (the dispatcher shares the CUs as queues drain);
    // otherwise the groups of a branch run one after another on its share
    const bool own = nb == ng;
    std::vector<int> order(ng), branch_of(ng), grid(ng);
    for (int i = 0; i < ng; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return P.groups[x].work > P.groups[y].work; });
    std::vector<double> load(nb, 0.0);
    for (int i : order) {
        const int b = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
        branch_of[i] = b;
        load[b] += P.groups[i].work;
        int pc = 1;
        if ((s = per_cu(P.groups[i].variant, &pc)) != OTM_OK) return s;
        const int want = own ? cus * pc : (cus * pc + nb - 1) / nb;
        grid[i] = std::max(1, std::min(P.groups[i].count, want));
    }
    const BatchJob* jobs = static_cast<const BatchJob*>(image);
    const BatchProblem* probs =
        reinterpret_cast<const BatchProblem*>(static_cast<const char*>(image) + P.problems_offset);
    if (ng == 1) {
        const auto& g = P.groups[0];
        hipLaunchKernelGGL(variant_kernel(g.variant), dim3(grid[0]), dim3(kThreads), 0, st, jobs + g.first, g.count,
                           counters);
        if ((s = check_launch("sgd_persistent_kernel")) != OTM_OK) return s;
    } else {
        Branches* B = nullptr;
        if ((s = branches(&B)) != OTM_OK) return s;
        hipError_t e = hipEventRecord(B->fork, st);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        for (int b = 0; b < nb; ++b)
            if ((e = hipStreamWaitEvent(B->stream[b], B->fork, 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        for (int i : order) {
            const auto& g = P.groups[i];
            hipLaunchKernelGGL(variant_kernel(g.variant), dim3(grid[i]), dim3(kThreads), 0, B->stream[branch_of[i]],
                               jobs + g.first, g.count, counters + i);
            if ((s = check_launch("sgd_persistent_kernel")) != OTM_OK) return s;
        }
        for (int b = 0; b < nb; ++b) {
            if ((e = hipEventRecord(B->join[b], B->stream[b])) != hipSuccess) return hip_fail(e, "hipEventRecord");
            if ((e = hipStreamWaitEvent(st, B->join[b], 0)) != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
        }
    }
    hipLaunchKernelGGL(select_best_kernel, dim3((P.n_problems + 255) / 256), dim3(256), 0, st, probs, P.n_problems,
                       P.best);
    return check_launch("select_best_kernel");
}

}  // namespace
}  // namespace otm

using namespace otm;

// ------------------------------------------------------------------ score
extern "C" size_t otm_sgd_score_workspace(int32_t restarts) {
    if (restarts < 1) return 0;
    return ws_round(sizeof(BatchJob) * (size_t)restarts) + 256;
}

extern "C" int otm_sgd_score(const otm_sgd_params* p, int32_t n, const void* YA, const void* YB, const void* YC,
                             const float* ybar, const float* Phi, int32_t restarts, double* score, void* ws,
                             size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(p != nullptr, OTM_EINVAL, "params is NULL");
    OTM_REQUIRE(YA && YB && YC && ybar && Phi && score, OTM_EINVAL, "null data pointer");
    OTM_REQUIRE(p->y_dtype == OTM_F32, OTM_EDTYPE, "the score takes FP32 rows");
    OTM_REQUIRE(restarts >= 1, OTM_ESHAPE, "restarts must be >= 1");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_sgd_score_workspace(restarts), OTM_EWORKSPACE,
                "score workspace too small");
    otm_sgd_params q = *p;
    q.passes = 1;
    BatchJob J;
    std::memset(&J, 0, sizeof J);
    int s = fill_scalars(n, p->k, p->ldy, p->alpha0, &q, 0, 0, J.args);   // no training step
    if (s != OTM_OK) return s;
    SgdArgs& a = J.args;
    a.YA = YA; a.YB = YB; a.YC = YC; a.ybar = ybar;
    a.Phi0 = Phi; a.Phi = const_cast<float*>(Phi);   // written back unchanged
    a.score = score;
    const bool three = !((YA == YB) && (YB == YC));
    const int v = variant_id((p->k + 15) / 16 - 1, 0, three ? 1 : 0);
    hipStream_t st = as_stream(stream);
    BatchJob* jobs = static_cast<BatchJob*>(ws);
    int32_t* counter = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + ws_round(sizeof(BatchJob) * (size_t)restarts));
    hipLaunchKernelGGL(write_jobs_kernel, dim3((restarts + 63) / 64), dim3(64), 0, st, J, restarts, jobs);
    if ((s = check_launch("write_jobs_kernel")) != OTM_OK) return s;
    hipLaunchKernelGGL(batched_reset_kernel, dim3(1), dim3(64), 0, st, counter, 1, static_cast<int32_t*>(nullptr));
    if ((s = check_launch("batched_reset_kernel")) != OTM_OK) return s;
    int cus = 0, pc = 1;
    if ((s = device_info(&cus)) != OTM_OK || (s = per_cu(v, &pc)) != OTM_OK) return s;
    hipLaunchKernelGGL(variant_kernel(v), dim3(std::min(restarts, cus * pc)), dim3(kThreads), 0, st, jobs, restarts,
                       counter);
    return check_launch("sgd_persistent_kernel");
}

// --------------------------------------------------------------- planning
extern "C" int otm_sgd_batched_plan(const otm_problem* problems, int32_t n_problems, int32_t restarts,
                                    const otm_sgd_params* p, const char* tune_cache, int32_t* best,
                                    int32_t* nonfinite, otm_plan* plan) {
    OTM_REQUIRE(problems && p && best && plan, OTM_EINVAL, "null argument");
    *plan = nullptr;
    OTM_REQUIRE(n_problems >= 1 && restarts >= 1, OTM_ESHAPE, "need n_problems >= 1 and restarts >= 1");
    OTM_REQUIRE((int64_t)n_problems * restarts < (int64_t(1) << 30), OTM_ECAPACITY, "too many jobs");
    OTM_REQUIRE(p->y_dtype == OTM_F32, OTM_EDTYPE, "the batched path takes FP32 rows");
    const TuneMap tune = read_cache(tune_cache);
    const int nj = n_problems * restarts;
    std::vector<BatchJob> proto(n_problems);
    std::vector<int> var(n_problems);
    std::vector<double> cost(n_problems);
    for (int i = 0; i < n_problems; ++i) {
        const otm_problem& P = problems[i];
        int s = fill_problem_job(P, p, restarts, proto[i]);
        if (s != OTM_OK) return fail(s, "problem " + std::to_string(i) + ": " + otm_last_error());
        const int cls = (P.k + 15) / 16 - 1, kp = 16 * (cls + 1);
        const int views = (P.YA == P.YB && P.YB == P.YC) ? 1 : 3;
        auto it = tune.find({kp, views});
        const int layout = it != tune.end() ? it->second.layout : 0;
        double us = model_us_step(kp, p->batch);
        if (it != tune.end()) us = layout == 0 ? it->second.us0 : it->second.us1;
        var[i] = variant_id(cls, layout, views == 3 ? 1 : 0);
        proto[i].problem = i;
        cost[i] = double(proto[i].args.spp) * (p->passes + 1) * us;
    }
    // jobs grouped by variant, longest first inside a group (ties: problem, restart)
    std::vector<std::tuple<int, double, int, int>> order;
    order.reserve(nj);
    for (int i = 0; i < n_problems; ++i)
        for (int r = 0; r < restarts; ++r) order.emplace_back(var[i], -cost[i], i, r);
    std::stable_sort(order.begin(), order.end());
    auto* P = new otm_plan_s;
    P->n_jobs = nj;
    P->n_problems = n_problems;
    P->best = best;
    P->nonfinite = nonfinite;
    P->problems_offset = ws_round(sizeof(BatchJob) * (size_t)nj);
    P->image.assign(P->problems_offset + sizeof(BatchProblem) * (size_t)n_problems, 0);
    BatchJob* jobs = reinterpret_cast<BatchJob*>(P->image.data());
    BatchProblem* probs = reinterpret_cast<BatchProblem*>(P->image.data() + P->problems_offset);
    for (int j = 0; j < nj; ++j) {
        const int v = std::get<0>(order[j]), i = std::get<2>(order[j]), r = std::get<3>(order[j]);
        jobs[j] = proto[i];
        jobs[j].r_id = r;
        jobs[j].args.nonfinite = nonfinite;
        if (P->groups.empty() || P->groups.back().variant != v) P->groups.push_back({v, j, 0, 0.0});
        P->groups.back().count += 1;
        P->groups.back().work += cost[i];
    }
    for (int i = 0; i < n_problems; ++i) {
        probs[i].score = problems[i].score;
        probs[i].restarts = restarts;
    }
    *plan = P;
    return OTM_OK;
}

extern "C" size_t otm_plan_size(otm_plan plan) { return plan ? plan->image.size() : 0; }
extern "C" const void* otm_plan_image(otm_plan plan) { return plan ? plan->image.data() : nullptr; }
extern "C" int32_t otm_plan_groups(otm_plan plan) { return plan ? static_cast<int32_t>(plan->groups.size()) : 0; }
extern "C" int otm_plan_group_info(otm_plan plan, int32_t group, int32_t* kp, int32_t* layout, int32_t* views,
                                   int32_t* jobs) {
    OTM_REQUIRE(plan != nullptr && kp && layout && views && jobs, OTM_EINVAL, "null argument");
    OTM_REQUIRE(group >= 0 && group < static_cast<int32_t>(plan->groups.size()), OTM_ESHAPE, "no such group");
    const auto& g = plan->groups[group];
    *kp = 16 * (g.variant / 4 + 1);
    *layout = (g.variant / 2) % 2;
    *views = (g.variant % 2) ? 3 : 1;
    *jobs = g.count;
    return OTM_OK;
}

extern "C" int otm_plan_free(otm_plan plan) {
    delete plan;
    return OTM_OK;
}

extern "C" size_t otm_sgd_batched_workspace(otm_plan plan) {
    if (plan == nullptr) return 0;
    return ws_round(sizeof(int32_t) * plan->groups.size());
}

extern "C" int otm_sgd_batched(otm_plan plan, const void* image, void* ws, size_t ws_bytes, otm_stream stream) {
    OTM_REQUIRE(plan != nullptr && image != nullptr, OTM_EINVAL, "plan and image must not be NULL");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_sgd_batched_workspace(plan), OTM_EWORKSPACE,
                "batched workspace too small");
    return enqueue_plan(*plan, image, static_cast<int32_t*>(ws), as_stream(stream));
}

// ------------------------------------------------------------------ graphs
struct otm_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

extern "C" int otm_sgd_batched_graph(otm_plan plan, const void* image, void* ws, size_t ws_bytes, otm_stream stream,
                                     otm_graph* graph) {
    OTM_REQUIRE(plan != nullptr && image != nullptr && graph != nullptr, OTM_EINVAL, "null argument");
    OTM_REQUIRE(stream != nullptr, OTM_EINVAL, "capture needs a stream other than the null stream");
    OTM_REQUIRE(ws != nullptr && ws_bytes >= otm_sgd_batched_workspace(plan), OTM_EWORKSPACE,
                "batched workspace too small");
    hipStream_t st = as_stream(stream);
    Branches* B = nullptr;
    int s = branches(&B);   // created before the capture starts
    if (s != OTM_OK) return s;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    s = enqueue_plan(*plan, image, static_cast<int32_t*>(ws), st);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (s != OTM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    auto* out = new otm_graph_s;
    out->graph = g;
    e = hipGraphInstantiate(&out->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete out;
        return hip_fail(e, "hipGraphInstantiate");
    }
    *graph = out;
    return OTM_OK;
}

extern "C" int otm_graph_launch(otm_graph graph, otm_stream stream) {
    OTM_REQUIRE(graph != nullptr && graph->exec != nullptr, OTM_EINVAL, "graph is NULL");
    hipError_t e = hipGraphLaunch(graph->exec, as_stream(stream));
    return e == hipSuccess ? OTM_OK : hip_fail(e, "hipGraphLaunch");
}

extern "C" int otm_graph_destroy(otm_graph graph) {
    if (graph == nullptr) return OTM_OK;
    hipError_t e1 = graph->exec ? hipGraphExecDestroy(graph->exec) : hipSuccess;
    hipError_t e2 = graph->graph ? hipGraphDestroy(graph->graph) : hipSuccess;
    delete graph;
    if (e1 != hipSuccess) return hip_fail(e1, "hipGraphExecDestroy");
    return e2 == hipSuccess ? OTM_OK : hip_fail(e2, "hipGraphDestroy");
}

// ------------------------------------------------------------------ tuning
namespace {

// deterministic probe data: uniform values in [-s, s] from an integer hash
__global__ void probe_fill_kernel(float* y, size_t count, float s, uint32_t salt) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t h = static_cast<uint32_t>(i) * 0x9E3779B1u ^ salt;
        h ^= h >> 15;
        h *= 0x85EBCA77u;
        h ^= h >> 13;
        h *= 0xC2B2AE3Du;
        h ^= h >> 16;
        y[i] = s * (static_cast<float>(h >> 8) * (2.0f / 16777216.0f) - 1.0f);
    }
}

}  // namespace

extern "C" int otm_sgd_autotune(const int32_t* ks, int32_t n_k, int32_t batch, const char* cache_path,
                                otm_stream stream) {
    OTM_REQUIRE(ks != nullptr && n_k >= 1 && cache_path != nullptr, OTM_EINVAL, "null argument");
    OTM_REQUIRE(batch >= 1 && batch <= kMaxBatch, OTM_ECAPACITY, "batch must be in [1, 128]");
    std::vector<int> kps;
    for (int i = 0; i < n_k; ++i) {
        OTM_REQUIRE(ks[i] >= 1 && ks[i] <= kMaxK, OTM_ECAPACITY, "k must be in [1, 128]");
        kps.push_back(16 * ((ks[i] + 15) / 16));
    }
    std::sort(kps.begin(), kps.end());
    kps.erase(std::unique(kps.begin(), kps.end()), kps.end());
    hipStream_t st = as_stream(stream);
    int cus = 0;
    int s = device_info(&cus);
    if (s != OTM_OK) return s;
    // jobs per probe: two per CU at the widest occupancy of any variant
    int most = 1;
    for (int v = 0; v < kVariants; ++v) {
        int pc = 1;
        if ((s = per_cu(v, &pc)) != OTM_OK) return s;
        most = std::max(most, pc);
    }
    const int n = 8 * batch, kmax = kMaxK, jobs_n = 2 * cus * most;
    const size_t yb = sizeof(float) * (size_t)n * kmax;
    float *Y = nullptr, *ybar = nullptr, *Phi0 = nullptr, *Phi = nullptr;
    double* score = nullptr;
    BatchJob* jobs = nullptr;
    int32_t* counter = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        (void)hipFree(Y); (void)hipFree(ybar); (void)hipFree(Phi0); (void)hipFree(Phi);
        (void)hipFree(score); (void)hipFree(jobs); (void)hipFree(counter);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    hipError_t e = hipSuccess;
    const size_t phi_bytes = sizeof(float) * (size_t)jobs_n * kmax * kmax;
    if ((e = hipMalloc(&Y, 3 * yb)) != hipSuccess || (e = hipMalloc(&ybar, sizeof(float) * 3 * kmax)) != hipSuccess ||
        (e = hipMalloc(&Phi0, phi_bytes)) != hipSuccess || (e = hipMalloc(&Phi, phi_bytes)) != hipSuccess ||
        (e = hipMalloc(&score, sizeof(double) * (size_t)jobs_n)) != hipSuccess ||
        (e = hipMalloc(&jobs, sizeof(BatchJob) * (size_t)jobs_n)) != hipSuccess ||
        (e = hipMalloc(&counter, 256)) != hipSuccess || (e = hipEventCreate(&e0)) != hipSuccess ||
        (e = hipEventCreate(&e1)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "autotune buffers");
    }
    TuneMap cache = read_cache(cache_path);
    int status = OTM_OK;
    for (int kp : kps) {
        const int cls = kp / 16 - 1;
        hipLaunchKernelGGL(probe_fill_kernel, dim3(256), dim3(256), 0, st, Y, 3 * yb / sizeof(float),
                           1.0f / std::sqrt(static_cast<float>(kp)), 0x51ed27u + kp);
        hipLaunchKernelGGL(probe_fill_kernel, dim3(4), dim3(256), 0, st, ybar, (size_t)3 * kmax, 0.01f, 0x1234u);
        hipLaunchKernelGGL(probe_fill_kernel, dim3(512), dim3(256), 0, st, Phi0, phi_bytes / sizeof(float),
                           1.0f / std::sqrt(static_cast<float>(kp)), 0x777u);
        if ((status = check_launch("probe_fill_kernel")) != OTM_OK) break;
        for (int views : {1, 3}) {
            double us[2] = {0, 0};
            for (int layout = 0; layout < 2 && status == OTM_OK; ++layout) {
                otm_sgd_params q{};
                q.k = kp; q.batch = batch; q.passes = 1; q.ldy = kp; q.y_dtype = OTM_F32; q.compensated = 1;
                q.alpha0 = 0.5; q.theta = 1.0; q.beta0 = 1e-4; q.beta_tau = 1e9;
                BatchJob J;
                std::memset(&J, 0, sizeof J);
                if ((status = fill_scalars(n, kp, kp, q.alpha0, &q, 0, -1, J.args)) != OTM_OK) break;
                SgdArgs& a = J.args;
                a.YA = Y;
                a.YB = views == 3 ? Y + (size_t)n * kmax : Y;
                a.YC = views == 3 ? Y + 2 * (size_t)n * kmax : Y;
                a.ybar = ybar; a.Phi0 = Phi0; a.Phi = Phi; a.score = score;
                const int v = variant_id(cls, layout, views == 3 ? 1 : 0);
                int pc = 1;
                if ((status = per_cu(v, &pc)) != OTM_OK) break;
                // every job (r_id = its index) writes its own Phi and score slot
                hipLaunchKernelGGL(write_jobs_kernel, dim3((jobs_n + 63) / 64), dim3(64), 0, st, J, jobs_n, jobs);
                if ((status = check_launch("write_jobs_kernel")) != OTM_OK) break;
                float best_ms = 1e30f;
                for (int rep = 0; rep < 4 && status == OTM_OK; ++rep) {
                    hipLaunchKernelGGL(batched_reset_kernel, dim3(1), dim3(64), 0, st, counter, 1,
                                       static_cast<int32_t*>(nullptr));
                    if ((e = hipEventRecord(e0, st)) != hipSuccess) { status = hip_fail(e, "hipEventRecord"); break; }
                    hipLaunchKernelGGL(variant_kernel(v), dim3(std::min(jobs_n, cus * pc)), dim3(kThreads), 0, st,
                                       jobs, jobs_n, counter);
                    if ((status = check_launch("sgd_persistent_kernel")) != OTM_OK) break;
                    if ((e = hipEventRecord(e1, st)) != hipSuccess) { status = hip_fail(e, "hipEventRecord"); break; }
                    if ((e = hipEventSynchronize(e1)) != hipSuccess) { status = hip_fail(e, "hipEventSynchronize"); break; }
                    float ms = 0.f;
                    if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) { status = hip_fail(e, "hipEventElapsedTime"); break; }
                    if (rep > 0) best_ms = std::min(best_ms, ms);   // the first run warms up
                }
                // cost of one step in CU-microseconds: elapsed time over the job-steps,
                // times the CUs (the inverse of the throughput per CU)
                const double steps = 2.0 * ((n + batch - 1) / batch);   // one pass + the scoring pass
                us[layout] = best_ms * 1e3 * cus / (double(jobs_n) * steps);
            }
            if (status != OTM_OK) break;
            cache[{kp, views}] = TuneEntry{us[1] < us[0] ? 1 : 0, us[0], us[1]};
        }
        if (status != OTM_OK) break;
    }
    cleanup();
    if (status != OTM_OK) return status;
    return write_cache(cache_path, cache);
}
