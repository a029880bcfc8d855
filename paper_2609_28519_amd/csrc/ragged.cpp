// Ragged batches: thousands of arrays of different shapes (square blocks 8..256 and
// whole images up to 1024 per axis) transformed by one hipGraphLaunch.
//
// Plan creation (host, once): the descriptors are validated and grouped into shape
// classes; each class gets a device-resident list of element offsets and the kernel
// configuration of the frozen per-size policy (the same table the autotuner fills for
// the basic calls, Section 3.2: variants fixed before measurement), with grid-stride
// schedules replaced by one tile per workgroup, since the classes share the GPU.  Image classes
// with power-of-two axes and an axis of 512 or 1024 run the two-pass long-axis kernels in
// place on the batch (no workspace); image classes with an axis that is not a power of two
// (such as 384) get dense float32 Q tables and a workspace.  The whole batch is then
// recorded once into a HIP graph: one fork-join branch per class, so independent
// classes run concurrently.  Kernels read the batch base pointer from a plan-owned
// device slot, so the recorded graph replays on any buffer.
//
// Execute: if the base differs from the one in the slot, one 8-byte copy updates the
// slot (stream-ordered before the graph); then a single hipGraphLaunch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "internal.hpp"

using namespace dct;

namespace {

struct ClassRec {
    int rows, cols;
    int64_t count;
    int64_t* d_off = nullptr; // device offsets (floats from base)
    bool dense = false;       // dense axis passes through the workspace
    bool long_axes = false;   // two-pass long-axis kernels (an axis of 512 or 1024)
    float* q_rows = nullptr;  // dense Q_rows (column pass)
    float* q_cols = nullptr;  // dense Q_cols (row pass)
    float* ws = nullptr;      // workspace, count * rows * cols floats
};

bool fast_shape(int r, int c)
{
    return is_pow2(r) && is_pow2(c) && r >= 8 && r <= 256 && c >= 8 && c <= 256;
}

bool long_shape(int r, int c)
{
    return is_pow2(r) && is_pow2(c) && r >= 8 && c >= 8 && r <= 1024 && c <= 1024 && (r > 256 || c > 256);
}

bool dense_shape(int r, int c) { return !fast_shape(r, c) && !long_shape(r, c); }

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

} // namespace

struct dct2d_ragged_plan {
    int device = -1;
    int dir = 0, prec = 0;
    int64_t items = 0;
    void* dmem = nullptr;
    float** d_slot = nullptr;
    float* bound = nullptr; // base currently in the slot
    std::vector<ClassRec> cls;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int nodes = 0;
    std::mutex mu;
};

namespace {

void release(dct2d_ragged_plan* p)
{
    if (!p) return;
    int prev = 0;
    hipGetDevice(&prev);
    if (p->device >= 0) hipSetDevice(p->device);
    if (p->exec) hipGraphExecDestroy(p->exec);
    if (p->graph) hipGraphDestroy(p->graph);
    for (auto e : p->events) hipEventDestroy(e);
    for (auto s : p->streams) hipStreamDestroy(s);
    if (p->dmem) {
        hipDeviceSynchronize();
        hipFree(p->dmem);
    }
    hipSetDevice(prev);
    delete p;
}

// Records the work of one class on stream s.
int record_class(const DeviceTables* t, dct2d_ragged_plan* p, const ClassRec& c, hipStream_t s)
{
    if (!c.dense) {
        Job j{p->dir, nullptr, nullptr, c.count, c.rows, c.cols, 0, 0, s, 0};
        j.in_idx = j.out_idx = c.d_off;
        j.in_slot = j.out_slot = p->d_slot;
        j.shared = true; // the classes run as concurrent branches of the graph
        // long axes: float32 whatever the plan's precision (the split paths cover axes <= 256)
        if (c.long_axes) return launch_long(t, j);
        return dispatch(t, j, p->prec);
    }
    // dense image passes: base(indexed) <-> workspace(packed), ping-pong
    const int64_t n = (int64_t)c.rows * c.cols;
    const Addr to_ws{nullptr, c.ws, 0, n, c.d_off, nullptr, p->d_slot, nullptr};
    const Addr to_base{c.ws, nullptr, n, 0, nullptr, c.d_off, nullptr, p->d_slot};
    const Addr base_to_ws = to_ws, ws_to_base = to_base;
    int rc;
    switch (p->dir) {
    case DCT2D_FORWARD:
        rc = launch_dense_axis(base_to_ws, c.count, c.rows, c.cols, false, false, c.q_cols, s);
        if (rc) return rc;
        return launch_dense_axis(ws_to_base, c.count, c.rows, c.cols, true, false, c.q_rows, s);
    case DCT2D_INVERSE:
        rc = launch_dense_axis(base_to_ws, c.count, c.rows, c.cols, false, true, c.q_cols, s);
        if (rc) return rc;
        return launch_dense_axis(ws_to_base, c.count, c.rows, c.cols, true, true, c.q_rows, s);
    default:
        rc = launch_dense_axis(base_to_ws, c.count, c.rows, c.cols, false, false, c.q_cols, s);
        if (rc) return rc;
        rc = launch_dense_axis(ws_to_base, c.count, c.rows, c.cols, true, false, c.q_rows, s);
        if (rc) return rc;
        rc = launch_dense_axis(base_to_ws, c.count, c.rows, c.cols, true, true, c.q_rows, s);
        if (rc) return rc;
        return launch_dense_axis(ws_to_base, c.count, c.rows, c.cols, false, true, c.q_cols, s);
    }
}

} // namespace

extern "C" {

int dct2d_ragged_plan_create(const dct2d_block* blocks, int64_t count, int dir, int precision,
                             dct2d_ragged_plan** out_plan)
{
    if (!out_plan) return DCT2D_ERR_ARG;
    *out_plan = nullptr;
    if (count <= 0 || !blocks || dir < DCT2D_FORWARD || dir > DCT2D_ROUNDTRIP) return DCT2D_ERR_ARG;
    if (precision != DCT2D_FP32 && precision != DCT2D_AUTO && precision != DCT2D_SPLIT_BF16X6 &&
        precision != DCT2D_SPLIT_FP16X3)
        return DCT2D_ERR_PRECISION;
    // validate and group
    std::map<std::pair<int, int>, std::vector<int64_t>> groups;
    std::vector<std::pair<int64_t, int64_t>> spans;
    spans.reserve((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        const dct2d_block& b = blocks[i];
        if (b.rows < 8 || b.cols < 8 || b.rows > 1024 || b.cols > 1024) return DCT2D_ERR_SIZE;
        if (b.offset < 0 || (b.offset & 3)) return DCT2D_ERR_ALIGN;
        if ((b.cols & 3) != 0) return DCT2D_ERR_SIZE; // rows are read as 16-byte vectors
        groups[{b.rows, b.cols}].push_back(b.offset);
        spans.push_back({b.offset, b.offset + (int64_t)b.rows * b.cols});
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second) return DCT2D_ERR_ARG; // overlapping arrays
    for (auto& g : groups) {
        const bool fast = fast_shape(g.first.first, g.first.second);
        if (!fast && g.second.size() > 65535) return DCT2D_ERR_ARG;
        if (fast && precision != DCT2D_FP32 && precision != DCT2D_AUTO &&
            !mfma_supported(g.first.first, g.first.second, precision))
            return DCT2D_ERR_PRECISION;
    }
    int rc = DCT2D_OK;
    const DeviceTables* t = tables_current(&rc);
    if (!t) return rc;

    dct2d_ragged_plan* p = new dct2d_ragged_plan();
    p->dir = dir;
    p->prec = precision;
    p->items = count;
    hipGetDevice(&p->device);
    // device memory layout: slot | offsets per class | dense Q tables | workspaces
    size_t bytes = 256;
    std::map<int, size_t> qoff;
    for (auto& g : groups) bytes = align256(bytes + g.second.size() * sizeof(int64_t));
    for (auto& g : groups) {
        if (!dense_shape(g.first.first, g.first.second)) continue;
        for (int L : {g.first.first, g.first.second})
            if (!qoff.count(L)) {
                qoff[L] = bytes;
                bytes = align256(bytes + (size_t)L * L * 4);
            }
    }
    std::vector<size_t> wsoff;
    for (auto& g : groups) {
        if (!dense_shape(g.first.first, g.first.second)) {
            wsoff.push_back(0);
            continue;
        }
        wsoff.push_back(bytes);
        bytes = align256(bytes + g.second.size() * (size_t)g.first.first * g.first.second * 4);
    }
    if (hipMalloc(&p->dmem, bytes) != hipSuccess) {
        p->dmem = nullptr;
        release(p);
        return DCT2D_ERR_NOMEM;
    }
    char* base = static_cast<char*>(p->dmem);
    p->d_slot = reinterpret_cast<float**>(base);
    size_t off = 256;
    int gi = 0;
    for (auto& g : groups) {
        ClassRec c;
        c.rows = g.first.first;
        c.cols = g.first.second;
        c.count = (int64_t)g.second.size();
        c.d_off = reinterpret_cast<int64_t*>(base + off);
        off = align256(off + g.second.size() * sizeof(int64_t));
        if (hipMemcpy(c.d_off, g.second.data(), g.second.size() * sizeof(int64_t), hipMemcpyHostToDevice) !=
            hipSuccess) {
            release(p);
            return DCT2D_ERR_HIP;
        }
        c.long_axes = long_shape(c.rows, c.cols);
        if (dense_shape(c.rows, c.cols)) {
            c.dense = true;
            c.q_rows = reinterpret_cast<float*>(base + qoff[c.rows]);
            c.q_cols = reinterpret_cast<float*>(base + qoff[c.cols]);
            c.ws = reinterpret_cast<float*>(base + wsoff[gi]);
        }
        p->cls.push_back(c);
        ++gi;
    }
    for (auto& q : qoff)
        if (tables_dense_q(q.first, reinterpret_cast<float*>(base + q.second), nullptr) != DCT2D_OK) {
            release(p);
            return DCT2D_ERR_HIP;
        }
    float* null_base = nullptr;
    if (hipMemcpy(p->d_slot, &null_base, sizeof(float*), hipMemcpyHostToDevice) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        release(p);
        return DCT2D_ERR_HIP;
    }
    // record the graph: fork one branch per class from s0, join back
    const size_t ncls = p->cls.size();
    p->streams.resize(ncls + 1, nullptr);
    p->events.resize(ncls + 1, nullptr);
    for (size_t i = 0; i <= ncls; ++i) {
        if (hipStreamCreateWithFlags(&p->streams[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->events[i], hipEventDisableTiming) != hipSuccess) {
            release(p);
            return DCT2D_ERR_HIP;
        }
    }
    hipStream_t s0 = p->streams[0];
    if (hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        release(p);
        return DCT2D_ERR_HIP;
    }
    rc = hipEventRecord(p->events[0], s0) == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
    for (size_t i = 0; i < ncls && rc == DCT2D_OK; ++i) {
        hipStream_t si = p->streams[i + 1];
        if (hipStreamWaitEvent(si, p->events[0], 0) != hipSuccess) rc = DCT2D_ERR_HIP;
        if (rc == DCT2D_OK) rc = record_class(t, p, p->cls[i], si);
        if (rc == DCT2D_OK && hipEventRecord(p->events[i + 1], si) != hipSuccess) rc = DCT2D_ERR_HIP;
        if (rc == DCT2D_OK && hipStreamWaitEvent(s0, p->events[i + 1], 0) != hipSuccess) rc = DCT2D_ERR_HIP;
    }
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s0, &g);
    p->graph = g;
    if (rc != DCT2D_OK || ec != hipSuccess || !g) {
        release(p);
        return rc != DCT2D_OK ? rc : DCT2D_ERR_HIP;
    }
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess) {
        p->exec = nullptr;
        release(p);
        return DCT2D_ERR_HIP;
    }
    size_t nn = 0;
    hipGraphGetNodes(p->graph, nullptr, &nn);
    p->nodes = (int)nn;
    *out_plan = p;
    return DCT2D_OK;
}

int dct2d_ragged_execute(dct2d_ragged_plan* plan, float* base, void* stream)
{
    if (!plan || !base) return DCT2D_ERR_ARG;
    if ((reinterpret_cast<uintptr_t>(base) & 15u) != 0) return DCT2D_ERR_ALIGN;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(plan->mu);
    if (plan->bound != base) {
        // pageable source: the runtime stages the 8 bytes before returning
        if (hipMemcpyAsync(plan->d_slot, &base, sizeof(float*), hipMemcpyHostToDevice, s) != hipSuccess)
            return DCT2D_ERR_HIP;
        plan->bound = base;
    }
    return hipGraphLaunch(plan->exec, s) == hipSuccess ? DCT2D_OK : DCT2D_ERR_HIP;
}

void dct2d_ragged_plan_destroy(dct2d_ragged_plan* plan) { release(plan); }

int dct2d_ragged_plan_info(const dct2d_ragged_plan* plan, int64_t* items, int32_t* classes, int32_t* graph_nodes)
{
    if (!plan) return DCT2D_ERR_ARG;
    if (items) *items = plan->items;
    if (classes) *classes = (int32_t)plan->cls.size();
    if (graph_nodes) *graph_nodes = plan->nodes;
    return DCT2D_OK;
}

} // extern "C"
