// Structures shared by the persistent / batched kernels and the host driver.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_device.h"

namespace mf {
// Events that a timed launch records from its own dispatch (start and end
// of the kernel's execution); null = untimed.
struct KEv {
    hipEvent_t a = nullptr, b = nullptr;
};
}  // namespace mf

namespace mf {

// Grid barrier state: arrivals and the generation that waiting blocks poll
// sit on separate 128-byte lines.
struct GridBar {
    unsigned count;
    int pad0[31];
    unsigned gen;
    int abort;
    int pad1[30];
};

// A short list of breadth-first levels (passed by value to k_gr_slots).
struct LevelSet {
    int count;
    int lv[15];
};

struct PhaseParams {
    int sink, other;
    int64_t freq_num, freq_den, alpha, beta, round_charge, level_charge, max_rounds;
    int64_t dense_threshold, bu_factor;
    int hubdeg;
    int simple;              // rounds of the simple synchronous variant (RoundParams::simple)
    uint64_t limit_ticks;    // grid-barrier wait limit in wall-clock ticks
};

// One instance of a batch (device memory).
struct BatchItem {
    GraphView g;
    StateView st;          // st.ctl unused
    Ctl *ctl;              // [5]: [0] outputs, [1..3] round ring, [4] global relabel
    int32_t *flow;         // [slots] or null
    uint8_t *side;         // [n] or null (then st.touched is used as scratch)
    PhaseParams p;         // schedule; sink / other are set per phase
    int32_t G;             // lanes per vertex: 4, 8, 16 or 32
    int32_t preflow_only;
    // Served requests only (null in a batch): the graph as received, in
    // pinned coherent host memory (int64 offsets and reverse slots, int32
    // heads and capacities, each 256-byte aligned), which the block that
    // takes the request pulls into device memory and checks; and host
    // buffers that receive the sink side and the flow at the end.
    const int64_t *off64;
    const int64_t *rev64;
    const int32_t *head_h;
    const int32_t *cap_h;
    uint8_t *side_h;
    int32_t *flow_h;
};

struct BatchResult {
    int64_t value, cut, rounds, rounds2, grs, grs2, levels, pushes, relabels;
    int64_t t_start, t_end;          // wall-clock ticks
    int64_t t_solve;                 // served: when the pull and checks ended
    int64_t t_phase1;                // when the maximum preflow was reached
    int32_t status, block;
};

// Threads of a workgroup that solves one instance (batched and served forms,
// small graphs): 512 threads fit one workgroup per compute unit at the
// solver's register count and give each instance twice the lanes of 256.
constexpr int BATCH_BLOCK = 512;

struct BatchQueue {
    int32_t next;     // next position of `order` to hand out
    int32_t count;    // number of positions
};

// Served requests: queues in coherent host memory written by the host; `next`
// lives in device memory and is advanced by compare-and-swap.
constexpr int SERVE_CAP = 4096;          // queue slots (ring)

struct ServeHostQueue {                  // pinned, coherent host memory
    int32_t count;                       // items published (grows; slot = index % SERVE_CAP)
    int32_t shutdown;
    int32_t pad[14];
    BatchItem items[SERVE_CAP];
    BatchResult results[SERVE_CAP];
    int32_t done[SERVE_CAP];             // index + 1 when results[slot] holds that index's result
};

// next: device memory, [0] next index to claim, [4..7] mirror of the host
// queue (published count, shutdown, number of requests finished, epoch of the
// launch whose watcher has left); zeroed once when the queue is created and
// kept across launches.  epoch: 1, 2, ... per launch.
hipError_t launch_serve(int G, int grid, ServeHostQueue *hq, int32_t *next, uint64_t idle_ticks, int epoch,
                        hipStream_t s);
int serve_blocks_per_cu(int G);

hipError_t launch_phase(int G, int grid, GraphView g, StateView st, PhaseParams P, Ctl *ring, Ctl *gc,
                        GridBar *bar, hipStream_t s);
int phase_blocks_per_cu(int G);
hipError_t launch_batch(int G, int grid, const BatchItem *items, const int32_t *order, BatchResult *results,
                        BatchQueue *q, hipStream_t s);
void launch_queue_init(BatchQueue *q, int count, hipStream_t s);
int batch_blocks_per_cu(int G);

}  // namespace mf
