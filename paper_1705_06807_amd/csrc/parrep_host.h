// parrep_host.h -- host-side internals of libparrep shared by the C-ABI
// translation units: handles, validation, device descriptors, scratch, and
// the launch sequence of a batch.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "parrep_internal.h"

struct parrep_ctx {
    int device = 0;
    int n_cu = 256;  // compute units of the device
    std::mutex mu;
    double* logtab = nullptr;  // device copy of the -log(u) reduction table
    // Streams (default priority) on which the launch groups of a batch run
    // side by side; created on first use.
    std::vector<hipStream_t> aux;
    // Autotuned launch shapes: (replica-count bucket, species, reaction class)
    // -> (replicas per lane, waves, histogram staging: DevInst::stage_flush).
    std::map<std::tuple<int, int, int>, std::tuple<int, int, int>> tuned;
    // Device address of this device's fixed scratch array (parrep_solve_noalloc).
    char* noalloc_scratch = nullptr;
    double wall_hz = 1e8;  // rate of the device's constant wall clock
    int max_wide_groups = 0;  // co-resident workgroups of the wide kernel (0: not yet known)
};

struct parrep_net {
    parrep_ctx* ctx = nullptr;
    parrep::DevNet net{};
};

namespace parrep {

// Multi-run estimators: d_stats is a device array of n device pointers.
hipError_t launch_estimate(const double* const* d_stats, int n, int np, int ns, double window,
                           double* out, hipStream_t stream);

namespace host {

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
int set_device(parrep_ctx* ctx);

int validate_problem(const parrep_net* net, const parrep_problem* p, int64_t* nbins_out);
void fill_inst(DevInst& d, const parrep_net* net, const parrep_problem* p, int64_t nbins);
int check_result(const parrep_result* r);
void attach_result(DevInst& d, const parrep_result* r);

// Device memory of one batch: the descriptor array then per-instance scratch
// (propensity tables shared by equal (network, c, table length), outside-box
// accumulators, spill table, exchange and scan buffers).
// share_tables = false gives every instance a table of its own (plans, whose
// instances may later change their rate vector).
size_t arena_bytes(std::vector<DevInst>& insts, bool share_tables = true);
// Points insts[i]'s scratch into base (arena_bytes of device memory); the
// descriptors are then copied to base by the caller.
void place_arena(std::vector<DevInst>& insts, char* base, bool share_tables = true);

// Replica-count bucket used by the autotune table.
int shape_bucket(int R);
// Launch shape for an instance: in a sparse batch (no more instances than
// the device has CUs) the latency shape; else the autotuned one when there
// is one, else the library's default for R.
LaunchShape pick_shape(parrep_ctx* ctx, int R, int ns, int m, bool sparse);

// A batch after grouping: instances reordered so that each launch-shape
// group is contiguous, each group's instances by decreasing expected work
// (longest first, so the hardware's dispatch order fills the tail).
struct Group {
    LaunchShape shape;
    int first, count, tab_lds;
};
std::vector<Group> group_batch(parrep_ctx* ctx, std::vector<DevInst>& insts,
                               std::vector<int>* order, const LaunchShape* forced,
                               bool persist = false);

// Enqueue setup, zero, the group launches (side by side on the context's
// auxiliary streams, joined back into st), finalize.  d: device copy of the
// grouped descriptors.  Events ev_b/ev_a (optional) bracket the instance
// kernels on st.
// The fork/join events are appended to *keep when it is given (stream
// capture: they are destroyed after the capture ends), else destroyed once
// enqueued.
int enqueue_batch(parrep_ctx* ctx, DevInst* d, int n, const std::vector<Group>& groups,
                  int mode, uint32_t hook_cycle, int64_t hook_max_rounds, hipStream_t st,
                  hipEvent_t ev_b, hipEvent_t ev_a, std::vector<hipEvent_t>* keep = nullptr);

// How a single-instance solve may be spread over the workgroups of a
// cooperative launch (parrep_launch's fields).
struct WideReq {
    int workgroups = 0;  // 0 library choice (spread when R >= kWideMinR), 1 never, > 1 that many
    int rpl = 0;         // replicas per lane, 1 or 4 (0: 1)
    int s2 = 0, s3 = 0;  // chunk lengths in rounds (0: defaults)
    int wait_us = 0;     // longest wait at a grid barrier (0: 2 s)
    int persist = 0;     // 1: the persistent form of the groups' solve launches
};
// Rewrites the only group of a one-instance solve to the wide kernel when w
// asks for it or R is large, and sets the instance's wide fields (before
// the arena is laid out).  EINVAL when the request cannot hold R.
int apply_wide(parrep_ctx* ctx, std::vector<DevInst>& insts, std::vector<Group>& groups,
               const WideReq& w);

// Whole batch with a stream-ordered arena: allocate, upload, enqueue, free.
int run_batch(parrep_ctx* ctx, std::vector<DevInst>& insts, int mode, uint32_t hook_cycle,
              int64_t hook_max_rounds, hipStream_t st, hipEvent_t ev_b, hipEvent_t ev_a,
              const LaunchShape* forced, const WideReq* wide = nullptr);

}  // namespace host
}  // namespace parrep
