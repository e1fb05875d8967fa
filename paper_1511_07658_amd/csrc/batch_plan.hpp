// Schedule of one grouped batch on the manager's four streams, as a list of
// stream operations (host logic only, no HIP calls).  The HIP device walks the
// list eagerly, or inside a stream capture to build the batch's graph; a CPU
// test replays it against the dependency rules of streams and events and the
// capture rules (every stream forked into a capture joins its origin again).
//
// Streams: compute streams C0 and C1 carry the grouped launches (dealt round
// robin) and the small "local" copies of their own requests; H2D and D2H are
// the copy FIFOs, one per direction, in the role of the execution model's
// copy engines (Section 4.2.3).  C0 is the capture origin.
#pragma once

#include <cstdint>
#include <vector>

namespace gvm {

enum PlanStream : int { kPlanC0 = 0, kPlanC1 = 1, kPlanH2D = 2, kPlanD2H = 3, kPlanStreams = 4 };

enum PlanOpKind : int {
  kOpRecord = 0,   // record event `ev` on `stream`
  kOpWait = 1,     // `stream` waits for event `ev`
  kOpCopyIn = 2,   // whole copy-in of job `job` on `stream`
  kOpCopyOut = 3,  // copy-out of job `job` on `stream`
  kOpLaunch = 4,   // grouped launch of group `group` on `stream`; with ev >= 0,
                   // event `ev` is recorded right after it (end of that stream's kernels)
  kOpDone = 5,     // completion of job `job`: ev >= 0 names an event already
                   // recorded; otherwise a new one is recorded on `stream`
};

struct PlanOp {
  int kind;
  int stream;
  int ev;
  int job;
  int group;
};

// What the schedule needs to know of one request.
struct PlanJob {
  int kernel_id;
  uint64_t n;
  bool copy_in;
  bool copy_out;
  bool local;       // copies small enough to stay on the kernel's own stream
  bool pieces;      // input already queued piecewise on the H2D FIFO before the batch
  bool out_pieces;  // output leaves piecewise on the D2H FIFO, an event after each piece
};

// One grouped launch: requests of one kernel id, at most kPlanMaxGroup of
// them, SGEMM sizes from the largest down.  The launches come longest first
// (estimated device time), dealt round robin.
struct PlanGroup {
  int kernel_id;
  int stream;               // index into the stream list the groups are dealt to
  std::vector<int> jobs;    // indices into the job list, in launch order
};

constexpr int kPlanMaxGroup = 32;

// Eager batch: everything is in `ops`.  Graph batch: `pre` runs eagerly
// before the graph is launched on C0, `ops` is what the graph holds (captured
// once, replayed after), and `post` runs eagerly after the launch.  Event ids
// are shared by the three lists.
struct BatchPlan {
  std::vector<PlanOp> pre;
  std::vector<PlanOp> ops;
  std::vector<PlanOp> post;
  std::vector<PlanGroup> groups;
  std::vector<int> stream_of;  // per job: the compute stream of its kernel
  int events = 0;              // event ids 0 .. events-1
};

// The grouped launches of `jobs` dealt round robin over `nstreams` streams
// (one group per kernel id, split every kPlanMaxGroup requests).
// `longest_first` false: shortest first instead.
std::vector<PlanGroup> plan_groups(const std::vector<PlanJob>& jobs, int nstreams, bool longest_first = true);

// Grouped policy: copy-ins (local ones on C0 ahead of its kernels, the rest
// on the H2D FIFO), the grouped launches on C0 and C1 after the inputs they
// read, copy-outs (local ones on the launch's own stream, the rest on the
// D2H FIFO after the launch that computed them) and one completion per job.
// With `graph`: the graph forks from C0 into the other three streams and
// every one of them joins C0 again after its last operation.  Piecewise
// copies stay outside the graph, since the host stages them piece by piece:
// before the launch C0 waits for the H2D FIFO that holds the input pieces,
// and after it the output pieces leave on the D2H FIFO.  The completions
// follow the launch.
// `compute_streams` 1: every launch on C0, one after another, in the order
// `longest_first` gives.
BatchPlan plan_grouped(const std::vector<PlanJob>& jobs, bool graph, int compute_streams = 2,
                       bool longest_first = true);

}  // namespace gvm
