// Host-side construction of the tile DAG and of the ticket order the
// persistent device scheduler follows.
#pragma once
#include <stdint.h>

#include <vector>

#include "tq_sched.h"

// Fills the geometry fields of a descriptor (pointers untouched); p: number
// of row domains of the reduction tree (1: flat tree; clamped to [1, MT]).
void md_init(MatDesc &md, int64_t M, int64_t N, int nb, int ib, int w, int64_t nrhs, int p = 1);

// Rows of step k: the heads (GEQRT), the other rows (TSQRT), and the bottom
// heads of the merges in level order (TTQRT).
void tree_step(const MatDesc &md, int k, std::vector<int> &heads, std::vector<int> &rest,
               std::vector<int> &bottoms);

// Tasks of one matrix in the sequential program order of the tile algorithm
// (step k ascending; within a step the GEQRTs, the TSQRTs with i ascending,
// the merges in level order, then the LARFBs, SSRFBs and TTMQRs in the same
// row orders). This order is a topological order of the DAG.
void enum_factor_tasks(const MatDesc &md, int mat, std::vector<Task> &out);
void enum_apply_tasks(const MatDesc &md, int mat, std::vector<Task> &out);  // reversed if md.notrans

// Counts of GEQRT / TSQRT / LARFB / SSRFB tile tasks (strips not split).
void dag_tile_counts(int64_t M, int64_t N, int nb, int64_t counts[4]);

// Cost estimate (arbitrary time units) of one task, used only to order tasks.
double task_cost(const Task &t, const MatDesc &m);

// Builds the ticket order for the union of the matrices' DAGs: list
// scheduling on `workers` identical workers, ready tasks taken by largest
// bottom level (longest cost path to the end). The order is the order of
// start times, hence topological. Returns 0, or a negative code if the
// dependency protocol and the program order disagree (a bug).
int build_order(const std::vector<MatDesc> &mats, bool apply, int workers,
                std::vector<Task> &order, int64_t *counter_total);

// Replays `order` one task at a time with the counter protocol and checks
// that every wait is already satisfied when its turn comes (so the order can
// never block a scheduler whose workers take tickets in order). Returns the
// number of violations.
int64_t check_order_sequential(const std::vector<MatDesc> &mats, const std::vector<Task> &order);

// Randomised parallel replay: `workers` workers take tickets in order, wait
// on the counters like the device does, and run for random durations. Every
// pair of tasks that touch the same tile data (one of them writing) must run
// in the program order, without overlap. Returns the number of violations, or
// -1 on a deadlock.
int64_t stress_order(const std::vector<MatDesc> &mats, bool apply,
                     const std::vector<Task> &order, int workers, uint64_t seed);
