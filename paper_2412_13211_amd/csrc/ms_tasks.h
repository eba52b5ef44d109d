// ms_tasks.h -- launch interface of the subtask predicate / event kernels.
#pragma once
#include "../../include/ms_phys.h"
#include "ms_internal.h"

// the Python binding mirrors these layouts
static_assert(sizeof(ms_task) == 24, "ms_task layout");
static_assert(sizeof(ms_episode) == 72, "ms_episode layout");
static_assert(sizeof(ms_task_robot) == 136, "ms_task_robot layout");

namespace msk {

struct TaskArgs {
  const DModel* models;
  const DScene* scenes;
  const DAux* aux;
  const float* x;            // state
  const ms_task* tasks;      // [S]
  const float* robot_force;  // [S] (null: start of the episodes)
  const float* grip;         // [NF + NA][2] or null
  const uint8_t* mask;       // start: scenes to start (null: all)
  ms_episode* ep;            // [S]
  float* pred;               // [S][8] or null
  ms_task_robot robot;
  int S, NF, n_sub;
};

void launch_task_eval(const TaskArgs& a, hipStream_t st);
void launch_task_categorize(const ms_task* tasks, const ms_episode* ep, int32_t* mode, int S, hipStream_t st);

}  // namespace msk
