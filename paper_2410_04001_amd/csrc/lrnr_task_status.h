// Status bits of a task's device-side Adam step counter (KTask::step), shared
// by the per-task reduction that sets them and the serving engine that reads
// them back.
#pragma once

namespace lrnr {

// The loss or gradient of the step after the counted ones was non-finite:
// s was left unchanged and the task is finished (the counter now exceeds any
// step limit, so every kernel skips the task).
constexpr int kTaskFailed = 1 << 30;

}  // namespace lrnr
