// Panel width of the batched kernel per matrix order, measured on MI355X
// by paper_2411_09859_amd/tune_batched.py (written by the tuner).
#pragma once
namespace skl {
struct BatchedTune { int n_max; int bs; };
constexpr BatchedTune kBatchedTune[] = {
    {32, 16},
    {64, 16},
    {96, 16},
    {128, 16},
    {160, 16},
    {192, 16},
    {224, 16},
    {256, 16},
};
}  // namespace skl
