// Panel width of the batched kernel per matrix order, measured on MI355X
// by paper_2411_09859_amd/tune_batched.py (written by the tuner).
#pragma once
namespace skl {
struct BatchedTune { int n_max; int bs; };
constexpr BatchedTune kBatchedTune[] = {
    {32, 32},
    {64, 24},
    {96, 20},
    {128, 16},
    {160, 24},
    {192, 32},
    {224, 32},
    {256, 32},
};
}  // namespace skl
