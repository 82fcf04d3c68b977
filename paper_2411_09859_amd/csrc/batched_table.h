// Panel width of the batched kernel per matrix order and persistent
// workgroups per CU per largest order of a batch, measured on MI355X by
// paper_2411_09859_amd/tune_batched.py (written by the tuner).
#pragma once
namespace skl {
struct BatchedTune { int n_max; int bs; int wgpc; };
constexpr BatchedTune kBatchedTune[] = {
    {32, 16, 4},
    {64, 16, 4},
    {96, 16, 4},
    {128, 16, 4},
    {160, 16, 4},
    {192, 16, 4},
    {224, 16, 4},
    {256, 16, 4},
};
}  // namespace skl
