// Panel width of the single-matrix factorization per matrix order,
// measured on MI355X by paper_2411_09859_amd/tune_factor.py (written by
// the tuner): the first entry whose n_max is at least the order applies.
#pragma once
namespace skl {
struct FactorTune { int n_max; int b; };
constexpr FactorTune kFactorTune[] = {
    {362, 128},
    {724, 256},
    {1448, 256},
    {2896, 256},
    {5792, 256},
    {11585, 256},
    {1073741824, 256},
};
}  // namespace skl
