// The plain-atomic backward composite (a6) compiled with LLVM's atomic optimizer
// (DPP strategy), an ablation beside the hand-written reduction: the compiler
// turns each atomic add whose address is the same in every lane into a
// reduction over the active lanes and one lane's add, nine such reductions
// per visited entry. Built from the same source as k_composite.hip; only the
// compiler flag differs (the build gives this file
// -amdgpu-atomic-optimizer-strategy=DPP instead of None).
#define GSR_COMPOSITE_COMPILER_REDUCE 1
#include "k_composite.hip"
