// Storage for the emulated HIP built-ins (see hip_emu.h).
#include "hip_emu.h"
thread_local uint3_ threadIdx;
thread_local uint3_ blockIdx;
dim3 blockDim, gridDim;
emu::Block* emu::g_block = nullptr;
