// Storage for the emulated HIP built-ins (see hip_emu.h).
#include "hip_emu.h"
thread_local uint3_ threadIdx;
thread_local uint3_ blockIdx;
thread_local dim3 blockDim, gridDim;
thread_local emu::Block* emu::g_block = nullptr;
thread_local emu::CoopRun* emu::g_coop = nullptr;
