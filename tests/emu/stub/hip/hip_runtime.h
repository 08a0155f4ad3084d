// Empty stand-in: the CPU emulation declarations come from hip_emu.h,
// which the emulator build force-includes.
#pragma once
