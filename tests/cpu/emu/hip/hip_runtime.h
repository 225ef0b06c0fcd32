// CPU emulation of the few HIP device facilities that the workgroup FFT
// (paper_2511_02700_amd/csrc/fft.hpp) uses, for tests/cpu/fft_emu.cpp only:
// one OS thread per GPU thread of one workgroup, threadIdx.x a thread-local
// index, __syncthreads() a barrier over the workgroup's threads.  Test
// infrastructure: never part of the library build.
#pragma once

#include <barrier>

#define __device__
#define __host__
#define __forceinline__ inline

struct double2 { double x, y; };
struct float2 { float x, y; };
inline double2 make_double2(double x, double y) { return double2{x, y}; }
inline float2 make_float2(float x, float y) { return float2{x, y}; }

struct EmuThreadIdx { unsigned x; };
inline thread_local EmuThreadIdx threadIdx{0};

// the barrier of the workgroup being emulated (set before its threads start)
inline std::barrier<>* emu_block_barrier = nullptr;
inline void __syncthreads() { emu_block_barrier->arrive_and_wait(); }
// instruction-scheduling fence of the GPU compiler: nothing to do on the host
inline void __builtin_amdgcn_sched_barrier(int) {}
