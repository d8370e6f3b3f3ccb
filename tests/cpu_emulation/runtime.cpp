// Globals of the emulated HIP runtime (hip/hip_runtime.h in this folder) and its fiber switch.
#include "hip/hip_runtime.h"

dim3 threadIdx, blockIdx, blockDim, gridDim;
EmuBlock *emu_block = nullptr;
void (*emu_after_launch)(const void *) = nullptr;

// Fiber switch (x86-64 System V): push the callee-saved registers, save the stack pointer to
// *save_sp, load next_sp, pop the same registers and return into the other fiber.
asm(R"(
    .text
    .globl emu_ctx_switch
    .type emu_ctx_switch, @function
emu_ctx_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_ctx_switch, .-emu_ctx_switch
)");
