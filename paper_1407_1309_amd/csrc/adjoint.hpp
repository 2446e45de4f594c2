// adjoint.hpp -- internal interface of the reverse-mode (adjoint) step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace mp {

template <typename T> struct AdjArgs {
    Geom g;
    int n_iters;
    unsigned opts;
    const T *psi0;
    const T *G;
    const T *c[3];
    int n_steps, ckpt_every;
    const T *lambda_T;
    T *grad_psi0;
    T *grad_c[3];
    char *ws;   // adjoint scratch (adj_extra_bytes)
    // Optional forward step psi_in -> psi_out without records (the caller's
    // fastest kernel for this configuration), used wherever the sweep only
    // needs states: the checkpointing pass and the segment recomputation.
    hipError_t (*plain_step)(void *ctx, const T *in, T *out) = nullptr;
    void *plain_ctx = nullptr;
};

size_t adj_extra_bytes(const Geom &g, size_t es, int n_iters, unsigned opts, int n_steps,
                       int ckpt_every);

template <typename T>
void adj_fill_args(AdjArgs<T> &a, const Geom &g, int n_iters, unsigned opts, const T *psi0,
                   const T *G, const T *const *c, int n_steps, int ckpt_every, const T *lambda_T,
                   T *grad_psi0, T **grad_c, char *ws)
{
    a.g = g;
    a.n_iters = n_iters;
    a.opts = opts;
    a.psi0 = psi0;
    a.G = G;
    for (int d = 0; d < 3; d++) {
        a.c[d] = c[d];
        a.grad_c[d] = grad_c[d];
    }
    a.n_steps = n_steps;
    a.ckpt_every = ckpt_every;
    a.lambda_T = lambda_T;
    a.grad_psi0 = grad_psi0;
    a.ws = ws;
}

template <typename T> hipError_t adjoint_run(const AdjArgs<T> &a, hipStream_t s);

}  // namespace mp
