// Continuous batches on a plan: the interface between the solver driver
// (kp_solver.hip) and the request server (kp_server.cpp).  Plain C++.
#pragma once

#include "kp_state.h"

struct kp_plan;

namespace kp {

// Continuous batch on a plan (kp_solver.hip; used by the request server):
// slots_open binds max_batch slots of eta and u (device) and empties them;
// slots_mark sets a slot JOINING (its eta is staged) or CAPPED; slots_step
// enqueues one step of `iters` iterations (1..8; slots join only at a step's
// start, and no slot may pass its iteration cap inside one) over the first
// `nslots` slots (every busy slot among them; 0: all); slots_wait
// synchronises and returns the host mirror of the slots' states (null on a
// HIP error).
int slots_open(kp_plan* p, const double* eta, double* u, double tol, int flags);
int slots_mark(kp_plan* p, int slot, int code);
int slots_step(kp_plan* p, int iters = 1, int nslots = 0);
const RhsState* slots_wait(kp_plan* p);
void slots_close(kp_plan* p);

}  // namespace kp
