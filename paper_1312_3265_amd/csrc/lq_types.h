// Types shared by the host engine and the kernels.
#pragma once

#include <stdint.h>

namespace lq {

enum OpKind { OP_WILSON = 0, OP_SW_CORNERS = 1, OP_SW_OTF = 2, OP_WILSON_R = 3, OP_WILSON_EO = 4 };
enum Prec { P64 = 0, P32 = 1, P16 = 2 };

// Per-system solver state in device memory.  Written only by single-block
// "finish" kernels, by block 0 of the p-update kernel (into the ring entry of
// the next iteration parity), or by the host between steps; read by all.
struct SlotState {
  double rho[2];     // ||r_lo||^2 in storage units, ring indexed by iteration parity
  double bnorm2;     // ||b||^2, b = M^dag chi (FP64)
  double thr2;       // tol^2 * bnorm2
  double thr_lo2;    // thr2 / scale^2: the same target in storage units
  double scale;      // low-precision vectors hold (true value) / scale
  double scale_prev; // scale before the latest reliable update
  double mass;       // bare mass of this system
  double tol;
  double true_res2;  // ||b - A x_hi||^2 at the latest reliable update
  double iter_res2;  // ||r_lo||^2 * scale^2 at the latest iteration
  double rho_ru;     // ||r_lo||^2 right after the latest reliable update
  double rho_max;    // largest ||r_lo||^2 since the latest reliable update
  double delta2;     // request a reliable update once rho <= delta2 * rho_max (0: never)
  double alpha[4];   // alpha of the iterations of the current group of four (x is updated once per group)
  double bfull2;     // even-odd: ||M^dag chi||^2, the b of eq. (2) for the whole lattice
  double full_res2;  // even-odd: ||b - A x||^2 of eq. (2) at the latest reliable update
  double best2;      // smallest FP64 true residual^2 so far (stagnation watch)
  int32_t stop[2];   // ring: 1 = frozen until the next reliable update
  int32_t status;    // 0 empty, 1 running, 2 converged, 3 failed
  int32_t iter;      // CG iterations done
  int32_t ru;        // reliable updates done
  int32_t cand;      // reliable updates since the iterated residual met tol
  int32_t maxiter;
  int32_t flags;     // bit0 breakdown, bit1 maxiter reached, bit2 stagnation
  int32_t apps;      // applications of A (iterations + reliable updates + setup)
  int32_t ru_iter;   // iteration count at the latest reliable update
  int32_t want_ru;   // frozen because the residual dropped by delta (not converged)
  int32_t pend;      // terms alpha[j] * p_ring[j], j < pend, that x still lacks (frozen mid-group)
  int32_t stall;     // reliable updates since the true residual last halved
  int32_t grown;     // reliable updates in a row with the true residual 100x above its best
};

enum SlotStatus { SLOT_EMPTY = 0, SLOT_RUNNING = 1, SLOT_DONE = 2, SLOT_FAILED = 3 };

// A reliable update acts on slot k only when mask[k] != 0 (host-chosen per
// slot from that slot's own state), so a system's trajectory does not depend
// on which other systems share the batch.
__host__ __device__ inline bool ru_selected(const SlotState* st, const int* mask, int k) {
  return st[k].status == SLOT_RUNNING && (mask == nullptr || mask[k] != 0);
}

}  // namespace lq
