// Device interval core for gfx950: outward-rounded FP64 interval arithmetic
// with one hardware rounding mode per kernel.
//
// Representation.  An interval [lo, hi] is held as the pair (nlo, hi) with
// nlo = -lo.  Every kernel switches the wave's FP64 rounding mode to "toward
// +infinity" once, at entry; from then on every FP64 add and multiply the
// compiler emits rounds up.  The lower endpoint is obtained through
// RD(x) = -RU(-x): with nlo stored, a rounded-down lower bound is simply a
// rounded-up operation on negated operands, and the negations live in the data
// (negated coefficients, negated box endpoints), never in the instruction
// stream.
//
// Why inline asm for the mode switch.  The AMDGPU backend assumes round-to-
// nearest for every FP64 instruction and re-inserts a mode reset in front of
// them after a visible s_setreg; it also folds -((-x)*y) into x*y, which is
// only valid under round-to-nearest.  Writing the MODE register from inline
// asm hides the switch from that bookkeeping, and keeping negations out of the
// arithmetic (or behind `opaque`) leaves no fold that depends on the mode.
// Kernels must therefore (1) call `round_up_mode()` before any FP64 arithmetic,
// (2) never feed a negated value into a multiply or add without `opaque`,
// (3) be compiled with -ffp-contract=off (no fused multiply-add anywhere).
//
// Interval rules (Sec. 3.2 of Moroz, arXiv 2406.09857, names interval
// arithmetic and gives the sum; the product is the textbook min/max rule):
//   [a,b] + [c,d] = [RD(a+c), RU(b+d)]
//   [a,b] * [c,d] = [RD(min P), RU(max P)],  P = {ac, ad, bc, bd}.
// RD/RU are monotone, so RD(min P) = min RD(P): every formula below that picks
// a subset of P known to contain the extremum gives the same bits (up to the
// sign of a zero).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vx {

// Switch this wave's FP64 rounding mode to round-toward-+infinity
// (MODE.FP_ROUND bits [3:2] = 1).  The "memory" clobber keeps loads after it.
__device__ __forceinline__ void round_up_mode() {
  asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 1" ::: "memory");
}

// Hide a value's provenance from the optimizer (no instruction emitted).
__device__ __forceinline__ double opaque(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Sign class of a box interval on one axis.
enum : int { CLS_POS = 0, CLS_NEG = 1, CLS_STRADDLE = 2 };

// Grid cell enclosure on one axis (round-up mode must be active).
// Cell `label` of the 2^level grid on [dlo, dhi] is
//   [RD(dlo + RD(label * RD(dhi-dlo)) 2^-level), RU(dlo + RU((label+1) * RU(dhi-dlo)) 2^-level)].
// Returned as nlo = -lo and hi.  On dyadic domains such as [-1,1] both are exact.
// With centre = 1 the "cell" is the degenerate box of the cell's centre, the
// common endpoint of cells 2*label and 2*label+1 at level+1: its lower bound is
// the lower end of cell 2*label+1, its upper bound the upper end of cell
// 2*label (the centre enclosures of the Taylor forms).  With centre = 2 it is
// grid vertex `label` (0 .. 2^level), the common endpoint of cells label-1 and
// label: the lower end of cell label and the upper end of cell label-1 (the
// vertex enclosures of the inclusion criterion).
struct AxisGrid {
  double dlo, ndlo, dhi, ndhi;  // domain endpoints and their negations (host-negated)
  int level;
  int centre;                   // 0: cells, 1: cell centres, 2: grid vertices
};

__device__ __forceinline__ void cell(const AxisGrid& g, int32_t label, double& nlo, double& hi) {
  const double wu = g.dhi + g.ndlo;   // RU(dhi - dlo)
  const double nw = g.dlo + g.ndhi;   // RU(dlo - dhi) = -RD(dhi - dlo)
  const int sh = g.centre == 1 ? 1 : 0;  // centres are vertices of level + 1
  const int64_t base = (int64_t)label << sh;
  const int64_t a = base + (g.centre == 1 ? 1 : 0);  // lower end: of cell a
  const int64_t b = base + (g.centre == 2 ? 0 : 1);  // upper end: of cell b - 1
  nlo = g.ndlo + ldexp((double)a * nw, -(g.level + sh));
  hi = g.dlo + ldexp((double)b * wu, -(g.level + sh));
}

__device__ __forceinline__ int cell_class(double nlo, double hi) {
  // lo >= 0  <=>  nlo <= 0 ;  hi <= 0
  return nlo <= 0.0 ? CLS_POS : (hi <= 0.0 ? CLS_NEG : CLS_STRADDLE);
}

// Multiplier operands of a cell for its class.
//   POS (0 <= a <= b):  u = a,  v = b
//   NEG (a <= b <= 0):  u = -a, v = -b      (both >= 0)
//   STRADDLE:           a, b, na = -a, nb = -b
struct CellOps { double u, v, nu, nv; };

__device__ __forceinline__ CellOps cell_ops(double nlo, double hi, int cls) {
  CellOps o;
  if (cls == CLS_NEG) { o.u = nlo; o.v = opaque(-hi); o.nu = 0; o.nv = 0; }
  else { o.u = opaque(-nlo); o.v = hi; o.nu = nlo; o.nv = opaque(-hi); }
  return o;
}

// One Horner step J <- J*I + C for a cell of class POS: I = [u, v], u >= 0.
//   lo' = min(lo*u, lo*v)  ->  nlo' = max(RU(nlo*u), RU(nlo*v))
//   hi' = max(hi*u, hi*v)
__device__ __forceinline__ void step_pos(double& nlo, double& hi, double u, double v, double cn, double ch) {
  const double a = fmax(nlo * u, nlo * v);
  const double b = fmax(hi * u, hi * v);
  nlo = a + cn;
  hi = b + ch;
}

// Class NEG: I = [a, b] <= 0 with u = -a, v = -b:
//   lo' = min(hi*a, hi*b)  ->  nlo' = max(RU(hi*u), RU(hi*v))
//   hi' = max(lo*a, lo*b)  ->  hi'  = max(RU(nlo*u), RU(nlo*v))
__device__ __forceinline__ void step_neg(double& nlo, double& hi, double u, double v, double cn, double ch) {
  const double a = fmax(hi * u, hi * v);
  const double b = fmax(nlo * u, nlo * v);
  nlo = a + cn;
  hi = b + ch;
}

// General product (any signs): I = [a, b], na = -a, nb = -b.
//   nlo' = max RU(-p) over p in P = max(nlo*a, nlo*b, hi*na, hi*nb)
//   hi'  = max RU(p)               = max(nlo*na, nlo*nb, hi*a, hi*b)
__device__ __forceinline__ void step_gen(double& nlo, double& hi, const CellOps& o, double cn, double ch) {
  const double a = fmax(fmax(nlo * o.u, nlo * o.v), fmax(hi * o.nu, hi * o.nv));
  const double b = fmax(fmax(nlo * o.nu, nlo * o.nv), fmax(hi * o.u, hi * o.v));
  nlo = a + cn;
  hi = b + ch;
}

}  // namespace vx
