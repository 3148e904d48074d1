// One precision's instantiations of the evaluation kernel: this file is
// compiled once per precision with -DHOBO_EVAL_PREC=<Prec value>.
#include "eval_kernel.h"

#ifndef HOBO_EVAL_PREC
#error "compile with -DHOBO_EVAL_PREC=<precision>"
#endif

namespace hobo {

template <>
int dispatch_eval_prec<HOBO_EVAL_PREC>(const EvalParams& ep, int mode, int rt, int ct, long long B, hipStream_t st) {
  return mode == M_FIELDS ? dispatch_eval_shape<HOBO_EVAL_PREC, M_FIELDS>(ep, rt, ct, B, st)
                          : dispatch_eval_shape<HOBO_EVAL_PREC, M_ENERGY>(ep, rt, ct, B, st);
}

}  // namespace hobo
