#include "schedule.hpp"

namespace expint {

std::vector<TermOp> phi1_schedule(const StepBuffers& ws, int s, int m, double tau, const void* b, void* x_out,
                                  void* u) {
  enum class X { Zero, HB, Buf };
  std::vector<TermOp> ops;
  const double h = tau / s;
  X xk = X::Zero;
  int xa = 0;  // acc buffer holding x when xk == Buf
  for (int sig = 1; sig <= s; ++sig) {
    TermOp op{};
    int j_next;  // first term index handled by the generic loop below
    if (xk == X::Zero) {
      if (m == 1) {  // x_1 = h b: no sweep
        xk = X::HB;
        continue;
      }
      op.src = b;  // y_2 = (h/2) A (h b)
      op.c = h * h / 2.0;
      op.alpha = h;  // sum starts at y_1 = h b
      j_next = 3;
    } else if (xk == X::HB) {
      op.src = b;  // y_1 = h (A (h b) + b)
      op.bsrc = b;
      op.c = h * h;
      op.cb = h;
      op.alpha = h;  // sum starts at x = h b
      j_next = 2;
    } else {
      op.src = ws.acc[xa];  // y_1 = h (A x + b)
      op.bsrc = b;
      op.c = h;
      op.cb = h;
      op.alpha = 1.0;  // sum starts at x
      j_next = 2;
    }
    const int out = (xk == X::Buf) ? 1 - xa : 0;
    op.acc_out = ws.acc[out];
    int ycur = 0;
    op.y_out = j_next <= m ? ws.y[0] : nullptr;
    ops.push_back(op);
    for (int j = j_next; j <= m; ++j) {
      TermOp t{};
      t.src = ws.y[ycur];
      t.c = h / j;
      t.acc_in = ws.acc[out];
      t.acc_out = ws.acc[out];
      t.y_out = j < m ? ws.y[1 - ycur] : nullptr;
      ycur = 1 - ycur;
      ops.push_back(t);
    }
    xk = X::Buf;
    xa = out;
  }
  if (ops.empty()) {  // s == m == 1: x = tau b
    TermOp t{};
    t.src = b;
    t.c = 0.0;
    t.alpha = h;
    ops.push_back(t);
  }
  TermOp& last = ops.back();
  last.y_out = nullptr;
  if (u) {
    last.u = u;
    last.acc_out = nullptr;
  } else {
    last.acc_out = x_out;
  }
  return ops;
}

}  // namespace expint
