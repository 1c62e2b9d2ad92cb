#include "schedule.hpp"

namespace expint {

void classify_term(TermOp& op) {
  op.flavor = kGeneric;
  if (op.u || op.bsrc2) return;
  if (!op.bsrc && !op.acc_in && !op.acc_out && op.y_out) {
    op.flavor = kSkip;
  } else if (!op.bsrc && op.acc_in && op.ca == 1.0 && op.acc_out) {
    op.flavor = op.y_out ? kFlushY : kFlushNoY;
  } else if (op.bsrc && !op.acc_in && op.acc_out && op.y_out) {
    op.flavor = kFirst;
  }
}

std::vector<TermOp> phi1_schedule(const StepBuffers& ws, int s, int m, double tau, const void* b, void* x_out,
                                  void* u, const void* d) {
  enum class X { Zero, HB, Buf };
  std::vector<TermOp> ops;
  const double h = tau / s;
  X xk = X::Zero;  // what x (the state entering the sub-step) is: 0, h*b, or ws.acc[xa]
  int xa = 0;
  for (int sig = 1; sig <= s; ++sig) {
    const int out = (xk == X::Buf) ? 1 - xa : 0;
    void* A = ws.acc[out];  // running sum of this sub-step
    int ycur = 0;           // buffer with y_{j-1}
    bool pend = false;      // y_{j-1} not yet in the running sum
    bool pend_hb = false;   // the sum has not been started: it still lacks h*b
    int j0;
    if (xk == X::Zero) {
      if (m == 1) {  // x_1 = h b: no sweep
        xk = X::HB;
        continue;
      }
      // y_1 = h b is not stored (eta = (0, 1): no d yet); y_2 = (h/2) A (h b),
      // plus (h^2 / (2 tau)) d
      TermOp t;
      t.src = b;
      t.c = h * h / 2.0;
      if (d) {
        t.bsrc2 = d;
        t.cb2 = h * h / (2.0 * tau);
      }
      if (m == 2) {
        t.acc_out = A;
        t.cs = h;  // h b + y_2
        ops.push_back(t);
        xk = X::Buf;
        xa = out;
        continue;
      }
      t.y_out = ws.y[0];
      ops.push_back(t);
      pend = true;
      pend_hb = true;
      j0 = 3;
    } else {
      // y_1 = h (A x + b) (+ h (k h / tau) d in sub-step k + 1), sum = x + y_1
      TermOp t;
      t.src = (xk == X::HB) ? b : ws.acc[xa];
      t.bsrc = b;
      t.c = (xk == X::HB) ? h * h : h;  // x = h b: h A (h b)
      t.cb = h;
      if (d) {
        t.bsrc2 = d;
        t.cb2 = h * (sig - 1) * h / tau;
      }
      t.cs = (xk == X::HB) ? h : 1.0;
      t.acc_out = A;
      t.y_out = m >= 2 ? ws.y[0] : nullptr;
      ops.push_back(t);
      j0 = 2;
    }
    for (int j = j0; j <= m; ++j) {
      // y_j = (h/j) A y_{j-1}; add to the sum in pairs (y_{j-1} is the source
      // already in registers), or alone for the last term
      TermOp t;
      t.src = ws.y[ycur];
      t.c = h / j;
      if (d && j == 2) {  // y_2 = (h/2) A y_1 + (h^2 / (2 tau)) d
        t.bsrc2 = d;
        t.cb2 = h * h / (2.0 * tau);
      }
      const bool last = j == m;
      if (pend || last) {
        if (pend_hb) {
          t.acc_in = b;
          t.ca = h;
        } else {
          t.acc_in = A;
          t.ca = 1.0;
        }
        t.cs = pend ? 1.0 : 0.0;
        t.acc_out = A;
        pend = false;
        pend_hb = false;
      } else {
        pend = true;
      }
      t.y_out = last ? nullptr : ws.y[1 - ycur];
      ycur = 1 - ycur;
      ops.push_back(t);
    }
    xk = X::Buf;
    xa = out;
  }
  if (ops.empty()) {  // s == m == 1: x = tau b
    TermOp t;
    t.src = b;
    t.cs = h;
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
  for (TermOp& t : ops) classify_term(t);
  return ops;
}

std::vector<TermOp> phi1_schedule_pairs(const StepBuffers& ws, int s, int m, double tau, const void* b,
                                        void* x_out, void* u) {
  std::vector<TermOp> ops;
  if (m < 2) return ops;
  const double h = tau / s;
  int xa = -1;  // the sub-step's start state x: -1 for x = 0, else ws.acc[xa]
  for (int sig = 1; sig <= s; ++sig) {
    const int out = xa < 0 ? 0 : 1 - xa;
    void* A = ws.acc[out];  // running sum of this sub-step
    int ycur = -1;          // ws.y[ycur] holds the term the next sweep starts from
    bool first = true;
    for (int j = xa < 0 ? 2 : 1; j <= m;) {
      TermOp t;
      if (first && xa < 0) {
        // y_1 = h b is never stored: term 2 is (h^2/2) A b, the sum starts at h b
        t.src = b;
        t.c = h * h / 2.0;
        t.cs = h;
      } else if (first) {
        // y_1 = h (A x + b), the sum starts at x
        t.src = ws.acc[xa];
        t.bsrc = b;
        t.c = h;
        t.cb = h;
        t.cs = 1.0;
      } else {
        t.src = ws.y[ycur];
        t.c = h / j;
        t.acc_in = A;
        t.ca = 1.0;
      }
      const bool two = j < m;
      if (two) {
        t.pair = 1;
        t.c2 = h / (j + 1);
      }
      t.acc_out = A;
      const int next = j + (two ? 2 : 1);
      if (next <= m) {
        ycur = ycur == 0 ? 1 : 0;
        t.y_out = ws.y[ycur];
      }
      ops.push_back(t);
      first = false;
      j = next;
    }
    xa = out;
  }
  TermOp& last = ops.back();
  last.y_out = nullptr;
  if (u) {
    last.u = u;
    last.acc_out = nullptr;
  } else {
    last.acc_out = x_out;
  }
  for (TermOp& t : ops)
    if (!t.pair) classify_term(t);
  return ops;
}

void set_linearised(std::vector<TermOp>& ops, const void* un, double rho) {
  for (TermOp& t : ops) {
    t.ju = un;
    t.jrho = rho;
  }
}

}  // namespace expint
