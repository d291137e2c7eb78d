// Gate matrices from their definitions (q[0] is the most significant bit).
#include <cmath>

#include "internal.h"

namespace hsf {

namespace {
const cd I1(0.0, 1.0);

void set(std::vector<cd>& m, int d, std::initializer_list<cd> v) {
    m.assign(v.begin(), v.end());
    (void)d;
}
}  // namespace

bool gate_matrix(int kind, int nq, double t, const double* em, std::vector<cd>& m) {
    const double c = std::cos(0.5 * t), s = std::sin(0.5 * t);
    const double r2 = 1.0 / std::sqrt(2.0);
    switch (kind) {
        case HSF_GATE_U: {
            const int d = 1 << nq;
            m.resize((size_t)d * d);
            for (int i = 0; i < d * d; ++i) m[i] = cd(em[2 * i], em[2 * i + 1]);
            return true;
        }
        case HSF_GATE_H: set(m, 2, {r2, r2, r2, -r2}); return true;
        case HSF_GATE_X: set(m, 2, {0, 1, 1, 0}); return true;
        case HSF_GATE_Y: set(m, 2, {0, -I1, I1, 0}); return true;
        case HSF_GATE_Z: set(m, 2, {1, 0, 0, -1}); return true;
        case HSF_GATE_S: set(m, 2, {1, 0, 0, I1}); return true;
        case HSF_GATE_SDG: set(m, 2, {1, 0, 0, -I1}); return true;
        case HSF_GATE_T: set(m, 2, {1, 0, 0, std::polar(1.0, M_PI / 4)}); return true;
        case HSF_GATE_TDG: set(m, 2, {1, 0, 0, std::polar(1.0, -M_PI / 4)}); return true;
        // exp(-i t P / 2) = cos(t/2) 1 - i sin(t/2) P
        case HSF_GATE_RX: set(m, 2, {c, -I1 * s, -I1 * s, c}); return true;
        case HSF_GATE_RY: set(m, 2, {c, -s, s, c}); return true;
        case HSF_GATE_RZ: set(m, 2, {cd(c, -s), 0, 0, cd(c, s)}); return true;
        case HSF_GATE_PHASE: set(m, 2, {1, 0, 0, std::polar(1.0, t)}); return true;
        case HSF_GATE_CX:
            set(m, 4, {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0});
            return true;
        case HSF_GATE_CZ:
            set(m, 4, {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, -1});
            return true;
        case HSF_GATE_CP:
            set(m, 4, {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, std::polar(1.0, t)});
            return true;
        case HSF_GATE_RZZ: {
            // Z(x)Z = diag(1, -1, -1, 1)
            const cd e0(c, -s), e1(c, s);
            set(m, 4, {e0, 0, 0, 0, 0, e1, 0, 0, 0, 0, e1, 0, 0, 0, 0, e0});
            return true;
        }
        case HSF_GATE_SWAP:
            set(m, 4, {1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1});
            return true;
        case HSF_GATE_ISWAP:
            set(m, 4, {1, 0, 0, 0, 0, 0, I1, 0, 0, I1, 0, 0, 0, 0, 0, 1});
            return true;
        default:
            return false;
    }
}

bool gate_generator(int kind, int nq, std::vector<cd>& d) {
    // exp(-i t P / 2): dU/dt = (-i/2) P U;  diag(1, e^{it}): dU/dt = i |1><1| U
    const cd h(0.0, -0.5), one_i(0.0, 1.0);
    switch (kind) {
        case HSF_GATE_RX: set(d, 2, {0, h, h, 0}); return nq == 1;
        case HSF_GATE_RY: set(d, 2, {0, -h * cd(0, 1), h * cd(0, 1), 0}); return nq == 1;
        case HSF_GATE_RZ: set(d, 2, {h, 0, 0, -h}); return nq == 1;
        case HSF_GATE_PHASE: set(d, 2, {0, 0, 0, one_i}); return nq == 1;
        case HSF_GATE_RZZ:
            set(d, 4, {h, 0, 0, 0, 0, -h, 0, 0, 0, 0, -h, 0, 0, 0, 0, h});
            return nq == 2;
        case HSF_GATE_CP:
            set(d, 4, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, one_i});
            return nq == 2;
        default:
            return false;
    }
}

}  // namespace hsf
