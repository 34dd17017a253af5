"""Exact solution of the 1-D Riemann problem of an ideal ultrarelativistic
fluid (p = e/3) initially at rest on both sides, e_L > e_R: a rarefaction
fan moves into the left state and a shock into the right one.  The
large-cross-section limit of the kinetic evolution (the paper's Sec. 5
benchmark compares against it qualitatively): the cross-section scan
measures its distance to it, and tests pin the oracle's whole runs to it.  Written from the textbook
relations: the Riemann invariant arctanh(v) + (sqrt(3)/4) ln e across the
fan, and the Taub jump conditions across the shock."""
import math

from scipy import optimize

CS = 1.0 / math.sqrt(3.0)


def _v_rarefaction(e, eL):
    return math.tanh(math.sqrt(3.0) / 4.0 * math.log(eL / e))


def _v_shock(e, eR):
    p, pR = e / 3.0, eR / 3.0
    return math.sqrt((e - eR) * (p - pR) / ((eR + p) * (e + pR)))


def _t00(e, v):
    g2 = 1.0 / (1.0 - v * v)
    return (4.0 / 3.0) * e * g2 - e / 3.0


def _t0x(e, v):
    g2 = 1.0 / (1.0 - v * v)
    return (4.0 / 3.0) * e * g2 * v


class Riemann:
    def __init__(self, eL, eR):
        self.eL, self.eR = eL, eR
        self.es = optimize.brentq(lambda e: _v_rarefaction(e, eL) - _v_shock(e, eR),
                                  eR * (1 + 1e-12), eL * (1 - 1e-12), xtol=1e-15)
        self.vs = _v_shock(self.es, eR)
        # shock speed from energy conservation across the front
        self.shock = _t0x(self.es, self.vs) / (_t00(self.es, self.vs) - eR)
        self.head = -CS
        self.tail = (self.vs - CS) / (1.0 - self.vs * CS)

    def state(self, xi):
        """(e, v) at similarity coordinate xi = (x - x0) / t."""
        if xi <= self.head:
            return self.eL, 0.0
        if xi < self.tail:
            v = (xi + CS) / (1.0 + xi * CS)
            e = self.eL * math.exp(-4.0 / math.sqrt(3.0) * math.atanh(v))
            return e, v
        if xi < self.shock:
            return self.es, self.vs
        return self.eR, 0.0

    def profiles(self, xi):
        e, v = self.state(xi)
        return _t00(e, v), _t0x(e, v)

    def jump_residual(self):
        """Relative residuals of energy and momentum conservation across
        the shock (T^0x and T^xx fluxes)."""
        e, v, eR = self.es, self.vs, self.eR
        g2 = 1.0 / (1.0 - v * v)
        txx = (4.0 / 3.0) * e * g2 * v * v + e / 3.0
        r1 = (_t0x(e, v) - self.shock * (_t00(e, v) - eR)) / _t0x(e, v)
        r2 = ((txx - eR / 3.0) - self.shock * _t0x(e, v)) / txx
        return r1, r2
