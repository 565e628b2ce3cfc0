"""Fourier-space GridSPT recursion on a sparse spectrum -- test infrastructure.

For an input delta_1 made of a few plane waves, every order delta_n is a sum
over a small set of modes, so the recursion of Eq. 10 can be evaluated
exactly in Fourier space by explicit mode-pair sums, at any grid size: this
yields reference values for individual modes of very large grids.  Output
modes wrap as on the grid (k = q1 + q2 mod N), and per mode pair (q1 from
order m, q2 from order n - m) the sources take the coefficients of one of
the two forms (Sec. II C; Eq. 10 and the products of Eq. 15/16):

  divergence form ("D", what gridspt_orders evaluates), k the wrapped sum:
    S_delta(k) += (k.q2 / q2^2) delta_m(q1) theta_{n-m}(q2)
    S_theta(k) += (k^2/2)(q1.q2)/(q1^2 q2^2) theta_m(q1) theta_{n-m}(q2)
  printed form ("P", the products of Eq. 10 as written), from the
  derivatives of each factor, so the unwrapped q1 + q2 enters:
    S_delta(k) += ((q1 + q2).q2 / q2^2) delta_m(q1) theta_{n-m}(q2)
                  [(grad delta_m).u_{n-m} + delta_m theta_{n-m}]
    S_theta(k) += [(q1.q2)^2/(q1^2 q2^2) + q1.q2/q1^2] theta_m(q1) theta_{n-m}(q2)
                  [d_j u_{m,k} d_k u_{n-m,j} + u_m.grad theta_{n-m}]

  delta_n = W2 c_n [(n + 1/2) S_delta + S_theta],  theta_n = W2 c_n [3/2 S_delta + n S_theta]

with c_n = 2 / ((2n + 3)(n - 1)), delta_1 = theta_1 = W1 delta_0, and k = 0
removed.  The two forms agree whenever q1 + q2 does not wrap.  Pure-Python
loops: only for a handful of input modes.
"""
from __future__ import annotations


def _wrap(v: int, n: int) -> int:
    return (v + n // 2) % n - n // 2


def _der(v: int, n: int) -> int:
    return 0 if v == -n // 2 else v


def sparse_orders(modes1: dict, n: int, nmax: int, n2max1: int, n2max2: int, form: str = "D"):
    """modes1: {(a, b, c): amplitude} of the full (Hermitian) spectrum of the
    input field, signed modes.  form: "D" (divergence form) or "P" (the
    printed products).  Returns (deltas, thetas): lists of dicts."""
    printed = form.upper() == "P"
    d1 = {}
    for k, v in modes1.items():
        k = tuple(_wrap(int(x), n) for x in k)
        n2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2]
        if 0 < n2 <= n2max1 and v != 0:
            d1[k] = d1.get(k, 0) + complex(v)
    deltas, thetas = [d1], [d1]
    for order in range(2, nmax + 1):
        sd, st = {}, {}
        for m in range(1, order):
            dm, tm, tnm = deltas[m - 1], thetas[m - 1], thetas[order - m - 1]
            for q1, a_d in dm.items():
                a_t = tm.get(q1, 0)
                q1d = tuple(_der(x, n) for x in q1)
                s1 = q1[0] ** 2 + q1[1] ** 2 + q1[2] ** 2
                for q2, b in tnm.items():
                    k = tuple(_wrap(q1[i] + q2[i], n) for i in range(3))
                    s2 = q2[0] ** 2 + q2[1] ** 2 + q2[2] ** 2
                    kd = tuple(_der(x, n) for x in k)
                    q2d = tuple(_der(x, n) for x in q2)
                    dot_k2 = kd[0] * q2d[0] + kd[1] * q2d[1] + kd[2] * q2d[2]
                    dot_12 = q1d[0] * q2d[0] + q1d[1] * q2d[1] + q1d[2] * q2d[2]
                    nk2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
                    if printed:
                        alpha = (s2 + dot_12) / s2                  # (q1 + q2).q2 / q2^2, unwrapped
                        beta = dot_12 * dot_12 / (s1 * s2) + dot_12 / s1
                    else:
                        alpha = dot_k2 / s2
                        beta = 0.5 * nk2 * dot_12 / (s1 * s2)
                    sd[k] = sd.get(k, 0) + alpha * a_d * b
                    st[k] = st.get(k, 0) + beta * a_t * b
        c = 2.0 / ((2 * order + 3) * (order - 1))
        dn, tn = {}, {}
        for k in set(sd) | set(st):
            n2 = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
            if n2 == 0 or n2 > n2max2:
                continue
            a, b = sd.get(k, 0), st.get(k, 0)
            dn[k] = c * ((order + 0.5) * a + b)
            tn[k] = c * (1.5 * a + order * b)
        deltas.append(dn)
        thetas.append(tn)
    return deltas, thetas
