"""Writes sine_edisc.txt: closed-form discretization error of the 7-point
cell-centered Dirichlet Laplacian for u = sin(pi x) sin(pi y) sin(pi z).

The sampled u is an eigenvector of the discrete operator (Sec. 2 of the paper
defines the cell-centered grid), with eigenvalue -(12/h^2) sin^2(pi h/2), so
the discrete solution of L_h u_h = -3 pi^2 u is u_h = c u with
c = (pi h/2)^2 / sin^2(pi h/2); its max-norm error is (c - 1) max|u|, and
max|u| over cell centers is sin^3(pi (m+1/2)/N) at the middle cell.
Pure mathematics: no solver is called.
"""
import math
import os

rows = []
for N in (8, 16, 32, 64, 128, 256, 512):
    h = 1.0 / N
    c = (math.pi * h / 2) ** 2 / math.sin(math.pi * h / 2) ** 2
    umax = math.sin(math.pi * (N // 2 - 0.5) / N) ** 3
    rows.append("%d %.10e" % (N, (c - 1.0) * umax))
out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sine_edisc.txt")
with open(out, "w") as fh:
    fh.write("# N  max-norm discretization error, u = prod sin(pi x_d), 7-point cell-centered\n")
    fh.write("\n".join(rows) + "\n")
