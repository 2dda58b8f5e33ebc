"""Cost model of the two-pass gradient (paper, eqs. 1311A, 1211A, 0711C).

Cost(F_v) = K_F/c Cost(F), Cost(R_v) = K_R/c Cost(F), and the gradient of G
costs (2 K_F + K_R)/c per path: one forward pass for E y, then a forward
re-run plus the reverse sweep for every path.  On the GPU, with T_F the
measured time of the forward pass and T_2 the time of the second pass,
K_R/K_F = (T_2 - T_F)/T_F.
"""


def gradient_cost_over_paths_costF(kf_over_c: float, kr_over_c: float) -> float:
    """Cost(G) / (number_of_paths * Cost(F)) from eq. 0711C."""
    return 2.0 * kf_over_c + kr_over_c


def kr_over_kf(t_forward: float, t_pass2: float) -> float:
    """K_R/K_F from the two measured pass times: pass 2 costs K_F + K_R."""
    return (t_pass2 - t_forward) / t_forward


def gradient_over_forward(kr_over_kf_ratio: float) -> float:
    """Cost(G)/Cost(F_v) = (2 K_F + K_R)/K_F."""
    return 2.0 + kr_over_kf_ratio
