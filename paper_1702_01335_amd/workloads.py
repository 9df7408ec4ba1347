"""Named synthetic workloads (parameter sets only; no solver arithmetic).

Each workload is a dict of the parameters of one Couette instance plus the shared shape
(velocity set, node count, scheme).  Expansion orders follow the paper's choice
N_x = min(6, Qx - 1) and N = Q - 1 on y and z; time steps keep the Courant number near 0.4.

  couette_bgk_s64_v128     BGK (Pr = 1, mu ~ T), Kn = 0.1, u_w = 0.1, 64 equidistant nodes,
                           HHLB(3;4) x HLB(3;4) x HLB(3;4) (V = 128), 2nd-order upwind,
                           dt = 1e-3.
  couette_shakhov_s256_v800  Shakhov Pr = 2/3, mu ~ T^0.5, Kn = 1, u_w = 0.4, 256 nodes on
                           the tanh grid A = 0.98, HHLB(6;16) x HLB(4;5) x HLB(4;5) (V = 800),
                           WENO-5, dt = 1e-5.
  couette_shakhov_s512_v3600 Shakhov Pr = 2/3, mu ~ T^0.5, Kn = 100, u_w = 0.2, 512
                           equidistant nodes, HHLB(6;50) x HLB(5;6) x HLB(5;6) (V = 3600),
                           WENO-5, dt = 2.5e-5.
  paper_maxwell_s16_v686   the paper's Maxwell-molecule runs (Sec. V): Pr = 2/3, tau = Kn/n,
                           Kn = 0.1, u_w = 0.63, 16 nodes A = 0.98, HHLB(6;7) x HLB(6;7)
                           x HLB(6;7) (V = 686), WENO-5, dt = 5e-4.
  couette_shakhov_s256_reduced  the second workload's physics, grid and x, y velocity sets
                           with p_z integrated out as the paper does (reduced phi, chi
                           distributions of Sec. III): HHLB(6;16) x HLB(4;5), 160 velocities,
                           320 populations per node.
  paper_sutherland_s16_reduced  the paper's Sec. VI runs as printed in Tables III-VI: argon
                           (Sutherland, S = 0.5239), delta = 1, u_w = sqrt 2, 16 nodes A = 0.98,
                           HHLB(6;7) x HLB(6;7) reduced (98 velocities, 196 populations),
                           WENO-5, dt = 5e-4.
"""

WORKLOADS = {
    'couette_bgk_s64_v128': dict(Qx=4, Qy=4, Qz=4, S=64, scheme='upwind2',
                                 params=dict(kn=0.1, u_w=0.1, T_w=1.0, n0=1.0, pr=1.0, law='power', omega=1.0,
                                             A=0.0, dt=1e-3)),
    'couette_shakhov_s256_v800': dict(Qx=16, Qy=5, Qz=5, S=256, scheme='weno5',
                                      params=dict(kn=1.0, u_w=0.4, T_w=1.0, n0=1.0, pr=2.0 / 3.0, law='power',
                                                  omega=0.5, A=0.98, dt=1e-5)),
    'couette_shakhov_s512_v3600': dict(Qx=50, Qy=6, Qz=6, S=512, scheme='weno5',
                                       params=dict(kn=100.0, u_w=0.2, T_w=1.0, n0=1.0, pr=2.0 / 3.0, law='power',
                                                   omega=0.5, A=0.0, dt=2.5e-5)),
    'paper_maxwell_s16_v686': dict(Qx=7, Qy=7, Qz=7, S=16, scheme='weno5',
                                   params=dict(kn=0.1, u_w=0.63, T_w=1.0, n0=1.0, pr=2.0 / 3.0, law='power',
                                               omega=1.0, A=0.98, dt=5e-4)),
    'couette_shakhov_s256_reduced': dict(Qx=16, Qy=5, Qz=1, S=256, scheme='weno5', reduced=True,
                                         params=dict(kn=1.0, u_w=0.4, T_w=1.0, n0=1.0, pr=2.0 / 3.0, law='power',
                                                     omega=0.5, A=0.98, dt=1e-5)),
    'paper_sutherland_s16_reduced': dict(Qx=7, Qy=7, Qz=1, S=16, scheme='weno5', reduced=True,
                                         params=dict(kn=0.7071067811865476, u_w=1.4142135623730951, T_w=1.0,
                                                     n0=1.0, pr=2.0 / 3.0, law='sutherland', suth_S=0.5239,
                                                     omega=1.0, A=0.98, dt=5e-4)),
}


def workload(name):
    w = WORKLOADS[name]
    return dict(w, params=dict(w['params']))
