"""Single planted mistakes in copies of the oracle's sources, each with the
pins (tests/_pins.py) that must catch it.  A mistake is (file, exact text,
replacement); every text occurs once in its file."""

MUTANTS = {
    # robot / door-drawer contact rows
    "row_sign": ("ms_oracle.cpp", "    J[j] = v * sgn;", "    J[j] = -v * sgn;",
                 ["pin_robot_resting_moment", "pin_robot_speculative_landing", "pin_robot_hinge_momentum"]),
    "row_lever_origin": ("ms_oracle.cpp", "dot(d, cross(k.a[j], sub(p, k.o[j])))",
                         "dot(d, cross(k.a[j], sub(p, k.o[body])))", ["pin_robot_speculative_landing"]),
    "row_contact_point": ("ms_oracle.cpp", "art_row(am, kk, S.body, ct.p, rw.d[di], sgn, r.J);",
                          "art_row(am, kk, S.body, add(ct.p, scl(ct.n, T(0.02))), rw.d[di], sgn, r.J);",
                          ["pin_robot_hinge_momentum"]),
    "row_no_minv": ("ms_oracle.cpp", "          art_solve(S.art, r.w);\n", "",
                    ["pin_robot_resting_moment", "pin_robot_hinge_momentum"]),
    # implicit PD drive and damping
    "pd_no_h2kp": ("ms_oracle.cpp", "h * (kd + dmp) + h * h * kp)", "h * (kd + dmp))",
                   ["pin_pd_steady_state_and_stability"]),
    "pd_no_hqd": ("ms_oracle.cpp", "kp * (qt - st.q[j] - h * st.qd[j])", "kp * (qt - st.q[j])",
                  ["pin_pd_steady_state_and_stability"]),
    "pd_no_hkd": ("ms_oracle.cpp", "h * (kd + dmp) + h * h * kp)", "h * dmp + h * h * kp)",
                  ["pin_pd_steady_state_and_stability"]),
    "veldof_kp": ("ms_oracle.cpp", "      if (rm.veldof[j]) kp = 0.0;\n", "", ["pin_base_velocity_drive"]),
    "damping_explicit": ("ms_oracle.cpp", "arm[j] = T(rm.armature[j] + h * dmp);", "arm[j] = T(rm.armature[j]);",
                         ["pin_base_velocity_drive"]),
    # free-body gyroscopic term
    "gyro_transposed": ("ms_oracle.cpp", "    M3<T> Iw = mmt(mm(wk.fR[f], D), wk.fR[f]);",
                        "    M3<T> Rt;\n    for (int i = 0; i < 9; ++i) Rt[i] = wk.fR[f][(i % 3) * 3 + i / 3];\n"
                        "    M3<T> Iw = mmt(mm(Rt, D), Rt);", ["pin_gyroscopic_torque_free"]),
    "gyro_sign": ("ms_oracle.cpp", "wF[f] = sub(fs.w, scl(mv(wk.fIinv[f], gyro), T(h)));",
                  "wF[f] = add(fs.w, scl(mv(wk.fIinv[f], gyro), T(h)));", ["pin_gyroscopic_torque_free"]),
    # door / drawer joints and limit rows
    "limit_sign": ("ms_oracle.cpp", "lims.push_back({x, 1.0,", "lims.push_back({x, -1.0,",
                   ["pin_limit_lands_on_limit"]),
    "limit_bias": ("ms_oracle.cpp", "val(ghi) >= 0.0 ? ghi / h : pr.baumgarte * ghi / h",
                   "val(ghi) >= 0.0 ? pr.baumgarte * ghi / h : pr.baumgarte * ghi / h",
                   ["pin_limit_lands_on_limit"]),
    "aux_gravity": ("ms_oracle.cpp", "rnea(c.aux[x], wk.ak[x], qdx, (const T*)nullptr, pr.gravity, C);",
                    "const double g0[3] = {0.0, 0.0, 0.0};\n    rnea(c.aux[x], wk.ak[x], qdx, (const T*)nullptr, g0, C);",
                    ["pin_door_pendulum_period"]),
    "aux_com": ("ms_oracle.cpp", "    a.com[0][t] = sc->aux_box[x * 6 + t];", "    a.com[0][t] = 0.0;",
                ["pin_door_pendulum_period", "pin_door_hinge_momentum"]),
    # robot contact cap
    "no_robot_cap": ("ms_oracle.cpp", "if (ct.robot_owner && n_robot >= pr.robot_contact_cap)",
                     "if (false && ct.robot_owner && n_robot >= pr.robot_contact_cap)", ["pin_robot_contact_cap"]),
    # reverse-mode derivative rules
    "ad_div_sign": ("ms_ad.hpp", "  return mk2(r, a, 1.0 / b.v, b, -r / b.v);", "  return mk2(r, a, 1.0 / b.v, b, r / b.v);",
                    ["pin_sliding_sensitivity"]),
    "ad_sqrt": ("ms_ad.hpp", "  return mk1(r, a, r > 0.0 ? 0.5 / r : 0.0);", "  return mk1(r, a, r > 0.0 ? 1.0 / r : 0.0);",
                ["pin_sliding_sensitivity"]),
}
