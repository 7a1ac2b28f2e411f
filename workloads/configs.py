"""The five benchmark/parity workloads, as plain dictionaries."""

TGV_64 = {  # plain method, tiny
    "name": "tgv64", "nx": 64, "ny": 64, "nz": 64, "omega": 1.9, "steps": 50,
    "u0": 0.05, "storage": "f32", "bc_x": "periodic",
}

SINGLE_TURBINE = {  # one rotor, inflow/outflow
    "name": "single_turbine", "nx": 256, "ny": 128, "nz": 128, "omega": 1.9,
    "steps": 2000, "u_in": (0.05, 0.0, 0.0), "storage": "f32", "bc_x": "inout",
}

BANDWIDTH_512 = {  # the bandwidth-bound periodic box
    "name": "random_phase_512", "n": 512, "omega": 1.9, "steps": 200,
    "seed": 0, "k_peak": 8.0, "u_rms": 0.03,
}

CLOSURE_LES = {  # learned closure, coarse LES
    "name": "les128", "n_fine": 512, "n": 128, "filter": 4, "seeds": list(range(8)),
    "omega_fine": 1.9, "steps_coarse": 2000, "cs": 0.1,
}

TURBINE_ROW = {  # three rotors, sheared turbulent inflow
    "name": "turbine_row", "nx": 1024, "ny": 256, "nz": 256, "omega": 1.9,
    "steps": 5000, "storage": "f16", "closure": "mlp", "u_hub": 0.05,
    "hub_height": 128.0, "shear_exp": 0.14, "ti": 0.05, "turb_seed": 100,
}
