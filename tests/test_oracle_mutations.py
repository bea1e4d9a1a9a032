"""Each pin of the oracle tests must catch the plausible mistake it is there
for. A copy of oracle.c with that one mistake planted is built on the CPU (or,
for the merging of superparticles, written in Python, a copy of
Oracle.merge, or of a method of the axisymmetric oracle), and the pin, run
against the copy, must fail; the same pin passes on the real oracle in its
own test module."""
import inspect
import os
import textwrap

import pytest

import oracle
import oracle.rz as orz
import test_oracle_merging as M
import test_oracle_rz_collide as RZC
import test_oracle_pairing as PR
import test_oracle_readings as R
import test_oracle_surface as S
import test_oracle_weights as WT

_SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, text in oracle.c, planted replacement, pin that must fail)
MUTATIONS = [
    ("unshifted pairing",
     "int64_t shift = (int64_t)floor(uc * (double)NT);",
     "int64_t shift = 0 * (int64_t)floor(uc * (double)NT);", R.pin_pairing),
    ("tie goes to the neutral",
     "int a_is_proj = NA <= NB;", "int a_is_proj = NA < NB;", R.pin_pairing),
    ("targets in descending id order",
     "const entry* te = &ent[T0 + (shift + i) % NT];",
     "const entry* te = &ent[T0 + NT - 1 - (shift + i) % NT];", R.pin_pairing),
    ("R instead of its inverse for (theta, phi)",
     "    du[0] = ct * cp * w0 - sp * w1 + st * cp * w2;\n"
     "    du[1] = ct * sp * w0 + cp * w1 + st * sp * w2;\n"
     "    du[2] = -st * w0 + ct * w2;",
     "    du[0] = ct * cp * w0 + ct * sp * w1 - st * w2;\n"
     "    du[1] = -sp * w0 + cp * w1;\n"
     "    du[2] = st * cp * w0 + st * sp * w1 + ct * w2;", R.pin_elastic_du),
    ("R instead of its inverse for (theta', phi')",
     "double w0 = um * st2 * cos(ph2), w1 = um * st2 * sin(ph2), w2 = um * (ct2 - 1.0);",
     "double w0 = -um * st2, w1 = 0.0 * ph2, w2 = um * (ct2 - 1.0);", R.pin_elastic_du),
    ("no (e,Cu) exclusion in the (Cu+,Cu) pairing",
     "if (cls == 2 && used[sb][ib]) continue;", "", R.pin_priority),
    ("no impact exclusion in field ionization",
     "if (used[ORC_SP_NEU][p]) continue;", "", R.pin_priority),
    ("(Cu+,Cu) before (e,Cu)",
     "    if (flags & ORC_COLL_MCC1) mcc_class(c, step, 1, ent, ne, sp, used, prod, &nprod, spl, &nspl, o);\n"
     "    if (flags & ORC_COLL_MCC2) mcc_class(c, step, 2, ent, ne, sp, used, prod, &nprod, spl, &nspl, o);",
     "    if (flags & ORC_COLL_MCC2) mcc_class(c, step, 2, ent, ne, sp, used, prod, &nprod, spl, &nspl, o);\n"
     "    if (flags & ORC_COLL_MCC1) mcc_class(c, step, 1, ent, ne, sp, used, prod, &nprod, spl, &nspl, o);",
     R.pin_priority),
    ("emission field half a spacing out",
     "g[0] + g[3], g[1] + g[4], g[2] + g[5]) / h;",
     "g[0] + 0.5 * g[3], g[1] + 0.5 * g[4], g[2] + 0.5 * g[5]) / (0.5 * h);", R.pin_emission_field_point),
    ("emission field from the surface potential",
     "g[0] + g[3], g[1] + g[4], g[2] + g[5]) / h;", "g[0], g[1], g[2] + 1.0) / h;", R.pin_emission_field_point),
    ("evaporation exponent with the wrong sign",
     "(1.0 / T_BOIL_CU - 1.0 / T)", "(1.0 / T - 1.0 / T_BOIL_CU)", S.pin_evaporation_flux),
    ("evaporation flux without the thermal prefactor's square root",
     "P_ATM / sqrt(2.0 * PI * c->m_ion * K_B * T)", "P_ATM / (2.0 * PI * c->m_ion * K_B * T)",
     S.pin_evaporation_flux),
    ("half-Maxwellian instead of flux-weighted normal speeds",
     "double vn = sig * sqrt(-2.0 * log(w1));",
     "double vn = sig * fabs(sqrt(-2.0 * log(w1)) * cos(2.0 * PI * w2));", S.pin_evaporation_atoms),
    ("Shockley-Ramo current from the field instead of the weighting field",
     "orc_gather(c, E0, s->x[p], s->y[p], s->z[p], w);", "orc_gather(c, E, s->x[p], s->y[p], s->z[p], w);",
     S.pin_shockley_ramo_push),
    ("collision probability without the target weight",
     "double P = -expm1(-um * n * (double)wt * stot * dt);", "double P = -expm1(-um * n * 1.0 * stot * dt);",
     WT.pin_ncoll_binomial),
    ("the lighter superparticle as the target",
     "uint32_t wt = wa > wb ? wa : wb, npart = wa < wb ? wa : wb;",
     "uint32_t wt = wa < wb ? wa : wb, npart = wa < wb ? wa : wb;", WT.pin_ncoll_binomial),
    ("one field-ionization draw per neutral superparticle",
     "for (uint32_t q = 1; q < wgt(N, p); ++q) {", "for (uint32_t q = 1; q < 1u; ++q) {",
     WT.pin_weighted_field_ionization),
    ("injection weight without the geometric mean",
     "double r = sqrt(n_cell / c->n_max * (double)n_inj);", "double r = n_cell / c->n_max * (double)n_inj;",
     WT.pin_injection_weights),
    ("Cu-Cu collision probability without the density",
     "double P = -expm1(-um * n * c->sigma_nn * dt);", "double P = -expm1(-um * c->sigma_nn * dt);",
     PR.pin_nn_rate_and_isotropy),
    ("Cu-Cu scattering not isotropic (cos theta' = U)",
     "elastic_du(u, 2.0 * u3 - 1.0, 2.0 * PI * u4, du);\n                    double k = 0.5 * dt / h;",
     "elastic_du(u, u3, 2.0 * PI * u4, du);\n                    double k = 0.5 * dt / h;", PR.pin_nn_rate_and_isotropy),
    ("Cu-Cu kick without the reduced mass",
     "double k = 0.5 * dt / h;   /* mu / m = 1/2 */", "double k = dt / h;", PR.pin_nn_rate_and_isotropy),
    ("Takizuka-Abe variance with mu instead of mu^2",
     "(8.0 * PI * EPS0 * EPS0 * mu * mu * um * um * um)", "(8.0 * PI * EPS0 * EPS0 * mu * um * um * um)",
     PR.pin_coulomb_angle),
    ("Takizuka-Abe variance with u^2 instead of u^3",
     "(8.0 * PI * EPS0 * EPS0 * mu * mu * um * um * um)", "(8.0 * PI * EPS0 * EPS0 * mu * mu * um * um)",
     PR.pin_coulomb_angle),
    ("Takizuka-Abe angle theta = delta instead of 2 atan(delta)",
     "double ct = (1.0 - delta * delta) / (1.0 + delta * delta);", "double ct = cos(delta);", PR.pin_coulomb_angle),
    ("same-species pairs without the cyclic shift",
     "for (int64_t j = 0; j < N; ++j) q[j] = ent[a0 + (shift + j) % N].idx;",
     "for (int64_t j = 0; j < N; ++j) q[j] = ent[a0 + j].idx;", PR.pin_pairing_enumerated),
    ("e-Cu+ Coulomb with the larger density",
     "double n_l = (double)NF / vol;", "double n_l = (double)NM / vol;", PR.pin_coulomb_e_ion),
    ("recombination probability without the density",
     "double P = -expm1(-um * n * c->sigma_rec * dt);", "double P = -expm1(-um * c->sigma_rec * dt);",
     PR.pin_recombination),
    ("recombined atom with the ion's velocity",
     "r->v[0] = (M_EL * El->vx[ie] + c->m_ion * I->vx[ii]) / mt;", "r->v[0] = I->vx[ii];", PR.pin_recombination),
]


@pytest.mark.parametrize("name,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(tmp_path, name, old, new, pin):
    text = open(_SRC).read()
    assert text.count(old) == 1, f"mutation site not found: {name}"
    path = oracle.build_copy(text.replace(old, new), str(tmp_path))
    with oracle.use_library(path):
        with pytest.raises(AssertionError):
            pin()


# mistakes planted in the Python part of the oracle (merging of superparticles)
PY_MUTATIONS = [
    ("centre of mass with the weights swapped",
     "v[pa] = (fa * v[pa] + fb * v[pb]) / (fa + fb)", "v[pa] = (fb * v[pa] + fa * v[pb]) / (fa + fb)",
     M.pin_merge_conservation),
    ("pairs in descending id order",
     "order = np.lexsort((ids[cand], cell))", "order = np.lexsort((-ids[cand], cell))", M.pin_pair_choice),
    ("merging down to floor(N / 2) regardless of merge_max",
     "for q in range(min(N // 2, N - cfg.merge_max)):", "for q in range(N // 2):", M.pin_pair_choice),
    ("merged weights above w_max",
     "if w1 + w2 > cfg.w_max:", "if False:", M.pin_w_max_and_id_limit),
    ("products of this step's collisions merged",
     "cand = np.nonzero(ids < id_limit)[0]", "cand = np.arange(n)", M.pin_w_max_and_id_limit),
]


@pytest.mark.parametrize("name,old,new,pin", PY_MUTATIONS, ids=[m[0] for m in PY_MUTATIONS])
def test_merge_pin_catches_planted_mistake(monkeypatch, name, old, new, pin):
    src = textwrap.dedent(inspect.getsource(oracle.Oracle.merge))
    assert src.count(old) == 1, f"mutation site not found: {name}"
    ns = dict(vars(oracle))
    exec(src.replace(old, new), ns)
    monkeypatch.setattr(oracle.Oracle, "merge", ns["merge"])
    with pytest.raises(AssertionError):
        pin()


# mistakes planted in the axisymmetric oracle: (name, method, text, planted
# replacement, pin that must fail)
RZ_MUTATIONS = [
    ("cell volume without the ring factor", "collide",
     "vol = math.pi * (2 * int(c % (self.nr - 1)) + 1) * h * h * h", "vol = math.pi * h * h * h",
     RZC.pin_collision_rate),
    ("elastic kick with the masses swapped", "collide",
     "ka, kb = mu / ma * dt / h, mu / mb * dt / h", "ka, kb = mu / mb * dt / h, mu / ma * dt / h",
     RZC.pin_elastic_conservation),
    ("charge exchange copying one way", "collide",
     "A[k][xa], N[k][xb] = N[k][xb], A[k][xa]", "A[k][xa] = N[k][xb]", RZC.pin_cx_swap),
    ("ionization energy without the threshold", "collide", "erem = E - self.xi", "erem = E",
     RZC.pin_ionization),
    ("ion id one too high", "collide",
     'ions["id"].append(self.next_id)', 'ions["id"].append(self.next_id + 1)', RZC.pin_ionization),
    ("field-ionization probability with dt in seconds", "collide",
     "pdt = self.adk_rate(Eg) * (dt * 1e15)", "pdt = self.adk_rate(Eg) * dt", RZC.pin_field_ionization),
    ("field ionization above the barrier-suppression field", "collide",
     "if Eg > ebsi:\n            continue", "if False:\n            continue",
     RZC.pin_field_ionization),
    ("emission field taken on the surface", "emit",
     "F = self.interp(self.phi, r + nr_, z + nz_) / self.h", "F = self.interp(self.phi, r, z) / self.h",
     RZC.pin_emission_count),
    ("no side rings", "patches", "return self.fn_rings + max(int(math.ceil(zc)), 0)", "return self.fn_rings",
     RZC.pin_emission_geometry),
    ("electrons started on the surface", "emit", "new[\"r\"].append(r + 1e-3 * nr_)", "new[\"r\"].append(r)",
     RZC.pin_emission_geometry),
    ("double ionization without the second threshold", "collide", "rest = E - self.xi - self.xi2",
     "rest = E - self.xi", RZC.pin_double_ionization),
    ("Cu2+ ionized again", "collide", " or B[\"q\"][xb] != 1", "", RZC.pin_ion_ionization),
    ("Cu+ ionization above xi instead of xi2", "collide", "rest3 = E - self.xi2", "rest3 = E - self.xi",
     RZC.pin_ion_ionization),
    ("Cu+ ionization density over the full cell volume h^3", "collide",
     "vol = math.pi * (2 * int(c % (self.nr - 1)) + 1) * h * h * h", "vol = h * h * h",
     RZC.pin_ion_ionization_rate),
    ("Cu2+ kick as for Cu+", "push", "kq = kq0 * float(d[\"q\"][p]) if s == 1 else kq0", "kq = kq0",
     RZC.pin_cu2_push_deposit),
    ("Cu2+ deposit as for Cu+", "deposit", "sign = sign0 * (int(d[\"q\"][p]) if s == 1 else 1)",
     "sign = sign0", RZC.pin_cu2_push_deposit),
]


@pytest.mark.parametrize("name,method,old,new,pin", RZ_MUTATIONS, ids=[m[0] for m in RZ_MUTATIONS])
def test_rz_pin_catches_planted_mistake(monkeypatch, name, method, old, new, pin):
    src = textwrap.dedent(inspect.getsource(getattr(orz.RZ, method)))
    assert src.count(old) == 1, f"mutation site not found: {name}"
    ns = dict(vars(orz))
    exec(src.replace(old, new), ns)
    monkeypatch.setattr(orz.RZ, method, ns[method])
    with pytest.raises(AssertionError):
        pin()
