"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case monkeypatches one plausible slip into ``oracle.relnn_oracle`` (a
dropped term, a wrong sign or index, a transposed operand, a swapped order)
and runs the pins; at least one of them must fail.
"""
import numpy as np
import pytest

from oracle import relnn_oracle as orc
from tests import test_oracle_pins as pins

PIN_SET = [
    pins.test_golden_index,
    lambda: pins.test_golden_forward("sum", "sum_pre"),
    lambda: pins.test_golden_forward("mean", "mean_pre"),
    lambda: pins.test_golden_forward("max", "max_pre"),
    pins.test_golden_relu_and_grad,
    pins.test_sum_closed_form,
    pins.test_mean_closed_form,
    pins.test_max_properties,
    lambda: pins.test_layer_matches_brute("sum", pins.CASES[0], ("none", "relu")),
    lambda: pins.test_layer_matches_brute("max", pins.CASES[3], ("relu", "none")),
    lambda: pins.test_grad_finite_differences("mean", "none"),
    lambda: pins.test_grad_finite_differences("max", "relu"),
    pins.test_grad_closed_form_sum,
    lambda: pins.test_join_matches_nested_loop(pins.CASES[7]),
]


def caught(mp):
    for pin in PIN_SET:
        try:
            pin()
        except (AssertionError, ValueError, IndexError):
            return True
    return False


orig_gather = orc.gather_concat
orig_transform = orc.transform
orig_fwd = orc.layer_fwd
orig_bwd = orc.layer_bwd
orig_lookup = orc.lookup_rows


def m_concat_reversed(idx, embs, sel=slice(None)):
    parts = [np.asarray(e, np.float64)[r[sel]] for e, r in zip(embs, idx.rows)]
    return np.concatenate(parts[::-1], axis=1)


def m_bias_dropped(x, W, b, act_pre):
    return orig_transform(x, W, np.zeros_like(b), act_pre)


def m_bias_sign(x, W, b, act_pre):
    return orig_transform(x, W, -np.asarray(b), act_pre)


def m_mean_off_by_one(idx, embs, W, b, agg="sum", act_pre="none", act_post="none", groups=None):
    out, pre, am = orig_fwd(idx, embs, W, b, agg, act_pre, act_post, groups)
    if agg == "mean":
        cnt = np.diff(idx.offsets)[orc._groups(idx, groups)].astype(np.float64)
        pre = pre * cnt[:, None] / (cnt[:, None] + 1)
        out = orc._act(act_post, pre)
    return out, pre, am


def m_argmax_last(idx, embs, W, b, agg="sum", act_pre="none", act_post="none", groups=None):
    out, pre, am = orig_fwd(idx, embs, W, b, agg, act_pre, act_post, groups)
    if agg == "max":
        for q, g in enumerate(orc._groups(idx, groups)):
            s, e = int(idx.offsets[g]), int(idx.offsets[g + 1])
            y = orc.transform(orc.gather_concat(idx, embs, slice(s, e)), W, b, act_pre)
            am[q] = s + (e - s - 1) - np.argmax(y[::-1], axis=0)
    return out, pre, am


def m_bwd_mean_no_scale(idx, embs, W, b, pre, argmax, dout, agg="sum", act_pre="none", act_post="none"):
    if agg == "mean":
        agg = "sum"
    return orig_bwd(idx, embs, W, b, pre, argmax, dout, agg, act_pre, act_post)


def m_bwd_relu_grad_at_zero(idx, embs, W, b, pre, argmax, dout, agg="sum", act_pre="none", act_post="none"):
    pre = np.where(np.asarray(pre) == 0, 1.0, pre)
    return orig_bwd(idx, embs, W, b, pre, argmax, dout, agg, act_pre, act_post)


def m_bwd_transposed_roles(idx, embs, W, b, pre, argmax, dout, agg="sum", act_pre="none", act_post="none"):
    demb, dW, db = orig_bwd(idx, embs, W, b, pre, argmax, dout, agg, act_pre, act_post)
    if len(demb) == 2 and demb[0].shape == demb[1].shape:
        demb = [demb[1], demb[0]]
    return demb, dW, db


def m_lookup_off_by_one(n_rows, keys, values):
    r = orig_lookup(n_rows, keys, values)
    if keys is None:
        values = np.asarray(values, np.int64)
        r = np.where((values >= 0) & (values <= n_rows) & (values < n_rows + 1), values, -1)
        r = np.where(r == n_rows, -1, r)
        r = np.where(r >= 1, r - 1, r)
    return r


MUTANTS = {
    "concat_reversed": ("gather_concat", m_concat_reversed),
    "bias_dropped": ("transform", m_bias_dropped),
    "bias_sign": ("transform", m_bias_sign),
    "mean_off_by_one": ("layer_fwd", m_mean_off_by_one),
    "argmax_last": ("layer_fwd", m_argmax_last),
    "bwd_mean_no_scale": ("layer_bwd", m_bwd_mean_no_scale),
    "bwd_relu_grad_at_zero": ("layer_bwd", m_bwd_relu_grad_at_zero),
    "bwd_transposed_roles": ("layer_bwd", m_bwd_transposed_roles),
    "lookup_off_by_one": ("lookup_rows", m_lookup_off_by_one),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTANTS[name]
    monkeypatch.setattr(orc, attr, fn)
    assert caught(monkeypatch), f"no pin caught the planted mistake {name}"


def test_unmutated_oracle_passes_every_pin(monkeypatch):
    assert not caught(monkeypatch)


# ------------------------------------------------------------ serving oracle
# Each mutant is a one-token slip applied to the source text of
# oracle/serve_oracle.py; the mutated module replaces the real one and the
# serving pins run against it.
import inspect
import sys
import types

from oracle import serve_oracle as so
from tests import test_serve_oracle as serve_pins

SERVE_PINS = [
    serve_pins.test_evaluate_golden_two_seeds,
    serve_pins.test_evaluate_single_buyer_reduces_to_layer_formulas,
    serve_pins.test_evaluate_matches_layer_oracle_on_sampled_rows,
    serve_pins.test_splitmix64_published_vectors,
    serve_pins.test_floyd_takes_everything_when_k_equals_n,
    serve_pins.test_adjacency_orders,
]

SERVE_MUTANTS = {
    "user_mean_as_sum": (".sum(axis=0) / k2", ".sum(axis=0)"),
    "layer2_concat_swapped": ("[np.array(u1), np.repeat(i1[None], k1, 0)", "[np.repeat(i1[None], k1, 0), np.array(u1)"),
    "k2_without_min": ("k2 = min(fanout2, du)", "k2 = fanout2"),
    "layer2_bias_dropped": ("_lin(x, W[2], b[2])", "_lin(x, W[2], None)"),
    "item1_cat_of_first_item": ("c = int(item_cat[s])", "c = int(item_cat[0])"),
    "user_layer_no_relu": ("u1.append(np.maximum(_lin(x, W[0], b[0]).sum(axis=0) / k2, 0.0))",
                           "u1.append(_lin(x, W[0], b[0]).sum(axis=0) / k2)"),
}


def _serve_caught():
    for pin in SERVE_PINS:
        try:
            pin()
        except Exception:
            return True
    return False


@pytest.mark.parametrize("name", sorted(SERVE_MUTANTS))
def test_planted_serving_mistake_is_caught(name, monkeypatch):
    old, new = SERVE_MUTANTS[name]
    src = inspect.getsource(so)
    assert src.count(old) == 1, f"mutant {name} no longer matches the oracle's source"
    mod = types.ModuleType("serve_oracle_mutant")
    exec(compile(src.replace(old, new), "<serve_oracle mutant>", "exec"), mod.__dict__)
    for attr in ("mix64", "splitmix64_stream", "stream_base", "draw", "floyd", "adjacency", "evaluate"):
        monkeypatch.setattr(so, attr, getattr(mod, attr))
    assert _serve_caught(), f"no pin caught the planted serving mistake {name}"


def test_unmutated_serving_oracle_passes_every_pin():
    assert not _serve_caught()


# ------------------------------------------------- selection and general joins
# One-token slips in the source text of the join steps and the selection of
# oracle/relnn_oracle.py; the mutated functions replace the real ones and the
# pins of tests/test_oracle_joins.py run against them.
from tests import test_oracle_joins as join_pins

JOIN_PINS = [
    lambda: join_pins.test_selection_matches_nested_loop(0, "sum"),
    lambda: join_pins.test_selection_matches_nested_loop(2, "max"),
    lambda: join_pins.test_selection_matches_nested_loop(4, "mean"),
    join_pins.test_selection_closed_form,
    lambda: join_pins.test_many_to_many_join_matches_nested_loop("sum"),
    join_pins.test_triangle_join_matches_nested_loop,
    join_pins.test_triangle_count_is_diagonal_of_A_cubed,
    join_pins.test_triangle_linear_closed_form,
    join_pins.test_step_with_no_match_and_filter_rejecting_all,
    join_pins.test_filter_applies_to_derived_columns,
]

JOIN_MUTANTS = {
    "step_second_pair_ignored": [("for k in step.key)", "for k in step.key[:1])"),
                                 ("for o in step.on)", "for o in step.on[:1])")],
    "step_rows_in_reverse": [("for k in step.key), []).append(r)", "for k in step.key), []).insert(0, r)")],
    "lt_as_le": [('"lt": np.less,', '"lt": np.less_equal,')],
    "mul_b_sign": [("v = v + p.mul_b *", "v = v - p.mul_b *")],
    "filter_dropped": [('valid &= selection(cols, getattr(rule, "preds", ()))', "valid &= True")],
    "step_matches_any_key": [("rows_of.get(tuple(int(cols[o][i]) for o in step.on), ())",
                              "[r for v in rows_of.values() for r in v]")],
}


def _join_caught():
    for pin in JOIN_PINS:
        try:
            pin()
        except Exception:
            return True
    return False


@pytest.mark.parametrize("name", sorted(JOIN_MUTANTS))
def test_planted_join_mistake_is_caught(name, monkeypatch):
    src = inspect.getsource(orc)
    for old, new in JOIN_MUTANTS[name]:
        assert src.count(old) == 1, f"mutant {name} no longer matches the oracle's source"
        src = src.replace(old, new)
    mod = types.ModuleType("relnn_oracle_mutant")
    monkeypatch.setitem(sys.modules, "relnn_oracle_mutant", mod)      # dataclasses look their module up
    exec(compile(src, "<relnn_oracle mutant>", "exec"), mod.__dict__)
    for attr in ("join_step", "selection", "build_index"):
        monkeypatch.setattr(orc, attr, getattr(mod, attr))
    assert _join_caught(), f"no pin caught the planted join mistake {name}"


def test_unmutated_join_oracle_passes_every_pin():
    assert not _join_caught()


# --------------------------------------------------------- projected union
from tests import test_oracle_union as union_pins

UNION_PINS = [
    lambda: union_pins.test_union_matches_nested_loop("mean", 2),
    lambda: union_pins.test_union_matches_nested_loop("max", 3),
    lambda: union_pins.test_union_matches_nested_loop("sum", 3),
    lambda: union_pins.test_union_of_one_is_the_projection("max"),
    union_pins.test_self_union,
    union_pins.test_mean_is_applied_once_across_relations,
    union_pins.test_keys_are_the_union_of_the_branches,
    union_pins.test_union_rule_transform_after_the_union,
]

UNION_MUTANTS = {
    "mean_of_means": [("pre[q] = y.sum(axis=0) / y.shape[0]",
                       "pre[q] = np.mean([v.mean(axis=0) for v in ys], axis=0)")],
    "keys_intersected": [("keys = sorted(set().union(*", "keys = sorted(set.intersection(*")],
    "max_last_branch_first": [("y = np.concatenate(ys, axis=0)", "y = np.concatenate(ys[::-1], axis=0)")],
    "post_bias_dropped": [("pre @ np.asarray(W_post, np.float64) + (\n        0.0 if b_post is None else np.asarray(b_post, np.float64))",
                           "pre @ np.asarray(W_post, np.float64) + (\n        0.0)")],
}


def _union_caught():
    for pin in UNION_PINS:
        try:
            pin()
        except Exception:
            return True
    return False


@pytest.mark.parametrize("name", sorted(UNION_MUTANTS))
def test_planted_union_mistake_is_caught(name, monkeypatch):
    src = inspect.getsource(orc)
    for old, new in UNION_MUTANTS[name]:
        assert src.count(old) == 1, f"mutant {name} no longer matches the oracle's source"
        src = src.replace(old, new)
    mod = types.ModuleType("relnn_oracle_union_mutant")
    monkeypatch.setitem(sys.modules, "relnn_oracle_union_mutant", mod)
    exec(compile(src, "<relnn_oracle mutant>", "exec"), mod.__dict__)
    monkeypatch.setattr(orc, "union_fwd", mod.union_fwd)
    assert _union_caught(), f"no pin caught the planted union mistake {name}"


def test_unmutated_union_oracle_passes_every_pin():
    assert not _union_caught()


# -------------------------------------------------------- segmented softmax
from tests import test_oracle_attention as attn_pins

ATTN_PINS = [attn_pins.test_golden_forward, attn_pins.test_golden_backward, attn_pins.test_shift_invariance,
             attn_pins.test_special_cases, attn_pins.test_matches_torch_softmax_and_autograd]

ATTN_MUTANTS = {
    "lse_without_max": [("        lse[g] = m + np.log(l)", "        lse[g] = np.log(l)")],
    "softmax_over_heads": [("        l = ex.sum(axis=0)\n", "        l = ex.sum(axis=1, keepdims=True)\n")],
    "scale_dropped": [("    return scale * (qr * kr)", "    return (qr * kr)")],
    "ds_without_centering": [("ds = a * (dp - (a * dp).sum(axis=0))", "ds = a * dp")],
    "dk_from_keys": [("np.add.at(dk, rk, (scale * ds[:, :, None] * Qh)", "np.add.at(dk, rk, (scale * ds[:, :, None] * Kh)")],
    "value_head_misaligned": [("V = v[rv].reshape(n, heads, dv // heads)", "V = v[rv].reshape(n, dv // heads, heads).transpose(0, 2, 1)")],
}


def _attn_caught():
    for pin in ATTN_PINS:
        try:
            pin()
        except Exception:
            return True
    return False


@pytest.mark.parametrize("name", sorted(ATTN_MUTANTS))
def test_planted_attention_mistake_is_caught(name, monkeypatch):
    src = inspect.getsource(orc)
    for old, new in ATTN_MUTANTS[name]:
        assert src.count(old) == 1, f"mutant {name} no longer matches the oracle's source"
        src = src.replace(old, new)
    mod = types.ModuleType("relnn_oracle_attn_mutant")
    monkeypatch.setitem(sys.modules, "relnn_oracle_attn_mutant", mod)
    exec(compile(src, "<relnn_oracle mutant>", "exec"), mod.__dict__)
    monkeypatch.setattr(orc, "attention_fwd", mod.attention_fwd)
    monkeypatch.setattr(orc, "attention_bwd", mod.attention_bwd)
    assert _attn_caught(), f"no pin caught the planted attention mistake {name}"


def test_unmutated_attention_oracle_passes_every_pin():
    assert not _attn_caught()


# --------------------------------------------------------- product transform
from tests import test_oracle_product as prod_pins

PROD_PINS = [lambda: prod_pins.test_product_matches_nested_loop("sum", "none"),
             lambda: prod_pins.test_product_matches_nested_loop("max", "relu"),
             prod_pins.test_product_closed_forms]

PROD_MUTANTS = {
    "product_as_sum": [("        y = y * np.asarray(e)[r[sel]].astype(np.float64)",
                        "        y = y + np.asarray(e)[r[sel]].astype(np.float64)")],
    "product_drops_atoms": [("for e, r in zip(embs[1:], idx.rows[1:]):", "for e, r in zip(embs[1:1], idx.rows[1:1]):")],
    "product_act_pre_ignored": [("    return _act(act_pre, y)\n", "    return y\n")],
}


@pytest.mark.parametrize("name", sorted(PROD_MUTANTS))
def test_planted_product_mistake_is_caught(name, monkeypatch):
    src = inspect.getsource(orc)
    for old, new in PROD_MUTANTS[name]:
        assert src.count(old) == 1, f"mutant {name} no longer matches the oracle's source"
        src = src.replace(old, new)
    mod = types.ModuleType("relnn_oracle_prod_mutant")
    monkeypatch.setitem(sys.modules, "relnn_oracle_prod_mutant", mod)
    exec(compile(src, "<relnn_oracle mutant>", "exec"), mod.__dict__)
    monkeypatch.setattr(orc, "product", mod.product)
    caught = False
    for pin in PROD_PINS:
        try:
            pin()
        except Exception:
            caught = True
            break
    assert caught, f"no pin caught the planted product mistake {name}"


PROD_BWD_PINS = [lambda: prod_pins.test_product_backward_finite_differences("sum", "none"),
                 lambda: prod_pins.test_product_backward_finite_differences("mean", "relu"),
                 lambda: prod_pins.test_product_backward_finite_differences("max", "relu"),
                 prod_pins.test_product_backward_closed_form]

PROD_BWD_MUTANTS = {
    "product_bwd_includes_own_row": [("            if i != j:\n", "            if True:\n")],
    "product_bwd_mask_ignored": [("            dY = dY * _act_grad(act_pre, full)\n", "            dY = dY\n")],
    "product_bwd_mean_undivided": [("        dY = dA[g] / cnt[g][:, None]\n", "        dY = dA[g]\n")],
    "product_bwd_max_unrouted": [("        dY = np.where(np.asarray(argmax)[g] == pos, dA[g], 0.0)\n",
                                  "        dY = dA[g]\n")],
}


@pytest.mark.parametrize("name", sorted(PROD_BWD_MUTANTS))
def test_planted_product_backward_mistake_is_caught(name, monkeypatch):
    src = inspect.getsource(orc.product_bwd)
    for old, new in PROD_BWD_MUTANTS[name]:
        assert src.count(old) == 1, f"mutant {name} no longer matches the oracle's source"
        src = src.replace(old, new)
    ns = dict(orc.__dict__)
    exec(compile(src, "<product_bwd mutant>", "exec"), ns)
    monkeypatch.setattr(orc, "product_bwd", ns["product_bwd"])
    caught = False
    for pin in PROD_BWD_PINS:
        try:
            pin()
        except Exception:
            caught = True
            break
    assert caught, f"no pin caught the planted product-backward mistake {name}"


def test_unmutated_product_backward_passes_every_pin():
    for pin in PROD_BWD_PINS:
        pin()


# ---------------------------------------------------------------------------
# union backward
# ---------------------------------------------------------------------------
from tests import test_oracle_union as union_pins  # noqa: E402

UNION_BWD_PINS = [lambda agg=agg, post=post: union_pins.test_union_backward_finite_differences(agg, post)
                  for agg in ("sum", "mean", "max") for post in (False, True)]
UNION_BWD_PINS += [lambda agg=agg: union_pins.test_union_backward_of_one_is_the_layer_backward(agg)
                   for agg in ("sum", "mean", "max")]
UNION_BWD_PINS += [union_pins.test_self_union_backward, union_pins.test_union_backward_mean_counts_every_relation]

UNION_BWD_MUTANTS = {
    "union_bwd_mean_per_branch_count": [("            dY = dV[t] / members[t][:, None]\n",
                                         "            dY = dV[t] / np.diff(idx.offsets)[idx.tuple_group][:, None]\n")],
    "union_bwd_max_ignores_the_branch": [("            mine = (a[..., 0] == bi) & (a[..., 1] == np.arange(idx.E)[:, None])\n",
                                          "            mine = a[..., 1] == np.arange(idx.E)[:, None]\n")],
    "union_bwd_post_mask_without_bias": [("        u = v @ Wp + (0.0 if b_post is None else np.asarray(b_post, np.float64))\n",
                                          "        u = v @ Wp\n")],
    "union_bwd_db_post_from_dout": [("        db_post = dU.sum(axis=0)\n", "        db_post = dout.sum(axis=0)\n")],
    "union_bwd_act_pre_ignored": [(
        "                dY = dY * _act_grad(act_pre, x @ W64 + (0.0 if b is None else np.asarray(b, np.float64)))\n",
        "                dY = dY\n")],
    "union_bwd_post_mask_ignored": [("        dV = dout * _act_grad(act_post, v)\n", "        dV = dout\n")],
}


@pytest.mark.parametrize("name", sorted(UNION_BWD_MUTANTS))
def test_planted_union_backward_mistake_is_caught(name, monkeypatch):
    src = inspect.getsource(orc.union_bwd)
    for old, new in UNION_BWD_MUTANTS[name]:
        assert src.count(old) == 1, f"mutant {name} no longer matches the oracle's source"
        src = src.replace(old, new)
    ns = dict(orc.__dict__)
    exec(compile(src, "<union_bwd mutant>", "exec"), ns)
    monkeypatch.setattr(orc, "union_bwd", ns["union_bwd"])
    caught = False
    for pin in UNION_BWD_PINS:
        try:
            pin()
        except Exception:
            caught = True
            break
    assert caught, f"no pin caught the planted union-backward mistake {name}"


def test_unmutated_union_backward_passes_every_pin():
    for pin in UNION_BWD_PINS:
        pin()
