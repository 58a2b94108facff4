"""Error measures and ensemble statistics (oracle).

Test infrastructure (oracle).

- Sec. 4: the space average <f> over all N points, and the averages over the
  boundary set I_B and the interior set I_I; the ensemble average over delay
  realisations.
- Sec. 5.1: the pointwise error E_i^n = u_i^n - u_a(x_i, t_n).

The paper averages the signed error; its plots are on log axes, so this oracle
reports magnitudes instead: mean |E| (L1), root-mean-square E (L2) and
max |E| (Linf), over I, I_B and I_I.
"""
import torch


def error_norms(u, ref, bmask=None):
    e = (u - ref).to(torch.float64)
    out = {
        "l1": float(e.abs().mean()),
        "l2": float(torch.sqrt((e * e).mean())),
        "linf": float(e.abs().max()),
    }
    if bmask is not None:
        eb = e[bmask]
        ei = e[~bmask]
        out["l2_b"] = float(torch.sqrt((eb * eb).mean())) if eb.numel() else 0.0
        out["l2_i"] = float(torch.sqrt((ei * ei).mean())) if ei.numel() else 0.0
        out["l1_b"] = float(eb.abs().mean()) if eb.numel() else 0.0
        out["l1_i"] = float(ei.abs().mean()) if ei.numel() else 0.0
    return out


def ensemble_mean_var(values):
    """Ensemble mean and unbiased variance of a list of per-realisation numbers."""
    v = torch.as_tensor(values, dtype=torch.float64)
    if v.numel() < 2:
        return float(v.mean()), 0.0
    return float(v.mean()), float(v.var(unbiased=True))


def binned_mean_var(dx, values, groups, edges, ngroups=3):
    """Ensemble mean and unbiased variance of per-member values binned by grid
    spacing (Sec. 4 ensemble averages, taken over the members that share a
    range of dx). Member i falls in group groups[i] and in bin j when
    edges[j] <= dx[i] < edges[j + 1]. Returns a list over groups of lists over
    bins of (count, mean dx, mean value, unbiased variance)."""
    out = []
    for g in range(ngroups):
        row = []
        for j in range(len(edges) - 1):
            sel = [i for i in range(len(values)) if groups[i] == g and edges[j] <= dx[i] < edges[j + 1]]
            if not sel:
                row.append((0, 0.0, 0.0, 0.0))
                continue
            m, v = ensemble_mean_var([values[i] for i in sel])
            row.append((len(sel), sum(dx[i] for i in sel) / len(sel), m, v))
        out.append(row)
    return out
