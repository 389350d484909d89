"""The C-ABI library loads and exports every symbol the header declares (CPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2410_08859_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dd_uot.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(dd_uot_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(binding.EXPORTED)


def test_struct_layouts_match_the_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "dd_uot.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(dduot_config),'
                   'sizeof(dduot_iter_stats), sizeof(dduot_score), offsetof(dduot_config, box_cap),'
                   'offsetof(dduot_score, overflow), offsetof(dduot_iter_stats, n_cells),'
                   'sizeof(dduot_multiscale), offsetof(dduot_multiscale, stage_gap),'
                   'offsetof(dduot_multiscale, target_rel_gap));'
                   'printf("%zu %zu %zu ", offsetof(dduot_multiscale, dd_from), '
                   'offsetof(dduot_multiscale, global_tol), offsetof(dduot_multiscale, coarse_lenience));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    got = [int(v) for v in out]
    want = [ctypes.sizeof(binding.dduot_config), ctypes.sizeof(binding.dduot_iter_stats),
            ctypes.sizeof(binding.dduot_score), binding.dduot_config.box_cap.offset,
            binding.dduot_score.overflow.offset, binding.dduot_iter_stats.n_cells.offset,
            ctypes.sizeof(binding.dduot_multiscale), binding.dduot_multiscale.stage_gap.offset,
            binding.dduot_multiscale.target_rel_gap.offset,
            binding.dduot_multiscale.dd_from.offset, binding.dduot_multiscale.global_tol.offset,
            binding.dduot_multiscale.coarse_lenience.offset]
    assert got == want


def test_default_config_values():
    cfg = binding.dd_uot_default_config()
    assert cfg.sinkhorn_err == 2e-5 and cfg.trunc == 1e-15 and cfg.lenience == 0.005
    assert cfg.getweights == binding.GW_SWIFT and cfg.precision == 32 and cfg.translate == 1


@pytest.mark.parametrize("field,value", [("n1", 30), ("cell", 0), ("cell", 9), ("eps", 0.0),
                                         ("lambda_", -1.0), ("precision", 16), ("box_cap", 4),
                                         ("getweights", 7), ("getweights", 6), ("translate", 2),
                                         ("balance", 2)])
def test_invalid_configs_are_rejected_before_any_device_work(field, value):
    import numpy as np
    cfg = binding.dd_uot_default_config(n1=32, n2=32, h=1 / 32, eps=1 / 1024)
    setattr(cfg, field, value)
    n = 32 * 32 if field != "n1" else 30 * 32
    mu = np.full(n, 1.0 / n)
    with pytest.raises(binding.DDUOTError) as e:
        binding.dd_uot_init(cfg, mu, mu.copy())
    assert e.value.code == binding.EINVAL


def test_nonpositive_mass_is_rejected():
    import numpy as np
    cfg = binding.dd_uot_default_config(n1=16, n2=16, h=1 / 16, eps=1 / 256)
    mu = np.full(256, 1.0 / 256)
    nu = mu.copy()
    nu[7] = 0.0
    with pytest.raises(binding.DDUOTError) as e:
        binding.dd_uot_init(cfg, mu, nu)
    assert e.value.code == binding.EINVAL
    nu[7] = np.nan
    with pytest.raises(binding.DDUOTError):
        binding.dd_uot_init(cfg, mu, nu)


def test_balancing_with_moved_points_is_rejected():
    import numpy as np
    cfg = binding.dd_uot_default_config(n1=16, n2=16, h=1 / 16, eps=1 / 256, balance=1)
    mu = np.full(256, 1.0 / 256)
    y = np.stack(np.meshgrid(np.arange(16), np.arange(16), indexing="ij"), -1) / 16.0
    with pytest.raises(binding.DDUOTError) as e:
        binding.dd_uot_init_moved(cfg, mu, mu.copy(), y)
    assert e.value.code == binding.EINVAL
    assert "balancing" in str(e.value)
