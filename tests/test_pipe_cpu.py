"""Pipes without a GPU: the T_control chooser (Section 4.3: the control
kernel's workgroup size is the largest member of the intersection of its
kernels' sets; an empty intersection means no outlining), the constraints the
library's bodies declare, and the structural check of pipe programs."""
import pytest

from paper_1607_05707_amd import irgl

E, S, F = irgl.IRGL_BLOCK_ELASTIC, irgl.IRGL_BLOCK_SHRINKABLE, irgl.IRGL_BLOCK_FIXED
LDS = 65536


def _config_error(fn, *a, **k):
    with pytest.raises(irgl.IrglError) as e:
        fn(*a, **k)
    return e.value.status


def test_chooser_takes_the_largest_common_size():
    assert irgl.irgl_control_block([(E, 0, 0, 0)], LDS) == 1024
    assert irgl.irgl_control_block([(E, 0, 0, 0), (F, 256, 0, 0)], LDS) == 256
    assert irgl.irgl_control_block([(E, 0, 0, 0), (S, 512, 0, 0)], LDS) == 512
    assert irgl.irgl_control_block([(S, 512, 0, 0), (S, 128, 0, 0)], LDS) == 128
    assert irgl.irgl_control_block([(S, 300, 0, 0)], LDS) == 256      # sizes are powers of two
    assert irgl.irgl_control_block([], LDS) == 1024                    # no constraint at all
    # LDS sized by the workgroup bounds the set: 100 B per thread fits 512 of them in 64 KiB
    assert irgl.irgl_control_block([(E, 0, 0, 100)], LDS) == 512
    assert irgl.irgl_control_block([(E, 0, 4097, 60)], LDS) == 512    # 4097 + 60 * 1024 > 64 KiB
    assert irgl.irgl_control_block([(E, 0, 4096, 60)], LDS) == 1024   # exactly 64 KiB fits
    assert irgl.irgl_control_block([(F, 64, 0, 0), (E, 0, 0, 0)], LDS) == 64


def test_chooser_empty_intersection_is_a_config_error():
    assert _config_error(irgl.irgl_control_block, [(F, 256, 0, 0), (S, 128, 0, 0)], LDS) == irgl.IRGL_ERR_CONFIG
    assert _config_error(irgl.irgl_control_block, [(F, 256, 0, 0), (F, 512, 0, 0)], LDS) == irgl.IRGL_ERR_CONFIG
    assert _config_error(irgl.irgl_control_block, [(F, 1024, 0, 100)], LDS) == irgl.IRGL_ERR_CONFIG
    assert _config_error(irgl.irgl_control_block, [(S, 32, 0, 0)], LDS) == irgl.IRGL_ERR_CONFIG
    assert _config_error(irgl.irgl_control_block, [(E, 0, 70000, 0)], LDS) == irgl.IRGL_ERR_CONFIG
    assert _config_error(irgl.irgl_control_block, [(E, 0, 0, 0)], 0) == irgl.IRGL_ERR_INVALID_ARGUMENT


def test_body_constraints_come_from_their_layout():
    push = irgl.irgl_pipe_body_constraint(irgl.IRGL_BODY_BFS_PUSH)
    pull = irgl.irgl_pipe_body_constraint(irgl.IRGL_BODY_BFS_PULL)
    init = irgl.irgl_pipe_body_constraint(irgl.IRGL_BODY_MST_INIT)
    hook = irgl.irgl_pipe_body_constraint(irgl.IRGL_BODY_MST_HOOK)
    # the nested scheduler keeps a gather window per thread and push queues per
    # wavefront: more LDS per thread than a body with push queues alone
    assert push[0] == E and push[3] > pull[3] > 0
    assert init[0] == F and init[1] == 256
    assert hook == (E, 1024, 0, 0)  # no LDS, no worklist
    assert _config_error(irgl.irgl_pipe_body_constraint, irgl.IRGL_BODY_COUNT) == irgl.IRGL_ERR_INVALID_ARGUMENT
    # the batched control kernel's sizes are derived the same way (both bodies
    # run the nested scheduler; its LDS fits every compiled size)
    assert irgl.irgl_control_block_sizes() == [256, 512, 1024]


def test_program_control_block():
    bfs = irgl.pipe_bfs_program()
    mst = irgl.pipe_boruvka_program()
    assert irgl.irgl_pipe_control_block(bfs, lds_limit=LDS) == 1024
    assert irgl.irgl_pipe_control_block(bfs, requested=128, lds_limit=LDS) == 128
    # a smaller LDS: the nested scheduler no longer fits 1024 threads
    push_per_thread = irgl.irgl_pipe_body_constraint(irgl.IRGL_BODY_BFS_PUSH)[3]
    assert irgl.irgl_pipe_control_block(bfs, lds_limit=push_per_thread * 1024 - 1) == 512
    # the Boruvka pipe holds a FixedBlock(256) body
    assert irgl.irgl_pipe_control_block(mst, lds_limit=LDS) == 256
    assert _config_error(irgl.irgl_pipe_control_block, mst, requested=512, lds_limit=LDS) == irgl.IRGL_ERR_CONFIG
    both = mst + [(irgl.IRGL_PIPE_INIT_SOURCE,), (irgl.IRGL_PIPE_INVOKE, irgl.IRGL_BODY_BFS_PUSH)]
    assert irgl.irgl_pipe_control_block(both, lds_limit=LDS) == 256


def test_program_check():
    I, IT, BG, EN, IF, J, SRC = (irgl.IRGL_PIPE_INVOKE, irgl.IRGL_PIPE_ITERATE, irgl.IRGL_PIPE_BEGIN,
                                 irgl.IRGL_PIPE_END, irgl.IRGL_PIPE_IF, irgl.IRGL_PIPE_JUMP,
                                 irgl.IRGL_PIPE_INIT_SOURCE)
    irgl.irgl_pipe_check(irgl.pipe_bfs_program())
    irgl.irgl_pipe_check(irgl.pipe_boruvka_program())
    irgl.irgl_pipe_check([(SRC,), (IT, irgl.IRGL_BODY_BFS_PUSH)])
    irgl.irgl_pipe_check([(BG, 1), (I, irgl.IRGL_BODY_MST_HOOK), (EN,)])  # Pipe Once needs no worklist body
    bad = [
        [(BG, 0), (I, 0)],                                   # unbalanced
        [(EN,)],
        [(BG, 0), (I, irgl.IRGL_BODY_MST_HOOK), (EN,)],     # looping pipe that never changes `in`
        [(SRC,), (J, 0)],                                    # backward jump
        [(SRC,), (IF, 0, 1)],                                # target not forward
        [(SRC,), (IF, 0, 9)],                                # target out of range
        [(SRC,), (IF, 7, 2)],                                # unknown condition
        [(IT, irgl.IRGL_BODY_MST_HOOK)],                     # Iterate of a body that ends neither way
        [(I, 99)],                                           # unknown body
        [(42,)],                                             # unknown statement
        [(BG, 2), (EN,)],                                    # BEGIN neither loop nor once
        [(BG, 1)] * 9 + [(EN,)] * 9,                         # nested deeper than 8
    ]
    for prog in bad:
        assert _config_error(irgl.irgl_pipe_check, prog) == irgl.IRGL_ERR_INVALID_ARGUMENT, prog
